/*
 * Runs the oracle's routines under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (built by tests/test_oracle_sanitized.py with gcc; host code
 * only).  Every routine is driven over the paper's worked example (Sec. 3.1
 * to 3.3), brute force over a tiny GF(2^4) code, and random round trips of
 * the benchmark's codes with ragged block sizes; any memory error, undefined
 * behaviour or wrong result ends the program with a non-zero status.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "rs_oracle.h"

static int failures;

#define CHECK(cond, ...)                         \
  do {                                           \
    if (!(cond)) {                               \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      fprintf(stderr, __VA_ARGS__);              \
      fputc('\n', stderr);                       \
      ++failures;                                \
    }                                            \
  } while (0)

static unsigned rnd_state = 0x13125155u;
static unsigned rnd(void) {   /* xorshift32: deterministic test data */
  rnd_state ^= rnd_state << 13;
  rnd_state ^= rnd_state >> 17;
  rnd_state ^= rnd_state << 5;
  return rnd_state;
}

/* t distinct indices below n */
static void pick(int n, int t, int *out) {
  for (int i = 0; i < t;) {
    int x = (int)(rnd() % (unsigned)n), dup = 0;
    for (int j = 0; j < i; ++j) dup |= out[j] == x;
    if (!dup) out[i++] = x;
  }
}

static void worked_example(void) {
  rso_field F;
  CHECK(rso_field_init(&F, 8, 0x11D) == 0, "field 0x11D");
  CHECK(rso_alpha_pow(&F, 8) == 29 && rso_alpha_pow(&F, 10) == 116, "alpha^8, alpha^10");
  uint8_t g[4];
  CHECK(rso_genpoly(&F, 3, g) == 0, "genpoly");
  CHECK(g[0] == 8 && g[1] == 14 && g[2] == 7 && g[3] == 1, "g = (8,14,7,1)");
  const uint8_t data[4] = {48, 6, 112, 70};
  uint8_t par[3];
  CHECK(rso_encode(&F, 4, 3, data, par, 1) == 0, "encode");
  CHECK(par[0] == 243 && par[1] == 125 && par[2] == 142, "parity (243,125,142)");
  uint8_t word[7] = {48, 6, 112, 70, 243, 125, 142};
  const int er[3] = {0, 1, 2};
  uint8_t S[3], V[9], Vi[9];
  CHECK(rso_syndromes(&F, 4, 3, word, er, 3, S) == 0, "syndromes");
  CHECK(S[0] == 70 && S[1] == 91 && S[2] == 171, "S = (70,91,171)");
  CHECK(rso_vandermonde(&F, 4, 3, er, 3, V) == 0, "vandermonde");
  const uint8_t Vp[9] = {1, 1, 1, 8, 16, 32, 64, 29, 116};
  CHECK(memcmp(V, Vp, 9) == 0, "printed V");
  CHECK(rso_invert(&F, 3, V, Vi) == 0, "invert");
  memset(word, 0, 3);
  CHECK(rso_decode(&F, 4, 3, word, 1, er, 3) == 0, "decode");
  CHECK(word[0] == 48 && word[1] == 6 && word[2] == 112, "recovered (48,6,112)");
}

/* Every data vector and every erasure pattern of RS(2,2) over GF(2^4). */
static void brute_force_gf16(void) {
  rso_field F;
  CHECK(rso_field_init(&F, 4, 0x13) == 0, "field 0x13");
  const int k = 2, m = 2, n = 4;
  for (int v = 0; v < 256; ++v) {
    uint8_t blocks[4];
    blocks[0] = (uint8_t)(v & 15);
    blocks[1] = (uint8_t)(v >> 4);
    CHECK(rso_encode(&F, k, m, blocks, blocks + k, 1) == 0, "encode gf16");
    for (int mask = 0; mask < (1 << n); ++mask) {
      int er[4], t = 0;
      for (int b = 0; b < n; ++b)
        if (mask >> b & 1) er[t++] = b;
      if (t > m) continue;
      uint8_t w[4];
      memcpy(w, blocks, 4);
      for (int i = 0; i < t; ++i) w[er[i]] = 0x0F;
      CHECK(rso_decode(&F, k, m, w, 1, er, t) == 0, "decode gf16");
      CHECK(memcmp(w, blocks, 4) == 0, "gf16 v=%d mask=%d", v, mask);
    }
  }
}

/* Encode, linearity, and decode round trips of random stripes. */
static void round_trips(int k, int m, size_t B, int trials) {
  rso_field F;
  rso_field_init(&F, 8, 0x11D);
  const int n = k + m;
  uint8_t *a = malloc((size_t)n * B), *b = malloc((size_t)n * B), *c = malloc((size_t)n * B);
  uint8_t *w = malloc((size_t)n * B);
  for (size_t i = 0; i < (size_t)k * B; ++i) {
    a[i] = (uint8_t)rnd();
    b[i] = (uint8_t)rnd();
    c[i] = a[i] ^ b[i];
  }
  CHECK(rso_encode(&F, k, m, a, a + (size_t)k * B, B) == 0, "encode a");
  CHECK(rso_encode(&F, k, m, b, b + (size_t)k * B, B) == 0, "encode b");
  CHECK(rso_encode(&F, k, m, c, c + (size_t)k * B, B) == 0, "encode a^b");
  for (size_t i = (size_t)k * B; i < (size_t)n * B; ++i)
    CHECK((a[i] ^ b[i]) == c[i], "linearity RS(%d,%d) at %zu", k, m, i);
  for (int tr = 0; tr < trials; ++tr) {
    int er[RSO_MAX_M];
    const int t = 1 + (int)(rnd() % (unsigned)m);
    pick(n, t, er);
    memcpy(w, a, (size_t)n * B);
    for (int i = 0; i < t; ++i) memset(w + (size_t)er[i] * B, 0xA5, B);
    CHECK(rso_decode(&F, k, m, w, B, er, t) == 0, "decode RS(%d,%d)", k, m);
    CHECK(memcmp(w, a, (size_t)n * B) == 0, "round trip RS(%d,%d) t=%d", k, m, t);
  }
  /* rejected arguments stay rejected without touching memory */
  int bad[2] = {0, 0};
  CHECK(rso_decode(&F, k, m, w, B, bad, 2) != 0 || m < 2, "duplicate erasure");
  int over[RSO_MAX_M + 1];
  for (int i = 0; i <= m; ++i) over[i] = i;
  CHECK(rso_decode(&F, k, m, w, B, over, m + 1) != 0, "t > m");
  free(a);
  free(b);
  free(c);
  free(w);
}

int main(void) {
  worked_example();
  brute_force_gf16();
  round_trips(6, 3, 1001, 40);
  round_trips(10, 4, 4097, 20);
  round_trips(12, 4, 333, 20);
  round_trips(32, 8, 2049, 10);
  round_trips(247, 8, 17, 5);
  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("oracle sanitized run: ok\n");
  return 0;
}
