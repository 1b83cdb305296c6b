/*
 * Plain CPU oracle for polynomial Reed-Solomon RS(k,m) over GF(2^w).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the GPU path.
 *
 * Every routine is the literal definition from the paper, written for a
 * reader to check by eye, with no blocking, fusion or reordering:
 *   - field:   powers of the primitive root alpha = 2 by repeated
 *              multiplication by x with reduction (Sec. 3.1 example; Sec. 5.1
 *              says multiplication/division tables are precomputed), plus a
 *              full product table built by shift-and-add, independently of
 *              the power table;
 *   - g(x):    product of (x + alpha^i), i = 0..m-1 (Sec. 3.1);
 *   - encode:  parity = x^m d(x) mod g(x) by schoolbook long division, one
 *              byte column (codeword) at a time (Sec. 3.2, eq. (1)-(2));
 *   - decode:  step 1 evaluates the received word with the erased symbols
 *              dropped at alpha^0..alpha^(t-1) over all n-t survivors (Sec.
 *              3.3 step 1, with Opt2 of Sec. 4: erased indexes are skipped);
 *              step 2 solves the t x t Vandermonde system, inverted once per
 *              erasure pattern by Gauss-Jordan elimination (Sec. 3.3 step 2,
 *              Opt3 of Sec. 4).
 *
 * Codeword layout (Sec. 3.2, eq. (2)): parity p_i is the coefficient of x^i
 * (0 <= i < m) and data d_j the coefficient of x^(m+j) (0 <= j < k).
 * API block order: block b < k is d_b, block b >= k is p_(b-k).
 * Symbols are stored one per byte, also for w = 4 (low nibble).
 */
#include "rs_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- field -- */

/* Carry-less product of a and b reduced modulo the field polynomial, done the
 * schoolbook way: add a shifted copy of a for every set bit of b, reducing a
 * by the field polynomial whenever its degree reaches w. */
static int slow_mul(int w, unsigned poly, int a, int b)
{
    int q = 1 << w;
    int acc = 0;
    for (int bit = 0; bit < w; bit++) {
        if (b & (1 << bit))
            acc ^= a;
        a <<= 1;                 /* a := a * x */
        if (a & q)
            a ^= (int)poly;      /* reduce: x^w = (poly - x^w) */
    }
    return acc;
}

int rso_field_init(rso_field *F, int w, unsigned poly)
{
    if (!F || (w != 4 && w != 8))
        return -1;
    int q = 1 << w;
    if ((poly >> w) != 1u)       /* the polynomial must have degree exactly w */
        return -1;
    memset(F, 0, sizeof(*F));
    F->w = w;
    F->poly = poly;
    F->q = q;
    F->order = q - 1;

    /* alpha^e for e = 0 .. q-2 by repeated multiplication by alpha = x. */
    for (int e = 0; e < q; e++)
        F->log[e] = -1;
    int v = 1;
    for (int e = 0; e < q - 1; e++) {
        if (F->log[v] != -1)     /* a power repeated early: x is not primitive */
            return -1;
        F->exp[e] = (uint8_t)v;
        F->log[v] = e;
        v <<= 1;
        if (v & q)
            v ^= (int)poly;
    }
    if (v != 1)                  /* alpha^(q-1) must come back to 1 */
        return -1;

    /* Full product table, built without the power table. */
    for (int a = 0; a < q; a++)
        for (int b = 0; b < q; b++)
            F->mul[a][b] = (uint8_t)slow_mul(w, poly, a, b);
    return 0;
}

uint8_t rso_mul(const rso_field *F, uint8_t a, uint8_t b)
{
    return F->mul[a][b];
}

uint8_t rso_alpha_pow(const rso_field *F, long e)
{
    long r = e % F->order;
    if (r < 0)
        r += F->order;
    return F->exp[r];
}

/* Multiplicative inverse by search in the product table: the element b with
 * a*b = 1.  a must be nonzero. */
static uint8_t inv(const rso_field *F, uint8_t a)
{
    for (int b = 1; b < F->q; b++)
        if (F->mul[a][b] == 1)
            return (uint8_t)b;
    return 0;
}

/* ----------------------------------------------------- generator g(x) -- */

int rso_genpoly(const rso_field *F, int m, uint8_t *g)
{
    if (!F || !g || m < 1 || m >= F->q)
        return -1;
    /* g := 1 */
    memset(g, 0, (size_t)m + 1);
    g[0] = 1;
    int deg = 0;
    /* g := g * (x + alpha^i) for i = 0 .. m-1 */
    for (int i = 0; i < m; i++) {
        uint8_t root = rso_alpha_pow(F, i);
        uint8_t next[RSO_MAX_N + 1];
        memset(next, 0, sizeof(next));
        for (int d = 0; d <= deg; d++) {
            next[d + 1] ^= g[d];                       /* g_d * x       */
            next[d] ^= rso_mul(F, g[d], root);         /* g_d * alpha^i */
        }
        deg++;
        memcpy(g, next, (size_t)deg + 1);
    }
    return 0;
}

/* --------------------------------------------------------------- encode -- */

static int check_code(const rso_field *F, int k, int m)
{
    if (!F || k < 1 || m < 1 || k + m > F->order || k + m > RSO_MAX_N)
        return -1;
    return 0;
}

int rso_encode(const rso_field *F, int k, int m, const uint8_t *data,
               uint8_t *parity, size_t B)
{
    if (check_code(F, k, m) != 0 || (!data && B) || (!parity && B))
        return -1;
    uint8_t g[RSO_MAX_N + 1];
    rso_genpoly(F, m, g);
    int n = k + m;
    uint8_t c[RSO_MAX_N];
    for (size_t col = 0; col < B; col++) {
        /* c(x) = x^m d(x): d_j sits on degree m + j, degrees below m are 0. */
        memset(c, 0, sizeof(c));
        for (int j = 0; j < k; j++)
            c[m + j] = data[(size_t)j * B + col];
        /* Long division by the monic g(x): cancel the leading coefficient
         * from the top degree down to degree m. */
        for (int deg = n - 1; deg >= m; deg--) {
            uint8_t f = c[deg];
            if (f == 0)
                continue;
            for (int i = 0; i <= m; i++)
                c[deg - m + i] ^= rso_mul(F, f, g[i]);
        }
        /* The remainder's coefficients are the parity symbols. */
        for (int i = 0; i < m; i++)
            parity[(size_t)i * B + col] = c[i];
    }
    return 0;
}

/* --------------------------------------------------------------- decode -- */

int rso_position(int k, int m, int b)
{
    return b < k ? m + b : b - k;
}

static int check_erasures(int n, int m, const int *erasures, int t)
{
    if (t < 0 || t > m || (t > 0 && !erasures))
        return -1;
    for (int a = 0; a < t; a++) {
        if (erasures[a] < 0 || erasures[a] >= n)
            return -1;
        for (int b = 0; b < a; b++)
            if (erasures[a] == erasures[b])
                return -1;
    }
    return 0;
}

int rso_vandermonde(const rso_field *F, int k, int m, const int *erasures,
                    int t, uint8_t *V)
{
    if (check_code(F, k, m) != 0 || check_erasures(k + m, m, erasures, t) != 0)
        return -1;
    /* Row i holds alpha^(i * pos(e_j)): the coefficient of the unknown symbol
     * e_j in D(alpha^i). */
    for (int i = 0; i < t; i++)
        for (int j = 0; j < t; j++)
            V[i * t + j] = rso_alpha_pow(F, (long)i * rso_position(k, m, erasures[j]));
    return 0;
}

int rso_invert(const rso_field *F, int t, const uint8_t *A, uint8_t *Ainv)
{
    uint8_t M[RSO_MAX_M][2 * RSO_MAX_M];
    if (t < 0 || t > RSO_MAX_M)
        return -1;
    /* Augment [A | I] and reduce A to I by Gauss-Jordan elimination. */
    for (int i = 0; i < t; i++)
        for (int j = 0; j < 2 * t; j++)
            M[i][j] = j < t ? A[i * t + j] : (uint8_t)(j - t == i);
    for (int col = 0; col < t; col++) {
        int piv = -1;
        for (int r = col; r < t; r++)
            if (M[r][col] != 0) {
                piv = r;
                break;
            }
        if (piv < 0)
            return -1;           /* singular */
        if (piv != col)
            for (int j = 0; j < 2 * t; j++) {
                uint8_t tmp = M[col][j];
                M[col][j] = M[piv][j];
                M[piv][j] = tmp;
            }
        uint8_t s = inv(F, M[col][col]);
        for (int j = 0; j < 2 * t; j++)
            M[col][j] = rso_mul(F, M[col][j], s);
        for (int r = 0; r < t; r++) {
            if (r == col || M[r][col] == 0)
                continue;
            uint8_t f = M[r][col];
            for (int j = 0; j < 2 * t; j++)
                M[r][j] ^= rso_mul(F, f, M[col][j]);
        }
    }
    for (int i = 0; i < t; i++)
        for (int j = 0; j < t; j++)
            Ainv[i * t + j] = M[i][t + j];
    return 0;
}

int rso_syndromes(const rso_field *F, int k, int m, const uint8_t *word,
                  const int *erasures, int t, uint8_t *S)
{
    if (check_code(F, k, m) != 0 || check_erasures(k + m, m, erasures, t) != 0)
        return -1;
    int n = k + m;
    for (int i = 0; i < t; i++) {
        uint8_t acc = 0;
        for (int b = 0; b < n; b++) {
            int erased = 0;
            for (int a = 0; a < t; a++)
                if (erasures[a] == b)
                    erased = 1;
            if (erased)
                continue;        /* Opt2: no product for an erased index */
            long e = (long)i * rso_position(k, m, b);
            acc ^= rso_mul(F, word[b], rso_alpha_pow(F, e));
        }
        S[i] = acc;
    }
    return 0;
}

int rso_decode(const rso_field *F, int k, int m, uint8_t *blocks, size_t B,
               const int *erasures, int t)
{
    if (check_code(F, k, m) != 0 || check_erasures(k + m, m, erasures, t) != 0)
        return -1;
    if (t == 0 || B == 0)
        return 0;
    if (!blocks)
        return -1;
    int n = k + m;
    uint8_t V[RSO_MAX_M * RSO_MAX_M], Vinv[RSO_MAX_M * RSO_MAX_M];
    rso_vandermonde(F, k, m, erasures, t, V);
    if (rso_invert(F, t, V, Vinv) != 0)
        return -1;
    uint8_t word[RSO_MAX_N], S[RSO_MAX_M];
    for (size_t col = 0; col < B; col++) {
        for (int b = 0; b < n; b++)
            word[b] = blocks[(size_t)b * B + col];
        rso_syndromes(F, k, m, word, erasures, t, S);
        /* lost = V^-1 S */
        for (int j = 0; j < t; j++) {
            uint8_t acc = 0;
            for (int i = 0; i < t; i++)
                acc ^= rso_mul(F, Vinv[j * t + i], S[i]);
            blocks[(size_t)erasures[j] * B + col] = acc;
        }
    }
    return 0;
}
