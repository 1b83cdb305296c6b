/*
 * Plain CPU oracle for polynomial Reed-Solomon RS(k,m) over GF(2^w).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark to check the GPU library.  The product
 * library never includes, links or calls it, and it includes nothing of the
 * product.  See rs_oracle.c for what each routine follows in the paper.
 *
 * All buffers are host memory.  Blocks are stored one after another with a
 * stride of B bytes: data[j*B + c] is byte column c of data block d_j.
 * Return value 0 is success, -1 a rejected argument.
 */
#ifndef RS_ORACLE_H
#define RS_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSO_MAX_N 255   /* n = k + m must stay below the multiplicative order */
#define RSO_MAX_M 16

typedef struct rso_field {
    int w;              /* 4 or 8 */
    unsigned poly;      /* full field polynomial, bit w set (0x11D, 0x13, ...) */
    int q;              /* 2^w */
    int order;          /* 2^w - 1, the multiplicative order of alpha */
    uint8_t exp[256];   /* exp[e] = alpha^e, 0 <= e < order */
    int log[256];       /* log[alpha^e] = e; log[0] = -1 */
    uint8_t mul[256][256];
} rso_field;

/* Builds the field; fails if poly has not degree w or x is not primitive. */
int rso_field_init(rso_field *F, int w, unsigned poly);
uint8_t rso_mul(const rso_field *F, uint8_t a, uint8_t b);
uint8_t rso_alpha_pow(const rso_field *F, long e);

/* g[0..m] = coefficients of prod_{i<m} (x + alpha^i), low degree first. */
int rso_genpoly(const rso_field *F, int m, uint8_t *g);

/* parity[i*B + c] = coefficient i of x^m d(x) mod g(x) for column c. */
int rso_encode(const rso_field *F, int k, int m, const uint8_t *data,
               uint8_t *parity, size_t B);

/* Degree of API block b in the codeword polynomial. */
int rso_position(int k, int m, int b);

/* V[i*t + j] = alpha^(i * pos(e_j)). */
int rso_vandermonde(const rso_field *F, int k, int m, const int *erasures,
                    int t, uint8_t *V);

/* Ainv = A^-1 for a t x t matrix (row-major); -1 if singular. */
int rso_invert(const rso_field *F, int t, const uint8_t *A, uint8_t *Ainv);

/* S[i] = sum over surviving blocks b of word[b] * alpha^(i*pos(b)), i < t:
 * the paper's step-1 values D(alpha^i) for one codeword (word[b] = symbol of
 * API block b; erased entries are ignored). */
int rso_syndromes(const rso_field *F, int k, int m, const uint8_t *word,
                  const int *erasures, int t, uint8_t *S);

/* Rebuilds, in place, the t erased blocks of blocks[0 .. (k+m)*B). */
int rso_decode(const rso_field *F, int k, int m, uint8_t *blocks, size_t B,
               const int *erasures, int t);

#ifdef __cplusplus
}
#endif

#endif
