/*
 * rs_poly.h -- C ABI of librs_poly.so: polynomial (generator-polynomial)
 * Reed-Solomon RS(k,m) erasure coding over GF(2^w) on AMD Instinct MI355X
 * (gfx950).
 *
 * The operations follow the paper "On the Effectiveness of Polynomial
 * Realization of Reed-Solomon Codes for Storage Systems" (Sheykh Esmaili,
 * Datta):
 *   - Sec. 1: an object of k symbols is encoded into n = k + m blocks so that
 *     any k of the n blocks recreate it; symbols live in GF(2^w);
 *   - Sec. 3.1: g(x) = (x + alpha^0)(x + alpha^1)...(x + alpha^(m-1)), with
 *     primitive root alpha = 2;
 *   - Sec. 3.2, eq. (1)-(2): the parity symbols are the coefficients of
 *     x^m d(x) mod g(x), data symbol d_j on degree m+j, parity p_i on degree i;
 *   - Sec. 3.3: decoding evaluates the received word, erasures dropped, at
 *     the roots of g (step 1) and solves the Vandermonde system in the erased
 *     symbols (step 2), with the matrix inverted once per erasure pattern
 *     (Opt3 of Sec. 4).
 *
 * Stripe and block layout.  A stripe is n blocks of block_bytes bytes each.
 * Byte column c of the stripe (byte c of every block) is one codeword.  The
 * API numbers blocks 0..n-1: block b < k is data d_b, block b >= k is parity
 * p_(b-k).  Symbols are stored one per byte; for w = 4 only the low nibble is
 * used and the high nibble must be zero (other bytes give unspecified output
 * but are memory-safe).
 *
 * Memory and ownership.  Block pointers are DEVICE pointers (e.g. from
 * hipMalloc or torch.empty(..., device="cuda").data_ptr()) on the device that
 * is current when the call is made; the arrays holding them are HOST arrays
 * read during the call only.  The caller owns every block buffer.  The
 * library owns the code handle and everything hung off it (tables, the
 * per-erasure-pattern coefficient cache, batch descriptors, graphs), released
 * by the matching *_free call.  Full speed needs 16-byte-aligned block
 * pointers and block sizes that are a multiple of 16.  The one-stripe
 * encode, decode and update accept any alignment and size (smaller
 * alignments take slower load paths); the batch calls and the bit-sliced
 * encode require 16-byte-aligned pointers (any size).
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the legacy
 * default stream).  Encode and decode are asynchronous: they enqueue work on
 * `stream` and return; results are valid once the stream has synchronized.
 * A handle may be used from several host threads; calls are serialized
 * inside the library.
 *
 * Errors.  Every call returns 0 (RS_OK) or a negative RS_E* code.  Arguments
 * are validated on the host before any HIP call is made, so a rejected call
 * has no effect.  RS_EDEVICE reports a HIP runtime error; an asynchronous
 * device fault of earlier work can surface as RS_EDEVICE on a later call.
 */
#ifndef RS_POLY_H
#define RS_POLY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RS_POLY_MAX_M 8      /* most parity blocks a code may have        */
#define RS_POLY_MAX_N 255    /* n = k + m must stay below 2^w (Sec. 1)     */

/* Status codes. */
#define RS_OK         0
#define RS_EINVAL    -1   /* bad k, m, w, field polynomial, flags or size  */
#define RS_ERANGE    -2   /* erasure index outside [0,n) or repeated       */
#define RS_ETOOMANY  -3   /* more erasures than parity blocks (t > m)      */
#define RS_ENULL     -4   /* a required pointer is NULL                    */
#define RS_EDEVICE   -5   /* HIP runtime error                             */
#define RS_ENOMEM    -6   /* host or device allocation failed              */
#define RS_EBUSY     -7   /* resource in use (e.g. a full serving queue)   */

/* Decode flag: read every surviving block (n - t of them) instead of the
 * minimum k.  Sec. 3.3 remarks that decoding may use more than k survivors;
 * the output is identical, only the bytes read differ. */
#define RS_POLY_FLAG_ALL_SURVIVORS 1u

typedef struct rs_poly rs_poly_t;

/* Creates a code handle for RS(k,m) over GF(2^w).  Host only: no HIP call is
 * made, no device memory is allocated.
 *   k          data blocks, k >= 1
 *   m          parity blocks, 1 <= m <= RS_POLY_MAX_M
 *   w          symbol width in bits, 4 or 8
 *   prim_poly  field polynomial with bit w set, e.g. 0x11D (w=8) or 0x13 (w=4);
 *              it must be primitive, i.e. alpha = 2 = x generates the field
 *              (the Sec. 3.1 example takes 2 as the primitive root)
 *   out        receives the handle
 * Errors: RS_ENULL (out), RS_EINVAL (k, m, w or prim_poly, or k+m > 2^w - 1:
 * the n positions alpha^pos must be distinct), RS_ENOMEM. */
int rs_poly_init(int k, int m, int w, unsigned prim_poly, rs_poly_t **out);

/* Releases the handle and everything it owns.  Waits for nothing: the
 * caller must not free a handle with its work still queued.  NULL is a
 * no-op. */
void rs_poly_free(rs_poly_t *h);

/* Static message for a status code; never NULL. */
const char *rs_poly_strerror(int err);

/* Copies the m+1 coefficients of g(x) (Sec. 3.1), low degree first, into g.
 * Host only.  Errors: RS_ENULL. */
int rs_poly_generator(const rs_poly_t *h, uint8_t *g);

/* Encode (Sec. 3.2, eq. (1)-(2)): for every byte column c < block_bytes,
 * parity[i][c] = coefficient i of x^m * sum_j data[j][c] x^j mod g(x).
 *   data     host array of k device pointers to the data blocks (read only)
 *   parity   host array of m device pointers to the parity blocks (written)
 *   block_bytes  bytes per block; 0 is a successful no-op
 * Parity buffers must not overlap data buffers.
 * Errors: RS_ENULL (h, data, parity, or any of their entries), RS_EDEVICE. */
int rs_poly_encode(rs_poly_t *h, const uint8_t *const *data,
                   uint8_t *const *parity, size_t block_bytes, void *stream);

/* Encode in bit-matrix (XOR-only) form, the multiplication-free direction
 * that Sec. 6 proposes: the same parity bytes as rs_poly_encode, computed as
 * parity p_i = sum_j c_ij d_j with c_ij the coefficient of x^i in
 * x^(m+j) mod g(x) (the generator-matrix columns of Sec. 6), where each
 * product by c_ij is an 8 x 8 matrix over GF(2) applied to the bit planes
 * of the data bytes.  Codes with k <= 32 run, over either field: for
 * RS(6,3), RS(10,4), RS(12,4) and RS(32,8) over GF(2^8) with polynomial
 * 0x11D the XOR networks are compiled into straight-line code; every other
 * code takes its matrices at run time (8 masked XORs per matrix row).
 *   data, parity, block_bytes  as rs_poly_encode; every pointer must be
 *            16-byte aligned (any block_bytes)
 * Errors: RS_ENULL (h, data, parity, or an entry), RS_EINVAL (k > 32, or a
 * pointer not 16-byte aligned), RS_EDEVICE. */
int rs_poly_encode_bitmatrix(rs_poly_t *h, const uint8_t *const *data,
                             uint8_t *const *parity, size_t block_bytes, void *stream);

/* 1 if rs_poly_encode_bitmatrix runs the code (k, m) over GF(2^w) with
 * polynomial prim_poly (a code rs_poly_init accepts, with k <= 32), else 0.
 * Host only. */
int rs_poly_bitmatrix_supported(int k, int m, int w, unsigned prim_poly);

/* Encode in generator-matrix form (Sec. 6): the same parity bytes as
 * rs_poly_encode, computed as p = sum_j P[:, j] d_j with column P[:, j] the
 * remainder of x^(m+j) mod g(x), one packed table lookup per data block and
 * column and no serial LFSR chain.  Codes with k <= 8 run the kernel of
 * rs_poly_update's matrix form (the k tables share one LDS row set),
 * updating zero parity by the data; codes with 8 < k <= 32
 * (RS_POLY_MATRIX_MAX_K) a wide form whose 32 tables fill two LDS regions.
 *   data, parity, block_bytes  as rs_poly_encode (any alignment)
 * Errors: RS_ENULL (h, data, parity, or an entry), RS_EINVAL (k > 32),
 * RS_EDEVICE. */
#define RS_POLY_MATRIX_MAX_K 32
int rs_poly_encode_matrix(rs_poly_t *h, const uint8_t *const *data,
                          uint8_t *const *parity, size_t block_bytes, void *stream);

/* Delta-parity update (the update property of Sec. 3.2): encoding is
 * linear, so when data blocks change, the parity of the new data is the old
 * parity plus the encoding of the data difference.  For every byte column c,
 *     parity[i][c] ^= coefficient i of x^m * sum_j delta[j][c] x^j mod g(x),
 * in one pass that reads the delta blocks and the parity and writes the
 * parity in place.  Up to 8 changed blocks use the generator-matrix columns
 * x^(m+j) mod g(x) of Sec. 6 (one table lookup per changed block); more use
 * the encode LFSR.  Both give the same bytes.
 *   delta    host array of k device pointers; delta[j] is the XOR of new and
 *            old data block j (read only), or NULL for an unchanged block,
 *            which is not read.  All NULL is a successful no-op.
 *   parity   host array of m device pointers to the current parity blocks
 *            (read and overwritten)
 *   block_bytes  bytes per block; 0 is a successful no-op
 * Applying the same delta twice restores the parity.  Parity buffers must
 * not overlap delta buffers or each other.
 * Errors: RS_ENULL (h, delta, parity, or a parity entry), RS_EDEVICE. */
int rs_poly_update(rs_poly_t *h, const uint8_t *const *delta,
                   uint8_t *const *parity, size_t block_bytes, void *stream);

/* The same delta-parity update as rs_poly_update (Sec. 3.2 update property,
 * generator-matrix columns of Sec. 6), computed with the split-nibble
 * multiply held in registers instead of LDS tables: per changed block j and
 * parity i, P[i][j] * x = P[i][j] * (x & 15) ^ P[i][j] * (x & 0xF0), each a
 * 16-entry table looked up 4 bytes at a time.  No LDS, no transposes; one
 * pass reading the changed blocks and the parity, writing the parity.
 *   delta, parity, block_bytes, stream  as for rs_poly_update
 * Limits: 1 or 2 changed (non-NULL) delta blocks with (changed * m) <= 8;
 * every changed delta block and every parity block 16-byte aligned (any
 * block_bytes: the last block_bytes mod 16 bytes are done byte by byte).
 * No changed block, or block_bytes = 0, is a successful no-op.
 * Errors: RS_ENULL (h, delta, parity, or a parity entry), RS_EINVAL (more
 * changed blocks or products than the limits, or an unaligned pointer),
 * RS_EDEVICE. */
int rs_poly_update_nibble(rs_poly_t *h, const uint8_t *const *delta,
                          uint8_t *const *parity, size_t block_bytes, void *stream);

/* Erasure decode (Sec. 3.3): rebuilds, in place, exactly the blocks named in
 * erasures[0..n_erasures), data or parity, from the surviving blocks.
 *   blocks      host array of n = k+m device pointers, API block order
 *   erasures    API indices of the lost blocks, any order, no repeats
 *   n_erasures  t, 0 <= t <= m; t = 0 is a successful no-op
 *   flags       0 or RS_POLY_FLAG_ALL_SURVIVORS
 * Erased buffers are outputs only and are never read.  By default the
 * library reads the k survivors of lowest degree in the code polynomial
 * (every surviving parity block, p_i at degree i, then the surviving data
 * blocks from d_0 up, d_j at degree m + j) and leaves the other m - t
 * surviving blocks, the highest data blocks, unread; their pointers may then
 * be NULL.  The LFSR starts at the highest data block read, so the unread
 * blocks cost neither traffic nor steps.
 * Errors: RS_ENULL, RS_EINVAL (n_erasures < 0, unknown flags),
 * RS_ETOOMANY (t > m), RS_ERANGE, RS_EDEVICE. */
int rs_poly_decode(rs_poly_t *h, uint8_t *const *blocks, size_t block_bytes,
                   const int *erasures, int n_erasures, unsigned flags,
                   void *stream);

/* Host-only view of the decode plan for an erasure pattern (the per-pattern
 * coefficients of Sec. 3.3 step 2, cached as Opt3 of Sec. 4 describes).
 *   read_set   receives the API indices of the blocks decode reads, in
 *              increasing order (capacity n); may be NULL
 *   n_read     receives their count; may be NULL
 *   coeffs     receives the t x m matrix C (row-major): rebuilt symbol e is
 *              sum_l C[e][l] * r_l, where r(x) = sum_l r_l x^l is the received
 *              word (erased and unread symbols set to 0) reduced mod g(x);
 *              may be NULL
 * Errors: as rs_poly_decode's validation. */
int rs_poly_decode_plan(rs_poly_t *h, const int *erasures, int n_erasures,
                        unsigned flags, int *read_set, int *n_read,
                        uint8_t *coeffs);

/* Measurement probe, not coding: streams `stripes` stripes of n_in input
 * and n_out output blocks of block_bytes each, block b of stripe s at
 * base + s * stripe_stride + b * block_stride (inputs b < n_in, outputs
 * n_in .. n_in + n_out - 1), reading every input byte once and writing
 * every output byte once (each output is the XOR of the inputs), with the
 * codec kernels' 16-byte non-temporal accesses and walks over column tiles
 * of tile_bytes (tile_order as in rs_poly_launch_t), but no table lookups.  Its rate is the HBM bandwidth this
 * part achieves for the read:write mix of an encode (n_in = k, n_out = m)
 * or a decode (k, t): the achievable roof beside the nominal peak.
 *   base        device pointer, 16-byte aligned; the caller owns the memory
 *               (outputs are overwritten)
 *   strides     multiples of 16; blocks and stripes must not overlap:
 *               block_bytes <= block_stride, (n_in + n_out) * block_stride
 *               <= stripe_stride
 *   n_in        0..RS_POLY_MAX_N;  n_out 0..RS_POLY_MAX_M, not both 0
 *               (n_out = 0 only reads, n_in = 0 only writes zeros: the
 *               rates of pure reads and pure writes)
 *   block_bytes multiple of 16, at most 2^31
 *   tile_bytes  columns per tile: a multiple of 16, >= 4096
 *   tile_order  0 or 1
 * Asynchronous on `stream`.  Errors: RS_ENULL, RS_EINVAL, RS_EDEVICE. */
int rs_poly_stream_probe(uint8_t *base, size_t stripe_stride, size_t block_stride,
                         int stripes, int n_in, int n_out, size_t block_bytes,
                         int tile_bytes, int tile_order, void *stream);

/* ------------------------------------------------------------ batches --
 *
 * Many stripes -- uneven block sizes, different codes -- go through ONE
 * persistent kernel launch per state width (codes with m <= 4, and codes
 * with 4 < m <= 8), replayed from a hipGraph captured once per batch object
 * and launch shape.  The columns of all stripes are cut into tiles that
 * persistent workgroups take from a device-side counter.  Arithmetic and
 * results are exactly those of rs_poly_encode / rs_poly_decode on each
 * stripe (Sec. 3.2 and 3.3); only the launch is shared.  Batching is not in
 * the paper; it is how the GPU is kept full with stripes of any size. */

/* One stripe of a batch call. */
typedef struct rs_poly_stripe {
    rs_poly_t *code;             /* its code handle                          */
    uint8_t *const *blocks;      /* host array of n = k+m device pointers,   *
                                  * API block order (encode: reads 0..k-1,   *
                                  * writes k..n-1; update: 0..k-1 are delta  *
                                  * blocks or NULL, k..n-1 the parity,       *
                                  * updated in place)                        */
    size_t block_bytes;          /* bytes per block; 0 = nothing to do       */
    const int *erasures;         /* decode only: lost API indices            */
    int n_erasures;              /* decode only: t, 0 <= t <= m              */
    unsigned flags;              /* decode only: 0 or RS_POLY_FLAG_ALL_SURVIVORS */
} rs_poly_stripe_t;

/* Launch shape of a batch kernel (what the autotuner chooses). */
typedef struct rs_poly_launch {
    int bytes_per_lane;   /* columns per lane per block: 4, 8 or 16            */
    int threads;          /* workgroup size: 256, 512, 768 or 1024; codes with *
                           * m <= 4 at 16 bytes per lane take at most 512      */
    int tile_bytes;       /* most columns per tile: a multiple of 16, >= 4096; *
                           * calls with few columns use smaller tiles so that  *
                           * every workgroup gets work                         */
    int wgs_per_cu;       /* persistent workgroups per CU: 1 or 2              */
    int table_placement;  /* LFSR tables in LDS: RS_POLY_TABLES_PACKED or      *
                           * RS_POLY_TABLES_NIBBLE; encode also                *
                           * RS_POLY_TABLES_BITMATRIX, update also             *
                           * RS_POLY_TABLES_REGISTERS (the update default)     */
    int tile_order;       /* 0: tiles handed out in order (the workgroups work *
                           * on neighbouring tiles); 1: each workgroup walks   *
                           * its own run of tiles (dynamic claims either way)  */
} rs_poly_launch_t;

/* Table placements of the LFSR feedback products T[f] (both give identical
 * results).  PACKED: one 256-entry table per rotation, one LDS lookup per
 * symbol.  NIBBLE: split-nibble tables, T[f] = T[f & 15] ^ T[f & 0xF0]
 * from two 16-entry tables, two lookups per symbol and 1/8 of the LDS. */
#define RS_POLY_TABLES_PACKED 0
#define RS_POLY_TABLES_NIBBLE 1
/* Encode only: no tables -- the bit-sliced XOR-only kernel of
 * rs_poly_encode_bitmatrix, for a state width whose stripes in the call all
 * use one code with k <= 32 (any other call runs
 * the PACKED tables with the same launch shape).  Tiles are rounded down to
 * a multiple of 2048 columns; bytes_per_lane does not apply. */
#define RS_POLY_TABLES_BITMATRIX 2
/* Update only: the split-nibble products held in registers, the kernel of
 * rs_poly_update_nibble, for a state width whose stripes in the call all
 * change at most 2 blocks with (changed blocks) * m <= 8 (any other call
 * runs the PACKED forms with the same launch shape).  No LDS; each thread
 * takes 16 bytes of every block per pass, so bytes_per_lane does not
 * apply.  The default placement of batched updates. */
#define RS_POLY_TABLES_REGISTERS 3

#define RS_POLY_OP_ENCODE 0
#define RS_POLY_OP_DECODE 1
#define RS_POLY_OP_UPDATE 2

typedef struct rs_poly_batch rs_poly_batch_t;

/* Creates a batch object: device descriptor buffers, pinned staging and
 * captured graphs, all grown on demand and owned by the object.  Binds to
 * the device current at creation; calls must be made with that device
 * current.  Errors: RS_ENULL, RS_ENOMEM, RS_EDEVICE. */
int rs_poly_batch_create(rs_poly_batch_t **out);

/* Waits for the object's own pending uploads, then frees it.  The caller
 * must not free it with its kernels still queued.  NULL is a no-op. */
void rs_poly_batch_free(rs_poly_batch_t *b);

/* Encodes every stripe (parity of Sec. 3.2, eq. (1)-(2)) with one graph
 * launch per state width on `stream`.  Every block pointer must be 16-byte
 * aligned (else RS_EINVAL; rs_poly_encode takes any alignment).  Outputs of
 * different stripes must not overlap.  The stripe array and the host arrays
 * it points to are read during the call only.
 * Errors: RS_ENULL, RS_EINVAL, RS_ENOMEM, RS_EDEVICE. */
int rs_poly_batch_encode(rs_poly_batch_t *b, const rs_poly_stripe_t *stripes,
                         int count, void *stream);

/* Erasure-decodes every stripe (Sec. 3.3), as rs_poly_decode would, with one
 * graph launch per state width.  Per-stripe erasure lists are validated as
 * in rs_poly_decode; any error rejects the whole call before any work.
 * Errors: RS_ENULL, RS_EINVAL, RS_ERANGE, RS_ETOOMANY, RS_ENOMEM,
 * RS_EDEVICE. */
int rs_poly_batch_decode(rs_poly_batch_t *b, const rs_poly_stripe_t *stripes,
                         int count, void *stream);

/* The same two calls under op-first names (rs_poly_<op>_batch); they
 * behave exactly as rs_poly_batch_encode and rs_poly_batch_decode. */
int rs_poly_encode_batch(rs_poly_batch_t *b, const rs_poly_stripe_t *stripes,
                         int count, void *stream);
int rs_poly_decode_batch(rs_poly_batch_t *b, const rs_poly_stripe_t *stripes,
                         int count, void *stream);

/* Delta-parity updates (as rs_poly_update) of every stripe, with one graph
 * launch per state width; a width uses the generator-matrix form when none
 * of its stripes changes more than 8 blocks, else the LFSR form.  Every
 * non-NULL block pointer must be 16-byte aligned; the parity of different
 * stripes must not overlap.
 * Errors: RS_ENULL, RS_EINVAL, RS_ENOMEM, RS_EDEVICE. */
int rs_poly_batch_update(rs_poly_batch_t *b, const rs_poly_stripe_t *stripes,
                         int count, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the batch calls with no
 * batch object.  rs_poly_batch_noalloc(op, ...) does what
 * rs_poly_batch_encode / _decode / _update do for op = RS_POLY_OP_ENCODE /
 * _DECODE / _UPDATE -- same validation, same kernels, same bytes -- at the
 * library's default launch shapes, but allocates no device memory, no
 * pinned host memory and no stream, event or graph: its zero page,
 * descriptor arena, tile map and tile counter live in one file-scope device
 * array of RS_POLY_NOALLOC_SCRATCH_BYTES per GPU, held until the process
 * ends (its address is looked up, and the array cleared, on the first call
 * on each device, which synchronizes `stream` once).  The descriptors reach
 * the array by an ordinary host-to-device copy on `stream` from library
 * memory (host-side planning uses the C++ heap, as every call does).
 * Limits, per state width (codes with m <= 4, and with 4 < m <= 8) of a
 * call: the packed descriptors of its stripes (about 0.2-0.7 KiB per stripe,
 * more for large k) must fit RS_POLY_NOALLOC_ARENA_BYTES and its tiles (of
 * 8-64 KiB of columns each) RS_POLY_NOALLOC_MAX_TILES; larger calls are
 * rejected with RS_EINVAL before any work.  Every call on a GPU uses that
 * GPU's one array: calls that overlap on the device (queued on different
 * streams without ordering between them) race and give undefined results;
 * calls on one stream are ordered.
 * Errors: as the batch calls, plus RS_EINVAL (op, or the limits above). */
#define RS_POLY_NOALLOC_ARENA_BYTES (512u << 10)
#define RS_POLY_NOALLOC_MAX_TILES (128u << 10)
#define RS_POLY_NOALLOC_SCRATCH_BYTES \
    ((64u << 10) + 2u * RS_POLY_NOALLOC_ARENA_BYTES + 2u * 4u * RS_POLY_NOALLOC_MAX_TILES)
int rs_poly_batch_noalloc(int op, const rs_poly_stripe_t *stripes, int count,
                          void *stream);

/* Pre-sizes the object's device descriptor buffers, tile map and pinned
 * staging for calls of up to max_stripes stripes of up to max_block_bytes
 * each (any codes), so such calls never allocate.  Larger calls still work:
 * buffers then grow, and replaced buffers are kept until rs_poly_batch_free
 * (no device-wide synchronization).  Errors: RS_ENULL, RS_EINVAL,
 * RS_ENOMEM. */
int rs_poly_batch_reserve(rs_poly_batch_t *b, int max_stripes, size_t max_block_bytes);

/* Reads or sets the launch shape used for (op, state width), where wide = 0
 * selects codes with m <= 4 and wide = 1 codes with 4 < m <= 8.  Shapes are
 * validated (RS_EINVAL). */
int rs_poly_batch_get_launch(const rs_poly_batch_t *b, int op, int wide,
                             rs_poly_launch_t *cfg);
int rs_poly_batch_set_launch(rs_poly_batch_t *b, int op, int wide,
                             const rs_poly_launch_t *cfg);

/* Autotuner: times every candidate launch shape (bytes per lane, threads,
 * tile, workgroups per CU, table placement, tile order) on these stripes (running
 * the real operation several times on `stream`: encode and decode are
 * idempotent, and an update runs an even number of times per candidate, so
 * the parity ends as it began -- tuning does not apply the update),
 * keeps the fastest for each state width present, and returns the shape
 * chosen for the width carrying the most bytes in *best (may be NULL).
 * Blocks until the timing runs finish.  If the environment variable
 * RS_POLY_TUNE_CACHE names a file, results are read from / appended to it
 * as JSON lines keyed by device architecture, op, width and block-size
 * bucket, and a cached entry skips the timing. */
int rs_poly_tune(rs_poly_batch_t *b, int op, const rs_poly_stripe_t *stripes,
                 int count, void *stream, rs_poly_launch_t *best);

/* ------------------------------------------------------------ serving --
 *
 * A continuous-batching request engine over the batch API (not in the
 * paper; it is how the codec is used under load).  Requests are encodes of
 * caller-resident data and degraded reads (decodes) of caller-resident
 * stripes.  A scheduler thread admits requests in arrival order while the
 * HBM budget and a free output buffer allow, groups the admitted ones into
 * a batch and launches it on one of `streams` streams, so batches formed
 * while others run overlap on the device.  Outputs (parity for encode,
 * rebuilt blocks for decode) are allocated from a device pool the engine
 * owns; they are bit-identical to what rs_poly_encode / rs_poly_decode
 * produce for the same request alone. */

typedef struct rs_serve rs_serve_t;

typedef struct rs_serve_config {
    size_t hbm_budget_bytes;  /* bytes admitted requests may charge at once;  *
                               * also the size of the output pool (> 0)       */
    int streams;              /* batches in flight at once, 1..8              */
    int max_batch;            /* most requests per batch, >= 1                */
    int auto_release;         /* 1: free outputs and budget at completion     *
                               * (completions then carry no output pointers) */
    size_t max_block_bytes;   /* largest block_bytes accepted (0 = any); the  *
                               * batch buffers are reserved for it up front   */
} rs_serve_config_t;

typedef struct rs_serve_request {
    int op;                   /* RS_POLY_OP_ENCODE or RS_POLY_OP_DECODE       */
    rs_poly_t *code;
    uint8_t *const *blocks;   /* n device pointers, API order.  Encode reads  *
                               * 0..k-1 (parity entries ignored); decode reads *
                               * survivors (erased entries ignored).  Must    *
                               * stay valid until the request completes.      */
    size_t block_bytes;       /* > 0                                          */
    const int *erasures;      /* decode: lost API indices                     */
    int n_erasures;           /* decode: 1..m                                 */
    unsigned flags;           /* decode: 0 or RS_POLY_FLAG_ALL_SURVIVORS      */
    uint64_t user_tag;        /* returned with the completion                 */
} rs_serve_request_t;

typedef struct rs_serve_completion {
    uint64_t ticket;
    uint64_t user_tag;
    int status;               /* RS_OK or the error of its batch             */
    int n_out;                /* m (encode) or t (decode)                    */
    uint8_t *out[RS_POLY_MAX_M]; /* encode: p_0..p_(m-1); decode: blocks in   *
                               * increasing erased index order; owned by the  *
                               * engine until released.  NULL with            *
                               * auto_release (the outputs were freed when    *
                               * the request completed)                       */
    int out_index[RS_POLY_MAX_M]; /* API index of each output block          */
    size_t charge_bytes;      /* budget held: (k+m)B encode, (k+t)B decode    */
    double queue_us;          /* submit -> batch launch                       */
    double latency_us;        /* submit -> completion observed by the engine  */
} rs_serve_completion_t;

typedef struct rs_serve_stats {
    uint64_t submitted, completed, batches;
    uint64_t user_bytes;      /* k*B summed over completed requests           */
    size_t budget_in_use;     /* now                                          */
    size_t budget_peak;       /* highest charge held at once                  */
    int peak_inflight_batches;
    int pending;              /* submitted, not yet admitted                  */
    double launch_host_us;    /* host time forming and enqueuing batches      */
    double batch_device_us;   /* summed device time of batches, from their    *
                               * first command to their completion event      */
    double admit_host_us;     /* host time reaping finished batches and       *
                               * admitting requests                           */
} rs_serve_stats_t;

/* Creates the engine on the current device: allocates the output pool and
 * starts the scheduler thread.  Errors: RS_ENULL, RS_EINVAL, RS_ENOMEM,
 * RS_EDEVICE. */
int rs_serve_create(const rs_serve_config_t *cfg, rs_serve_t **out);

/* Queues a request (validated here, as rs_poly_batch_* would) and returns
 * its ticket.  Non-blocking.  A request whose charge exceeds the whole
 * budget is rejected with RS_EINVAL. */
int rs_serve_submit(rs_serve_t *s, const rs_serve_request_t *req, uint64_t *ticket);

/* Replays a request trace from an engine-owned arrival thread: request i is
 * submitted arrival_us[i] microseconds after the call (non-decreasing
 * times).  Returns at once; tickets are 1 + the submission count so far. */
int rs_serve_replay(rs_serve_t *s, const rs_serve_request_t *reqs,
                    const double *arrival_us, int count);

/* Moves up to max finished requests into out (in completion order); waits
 * up to timeout_us for the first one (0 = do not wait).  *n_done receives
 * the count. */
int rs_serve_poll(rs_serve_t *s, rs_serve_completion_t *out, int max, int *n_done,
                  int timeout_us);

/* Returns a completed request's outputs to the pool and its charge to the
 * budget (no-op with auto_release).  Errors: RS_ERANGE (unknown ticket). */
int rs_serve_release(rs_serve_t *s, uint64_t ticket);

int rs_serve_stats(rs_serve_t *s, rs_serve_stats_t *out);

/* Stops accepting requests, waits for queued and running ones to finish,
 * stops the threads and frees the pool.  NULL is a no-op. */
void rs_serve_destroy(rs_serve_t *s);

#ifdef __cplusplus
}
#endif

#endif /* RS_POLY_H */
