// Internal interface between the host library (api.cpp, gf.cpp) and the HIP
// kernels (codec.hip).  Not installed; the public ABI is include/rs_poly.h.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace rsp {

constexpr int kMaxN = 255;
constexpr int kMaxM = 8;
// Most blocks the wide generator-matrix form takes (see Mode).
constexpr int kMatrixWideMaxBlocks = 32;

// ---------------------------------------------------------------- tables --
//
// Every table the kernels look up is a GF(2)-linear map of one byte, so it
// is fully described by the images of the 8 unit bytes 1, 2, 4, ..., 128
// ("basis").  The host computes basis values; each workgroup expands them
// into 256-entry tables in LDS.  A value is 4 bytes (codes with m <= 4) or 8
// bytes (m <= 8), stored as 1 or 2 dwords.
//
// LDS layout: entry e of every table starts at byte e * 256, so a single
// v_perm_b32 turns (index byte, lane offset byte) into an LDS address.  Each
// 256-byte entry row holds several tables side by side, each replicated so
// that lanes of a wave spread over banks; 64 KiB in all.
constexpr uint32_t kRowBytes = 256;

// State width in bytes for a code with m parity symbols.
inline int state_bytes(int m) { return m <= 4 ? 4 : 8; }

// Kernels address columns with 32-bit offsets: the host hands them blocks
// of at most this many bytes, splitting longer blocks into independent
// column ranges (every column is its own codeword).
constexpr uint64_t kMaxPieceBytes = 1ull << 31;

// Device buffer of zeros that stands in for blocks a kernel does not read,
// so that every load slot issues a real load (see load_item in codec.hip).
constexpr uint32_t kZeroPageBytes = 65536;

// Kernel arguments, passed by value (about 2.8 KiB, within the kernarg limit).
struct CodecParams {
  const uint8_t *data[kMaxN];     // d_j; nullptr = symbol 0, not read
  const uint8_t *par_in[kMaxM];   // decode/update: parity p_i read back, or nullptr
  uint8_t *out[kMaxM];            // encode/update: p_i; decode: i-th erased block
  uint64_t block_bytes;           // <= kMaxPieceBytes
  int32_t k;                      // data blocks
  int32_t m;                      // parity symbols (remainder bytes)
  int32_t k_pad;                  // k rounded up to the state width
  int32_t n_out;                  // blocks written
  const uint8_t *zero_page;       // kZeroPageBytes of zeros on the device
  uint32_t lfsr_basis[16];        // 8 values of T'(2^b), 1 or 2 dwords each
  uint32_t apply_basis[kMaxM][16];// decode: per remainder byte, 8 values;
                                  // matrix update: per changed block
  // Wide matrix form (up to kMatrixWideMaxBlocks blocks): the column of
  // changed block t is mat_coef[t][0..m) (coefficients of x^(m+j) mod g,
  // low degree first); the kernel builds its tables in GF(2^field_w) with
  // the field polynomial field_poly.
  uint8_t mat_coef[kMatrixWideMaxBlocks][kMaxM];
  uint32_t field_poly;
  int32_t field_w;
};

// kUpdate: parity ^= encode(delta) -- the encode LFSR over the changed data
// blocks, plus the old parity read back in place.  kUpdateMatrix: the same
// result from the generator-matrix columns of the (at most
// kMatrixMaxBlocks) changed blocks, one packed lookup per changed block and
// column; the apply bases then hold the columns' table bases.
// kUpdateMatrixWide: the matrix form for up to kMatrixWideMaxBlocks blocks,
// its tables in two 64 KiB LDS regions (plain launches only).
enum Mode : int { kEncode = 0, kDecode = 1, kUpdate = 2, kUpdateMatrix = 3, kUpdateMatrixWide = 11 };
constexpr int kMatrixMaxBlocks = 8;

struct BitmatrixCode;

// A launch configuration of the codec kernel.
struct LaunchCfg {
  int dwords_per_lane;   // 1, 2 or 4: bytes per lane per block = 4x this
  int threads;           // workgroup size, multiple of 64, <= 1024
  int grid;              // workgroups; 0 = pick from the size
  bool bytewise;         // byte loads/stores (for misaligned blocks)
  bool nibble;           // batch kernels: split-nibble LFSR tables
  const BitmatrixCode *bm = nullptr;   // batch encode: bit-sliced, of this code
  bool nibble_update = false;          // batch update: register split-nibble kernel
};

// Launches the codec kernel for one stripe.  Returns a hipError_t as int.
int launch_codec(Mode mode, int state_bytes, const CodecParams &p,
                 const LaunchCfg &cfg, void *stream);

// Bit-sliced encode of one code.  rows.r[j][i][b] has bit b' set when bit
// b of c_ij * 2^b' is, c_ij the coefficient of x^i in x^(m+j) mod g(x)
// (the product by c_ij as an 8 x 8 matrix over GF(2), row b); for w = 4
// the rows and bits from 4 up are zero.  `builtin`: the code's XOR network
// is compiled in (GF(2^8), polynomial 0x11D, a few (k, m)); otherwise the
// kernel takes the rows at run time.  `key` tells codes apart for cached
// launches: field polynomial, k and m.
constexpr int kBitmatrixMaxK = 32;
struct BitRows {
  uint8_t r[kBitmatrixMaxK][kMaxM][8];
};
struct BitmatrixCode {
  int k = 0, m = 0;
  bool builtin = false;
  const BitRows *rows = nullptr;
  int key = 0;
};
bool bitmatrix_builtin(int k, int m, int w, unsigned poly);

// ------------------------------------------------------------- batches --
//
// A batch group holds stripes whose codes share a state width.  Its columns
// are cut into tiles of tile_cols bytes (a stripe's last tile may be short);
// tiles are numbered stripe after stripe.

struct StripeDesc {
  uint64_t block_bytes;  // <= kMaxPieceBytes
  uint64_t tile_begin;   // first tile of the stripe
  uint64_t ptr_off;      // first pointer-table entry: k data, m parity-in, n_out out
  uint32_t lfsr_set;     // index of the stripe's LFSR basis set
  uint32_t apply_set;    // decode: index of its apply basis set
  int32_t k, m, k_pad, n_out;
};

// A group's arena starts with this header; the regions after it are packed
// per call and located by the byte offsets below, so one host-to-device copy
// uploads a whole batch and captured graphs never need new arguments.
struct BatchHeader {
  uint64_t upload_bytes; // bytes of this group's packed upload (header included)
  uint64_t total_tiles;
  uint64_t counter;      // next tile to hand out; cleared by the prepare kernel
  uint32_t n_stripes;
  uint32_t tile_cols;    // columns per tile for this call, multiple of 16
  uint32_t tile_order;   // 0: tiles in order; 1: each workgroup walks a run
  uint32_t pad_;
  uint64_t off_descs;    // StripeDesc[n_stripes]
  uint64_t off_ptrs;     // uint64_t device pointers
  uint64_t off_lfsr;     // 16 dwords per LFSR basis set
  uint64_t off_apply;    // kMaxM * 16 dwords per apply basis set
};

struct BatchGroup {            // device pointers
  uint8_t *arena;              // BatchHeader, then the packed regions
  uint32_t *tile_stripe;       // tile -> stripe, filled by the prepare kernel
  const uint8_t *zero_page;    // kZeroPageBytes of zeros
  const uint8_t *host_src;     // coherent pinned host copy of the upload
};

// kZeroPageBytes of zeros on the current device, allocated and cleared on
// first use (per device, kept until the process ends); nullptr on error.
const uint8_t *device_zero_page();

// Enqueues, for a group: the pull kernel (copies the upload from host_src to
// the arena; left out when pull is false, the arena then already holding
// it), the prepare kernel and the persistent batch kernel.  max_tiles (the
// tile-map capacity) sizes the prepare grid.  Returns a hipError_t as int.
int launch_batch(Mode mode, int state_bytes, const BatchGroup &g, uint64_t max_tiles,
                 const LaunchCfg &cfg, void *stream, bool pull = true);

// Bit-sliced encode (bitmatrix.hip) of any code with k <= kBitmatrixMaxK;
// blocks 16-byte aligned.  launch_bitmatrix encodes columns [offset,
// offset + block_bytes) (block_bytes <= kMaxPieceBytes);
// launch_bitmatrix_batch launches the persistent batch kernel for a group
// of encode stripes of that one code whose tile_cols is a multiple of
// kBitmatrixTileCols (after the pull and prepare kernels).  Both return a
// hipError_t as int.
int launch_bitmatrix(const BitmatrixCode &bc, const uint8_t *const *data,
                     uint8_t *const *parity, uint64_t offset, uint64_t block_bytes,
                     void *stream);
int launch_bitmatrix_batch(const BitmatrixCode &bc, const BatchGroup &g, int grid, int threads,
                           void *stream);
constexpr uint32_t kBitmatrixTileCols = 2048;

// Streaming probe (roof.hip): `stripes` stripes of n_in input and n_out
// output blocks of block_bytes (a multiple of 16) at base + s * stripe_stride
// + b * block_stride; every input byte read once, every output byte written
// once (the XOR of the inputs), tiles of tile_cols columns over `grid`
// workgroups in tile order 0 or 1.  Returns a hipError_t as int.
int launch_stream_probe(uint8_t *base, uint64_t stripe_stride, uint64_t block_stride,
                        uint32_t stripes, uint32_t n_in, uint32_t n_out, uint32_t block_bytes,
                        uint32_t tile_cols, uint32_t tile_order, int grid, void *stream);

// Register-resident split-nibble update (nibble.hip): parity[i] ^= sum_t
// P[i][j_t] * delta[t] for c changed blocks j_t, the product of each
// (t, i) constant as two 16-entry nibble tables in registers; every pointer
// 16-byte aligned, any block_bytes.
constexpr int kNibbleMaxBlocks = 2;
constexpr int kNibbleMaxProducts = 8;
struct NibbleParams {
  const uint8_t *delta[kNibbleMaxBlocks];
  uint8_t *parity[kMaxM];
  uint64_t block_bytes;
  int32_t c, m;
  // constant (t, i) at t * m + i: dwords 0-3 hold c * n for n < 16 (entry n
  // at byte n), dwords 4-7 hold c * (n << 4)
  uint32_t tab[kNibbleMaxProducts][8];
};
bool nibble_supported(int c, int m);
int launch_nibble_update(const NibbleParams &p, int grid, void *stream);
// The persistent batch kernel of the same update (after the pull and
// prepare kernels): per stripe, descriptor k = c changed blocks, pointer
// table = the c changed delta blocks then the m parity blocks, tables =
// apply set apply_set laid out as NibbleParams::tab.
int launch_nibble_batch(const BatchGroup &g, int grid, int threads, void *stream);
// Fills the c * m tables of the changed blocks which[0..c) of a code
// (layout of NibbleParams::tab) into out[c * m][8].
class Code;
void nibble_tables(const Code &code, const int *which, int c, uint32_t (*out)[8]);

// Resident workgroups per CU the kernel is sized for (LDS bound).
int codec_wgs_per_cu(Mode mode);
// Largest workgroup a variant is compiled for (register bound); 0 if the
// variant does not exist.
int codec_max_threads(Mode mode, int state_bytes, int dwords_per_lane);
// Widest loads (dwords per lane) of the one-stripe kernel for a state width.
int codec_plain_max_dwords(int state_bytes);

}  // namespace rsp
