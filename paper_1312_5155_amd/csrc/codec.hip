// HIP kernels for polynomial RS(k,m) encode and erasure decode on gfx950.
//
// Work decomposition.  Byte column c of a stripe (byte c of every block) is
// one codeword, independent of all others.  A lane owns 4*W consecutive
// columns (W dwords of every block, W in {1,2,4}), so the k data blocks are
// read with coalesced W-dword loads; a grid-stride loop walks the columns.
//
// Encode = the generator-polynomial LFSR of Sec. 3.2, eq. (1)-(2): x^m d(x)
// mod g(x), fed from the highest data degree (d_(k-1)) down to d_0.  With the
// remainder kept as an M-byte value u (M = 4 for m <= 4, 8 for m <= 8) whose
// byte b is remainder coefficient r_(m-1-b), one data symbol d is absorbed by
//     f = d ^ byte0(u);   u = (u >> 8) ^ T[f],
// T[f] = sum_b (g_(m-1-b) f) << 8b.  Two rewrites make a step cost one
// v_perm_b32, one LDS read and one XOR per M <= 4 (two XORs for M = 8):
//   * future data symbols are XORed into the free upper bytes of u ahead of
//     time ("augmented window"): u' = (u >> 8) ^ T[f] still holds, so M data
//     bytes enter with one XOR per M steps;
//   * the shift is removed by letting byte positions rotate: the register
//     holds P = rotl(u, 8t) at step t, the feedback byte is byte (t mod M) of
//     P, and P' = P ^ rotl(T'[f], 8(t+1)) with T'[f] = T[f] ^ (f << 8(M-1))
//     (the extra term clears the consumed byte).  The M rotated copies of
//     T' are separate LDS tables.
// k is padded at the top to a multiple of M with zero symbols (leading zeros
// leave a zero remainder unchanged), so the rotation is back at 0 at the end.
//
// Decode = Sec. 3.3 in remainder form.  The same LFSR over the symbols read
// (erased or unread ones are zero and never loaded: Opt2 of Sec. 4), XOR the
// parity read, gives r(x) = received word mod g(x), whose values at the roots
// alpha^i are the paper's step-1 values D(alpha^i).  The erased symbols are
// then C * r for a small per-pattern matrix C = V^-1 W (Vandermonde inverse
// computed once per pattern on the host: Opt3), applied as m packed product
// lookups, one per remainder byte (region-level multiply-XOR: Opt4); the
// interleaved m > 4 kernels look up the two nibbles of each byte in
// split-nibble tables instead.
//
// Update = the update property of Sec. 3.2: encoding is linear, so new
// parity = old parity + encode(delta), delta = new data - old data.  It is
// the encode LFSR over the delta blocks (unchanged blocks are zero), then
// the old parity is XORed in as decode does, and the result overwrites the
// parity in place: one read-modify-write pass.
//
// Matrix update = the generator-matrix form of Sec. 6 for an update of at
// most 8 blocks: the parity change is sum_j P[:, j] * delta_j, with column
// P[:, j] the remainder of x^(m+j) mod g(x).  Each changed block gets a
// packed 256-entry table (byte x -> the m products P[i][j] x), so a column
// costs one lookup per changed block, with no serial chain and no work for
// the unchanged blocks.
//
// LDS tables.  Each table is a GF(2)-linear map of one byte, expanded by
// every workgroup from 8 basis values passed in the kernel arguments.  Entry
// e of every table sits at byte e*256 plus the table's offset and the
// lane's replica offset, so one v_perm_b32 of (state, lane offset) yields
// the address (M = 4, and M = 8 in the interleaved layout of the 16-byte
// kernels; a v_perm and an OR in the narrower M = 8 kernels).  Replicas
// spread the lanes of a wave over banks, and lanes start at different
// rotation phases, so that one read spreads over all copies.  64 KiB per
// workgroup (8 KiB for split-nibble encode/update tables; 128 KiB for the
// narrow decode of m > 4; 128 KiB, 144 KiB for decode, in the interleaved
// layout, whose kernels run one workgroup per CU anyway).
//
// Memory-level parallelism.  The kernels stream every byte once; throughput
// is set by the bytes in flight per CU and by how local the concurrent
// accesses are.  Each lane walks its column chunks as a software pipeline
// that keeps the loads of the next M blocks in flight while the current M
// are absorbed.  The wide codes at 16 bytes per lane (16 columns, 8 blocks
// per item) keep one item buffer, reloaded as soon as it has been XORed into
// the states, so that 1024 threads fit (128 VGPRs).
#include <hip/hip_runtime.h>

#include "rs_internal.h"

namespace rsp {
namespace {

// A kernel variant (the MODE template argument below): the operation in the
// low two bits, the LFSR table placement in the next one, then the wide
// matrix form, then the interleaved M = 8 state layout.
constexpr int kNibbleBit = 4;
constexpr int kWideMatrixBit = 8;   // kUpdateMatrixWide = kUpdateMatrix | this
constexpr int kIlvBit = 16;
constexpr int op_of(int v) { return v & 3; }
constexpr bool nibble_of(int v) { return (v & kNibbleBit) != 0; }
constexpr bool wide_matrix_of(int v) { return (v & kWideMatrixBit) != 0; }
constexpr bool ilv_of(int v) { return (v & kIlvBit) != 0; }
static_assert(kUpdateMatrixWide == (kUpdateMatrix | kWideMatrixBit), "mode encoding");

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// An empty asm that takes and gives back two column states: code that
// reads them cannot move above it, code that writes them cannot move below.
template <int NQ>
__device__ __forceinline__ void pin_pair(uint32_t (&x)[NQ], uint32_t (&y)[NQ]) {
  if constexpr (NQ == 1)
    asm volatile("" : "+v"(x[0]), "+v"(y[0]));
  else
    asm volatile("" : "+v"(x[0]), "+v"(x[1]), "+v"(y[0]), "+v"(y[1]));
}

// a ^ b ^ c in one v_bitop3_b32 (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint32_t rotl32(uint32_t x, int s) {
  s &= 31;
  return s ? (x << s) | (x >> (32 - s)) : x;
}

__device__ __forceinline__ uint64_t rotl64(uint64_t x, int s) {
  s &= 63;
  return s ? (x << s) | (x >> (64 - s)) : x;
}

// 4x4 byte transpose: o_b = (i0.byte b, i1.byte b, i2.byte b, i3.byte b),
// as two rounds of v_perm.  Other selectors fold a byte rotation in: second
// round selectors rotated left by 8g bytes give rotl(o_b, 8g); first round
// selectors that read byte b + g give the transpose of inputs rotated by g.
constexpr uint32_t kT1a = 0x05010400u, kT1b = 0x07030602u;   // first round
constexpr uint32_t kT2a = 0x05040100u, kT2b = 0x07060302u;   // second round

__device__ __forceinline__ void transpose4(uint32_t i0, uint32_t i1, uint32_t i2, uint32_t i3,
                                           uint32_t &o0, uint32_t &o1, uint32_t &o2,
                                           uint32_t &o3, uint32_t s1a = kT1a,
                                           uint32_t s1b = kT1b, uint32_t s2a = kT2a,
                                           uint32_t s2b = kT2b) {
  const uint32_t lo01 = perm(i1, i0, s1a);  // i0.b0 i1.b0 i0.b1 i1.b1
  const uint32_t hi01 = perm(i1, i0, s1b);  // i0.b2 i1.b2 i0.b3 i1.b3
  const uint32_t lo23 = perm(i3, i2, s1a);
  const uint32_t hi23 = perm(i3, i2, s1b);
  o0 = perm(lo23, lo01, s2a);
  o1 = perm(lo23, lo01, s2b);
  o2 = perm(hi23, hi01, s2a);
  o3 = perm(hi23, hi01, s2b);
}

// Image of byte f under the linear map with basis values basis[0..7].
__device__ __forceinline__ uint32_t lin32(uint32_t f, const uint32_t *basis) {
  uint32_t v = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) v ^= basis[b] & (0u - ((f >> b) & 1u));
  return v;
}

__device__ __forceinline__ uint64_t lin64(uint32_t f, const uint32_t *basis) {
  uint64_t v = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t bv = (uint64_t)basis[2 * b] | ((uint64_t)basis[2 * b + 1] << 32);
    v ^= bv & (0ull - (uint64_t)((f >> b) & 1u));
  }
  return v;
}

__device__ __forceinline__ void st4(uint8_t *lds, uint32_t off, uint32_t a, uint32_t b,
                                    uint32_t c, uint32_t d) {
  *reinterpret_cast<uint4 *>(lds + off) = make_uint4(a, b, c, d);
}

// LDS row layout.  Row e (256 bytes at e*256) holds entry e of every table;
// a row spans the 64 banks once, so a lane's bank is set by its offset in
// the row alone.  LDS serves a wave's read in passes of 32 lanes, and a
// read is conflict-free when the 32 lanes of a pass use distinct banks.
// Encode and update: the M rotated copies of T' (copy v = rotation by v+1
// bytes), each kLfsrReps replicas wide.  Decode of m <= 4: the same copies
// at half the replication in bytes 0..127 and the apply tables U'_b (one
// per remainder byte) in bytes 128..255.  Decode of m > 4 (8-byte entries)
// needs whole rows for both, so in the narrower kernels its apply tables sit
// in a second 64 KiB region (128 KiB of LDS, one workgroup per CU); the
// interleaved layout (below) has regions of its own.
//
// Split-nibble placement (the alternative the autotuner can pick): each
// rotated copy of T' is two 16-entry tables, T'[n] in rows 0..15 and
// T'[n << 4] in rows 16..31 (T' is GF(2)-linear, so T'[f] is their XOR).  A
// step then makes two lookups instead of one; encode and update need 8 KiB
// of LDS instead of 64.
template <int M, int MODE>
struct Layout {
  static constexpr bool kNibble = nibble_of(MODE);
  static constexpr uint32_t kHiBase = 16 * kRowBytes;   // nibble: rows of T'[n << 4]
  static constexpr bool kTwoRegions = M == 8 && op_of(MODE) == kDecode;
  static constexpr uint32_t kEntry = M == 4 ? 4 : 8;              // bytes per value
  static constexpr uint32_t kCopies = M;                          // rotations 1..M bytes
  static constexpr uint32_t kLfsrReps =
      (op_of(MODE) == kDecode && !kTwoRegions ? 128 : 256) / (kCopies * kEntry);
  static constexpr uint32_t kCopyBytes = kLfsrReps * kEntry;      // one rotated copy
  static constexpr uint32_t kApplyReps = (kTwoRegions ? 256 : 128) / (M * kEntry);
  static constexpr uint32_t kTableBytes = kApplyReps * kEntry;    // one apply table
  static constexpr uint32_t kApplyBase = kTwoRegions ? 65536 : 128;
  // Wide matrix form: 32 tables in two 64 KiB regions of 16 tables each.
  static constexpr bool kWideMatrix = wide_matrix_of(MODE);
  // Interleaved M = 8 layout (see below): LFSR copies of even rotation
  // index in region 0, odd in region 1 (64 KiB each, 4 copies x 8
  // replicas per row); decode adds split-nibble apply tables in region 2
  // (64 rows: low-nibble and high-nibble tables of the even remainder
  // bytes, then of the odd ones, 4 tables x 8 replicas per row).
  static constexpr bool kIlv = M == 8 && ilv_of(MODE) && !kNibble && op_of(MODE) != kUpdateMatrix;
  static constexpr uint32_t kIlvReps = 8;
  static constexpr uint32_t kIlvTableBytes = kIlvReps * 8;
  static constexpr uint32_t kIlvApplyBase = 131072;
  static constexpr uint32_t kIlvApplyRows = 64;
  static constexpr uint32_t kLdsBytes =
      kIlv ? (op_of(MODE) == kDecode ? kIlvApplyBase + kIlvApplyRows * kRowBytes : 131072)
      : kTwoRegions || kWideMatrix ? 131072
      : kNibble && op_of(MODE) != kDecode ? 32 * kRowBytes : 65536;
  // Matrix update: one table per changed block, a group of M tables per
  // item (the item's M blocks), kMatReps replicas; 2 groups per row for
  // M = 4, 1 for M = 8 (8 tables at most).  Wide form: 4 (M = 4) or 2
  // (M = 8) groups per row, 16 tables per row and region.
  static constexpr uint32_t kMatReps = kWideMatrix ? (M == 4 ? 4 : 2) : (M == 4 ? 8 : 4);
  static constexpr uint32_t kMatTableBytes = kMatReps * kEntry;
  static constexpr uint32_t kMatGroupBytes = M * kMatTableBytes;
  // Lane groups at different rotation phases: in one LDS read group g uses
  // copy (q + g) mod M, so the 32 lanes of a pass cover 32 distinct
  // replica slots (banks).
  static constexpr uint32_t kPhases = M == 4 ? 32 / kLfsrReps : 8;
};

// Per-lane LDS addressing, computed once per kernel.  A lane of phase g keeps
// its state rotated by g more bytes than the step count says: at unrolled
// step q it reads feedback byte (q + g) mod M from copy (q + g) mod M.
// Decode lanes likewise walk the apply tables in rotated order.
//
// M = 4: the state stays rotated to the end of a chunk.  Items enter
// rotated by g bytes through the second transpose round, decode reads the
// apply index at byte (b + g) mod 4, and encode/update outputs leave
// through a first transpose round that reads byte b + g: the rotation costs
// no instruction.
//
// M = 8 in the narrower kernels: the state is two dwords, and byte
// (q + g) mod 8 may sit in either, so a step selects it with a v_perm over
// both dwords and ORs in the lane offset; rotations into and out of the
// phase are v_perm byte shuffles of the dword pair.
//
// Interleaved M = 8 (the wide kernels at 16 bytes per lane): the state
// keeps the even bytes of the 8-byte value in its first dword and the odd
// ones in its second, and only even phases g = 2h (h = 0..3) are used.  At
// step q every lane's feedback byte (q + g) mod 8 then sits in dword q & 1,
// at position (q/2 + h) mod 4, so one v_perm of (that dword, an offset
// register) forms the whole address: byte 1 the feedback byte, byte 0 the
// lane's slot in the row, byte 2 the region (copies of odd rotation index
// are 64 KiB up).  The 32 lanes of a pass use 4 copies (one parity) x 8
// replicas, all distinct banks.  Rotation by g moves bytes only within a
// dword, so items enter and parity leaves through the rotating transpose
// selectors, as for M = 4, and no state is ever rotated back.  The decode
// apply reads remainder byte (b - g) mod 8 at step b, which sits at the
// same position b/2 in every lane (a uniform selector), from split-nibble
// tables (two lookups per byte) that fit beside the 128 KiB of LFSR copies.
template <int M, int MODE>
struct Lanes {
  uint32_t lsel[M], loff[M];   // LFSR step q: v_perm selector, byte offset
  uint32_t loffhi[M];          // split-nibble: offset of the high-nibble table
  uint32_t tin[2], tout[2];    // M = 4: rotating transpose selectors (in, out)
  uint32_t rin[2], rout[2];    // M = 8: v_perm selectors (low, high dword)
  uint32_t asel[M], aoff[M];   // decode apply, slot b
  uint32_t isel[4];            // interleaved: selector of steps 2j, 2j + 1
  uint32_t ioff[4];            // interleaved: slot offsets, region 0 (x2), region 1 (x2)
  uint32_t iapp[2];            // interleaved decode: apply slot offsets, region 2
};

template <int M, int MODE>
__device__ __forceinline__ Lanes<M, MODE> make_lanes() {
  using L = Layout<M, MODE>;
  Lanes<M, MODE> t{};
  const uint32_t lane = threadIdx.x & 63;
  if constexpr (L::kIlv) {
    const uint32_t h = (lane >> 3) & 3, rep = lane & 7;
    uint32_t off[4], aof[4];
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      // steps 2j, 2j + 1 read copies 2((j + h) mod 4) and that plus one;
      // apply step 2j (+1) reads table 2((j - h) mod 4) (+1)
      off[j] = ((j + h) & 3) * L::kIlvTableBytes + rep * 8;
      aof[j] = ((j - h) & 3) * L::kIlvTableBytes + rep * 8;
      // byte 0 <- offset byte j & 1, byte 1 <- state byte (j + h) mod 4,
      // byte 2 <- offset byte 2 (the region), byte 3 <- 0
      t.isel[j] = (j & 1) | ((4 + ((j + h) & 3)) << 8) | (2u << 16) | (0x0Cu << 24);
    }
#pragma unroll
    for (uint32_t x = 0; x < 2; ++x) {
      t.ioff[x] = off[2 * x] | (off[2 * x + 1] << 8);
      t.ioff[2 + x] = t.ioff[x] | (1u << 16);
      t.iapp[x] = aof[2 * x] | (aof[2 * x + 1] << 8) | ((L::kIlvApplyBase >> 16) << 16);
    }
    t.tin[0] = rotl32(kT2a, 8 * h);
    t.tin[1] = rotl32(kT2b, 8 * h);
#pragma unroll
    for (uint32_t i = 0; i < 2; ++i) {
      t.tout[0] |= (((i + h) & 3) | (((4 + ((i + h) & 3))) << 8)) << (16 * i);
      t.tout[1] |= (((i + 2 + h) & 3) | (((4 + ((i + 2 + h) & 3))) << 8)) << (16 * i);
    }
    return t;
  }
  const uint32_t g = (lane / L::kLfsrReps) % L::kPhases;
  const uint32_t rep = lane & (L::kLfsrReps - 1);
#pragma unroll
  for (uint32_t q = 0; q < (uint32_t)M; ++q) {
    const uint32_t p = (q + g) & (M - 1);
    // M = 4: byte 1 <- state byte p, byte 0 <- lane offset.  M = 8: byte 1
    // <- byte p of the dword pair (selector p: 0..3 low dword, 4..7 high).
    t.lsel[q] = M == 4 ? 0x0C0C0400u | (p << 8) : 0x0C0C000Cu | (p << 8);
    t.loff[q] = p * L::kCopyBytes + rep * L::kEntry;
    t.loffhi[q] = L::kHiBase + t.loff[q];
  }
  t.tin[0] = rotl32(kT2a, 8 * g);
  t.tin[1] = rotl32(kT2b, 8 * g);
  t.tout[0] = t.tout[1] = 0;
#pragma unroll
  for (uint32_t i = 0; i < 2; ++i) {
    t.tout[0] |= (((i + g) & 3) | (((4 + ((i + g) & 3))) << 8)) << (16 * i);
    t.tout[1] |= (((i + 2 + g) & 3) | (((4 + ((i + 2 + g) & 3))) << 8)) << (16 * i);
  }
  // M = 8: rotl64 by g bytes takes result byte i from byte (i - g) mod 8;
  // the inverse from byte (i + g) mod 8.
  t.rin[0] = t.rin[1] = t.rout[0] = t.rout[1] = 0;
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i) {
    t.rin[0] |= ((i - g) & 7) << (8 * i);
    t.rin[1] |= ((i + 4 - g) & 7) << (8 * i);
    t.rout[0] |= ((i + g) & 7) << (8 * i);
    t.rout[1] |= ((i + 4 + g) & 7) << (8 * i);
  }
  if constexpr (op_of(MODE) == kUpdateMatrix) {
    // table of block slot tb of the item, read in per-lane rotated order
    const uint32_t arep = lane & (L::kMatReps - 1);
    const uint32_t ga = (lane / L::kMatReps) % M;
#pragma unroll
    for (uint32_t b = 0; b < (uint32_t)M; ++b) {
      const uint32_t tb = (b + ga) & (M - 1);
      t.asel[b] = M == 4 ? 0x0C0C0400u | (tb << 8) : 0x0C0C000Cu | (tb << 8);
      t.aoff[b] = tb * L::kMatTableBytes + arep * L::kEntry;
    }
  }
  if constexpr (op_of(MODE) == kDecode) {
    const uint32_t arep = lane & (L::kApplyReps - 1);
    const uint32_t ga = (lane / L::kApplyReps) % M;
#pragma unroll
    for (uint32_t b = 0; b < (uint32_t)M; ++b) {
      const uint32_t tb = (b + ga) & (M - 1);
      // M = 4: remainder byte tb sits at byte tb + g of the rotated state
      t.asel[b] = M == 4 ? 0x0C0C0400u | (((tb + g) & 3) << 8) : 0x0C0C000Cu | (tb << 8);
      t.aoff[b] = L::kApplyBase + tb * L::kTableBytes + arep * L::kEntry;
    }
  }
  return t;
}

// Fills `tables` tables of `table_bytes` each (replicas of one 4- or 8-byte
// entry) at byte `base` of rows 0..rows-1.  Thread idx computes entry
// idx / tables of table idx mod tables once, as a (low, high) dword pair (the
// same dword twice for 4-byte entries), and stores its 16-byte chunks
// starting at chunk (row mod chunks): the lanes of a wave that share a table
// but not a row then store to different banks.
template <class ValueFn>
__device__ __forceinline__ void fill_tables(uint8_t *lds, uint32_t rows, uint32_t base,
                                            uint32_t tables, uint32_t table_bytes,
                                            ValueFn value) {
  const uint32_t chunks = table_bytes / 16;   // 2 or 4
  for (uint32_t idx = threadIdx.x; idx < rows * tables; idx += blockDim.x) {
    const uint32_t r = idx / tables, t = idx % tables;
    const uint2 v = value(r, t);
    const uint32_t at = r * kRowBytes + base + t * table_bytes;
    for (uint32_t c = 0; c < chunks; ++c)
      st4(lds, at + 16 * ((c + r) & (chunks - 1)), v.x, v.y, v.x, v.y);
  }
}

template <int M>
__device__ __forceinline__ uint2 entry_of(uint32_t f, const uint32_t *basis, int rot_bytes) {
  if constexpr (M == 4) {
    const uint32_t v = rotl32(lin32(f, basis), 8 * rot_bytes);
    return make_uint2(v, v);
  } else {
    const uint64_t x = rotl64(lin64(f, basis), 8 * rot_bytes);
    return make_uint2((uint32_t)x, (uint32_t)(x >> 32));
  }
}

// An 8-byte entry in the interleaved layout: even bytes in the first dword,
// odd bytes in the second.
__device__ __forceinline__ uint2 interleave(uint2 v) {
  return make_uint2(perm(v.y, v.x, 0x06040200u), perm(v.y, v.x, 0x07050301u));
}

// Expands the LFSR tables: copy v (0..M-1) of entry f is rotl(T'[f], 8(v+1));
// split-nibble: row r < 16 holds entry r, row 16 + r entry r << 4;
// interleaved: copy v in region v & 1 at table v >> 1 of the row.
template <int M, int MODE>
__device__ void build_lfsr_tables(uint8_t *lds, const uint32_t *basis) {
  using L = Layout<M, MODE>;
  if constexpr (L::kIlv) {
#pragma unroll
    for (uint32_t region = 0; region < 2; ++region)
      fill_tables(lds + 65536 * region, 256, 0, 4, L::kIlvTableBytes,
                  [&](uint32_t f, uint32_t c) {
                    return interleave(entry_of<M>(f, basis, (int)(2 * c + region) + 1));
                  });
    return;
  }
  fill_tables(lds, L::kNibble ? 32 : 256, 0, L::kCopies, L::kCopyBytes,
              [&](uint32_t r, uint32_t v) {
                const uint32_t f = !L::kNibble ? r : r < 16 ? r : (r - 16) << 4;
                return entry_of<M>(f, basis, (int)v + 1);
              });
}

// Expands the decode apply tables U'_b, b < m (unused tables are zero).
// Interleaved: rows 16G + n of region 2 hold, for G = 0..3, the entries n
// (G even) or n << 4 (G odd) of the tables of remainder bytes b = 2c + G/2
// at table c of the row; the entries themselves keep the natural byte
// order (byte e the product for erased block e).
template <int M, int MODE>
__device__ void build_apply_tables(uint8_t *lds, const uint32_t *basis /* [kMaxM][16] */,
                                   int m) {
  using L = Layout<M, MODE>;
  if constexpr (L::kIlv) {
    fill_tables(lds + L::kIlvApplyBase, L::kIlvApplyRows, 0, 4, L::kIlvTableBytes,
                [&](uint32_t r, uint32_t c) {
                  const uint32_t grp = r >> 4, n = r & 15;
                  const uint32_t f = grp & 1 ? n << 4 : n;
                  const int b = (int)(2 * c + (grp >> 1));
                  return b < m ? entry_of<M>(f, basis + 16 * b, 0) : make_uint2(0u, 0u);
                });
    return;
  }
  fill_tables(lds, 256, L::kApplyBase, M, L::kTableBytes,
              [&](uint32_t f, uint32_t b) {
                return (int)b < m ? entry_of<M>(f, basis + 16 * b, 0) : make_uint2(0u, 0u);
              });
}

// Expands the matrix-update tables.  Window position pos (item pos / M,
// slot pos mod M; its table at byte pos * kMatTableBytes of the row) holds
// changed block t = k_pad - 1 - pos, as load_item places it; tables of
// positions with no block are zero.
template <int M>
__device__ void build_matrix_tables(uint8_t *lds, const uint32_t *basis /* [kMaxM][16] */,
                                    int c, int k_pad) {
  using L = Layout<M, kUpdateMatrix>;
  static_assert(L::kMatGroupBytes == M * L::kMatTableBytes &&
                    kMatrixMaxBlocks * L::kMatTableBytes == kRowBytes,
                "one row holds all tables, position after position");
  fill_tables(lds, 256, 0, kMatrixMaxBlocks, L::kMatTableBytes, [&](uint32_t f, uint32_t pos) {
    const int tt = k_pad - 1 - (int)pos;
    return tt >= 0 && tt < c ? entry_of<M>(f, basis + 16 * tt, 0) : make_uint2(0u, 0u);
  });
}

// Product of a and b in GF(2^w) with field polynomial poly (shift and add).
__device__ __forceinline__ uint32_t gf_mul(uint32_t a, uint32_t b, uint32_t poly, int w) {
  uint32_t r = 0;
  for (int i = 0; i < w; ++i) {
    if ((b >> i) & 1u) r ^= a;
    a <<= 1;
    if (a >> w) a ^= poly;
  }
  return r;
}

// Expands the wide matrix-form tables (up to 32 blocks).  Window position
// pos holds changed block t = k_pad - 1 - pos, its table in region pos / 16
// at table index pos mod 16 of the row (group (pos mod 16) / M, slot pos
// mod M).  The 8 basis values of each table (the products of its column
// by the unit bytes) are computed here, from the column coefficients, into
// `bases` first.
template <int M>
__device__ void build_wide_matrix_tables(uint8_t *lds, uint32_t (*bases)[16],
                                         const CodecParams &p) {
  using L = Layout<M, kUpdateMatrixWide>;
  static_assert(16 * L::kMatTableBytes == kRowBytes, "16 tables per row and region");
  const int m = p.m, c = p.k, k_pad = p.k_pad;
  for (uint32_t idx = threadIdx.x; idx < kMatrixWideMaxBlocks * 8; idx += blockDim.x) {
    const int pos = (int)idx / 8, b = (int)idx % 8;
    const int t = k_pad - 1 - pos;
    uint64_t v = 0;
    if (t >= 0 && t < c && b < p.field_w)
      for (int i = 0; i < m; ++i)   // byte i: coefficient m - 1 - i
        v |= (uint64_t)gf_mul(p.mat_coef[t][m - 1 - i], 1u << b, p.field_poly, p.field_w)
             << (8 * i);
    if constexpr (M == 4) {
      bases[pos][b] = (uint32_t)v;
    } else {
      bases[pos][2 * b] = (uint32_t)v;
      bases[pos][2 * b + 1] = (uint32_t)(v >> 32);
    }
  }
  __syncthreads();
  for (int region = 0; region < 2; ++region)
    fill_tables(lds + 65536 * region, 256, 0, 16, L::kMatTableBytes,
                [&](uint32_t f, uint32_t tt) { return entry_of<M>(f, bases[16 * region + tt], 0); });
}

// Block pointers always address global memory; saying so keeps the
// compiler on global (not flat) loads and stores, which leave the LDS
// wait counter alone.
template <class T>
using global_ptr = __attribute__((address_space(1))) T *;

template <class T>
__device__ __forceinline__ global_ptr<T> as_global(T *p) {
  return (global_ptr<T>)(uintptr_t)p;
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Loads W dwords (4*W byte columns starting at col) of one block.  The
// vector form needs the whole chunk inside the block; the byte form reads
// columns past the end of the block as zero.  Every block byte is read (and
// every output byte written) exactly once, so vector accesses carry the
// non-temporal hint.
template <int W, bool BYTEWISE>
__device__ __forceinline__ void load_cols(const uint8_t *ptr, uint32_t col, uint32_t B,
                                          uint32_t (&a)[W]) {
  const global_ptr<const uint8_t> g = as_global(ptr);
  if (!BYTEWISE) {
    const global_ptr<const uint8_t> q = g + col;
    if constexpr (W == 4) {
      const u32x4 v = __builtin_nontemporal_load((const global_ptr<const u32x4>)q);
      a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
    } else if constexpr (W == 2) {
      const u32x2 v = __builtin_nontemporal_load((const global_ptr<const u32x2>)q);
      a[0] = v.x; a[1] = v.y;
    } else {
      a[0] = __builtin_nontemporal_load((const global_ptr<const uint32_t>)q);
    }
  } else {
#pragma unroll
    for (int d = 0; d < W; ++d) {
      uint32_t v = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t c = col + 4 * d + i;
        if (c < B) v |= (uint32_t)g[c] << (8 * i);
      }
      a[d] = v;
    }
  }
}

template <int W, bool BYTEWISE>
__device__ __forceinline__ void store_cols(uint8_t *ptr, uint32_t col, uint32_t B,
                                           const uint32_t (&a)[W]) {
  const global_ptr<uint8_t> g = as_global(ptr);
  if (!BYTEWISE) {
    const global_ptr<uint8_t> q = g + col;
    if constexpr (W == 4) {
      __builtin_nontemporal_store(u32x4{a[0], a[1], a[2], a[3]}, (global_ptr<u32x4>)q);
    } else if constexpr (W == 2) {
      __builtin_nontemporal_store(u32x2{a[0], a[1]}, (global_ptr<u32x2>)q);
    } else {
      __builtin_nontemporal_store(a[0], (global_ptr<uint32_t>)q);
    }
  } else {
#pragma unroll
    for (int d = 0; d < W; ++d) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t c = col + 4 * d + i;
        if (c < B) g[c] = (uint8_t)(a[d] >> (8 * i));
      }
    }
  }
}

// One LFSR step at unrolled window position q for one column.
template <int M, int MODE>
__device__ __forceinline__ void lfsr_step(uint32_t (&s)[M / 4], const uint8_t *lds,
                                          const Lanes<M, MODE> &t, int q) {
  if constexpr (Layout<M, MODE>::kNibble) {
    // x = f << 8 (| the lane offset for M = 4); two lookups, rows f & 15
    // and 16 + (f >> 4)
    uint32_t lo, hi;
    if constexpr (M == 4) {
      const uint32_t x = perm(s[0], t.loff[q], t.lsel[q]);
      lo = x & 0xFFFu;
      hi = (x >> 4) & 0xF00u;
    } else {
      const uint32_t x = perm(s[1], s[0], t.lsel[q]);
      lo = (x & 0xF00u) | t.loff[q];
      hi = (x >> 4) & 0xF00u;
    }
    hi |= t.loffhi[q];
    if constexpr (M == 4) {
      s[0] ^= *reinterpret_cast<const uint32_t *>(lds + lo) ^
              *reinterpret_cast<const uint32_t *>(lds + hi);
    } else {
      const uint2 a = *reinterpret_cast<const uint2 *>(lds + lo);
      const uint2 b = *reinterpret_cast<const uint2 *>(lds + hi);
      s[0] ^= a.x ^ b.x;
      s[1] ^= a.y ^ b.y;
    }
  } else if constexpr (M == 4) {
    const uint32_t addr = perm(s[0], t.loff[q], t.lsel[q]);
    s[0] ^= *reinterpret_cast<const uint32_t *>(lds + addr);
  } else if constexpr (Layout<M, MODE>::kIlv) {
    // feedback byte in dword q & 1; region q & 1 comes with the offsets
    const uint32_t addr = perm(s[q & 1], t.ioff[2 * (q & 1) + (q >> 2)], t.isel[q >> 1]);
    const uint2 v = *reinterpret_cast<const uint2 *>(lds + addr);
    s[0] ^= v.x;
    s[1] ^= v.y;
  } else {
    const uint32_t addr = perm(s[1], s[0], t.lsel[q]) | t.loff[q];
    const uint2 v = *reinterpret_cast<const uint2 *>(lds + addr);
    s[0] ^= v.x;
    s[1] ^= v.y;
  }
}

// Where one stripe's blocks are: kernel arguments (plain launch) or a
// pointer table in device memory (batched launch).
struct PlainSrc {
  const CodecParams &p;
  __device__ const uint8_t *data(int j) const { return p.data[j]; }
  __device__ const uint8_t *par_in(int i) const { return p.par_in[i]; }
  __device__ const uint8_t *input(int x) const { return x < p.k ? p.data[x] : p.par_in[x - p.k]; }
  __device__ uint8_t *out(int o) const { return p.out[o]; }
  __device__ uint32_t B() const { return p.block_bytes; }
  __device__ int k() const { return p.k; }
  __device__ int m() const { return p.m; }
  __device__ int k_pad() const { return p.k_pad; }
  __device__ int n_out() const { return p.n_out; }
  __device__ const uint8_t *zero() const { return p.zero_page; }
};

// Batch tables (pointers, descriptors, bases, tile map) never change while
// a batch kernel runs: reading them through the constant address space lets
// the compiler use scalar loads for uniform indices.
template <class T>
using const_as = const __attribute__((address_space(4))) T *;

template <class T>
__device__ __forceinline__ const_as<T> as_const(const T *p) {
  return (const_as<T>)(uintptr_t)p;
}

__device__ __forceinline__ StripeDesc load_desc(const_as<StripeDesc> p) {
  StripeDesc d;
  d.block_bytes = p->block_bytes;
  d.tile_begin = p->tile_begin;
  d.ptr_off = p->ptr_off;
  d.lfsr_set = p->lfsr_set;
  d.apply_set = p->apply_set;
  d.k = p->k;
  d.m = p->m;
  d.k_pad = p->k_pad;
  d.n_out = p->n_out;
  return d;
}

struct TableSrc {
  const_as<uint64_t> ptrs;   // k data, then m parity inputs, then n_out outputs
  uint32_t bytes;
  int kk, mm, kp, no;
  const uint8_t *zp;
  __device__ const uint8_t *data(int j) const {
    return reinterpret_cast<const uint8_t *>(ptrs[j]);
  }
  __device__ const uint8_t *par_in(int i) const {
    return reinterpret_cast<const uint8_t *>(ptrs[kk + i]);
  }
  __device__ const uint8_t *input(int x) const {   // data x < k, then parity
    return reinterpret_cast<const uint8_t *>(ptrs[x]);
  }
  __device__ uint8_t *out(int o) const { return reinterpret_cast<uint8_t *>(ptrs[kk + mm + o]); }
  __device__ uint32_t B() const { return bytes; }
  __device__ int k() const { return kk; }
  __device__ int m() const { return mm; }
  __device__ int k_pad() const { return kp; }
  __device__ int n_out() const { return no; }
  __device__ const uint8_t *zero() const { return zp; }
};

// Loads item g of a column chunk: for g < k_pad/M the M data blocks of LFSR
// group g (window position q holds block k_pad-1-(g*M+q)); for decode and
// update, item k_pad/M holds the parity read, position b holding p_(m-1-b).  Blocks not
// read (erased, unread, padding) give zeros.  In the vector form of the
// wide (M = 8) kernels every slot issues its load -- an absent block reads
// the zero page at an offset kept inside it -- so the number of loads in
// flight never depends on the path and the compiler can wait for exactly
// the item it is about to use; the narrow kernels skip an absent block's
// loads (measured faster there, though the compiler then waits for every
// load in flight).  A dummy item (the prefetch slot after a lane's last
// item) has only absent slots: re-reading real blocks there would fetch them
// from HBM a second time, since block loads do not keep lines in L2.
template <int M, int W, int MODE, bool BYTEWISE, class Src>
__device__ __forceinline__ void load_item(const Src &src, uint32_t col, int g, int groups,
                                          bool dummy, uint32_t (&a)[M][W]) {
  const uint32_t B = src.B();
#pragma unroll
  for (int q = 0; q < M; ++q) {
    const uint8_t *ptr;
    if constexpr (M == 8) {
      // Input x of the stripe (data block x < k, then the parity read), one
      // table index for both kinds of item: a single uniform load per slot
      // (separate data and parity branches hold more scalar registers live,
      // more than the wide kernels have to spare).
      const bool par = op_of(MODE) != kEncode && g == groups;
      const int x = par ? src.k() + src.m() - 1 - q : src.k_pad() - 1 - (g * M + q);
      const bool ok = !dummy && (par ? q < src.m() : x < src.k());
      ptr = ok ? src.input(x) : nullptr;
    } else if (dummy) {
      ptr = nullptr;
    } else if (op_of(MODE) != kEncode && g == groups) {
      const int i = src.m() - 1 - q;
      ptr = i >= 0 ? src.par_in(i) : nullptr;
    } else {
      const int j = src.k_pad() - 1 - (g * M + q);
      ptr = j < src.k() ? src.data(j) : nullptr;
    }
    if constexpr (BYTEWISE) {
      if (ptr) {
        load_cols<W, true>(ptr, col, B, a[q]);
      } else {
#pragma unroll
        for (int w = 0; w < W; ++w) a[q][w] = 0;
      }
    } else if (M == 4 && ptr == nullptr) {
#pragma unroll
      for (int w = 0; w < W; ++w) a[q][w] = 0;
    } else {
      const bool absent = ptr == nullptr;
      load_cols<W, false>(absent ? src.zero() : ptr, absent ? col & (kZeroPageBytes - 16) : col,
                          B, a[q]);
    }
  }
}

// Matrix update: the packed products of one item (the M changed blocks of
// group gofs / kMatGroupBytes) for one column, whose M symbols are the bytes
// of d0 (and d1 for M = 8).  The group offset is an immediate of the reads.
template <int M, int MODE, uint32_t GOFS>
__device__ __forceinline__ void matrix_lookups(uint32_t d0, uint32_t d1, uint32_t (&acc)[M / 4],
                                               const uint8_t *lds, const Lanes<M, MODE> &t) {
#pragma unroll
  for (int b = 0; b < M; ++b) {
    if constexpr (M == 4) {
      const uint32_t addr = perm(d0, t.aoff[b], t.asel[b]);
      acc[0] ^= *reinterpret_cast<const uint32_t *>(lds + GOFS + addr);
    } else {
      const uint32_t addr = perm(d1, d0, t.asel[b]) | t.aoff[b];
      const uint2 v = *reinterpret_cast<const uint2 *>(lds + GOFS + addr);
      acc[0] ^= v.x;
      acc[1] ^= v.y;
    }
  }
}

// XORs item g into the column states.  The item is transposed so that each
// column's M symbols fill its state window.  An LFSR group is rotated into
// the lane's phase (for M = 4 and the interleaved layout every item is,
// since the state stays rotated; for the other M = 8 kernels only LFSR
// groups, since the state is brought back before the parity item), then
// runs its M steps.  The first `skip` steps are left
// out: they are the leading window positions of the first group that hold
// no block (padding or absent blocks above every present one), where the
// state is still zero, so the feedback is zero and a step changes nothing.
// A matrix-update item adds its blocks' packed products instead.  DATA:
// the item is a data group (else the parity item); a template argument, so
// that the rotation of data groups is code of its own rather than a
// per-column select between rotated and unrotated words.
template <int M, int W, int MODE, bool DATA>
__device__ __forceinline__ void absorb_xor_item(uint32_t (&s)[4 * W][M / 4],
                                                const uint32_t (&a)[M][W], int g,
                                                const uint8_t *lds, const Lanes<M, MODE> &t) {
  constexpr int NQ = M / 4;
  constexpr bool kMatrix = op_of(MODE) == kUpdateMatrix;
  constexpr bool data_item = DATA;
  constexpr bool lfsr = DATA && !kMatrix;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    uint32_t d[NQ][4];
    if constexpr (Layout<M, MODE>::kIlv) {
      // even window positions to dword 0, odd to dword 1, both rotated into
      // the lane's phase by the second round (data and parity items alike)
      transpose4(a[0][w], a[2][w], a[4][w], a[6][w], d[0][0], d[0][1], d[0][2], d[0][3],
                 kT1a, kT1b, t.tin[0], t.tin[1]);
      transpose4(a[1][w], a[3][w], a[5][w], a[7][w], d[NQ - 1][0], d[NQ - 1][1],
                 d[NQ - 1][2], d[NQ - 1][3], kT1a, kT1b, t.tin[0], t.tin[1]);
    } else {
#pragma unroll
      for (int h = 0; h < NQ; ++h) {
        if constexpr (M == 4 && !kMatrix)
          transpose4(a[4 * h][w], a[4 * h + 1][w], a[4 * h + 2][w], a[4 * h + 3][w], d[h][0],
                     d[h][1], d[h][2], d[h][3], kT1a, kT1b, t.tin[0], t.tin[1]);
        else
          transpose4(a[4 * h][w], a[4 * h + 1][w], a[4 * h + 2][w], a[4 * h + 3][w], d[h][0],
                     d[h][1], d[h][2], d[h][3]);
      }
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      if constexpr (kMatrix) {
        if constexpr (data_item) {
          uint32_t acc[NQ];
#pragma unroll
          for (int h = 0; h < NQ; ++h) acc[h] = 0;
          constexpr uint32_t kG = Layout<M, MODE>::kMatGroupBytes;
          if constexpr (Layout<M, MODE>::kWideMatrix) {
            // item g: region (g M) / 16, group ((g M) mod 16) / M of the row
            const uint8_t *rl = lds + ((g * M) >> 4) * 65536;
            const int gr = ((g * M) & 15) / M;
            if (gr == 0)
              matrix_lookups<M, MODE, 0>(d[0][x], d[NQ - 1][x], acc, rl, t);
            else if (gr == 1)
              matrix_lookups<M, MODE, kG>(d[0][x], d[NQ - 1][x], acc, rl, t);
            else if (gr == 2)
              matrix_lookups<M, MODE, 2 * kG>(d[0][x], d[NQ - 1][x], acc, rl, t);
            else
              matrix_lookups<M, MODE, 3 * kG>(d[0][x], d[NQ - 1][x], acc, rl, t);
          } else if (M == 8 || g == 0) {
            matrix_lookups<M, MODE, 0>(d[0][x], d[NQ - 1][x], acc, lds, t);
          } else {
            matrix_lookups<M, MODE, kG>(d[0][x], d[NQ - 1][x], acc, lds, t);
          }
#pragma unroll
          for (int h = 0; h < NQ; ++h) d[h][x] = acc[h];
        }
      } else if constexpr (M == 8 && !Layout<M, MODE>::kIlv) {
        if constexpr (lfsr) {
          const uint32_t lo = perm(d[1][x], d[0][x], t.rin[0]);
          const uint32_t hi = perm(d[1][x], d[0][x], t.rin[1]);
          d[0][x] = lo;
          d[1][x] = hi;
        }
      }
#pragma unroll
      for (int h = 0; h < NQ; ++h) s[4 * w + x][h] ^= d[h][x];
    }
  }
}

template <int M, int W, int MODE>
__device__ __forceinline__ void absorb_xor(uint32_t (&s)[4 * W][M / 4], const uint32_t (&a)[M][W],
                                           bool data_item, int g, const uint8_t *lds,
                                           const Lanes<M, MODE> &t) {
  if (op_of(MODE) == kEncode || data_item)   // an encode has no parity item
    absorb_xor_item<M, W, MODE, true>(s, a, g, lds, t);
  else
    absorb_xor_item<M, W, MODE, false>(s, a, g, lds, t);
}

// The M LFSR steps of a data item (after absorb_xor), less the first `skip`.
template <int M, int W, int MODE>
__device__ __forceinline__ void absorb_steps(uint32_t (&s)[4 * W][M / 4], bool data_item,
                                             int skip, const uint8_t *lds,
                                             const Lanes<M, MODE> &t) {
  constexpr int NC = 4 * W;
  if (data_item && op_of(MODE) != kUpdateMatrix) {
#pragma unroll
    for (int q = 0; q < M; ++q) {
      if (q < skip) continue;
#pragma unroll
      for (int c = 0; c < NC; ++c) lfsr_step<M, MODE>(s[c], lds, t, q);
    }
  }
}

template <int M, int W, int MODE>
__device__ __forceinline__ void absorb_item(uint32_t (&s)[4 * W][M / 4], const uint32_t (&a)[M][W],
                                            bool data_item, int g, int skip, const uint8_t *lds,
                                            const Lanes<M, MODE> &t) {
  absorb_xor<M, W, MODE>(s, a, data_item, g, lds, t);
  absorb_steps<M, W, MODE>(s, data_item, skip, lds, t);
}

// M = 8, narrower kernels: brings the column states back from the lane's
// rotation phase (M = 4 and the interleaved layout keep them rotated; see
// Lanes).
template <int M, int W, int MODE>
__device__ __forceinline__ void unrotate(uint32_t (&s)[4 * W][M / 4], const Lanes<M, MODE> &t) {
  if constexpr (M == 8 && !Layout<M, MODE>::kIlv) {
#pragma unroll
    for (int c = 0; c < 4 * W; ++c) {
      const uint32_t lo = perm(s[c][1], s[c][0], t.rout[0]);
      const uint32_t hi = perm(s[c][1], s[c][0], t.rout[1]);
      s[c][0] = lo;
      s[c][1] = hi;
    }
  }
}

// After the last item of a chunk: byte b of the state is remainder
// coefficient r_(m-1-b) (plus the parity read, for decode and update); for
// M = 4 the state is still rotated by the lane's phase g (byte b at b + g),
// and likewise in the interleaved layout (byte b at position (b + g) / 2 of
// dword b & 1).
// Decode maps it through the apply tables; the result is transposed back to
// blocks and stored: encode and update write parity p_(m-1-b) from byte b,
// decode writes erased block e from byte e.
template <int M, int W, int MODE, bool BYTEWISE, class Src>
__device__ __forceinline__ void finish_chunk(const Src &src, uint32_t col, bool active,
                                             uint32_t (&s)[4 * W][M / 4], const uint8_t *lds,
                                             const Lanes<M, MODE> &t) {
  constexpr int NQ = M / 4;
  constexpr int NC = 4 * W;
  const int m = src.m(), n_out = src.n_out();
  if constexpr (op_of(MODE) == kDecode) {
    // Column by column: every lane walks all M tables (those past m are
    // zero) in its rotated order, and the M products are summed three at a
    // time (v_bitop3_b32).  Other than in the interleaved layout (below),
    // two columns at a time: an empty asm that takes
    // and gives back the states of a pair of columns before and after their
    // lookups keeps the pairs in order; left free, the compiler issues the
    // lookups of every column at once and holds all their results
    // (8 columns x 8 products x 2 dwords).
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if constexpr (NC > 1 && !Layout<M, MODE>::kIlv) {
        if ((c & 1) == 0) pin_pair(s[c], s[c + 1]);
      }
      if constexpr (Layout<M, MODE>::kIlv) {
        // Nibbles of the remainder bytes, each with its table group's row
        // base (+16 high nibbles, +32 odd bytes); step b looks up both
        // nibbles of byte (b - g) mod 8, at position b/2 of dword b & 1.
        // The 16 lookups go in two halves, the second issued after the
        // first is summed (the empty asm), so that a column holds 8
        // products at a time.
        uint32_t nib[2][2];
        nib[0][0] = s[c][0] & 0x0F0F0F0Fu;
        nib[0][1] = __builtin_amdgcn_bitop3_b32(s[c][0] >> 4, 0x0F0F0F0Fu, 0x10101010u, 0xEA);
        nib[1][0] = __builtin_amdgcn_bitop3_b32(s[c][1], 0x0F0F0F0Fu, 0x20202020u, 0xEA);
        nib[1][1] = __builtin_amdgcn_bitop3_b32(s[c][1] >> 4, 0x0F0F0F0Fu, 0x30303030u, 0xEA);
        uint32_t acc[2] = {0u, 0u};
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          uint32_t v[M][2];
#pragma unroll
          for (int i = 0; i < M; ++i) {
            const int b = 4 * half + (i >> 1), hl = i & 1;
            const uint32_t j = b >> 1;
            const uint32_t sel = (j & 1) | ((4 + j) << 8) | (2u << 16) | (0x0Cu << 24);
            const uint32_t addr = perm(nib[b & 1][hl], t.iapp[j >> 1], sel);
            const uint2 x = *reinterpret_cast<const uint2 *>(lds + addr);
            v[i][0] = x.x;
            v[i][1] = x.y;
          }
#pragma unroll
          for (int h = 0; h < NQ; ++h) {
            uint32_t L = xor3(acc[h], v[0][h], v[1][h]);
            L = xor3(L, v[2][h], v[3][h]);
            L = xor3(L, v[4][h], v[5][h]);
            acc[h] = xor3(L, v[6][h], v[7][h]);
          }
          asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(nib[0][0]), "+v"(nib[0][1]),
                       "+v"(nib[1][0]), "+v"(nib[1][1]));
        }
        s[c][0] = acc[0];
        s[c][1] = acc[1];
        continue;
      }
      uint32_t v[M][NQ];
#pragma unroll
      for (int b = 0; b < M; ++b) {
        if constexpr (M == 4) {
          const uint32_t addr = perm(s[c][0], t.aoff[b], t.asel[b]);
          v[b][0] = *reinterpret_cast<const uint32_t *>(lds + addr);
        } else {
          // The apply tables sit 64 KiB above the LFSR copies at the same
          // per-lane offsets (same rotation phase and replica), so the
          // address is the LFSR one plus the region base in one v_or3_b32
          // (the base in an SGPR keeps it out of the per-lane registers).
          static_assert(Layout<M, MODE>::kApplyBase == 65536 &&
                            Layout<M, MODE>::kTableBytes == Layout<M, MODE>::kCopyBytes,
                        "apply offsets equal the LFSR offsets plus the base");
          const uint32_t p = perm(s[c][1], s[c][0], t.lsel[b]);
          uint32_t addr;
          asm("v_or3_b32 %0, %1, %2, %3"
              : "=v"(addr)
              : "v"(p), "v"(t.loff[b]), "s"(Layout<M, MODE>::kApplyBase));
          const uint2 x = *reinterpret_cast<const uint2 *>(lds + addr);
          v[b][0] = x.x;
          v[b][1] = x.y;
        }
      }
#pragma unroll
      for (int h = 0; h < NQ; ++h) {
        uint32_t L = xor3(v[0][h], v[1][h], v[2][h]);
        if constexpr (M == 4) {
          L ^= v[3][h];
        } else {
          L = xor3(L, v[3][h], v[4][h]);
          L = xor3(L, v[5][h], v[6][h]);
          L ^= v[7][h];
        }
        s[c][h] = L;
      }
      if constexpr (NC > 1) {
        if (c & 1) pin_pair(s[c - 1], s[c]);
      }
    }
  }
#pragma unroll
  for (int h = 0; h < NQ; ++h) {
    uint32_t o[4][W];
    // encode and update (M = 4 or interleaved): the state is still rotated
    // by the lane's phase; interleaved: output bb of dword h is byte 2bb + h
    constexpr bool kRotated = (M == 4 || Layout<M, MODE>::kIlv) && op_of(MODE) != kDecode &&
                              op_of(MODE) != kUpdateMatrix;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      if constexpr (kRotated)
        transpose4(s[4 * w][h], s[4 * w + 1][h], s[4 * w + 2][h], s[4 * w + 3][h], o[0][w],
                   o[1][w], o[2][w], o[3][w], t.tout[0], t.tout[1]);
      else
        transpose4(s[4 * w][h], s[4 * w + 1][h], s[4 * w + 2][h], s[4 * w + 3][h], o[0][w],
                   o[1][w], o[2][w], o[3][w]);
    }
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const int b = kRotated && M == 8 ? 2 * bb + h : 4 * h + bb;
      const int oi = op_of(MODE) == kDecode ? b : m - 1 - b;
      if (oi >= 0 && oi < n_out && active)
        store_cols<W, BYTEWISE>(src.out(oi), col, src.B(), o[bb]);
    }
  }
}

// An empty asm that takes and gives back every column state and may touch
// memory: the XORs of an item into the states complete before it, and no
// load is issued above it.  (A scheduling barrier alone leaves earlier
// passes free to sink the XORs below the next item's loads, which then need
// registers of their own.)
template <int W, int NQ>
__device__ __forceinline__ void fence_states(uint32_t (&s)[4 * W][NQ]) {
#pragma unroll
  for (int c = 0; c < 4 * W; c += 2) {
    if constexpr (NQ == 1)
      asm volatile("" : "+v"(s[c][0]), "+v"(s[c + 1][0])::"memory");
    else
      asm volatile("" : "+v"(s[c][0]), "+v"(s[c][1]), "+v"(s[c + 1][0]), "+v"(s[c + 1][1])::"memory");
  }
}

// Whether a variant keeps one item buffer instead of two (see
// process_columns): the wide codes at 16 bytes per lane, and the wide
// decode at 8, which then fit four waves per SIMD (at most 128 VGPRs).
template <int M, int W, int MODE>
constexpr bool kSingleBuffer() {
  return M == 8 && (W == 4 || (W == 2 && op_of(MODE) == kDecode));
}

// Encodes, updates or decodes chunks c0 + (r*lanes + lane)*NC, r = 0, 1,
// ..., of one stripe, for the n chunks starting at c0.  Control flow is
// uniform: every lane runs the same rounds, and a lane whose chunk index is
// past n works on chunk c0 again and stores nothing, so block pointers stay
// in SGPRs and the loads need no branches.  The walk is a software pipeline
// over items (LFSR groups, then for decode and update the parity item): the
// loads of the next item, also across chunks, are issued before the current
// item goes through the LFSR, so each lane keeps up to 2*M block loads in
// flight.  A chunk's parity is read (update) before the same lane writes it.
template <int M, int W, int MODE, bool BYTEWISE, class Src>
__device__ __forceinline__ void process_columns(const Src &src, uint32_t c0, uint32_t n,
                                                uint32_t lane, uint32_t lanes,
                                                const uint8_t *lds, const Lanes<M, MODE> &t) {
  constexpr uint32_t NC = 4 * W;
  if (n == 0) return;
  const int groups = src.k_pad() / M;
  const int items = groups + (op_of(MODE) == kEncode ? 0 : 1);
  const uint32_t rounds = (n + lanes - 1) / lanes;
  auto col_of = [&](uint32_t r) {
    const uint32_t idx = r * lanes + lane;
    return idx < n ? c0 + idx * NC : c0;
  };
  // Leading window positions of the first group with no block above any
  // present one: their LFSR steps are skipped (see absorb_item).
  int lead = 0;
#pragma unroll
  for (int q = 0; q < M - 1; ++q) {
    const int j = src.k_pad() - 1 - q;
    if (lead == q && (j >= src.k() || src.data(j) == nullptr)) lead = q + 1;
  }

  uint32_t s[4 * W][M / 4];
  uint32_t a[M][W], b[M][W];
#pragma unroll
  for (int c = 0; c < 4 * W; ++c)
#pragma unroll
    for (int h = 0; h < M / 4; ++h) s[c][h] = 0;

  uint32_t r = 0;   // round of the current item (uniform)
  int g = 0;        // item within the chunk (uniform)
  load_item<M, W, MODE, BYTEWISE>(src, col_of(0), 0, groups, false, a);

  if constexpr (kSingleBuffer<M, W, MODE>()) {
    // One item buffer: the item is XORed into the states first, then the
    // next item's loads are issued into the same registers and stay in
    // flight while the current one runs its LFSR steps.
    for (;;) {
      uint32_t nr = r;
      int ng = g + 1;
      if (ng == items) {
        ng = 0;
        ++nr;
      }
      const bool more = nr < rounds;
      absorb_xor<M, W, MODE>(s, a, g < groups, g, lds, t);
      // keeps the next loads after the XOR, so they reuse the registers
      fence_states<W>(s);
      load_item<M, W, MODE, BYTEWISE>(src, col_of(more ? nr : r), more ? ng : g, groups, !more,
                                      a);
      absorb_steps<M, W, MODE>(s, g < groups, g == 0 ? lead : 0, lds, t);
      if (op_of(MODE) != kUpdateMatrix && g == groups - 1) unrotate<M, W, MODE>(s, t);
      if (g == items - 1) {
        finish_chunk<M, W, MODE, BYTEWISE>(src, col_of(r), r * lanes + lane < n, s, lds, t);
#pragma unroll
        for (int c = 0; c < 4 * W; ++c)
#pragma unroll
          for (int h = 0; h < M / 4; ++h) s[c][h] = 0;
      }
      r = nr;
      g = ng;
      if (!more) return;
    }
  }

  // One pipeline stage: prefetch the item after (r, g) into nxt, consume cur.
  auto stage = [&](uint32_t (&cur)[M][W], uint32_t (&nxt)[M][W]) -> bool {
    uint32_t nr = r;
    int ng = g + 1;
    if (ng == items) {
      ng = 0;
      ++nr;
    }
    const bool more = nr < rounds;
    // past the last item the prefetch is a dummy (and is unused)
    load_item<M, W, MODE, BYTEWISE>(src, col_of(more ? nr : r), more ? ng : g, groups, !more,
                                    nxt);
    absorb_item<M, W, MODE>(s, cur, g < groups, g, g == 0 ? lead : 0, lds, t);
    if (op_of(MODE) != kUpdateMatrix && g == groups - 1) unrotate<M, W, MODE>(s, t);
    if (g == items - 1) {
      finish_chunk<M, W, MODE, BYTEWISE>(src, col_of(r), r * lanes + lane < n, s, lds, t);
#pragma unroll
      for (int c = 0; c < 4 * W; ++c)
#pragma unroll
        for (int h = 0; h < M / 4; ++h) s[c][h] = 0;
    }
    r = nr;
    g = ng;
    return more;
  };
  for (;;) {
    if (!stage(a, b)) break;
    if (!stage(b, a)) break;
  }
}

// Columns [c0, c1) of one stripe: full chunks by all lanes, then the last
// partial chunk (fewer than 4*W columns, only at the end of a block) by one
// thread with byte loads and stores.
template <int M, int W, int MODE, class Src>
__device__ __forceinline__ void process_range(const Src &src, uint32_t c0, uint32_t c1,
                                              uint32_t lane, uint32_t lanes, const uint8_t *lds,
                                              const Lanes<M, MODE> &t) {
  constexpr uint32_t NC = 4 * W;
  const uint32_t n_full = (c1 - c0) / NC;
  process_columns<M, W, MODE, false>(src, c0, n_full, lane, lanes, lds, t);
  const uint32_t tail = c0 + n_full * NC;
  if (tail < c1 && lane == 0)
    process_columns<M, 1, MODE, true>(src, tail, (c1 - tail + 3) / 4, 0, 1, lds, t);
}

// Workgroup size bound per variant: at most 128 VGPRs (four waves per SIMD)
// for 1024 threads.  The narrow codes at 16 bytes per lane hold two items
// of loads in flight and need more, so they take at most 512 threads; the
// wide codes at 16 bytes per lane fit with one item buffer.
template <int M, int W, int MODE>
constexpr int max_threads() {
  return W == 4 && M == 4 ? 512 : 1024;
}

// One stripe per launch: grid-stride loop over its column chunks.
template <int M, int W, int MODE, bool BYTEWISE>
__global__ void __launch_bounds__((max_threads<M, W, MODE>()))
__attribute__((amdgpu_waves_per_eu(M == 4 && !wide_matrix_of(MODE) ? 4 : 2)))
codec_kernel(CodecParams p) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[Layout<M, MODE>::kLdsBytes];
  if constexpr (Layout<M, MODE>::kWideMatrix) {
    __shared__ uint32_t bases[kMatrixWideMaxBlocks][16];
    build_wide_matrix_tables<M>(lds, bases, p);
  } else if constexpr (op_of(MODE) == kUpdateMatrix) {
    build_matrix_tables<M>(lds, &p.apply_basis[0][0], p.k, p.k_pad);
  } else {
    build_lfsr_tables<M, MODE>(lds, p.lfsr_basis);
    if constexpr (op_of(MODE) == kDecode)
      build_apply_tables<M, MODE>(lds, &p.apply_basis[0][0], p.m);
  }
  __syncthreads();

  constexpr uint32_t NC = 4 * W;
  const PlainSrc src{p};
  const Lanes<M, MODE> t = make_lanes<M, MODE>();
  const uint32_t lane = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t lanes = gridDim.x * blockDim.x;
  const uint32_t B = (uint32_t)p.block_bytes;
  if constexpr (BYTEWISE)
    process_columns<M, W, MODE, true>(src, 0, (B + NC - 1) / NC, lane, lanes, lds, t);
  else
    process_range<M, W, MODE>(src, 0, B, lane, lanes, lds, t);
}

__device__ __forceinline__ uint32_t uniform(uint32_t x) {
  return __builtin_amdgcn_readfirstlane(x);
}

// Copies a group's upload (header, descriptors, pointers, table bases) from
// coherent pinned host memory to the arena, 16 bytes per thread and step.
// The size is in the upload's own header.  Reading the host copy from the
// graph's first kernel keeps the upload on the launch queue.
__global__ void batch_pull_kernel(BatchGroup g) {
  const uint64_t bytes = reinterpret_cast<const BatchHeader *>(g.host_src)->upload_bytes;
  const uint4 *src = reinterpret_cast<const uint4 *>(g.host_src);
  uint4 *dst = reinterpret_cast<uint4 *>(g.arena);
  const uint64_t n = bytes / 16;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Fills the tile -> stripe map of a batch group (one thread per tile, a
// binary search over the stripes' first tiles) and clears the tile counter;
// runs before the persistent kernel in the same graph.  The grid covers the
// group's tile capacity; threads past the batch's tiles only exit.
__global__ void batch_prepare_kernel(BatchGroup g) {
  BatchHeader *hdr = reinterpret_cast<BatchHeader *>(g.arena);
  const StripeDesc *descs = reinterpret_cast<const StripeDesc *>(g.arena + hdr->off_descs);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) hdr->counter = 0;
  if (t >= hdr->total_tiles) return;
  uint32_t lo = 0, hi = hdr->n_stripes - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) / 2;
    if (descs[mid].tile_begin <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  g.tile_stripe[t] = lo;
}

// Persistent kernel over every tile of a batch group.  Each workgroup takes
// the next claim from an atomic counter (prefetched one claim ahead), maps
// it to a tile, finds the tile's stripe through the tile map, re-expands the
// LDS tables only when the stripe's code, erasure pattern or changed-block
// set differs from the one staged, and encodes, decodes or updates the
// tile's columns.  Every wave leaves the loop once the counter passes the
// last claim.
template <int M, int W, int MODE>
__global__ void __launch_bounds__((max_threads<M, W, MODE>()))
__attribute__((amdgpu_waves_per_eu(M == 4 ? 4 : 2))) batch_kernel(BatchGroup g) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[Layout<M, MODE>::kLdsBytes];
  __shared__ uint64_t next_claim;
  BatchHeader *hdr = reinterpret_cast<BatchHeader *>(g.arena);
  const_as<BatchHeader> chdr = as_const(hdr);
  const uint64_t total = chdr->total_tiles;
  const_as<StripeDesc> descs = as_const(reinterpret_cast<const StripeDesc *>(g.arena + chdr->off_descs));
  const_as<uint64_t> ptr_table = as_const(reinterpret_cast<const uint64_t *>(g.arena + chdr->off_ptrs));
  const uint32_t *lfsr_sets = reinterpret_cast<const uint32_t *>(g.arena + chdr->off_lfsr);
  const uint32_t *apply_sets = reinterpret_cast<const uint32_t *>(g.arena + chdr->off_apply);
  const_as<uint32_t> tile_stripe = as_const(g.tile_stripe);
  unsigned long long *counter = reinterpret_cast<unsigned long long *>(&hdr->counter);
  const uint32_t tile_cols = chdr->tile_cols;
  const Lanes<M, MODE> lt = make_lanes<M, MODE>();
  uint32_t staged_lfsr = ~0u, staged_apply = ~0u;

  // Claim c maps to tile c (order 0: at any moment the workgroups work on
  // neighbouring tiles) or to tile (c mod P) * run + c / P (order 1: a
  // workgroup's successive claims, about P apart, are neighbouring tiles of
  // its own run).  Which is faster depends on the workload; the order is a
  // launch parameter.  Claims past the last tile are skipped.
  const bool runs = chdr->tile_order != 0;
  const uint64_t P = gridDim.x;
  const uint64_t run = (total + P - 1) / P;
  const uint64_t claims = runs ? run * P : total;
  if (threadIdx.x == 0) next_claim = atomicAdd(counter, 1ull);
  __syncthreads();
  for (;;) {
    const uint64_t c =
        (uint64_t)uniform((uint32_t)(next_claim >> 32)) << 32 | uniform((uint32_t)next_claim);
    __syncthreads();   // every thread has read next_claim
    if (c >= claims) break;
    if (threadIdx.x == 0) next_claim = atomicAdd(counter, 1ull);
    const uint64_t tile = runs ? (c % P) * run + c / P : c;
    if (tile >= total) {
      __syncthreads();   // next_claim is about to change
      continue;
    }

    const uint32_t s = tile_stripe[tile];
    const StripeDesc d = load_desc(descs + s);
    constexpr bool kMatrix = op_of(MODE) == kUpdateMatrix;
    const bool new_lfsr = !kMatrix && d.lfsr_set != staged_lfsr;
    const bool new_apply =
        (op_of(MODE) == kDecode || kMatrix) && d.apply_set != staged_apply;
    if (new_lfsr || new_apply) {
      // The barrier at the end of the previous tile guarantees no wave still
      // reads the old tables.
      if (new_lfsr) build_lfsr_tables<M, MODE>(lds, lfsr_sets + 16 * d.lfsr_set);
      if constexpr (kMatrix) {
        if (new_apply)
          build_matrix_tables<M>(lds, apply_sets + kMaxM * 16 * d.apply_set, d.k, d.k_pad);
      } else {
        if (new_apply)
          build_apply_tables<M, MODE>(lds, apply_sets + kMaxM * 16 * d.apply_set, d.m);
      }
      staged_lfsr = d.lfsr_set;
      staged_apply = d.apply_set;
      __syncthreads();
    }

    const uint32_t bytes = (uint32_t)d.block_bytes;
    const TableSrc src{ptr_table + d.ptr_off, bytes, d.k, d.m, d.k_pad, d.n_out, g.zero_page};
    const uint32_t c0 = (uint32_t)(tile - d.tile_begin) * tile_cols;
    const uint32_t c1 = bytes - c0 > tile_cols ? c0 + tile_cols : bytes;
    process_range<M, W, MODE>(src, c0, c1, threadIdx.x, blockDim.x, lds, lt);
    __syncthreads();   // tables and next_claim are about to change
  }
}

using KernelFn = void (*)(CodecParams);
using BatchFn = void (*)(BatchGroup);

// The wide kernels at 16 bytes per lane take the interleaved M = 8 layout
// for the LFSR operations with packed tables: they run one workgroup per CU
// (128 VGPRs at 1024 threads) whatever their LDS, so its 128-144 KiB cost
// no occupancy.  Narrower kernels keep the 64 KiB layout.
constexpr int wide_mode(int mode) {
  return op_of(mode) == kUpdateMatrix || nibble_of(mode) ? mode : mode | kIlvBit;
}

template <int MODE>
KernelFn pick(int sb, int w, bool bytewise) {
  if (bytewise) return sb == 4 ? codec_kernel<4, 1, MODE, true> : codec_kernel<8, 1, MODE, true>;
  if (sb == 4) {
    if (w == 4) return codec_kernel<4, 4, MODE, false>;
    if (w == 2) return codec_kernel<4, 2, MODE, false>;
    return codec_kernel<4, 1, MODE, false>;
  }
  if (w == 4) return codec_kernel<8, 4, wide_mode(MODE), false>;
  if (w >= 2) return codec_kernel<8, 2, MODE, false>;
  return codec_kernel<8, 1, MODE, false>;
}

template <int MODE>
BatchFn pick_batch(int sb, int w) {
  if (sb == 4) {
    if (w == 4) return batch_kernel<4, 4, MODE>;
    if (w == 2) return batch_kernel<4, 2, MODE>;
    return batch_kernel<4, 1, MODE>;
  }
  if (w == 4) return batch_kernel<8, 4, wide_mode(MODE)>;
  if (w >= 2) return batch_kernel<8, 2, MODE>;
  return batch_kernel<8, 1, MODE>;
}

}  // namespace

int codec_wgs_per_cu(Mode) { return 2; }

int codec_plain_max_dwords(int) { return 4; }

int codec_max_threads(Mode mode, int sb, int dwords_per_lane) {
  return dwords_per_lane == 4 && sb == 4 ? 512 : 1024;
}

int launch_codec(Mode mode, int sb, const CodecParams &p, const LaunchCfg &cfg, void *stream) {
  const int w = cfg.dwords_per_lane;
  KernelFn fn;
  switch (mode) {
    case kEncode: fn = pick<kEncode>(sb, w, cfg.bytewise); break;
    case kDecode: fn = pick<kDecode>(sb, w, cfg.bytewise); break;
    case kUpdate: fn = pick<kUpdate>(sb, w, cfg.bytewise); break;
    case kUpdateMatrix: fn = pick<kUpdateMatrix>(sb, w, cfg.bytewise); break;
    case kUpdateMatrixWide: fn = pick<kUpdateMatrixWide>(sb, w, cfg.bytewise); break;
    default: return (int)hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(fn, dim3(cfg.grid), dim3(cfg.threads), 0,
                     reinterpret_cast<hipStream_t>(stream), p);
  return (int)hipGetLastError();
}

int launch_batch(Mode mode, int sb, const BatchGroup &g, uint64_t max_tiles,
                 const LaunchCfg &cfg, void *stream, bool pull) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (pull) {
    hipLaunchKernelGGL(batch_pull_kernel, dim3(64), dim3(256), 0, st, g);
    const int perr = (int)hipGetLastError();
    if (perr) return perr;
  }
  const uint32_t prep_threads = 256;
  const uint32_t prep_grid = (uint32_t)((max_tiles + prep_threads - 1) / prep_threads);
  hipLaunchKernelGGL(batch_prepare_kernel, dim3(prep_grid ? prep_grid : 1), dim3(prep_threads),
                     0, st, g);
  int err = (int)hipGetLastError();
  if (err) return err;
  if (cfg.bm) return launch_bitmatrix_batch(*cfg.bm, g, cfg.grid, cfg.threads, st);
  if (cfg.nibble_update) return launch_nibble_batch(g, cfg.grid, cfg.threads, st);
  const int w = cfg.dwords_per_lane;
  BatchFn fn;
  // (the matrix-form update has no LFSR tables: the placement does not apply)
  const bool nibble = cfg.nibble && mode != kUpdateMatrix;
  switch ((int)mode | (nibble ? kNibbleBit : 0)) {
    case kEncode: fn = pick_batch<kEncode>(sb, w); break;
    case kDecode: fn = pick_batch<kDecode>(sb, w); break;
    case kUpdate: fn = pick_batch<kUpdate>(sb, w); break;
    case kUpdateMatrix: fn = pick_batch<kUpdateMatrix>(sb, w); break;
    case kEncode | kNibbleBit: fn = pick_batch<kEncode | kNibbleBit>(sb, w); break;
    case kDecode | kNibbleBit: fn = pick_batch<kDecode | kNibbleBit>(sb, w); break;
    case kUpdate | kNibbleBit: fn = pick_batch<kUpdate | kNibbleBit>(sb, w); break;
    default: return (int)hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(fn, dim3(cfg.grid), dim3(cfg.threads), 0, st, g);
  return (int)hipGetLastError();
}

}  // namespace rsp
