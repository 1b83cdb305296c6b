// Bit-sliced (XOR-only) encode: the generator-matrix form of the
// polynomial code (Sec. 6), parity p_i = sum_j c_ij d_j with c_ij the
// coefficient of x^i in x^(m+j) mod g(x), where every product by c_ij is
// written as an 8 x 8 matrix over GF(2) acting on the 8 bit planes of the
// data bytes (Sec. 6 names this multiplication-free form as future work).
//
// The coefficients depend only on (k, m) and the field, so for the codes
// compiled in here they are compile-time constants and the whole XOR
// network unrolls into straight-line code: no tables, no LDS, no serial
// LFSR chain.  Any other code (k <= kBitmatrixMaxK, either field) takes its
// GF(2) rows with the launch and applies each row as masked XORs.  Each
// lane takes 32 byte columns (two 16-byte runs 1 KiB apart, so every load
// instruction of a wave is one contiguous 1 KiB), bit-transposes each
// block's 32 bytes into 8 planes of 32 bits, XORs the planes into the
// m x 8 parity planes, and transposes those back.
#include <hip/hip_runtime.h>

#include <utility>

#include "batch_tiles.h"
#include "rs_internal.h"

namespace rsp {
namespace {

// GF(2^8) of the library's default field: x^8 + x^4 + x^3 + x^2 + 1, alpha = 2.
constexpr unsigned kPoly = 0x11D;

constexpr uint8_t cmul(uint8_t a, uint8_t b) {
  unsigned r = 0, x = a;
  for (int i = 0; i < 8; ++i) {
    if ((b >> i) & 1) r ^= x;
    x <<= 1;
    if (x & 0x100) x ^= kPoly;
  }
  return (uint8_t)r;
}

template <int K, int M>
struct GenMatrix {
  uint8_t c[M][K];
};

// c[i][j] = coefficient of x^i in x^(M+j) mod g(x), g(x) = prod_{i<M}(x + alpha^i)
// (Sec. 3.1 for g; Sec. 6 for the generator-matrix columns).
template <int K, int M>
constexpr GenMatrix<K, M> gen_matrix() {
  uint8_t g[M + 1] = {};
  g[0] = 1;
  uint8_t root = 1;
  for (int i = 0; i < M; ++i) {   // g <- g * (x + root)
    for (int d = i + 1; d >= 1; --d) g[d] = g[d - 1] ^ cmul(g[d], root);
    g[0] = cmul(g[0], root);
    root = cmul(root, 2);
  }
  GenMatrix<K, M> out{};
  uint8_t r[M] = {};
  for (int i = 0; i < M; ++i) r[i] = g[i];   // x^M mod g (g monic, char 2)
  for (int j = 0; j < K; ++j) {
    for (int i = 0; i < M; ++i) out.c[i][j] = r[i];
    const uint8_t top = r[M - 1];             // r <- x r mod g
    for (int i = M - 1; i >= 1; --i) r[i] = r[i - 1] ^ cmul(top, g[i]);
    r[0] = cmul(top, g[0]);
  }
  return out;
}

template <int K, int M>
struct Coeffs {
  static constexpr GenMatrix<K, M> G = gen_matrix<K, M>();
};

// Calls f(integral_constant<int, 0>), ..., f(integral_constant<int, N-1>).
template <class F, int... I>
__device__ __forceinline__ void unroll_seq(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void unroll(F &&f) {
  unroll_seq(f, std::make_integer_sequence<int, N>{});
}

// Row b of the GF(2) matrix of the product by coef: bit b' is set when bit
// b of coef * 2^b' is.
constexpr unsigned product_row(uint8_t coef, int b) {
  unsigned row = 0;
  for (int bi = 0; bi < 8; ++bi)
    if ((cmul(coef, (uint8_t)(1u << bi)) >> b) & 1) row |= 1u << bi;
  return row;
}

// acc ^ (XOR of x[b'] over the bits b' of ROW), two planes per v_bitop3_b32
// (truth table 0x96: three-way XOR).
template <unsigned ROW>
__device__ __forceinline__ uint32_t xor_row(uint32_t acc, const uint32_t (&x)[8]) {
  if constexpr (ROW == 0) {
    return acc;
  } else {
    constexpr int a = __builtin_ctz(ROW);
    constexpr unsigned rest = ROW & (ROW - 1);
    if constexpr (rest == 0) {
      return acc ^ x[a];
    } else {
      constexpr int b = __builtin_ctz(rest);
      return xor_row<rest & (rest - 1)>(__builtin_amdgcn_bitop3_b32(acc, x[a], x[b], 0x96), x);
    }
  }
}

// In-place transpose of the 8 x 8 bit matrices formed by byte t of x[0..7]
// (row r = x[r], column b = bit b): afterwards bit b of byte t of x[r] is
// bit r of byte t of the old x[b].  Three rounds of block swaps; the
// transpose is its own inverse.
__device__ __forceinline__ void bit_transpose(uint32_t (&x)[8]) {
  auto swap = [](uint32_t &lo, uint32_t &hi, int k, uint32_t mask) {
    const uint32_t nlo = (lo & mask) | ((hi << k) & ~mask);
    const uint32_t nhi = ((lo >> k) & mask) | (hi & ~mask);
    lo = nlo;
    hi = nhi;
  };
#pragma unroll
  for (int r = 0; r < 4; ++r) swap(x[r], x[r + 4], 4, 0x0F0F0F0Fu);
#pragma unroll
  for (int r = 0; r < 8; r += 4) {
    swap(x[r], x[r + 2], 2, 0x33333333u);
    swap(x[r + 1], x[r + 3], 2, 0x33333333u);
  }
#pragma unroll
  for (int r = 0; r < 8; r += 2) swap(x[r], x[r + 1], 1, 0x55555555u);
}

using u32x4 = uint32_t __attribute__((ext_vector_type(4)));

template <class T>
using global_ptr = __attribute__((address_space(1))) T *;

// 16 columns starting at byte s of a block of B bytes.  FULL: all 16 lie
// inside the block (one 16-byte load); otherwise bytes past B read as zero.
template <bool FULL>
__device__ __forceinline__ void load16(const uint8_t *blk, uint64_t s, uint64_t B,
                                       uint32_t *w) {
  if constexpr (FULL) {
    const u32x4 v = __builtin_nontemporal_load((const global_ptr<const u32x4>)(blk + s));
    w[0] = v.x;
    w[1] = v.y;
    w[2] = v.z;
    w[3] = v.w;
  } else {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      uint32_t v = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint64_t at = s + 4 * d + t;
        if (at < B) v |= (uint32_t)blk[at] << (8 * t);
      }
      w[d] = v;
    }
  }
}

template <bool FULL>
__device__ __forceinline__ void store16(uint8_t *blk, uint64_t s, uint64_t B,
                                        const uint32_t *w) {
  if constexpr (FULL) {
    __builtin_nontemporal_store(u32x4{w[0], w[1], w[2], w[3]},
                                (global_ptr<u32x4>)(blk + s));
  } else {
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint64_t at = s + 4 * d + t;
        if (at < B) blk[at] = (uint8_t)(w[d] >> (8 * t));
      }
  }
}

struct BitmatrixParams {
  const uint8_t *data[kBitmatrixMaxK];
  uint8_t *parity[kMaxM];
  uint64_t block_bytes;
};

constexpr uint64_t kWaveCols = kBitmatrixTileCols;   // 64 lanes x 32 columns

// Block pointers of one stripe: kernel arguments (plain launch) or the
// batch pointer table (k data, m parity-in, then the m parity outputs).
struct ArgBlocks {
  const BitmatrixParams &p;
  __device__ const uint8_t *data(int j) const { return p.data[j]; }
  __device__ uint8_t *parity(int i) const { return p.parity[i]; }
};

template <class T>
using const_as = const __attribute__((address_space(4))) T *;

template <int K, int M>
struct TableBlocks {
  const_as<uint64_t> ptrs;
  __device__ const uint8_t *data(int j) const {
    return reinterpret_cast<const uint8_t *>(ptrs[j]);
  }
  __device__ uint8_t *parity(int i) const { return reinterpret_cast<uint8_t *>(ptrs[K + M + i]); }
};

// Blocks loaded ahead of the one being XORed in: each lane keeps
// kDepth + 1 blocks of 32 bytes in registers besides the m x 8 parity planes.
// Fewer loads in flight streamed faster (batched RS(10,4): 0.620 ms with one
// block ahead, 0.628 with two, 0.632 with three; RS(32,8): two ahead).
template <int M>
constexpr int bitmatrix_depth() { return M <= 4 ? 1 : 2; }

// One wave encodes 2048 columns of a stripe: lane l holds columns s0 ..
// s0 + 15 (dwords 0-3) and s1 = s0 + 1024 .. (dwords 4-7).  FULL: all of
// them lie below `lim`; otherwise columns from `lim` on are neither read
// nor written.
template <int K, int M, bool FULL, class Blocks>
__device__ __forceinline__ void encode_columns(const Blocks &src, uint64_t s0, uint64_t s1,
                                               uint64_t lim) {
  // (the byte-wise tail path loads one block ahead only)
  constexpr int kD = FULL ? bitmatrix_depth<M>() : 1;
  constexpr int D = kD < K ? kD : K;
  constexpr int R = D + 1;
  uint32_t par[M][8];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int b = 0; b < 8; ++b) par[i][b] = 0;

  uint32_t blk[R][8];   // block j in blk[j % R]
  unroll<D>([&](auto J) {
    constexpr int j = decltype(J)::value;
    load16<FULL>(src.data(j), s0, lim, blk[j]);
    load16<FULL>(src.data(j), s1, lim, blk[j] + 4);
  });
  unroll<K>([&](auto J) {
    constexpr int j = decltype(J)::value;
    if constexpr (j + D < K) {
      load16<FULL>(src.data(j + D), s0, lim, blk[(j + D) % R]);
      load16<FULL>(src.data(j + D), s1, lim, blk[(j + D) % R] + 4);
    }
    // keep the scheduler from hoisting later blocks' loads above this
    // block's work (their registers would not fit)
    __builtin_amdgcn_sched_barrier(0);
    uint32_t(&cur)[8] = blk[j % R];
    bit_transpose(cur);   // cur[b] = bit plane b of the lane's 32 columns
    unroll<M>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr uint8_t coef = Coeffs<K, M>::G.c[i][j];
      // plane b of coef * d = XOR of the planes b' of d in row b
      unroll<8>([&](auto Bo) {
        constexpr int b = decltype(Bo)::value;
        par[i][b] = xor_row<product_row(coef, b)>(par[i][b], cur);
        // an empty asm pins the partial sum here: without it the XORs of
        // all blocks are reassociated into one tree that keeps every
        // block's planes live at once
        asm volatile("" : "+v"(par[i][b]));
      });
    });
  });

#pragma unroll
  for (int i = 0; i < M; ++i) {
    bit_transpose(par[i]);
    store16<FULL>(src.parity(i), s0, lim, par[i]);
    store16<FULL>(src.parity(i), s1, lim, par[i] + 4);
  }
}

// Columns [c, min(c + 2048, lim)) by one wave.
template <int K, int M, class Blocks>
__device__ __forceinline__ void encode_chunk(const Blocks &src, uint64_t c, uint64_t lim,
                                             uint32_t lane) {
  const uint64_t s0 = c + 16 * lane, s1 = s0 + 1024;
  if (c + kWaveCols <= lim)
    encode_columns<K, M, true>(src, s0, s1, lim);
  else
    encode_columns<K, M, false>(src, s0, s1, lim);
}

// Register budget: M parity x 8 planes, kDepth + 1 blocks of 8 dwords,
// temporaries.
template <int M>
constexpr int bitmatrix_waves_per_eu() { return M <= 4 ? 5 : 4; }

constexpr int kBitmatrixThreads = 256;

template <int K, int M>
__global__ void __launch_bounds__(kBitmatrixThreads)
__attribute__((amdgpu_waves_per_eu(bitmatrix_waves_per_eu<M>()))) bitmatrix_kernel(BitmatrixParams p) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBitmatrixThreads + threadIdx.x) >> 6;
  const uint64_t c = wave * kWaveCols;
  if (c >= p.block_bytes) return;
  encode_chunk<K, M>(ArgBlocks{p}, c, p.block_bytes, threadIdx.x & 63);
}

__device__ __forceinline__ uint32_t uniform(uint32_t x) {
  return __builtin_amdgcn_readfirstlane(x);
}

// Persistent batch kernel of a compiled-in code: every stripe of the group
// is an RS(K, M) stripe.
// (at most 2 workgroups of at most 1024 threads per CU: 4 waves per SIMD at
// 512 threads, so the kernel may use 128 VGPRs; RS(10,4) spills nothing,
// the RS(32,8) network keeps a few values in scratch)
template <int K, int M>
__global__ void __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu(4))) bitmatrix_batch_kernel(BatchGroup g) {
  const uint32_t lane = threadIdx.x & 63, wave = uniform(threadIdx.x >> 6),
                 waves = blockDim.x >> 6;
  tiles::run(g, [&](tiles::cptr<StripeDesc>, const_as<uint64_t> ptrs, uint64_t c0, uint64_t c1) {
    // the waves take neighbouring 2048-column chunks of the tile
    for (uint64_t cc = c0 + (uint64_t)wave * kWaveCols; cc < c1; cc += (uint64_t)waves * kWaveCols)
      encode_chunk<K, M>(TableBlocks<K, M>{ptrs}, cc, c1, lane);
  });
}

// ---------------------------------------------------- runtime coefficients --
//
// Any code with k <= kBitmatrixMaxK over any field: the GF(2) rows of the
// products come with the launch (rows.r[j][i][b]: bit b' set when bit b of
// c_ij * 2^b' is), and each output plane is the XOR of the data planes its
// row selects, as AND with an all-ones or all-zero mask made from the row
// on the scalar unit: 8 vector operations per row whatever its bits, where
// the compiled-in networks skip the zero bits.

struct BitmatrixRtParams {
  BitmatrixParams io;
  int32_t k;
  BitRows rows;
};

struct BitmatrixRtBatch {
  BatchGroup g;
  int32_t k;
  BitRows rows;
};

// Pointer-table blocks with the code's k known at run time.
struct TableBlocksRt {
  const_as<uint64_t> ptrs;
  int k, m;
  __device__ const uint8_t *data(int j) const {
    return reinterpret_cast<const uint8_t *>(ptrs[j]);
  }
  __device__ uint8_t *parity(int i) const { return reinterpret_cast<uint8_t *>(ptrs[k + m + i]); }
};

// As encode_columns, for K = k blocks and the rows of `rows`; one block is
// loaded ahead of the one being XORed in.
template <int M, bool FULL, class Blocks>
__device__ __forceinline__ void encode_columns_rt(const Blocks &src, int k, const BitRows &rows,
                                                  uint64_t s0, uint64_t s1, uint64_t lim) {
  uint32_t par[M][8];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int b = 0; b < 8; ++b) par[i][b] = 0;
  uint32_t x[8], y[8];
  load16<FULL>(src.data(0), s0, lim, x);
  load16<FULL>(src.data(0), s1, lim, x + 4);
  auto step = [&](uint32_t (&cur)[8], uint32_t (&nxt)[8], int j) {
    if (j + 1 < k) {
      load16<FULL>(src.data(j + 1), s0, lim, nxt);
      load16<FULL>(src.data(j + 1), s1, lim, nxt + 4);
    }
    __builtin_amdgcn_sched_barrier(0);
    bit_transpose(cur);
    // the planes are materialised once (left free, the compiler folds the
    // transpose's last step into every one of their 8 * M uses)
#pragma unroll
    for (int b = 0; b < 8; ++b) asm volatile("" : "+v"(cur[b]));
#pragma unroll
    for (int i = 0; i < M; ++i) {
      uint64_t row8;   // the 8 rows of c_ij, row b in byte b
      __builtin_memcpy(&row8, rows.r[j][i], 8);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint32_t row = (uint32_t)(row8 >> (8 * b)) & 0xFFu;
        uint32_t acc = par[i][b];
#pragma unroll
        for (int bi = 0; bi < 8; ++bi)   // acc ^ (plane & mask), truth table 0x78
          acc = __builtin_amdgcn_bitop3_b32(acc, cur[bi], 0u - ((row >> bi) & 1u), 0x78);
        par[i][b] = acc;
        asm volatile("" : "+v"(par[i][b]));
      }
    }
  };
  for (int j = 0; j < k; j += 2) {
    step(x, y, j);
    if (j + 1 < k) step(y, x, j + 1);
  }
#pragma unroll
  for (int i = 0; i < M; ++i) {
    bit_transpose(par[i]);
    store16<FULL>(src.parity(i), s0, lim, par[i]);
    store16<FULL>(src.parity(i), s1, lim, par[i] + 4);
  }
}

template <int M, class Blocks>
__device__ __forceinline__ void encode_chunk_rt(const Blocks &src, int k, const BitRows &rows,
                                                uint64_t c, uint64_t lim, uint32_t lane) {
  const uint64_t s0 = c + 16 * lane, s1 = s0 + 1024;
  if (c + kWaveCols <= lim)
    encode_columns_rt<M, true>(src, k, rows, s0, s1, lim);
  else
    encode_columns_rt<M, false>(src, k, rows, s0, s1, lim);
}

template <int M>
__global__ void __launch_bounds__(kBitmatrixThreads)
__attribute__((amdgpu_waves_per_eu(bitmatrix_waves_per_eu<M>()))) bitmatrix_rt_kernel(
    BitmatrixRtParams p) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBitmatrixThreads + threadIdx.x) >> 6;
  const uint64_t c = wave * kWaveCols;
  if (c >= p.io.block_bytes) return;
  encode_chunk_rt<M>(ArgBlocks{p.io}, p.k, p.rows, c, p.io.block_bytes, threadIdx.x & 63);
}

template <int M>
__global__ void __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu(4))) bitmatrix_rt_batch_kernel(BitmatrixRtBatch a) {
  const uint32_t lane = threadIdx.x & 63, wave = uniform(threadIdx.x >> 6),
                 waves = blockDim.x >> 6;
  tiles::run(a.g, [&](tiles::cptr<StripeDesc>, const_as<uint64_t> ptrs, uint64_t c0,
                      uint64_t c1) {
    for (uint64_t cc = c0 + (uint64_t)wave * kWaveCols; cc < c1; cc += (uint64_t)waves * kWaveCols)
      encode_chunk_rt<M>(TableBlocksRt{ptrs, a.k, M}, a.k, a.rows, cc, c1, lane);
  });
}

using BitmatrixFn = void (*)(BitmatrixParams);
using BitmatrixBatchFn = void (*)(BatchGroup);

struct BitmatrixKernels {
  BitmatrixFn plain;
  BitmatrixBatchFn batch;
};

// The codes compiled in (GF(2^8), polynomial 0x11D).
BitmatrixKernels pick_bitmatrix(int k, int m) {
  if (k == 6 && m == 3) return {bitmatrix_kernel<6, 3>, bitmatrix_batch_kernel<6, 3>};
  if (k == 10 && m == 4) return {bitmatrix_kernel<10, 4>, bitmatrix_batch_kernel<10, 4>};
  if (k == 12 && m == 4) return {bitmatrix_kernel<12, 4>, bitmatrix_batch_kernel<12, 4>};
  if (k == 32 && m == 8) return {bitmatrix_kernel<32, 8>, bitmatrix_batch_kernel<32, 8>};
  return {nullptr, nullptr};
}

using BitmatrixRtFn = void (*)(BitmatrixRtParams);
using BitmatrixRtBatchFn = void (*)(BitmatrixRtBatch);

template <int M>
constexpr std::pair<BitmatrixRtFn, BitmatrixRtBatchFn> rt_pair() {
  return {bitmatrix_rt_kernel<M>, bitmatrix_rt_batch_kernel<M>};
}

std::pair<BitmatrixRtFn, BitmatrixRtBatchFn> pick_rt(int m) {
  switch (m) {
    case 1: return rt_pair<1>();
    case 2: return rt_pair<2>();
    case 3: return rt_pair<3>();
    case 4: return rt_pair<4>();
    case 5: return rt_pair<5>();
    case 6: return rt_pair<6>();
    case 7: return rt_pair<7>();
    case 8: return rt_pair<8>();
    default: return {nullptr, nullptr};
  }
}

bool valid_code(const BitmatrixCode &bc) {
  return bc.k >= 1 && bc.k <= kBitmatrixMaxK && bc.m >= 1 && bc.m <= kMaxM &&
         (bc.builtin ? pick_bitmatrix(bc.k, bc.m).plain != nullptr : bc.rows != nullptr);
}

}  // namespace

bool bitmatrix_builtin(int k, int m, int w, unsigned poly) {
  return w == 8 && poly == kPoly && pick_bitmatrix(k, m).plain != nullptr;
}

int launch_bitmatrix(const BitmatrixCode &bc, const uint8_t *const *data,
                     uint8_t *const *parity, uint64_t offset, uint64_t block_bytes,
                     void *stream) {
  if (!valid_code(bc) || block_bytes == 0 || block_bytes > kMaxPieceBytes)
    return (int)hipErrorInvalidValue;
  BitmatrixParams p{};
  for (int j = 0; j < bc.k; ++j) p.data[j] = data[j] + offset;
  for (int i = 0; i < bc.m; ++i) p.parity[i] = parity[i] + offset;
  p.block_bytes = block_bytes;
  const uint64_t waves = (block_bytes + kWaveCols - 1) / kWaveCols;
  const uint64_t wgs = (waves + kBitmatrixThreads / 64 - 1) / (kBitmatrixThreads / 64);
  if (bc.builtin) {
    hipLaunchKernelGGL(pick_bitmatrix(bc.k, bc.m).plain, dim3((uint32_t)wgs),
                       dim3(kBitmatrixThreads), 0, (hipStream_t)stream, p);
  } else {
    BitmatrixRtParams rp{};
    rp.io = p;
    rp.k = bc.k;
    rp.rows = *bc.rows;
    hipLaunchKernelGGL(pick_rt(bc.m).first, dim3((uint32_t)wgs), dim3(kBitmatrixThreads), 0,
                       (hipStream_t)stream, rp);
  }
  return (int)hipGetLastError();
}

int launch_bitmatrix_batch(const BitmatrixCode &bc, const BatchGroup &g, int grid, int threads,
                           void *stream) {
  if (!valid_code(bc) || threads < 64 || threads > 1024 || threads % 64 || grid < 1)
    return (int)hipErrorInvalidValue;
  if (bc.builtin) {
    hipLaunchKernelGGL(pick_bitmatrix(bc.k, bc.m).batch, dim3(grid), dim3(threads), 0,
                       (hipStream_t)stream, g);
  } else {
    BitmatrixRtBatch a{};
    a.g = g;
    a.k = bc.k;
    a.rows = *bc.rows;
    hipLaunchKernelGGL(pick_rt(bc.m).second, dim3(grid), dim3(threads), 0, (hipStream_t)stream,
                       a);
  }
  return (int)hipGetLastError();
}

}  // namespace rsp
