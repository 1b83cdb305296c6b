// Bit-sliced (XOR-only) encode: the generator-matrix form of the
// polynomial code (Sec. 6), parity p_i = sum_j c_ij d_j with c_ij the
// coefficient of x^i in x^(m+j) mod g(x), where every product by c_ij is
// written as an 8 x 8 matrix over GF(2) acting on the 8 bit planes of the
// data bytes (Sec. 6 names this multiplication-free form as future work).
//
// The coefficients depend only on (k, m) and the field, so for the codes
// compiled in here they are compile-time constants and the whole XOR
// network unrolls into straight-line code: no tables, no LDS, no serial
// LFSR chain.  Each lane takes 32 byte columns (two 16-byte runs 1 KiB
// apart, so every load instruction of a wave is one contiguous 1 KiB),
// bit-transposes each block's 32 bytes into 8 planes of 32 bits, XORs the
// planes into the m x 8 parity planes, and transposes those back.
#include <hip/hip_runtime.h>

#include <utility>

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

constexpr int kBitmatrixThreads = 256;
constexpr uint64_t kWaveCols = 2048;   // 64 lanes x 32 columns

// One wave encodes columns [c, c + 2048): lane l holds columns c + 16l ..
// c + 16l + 15 (dwords 0-3) and c + 1024 + 16l .. (dwords 4-7).  Blocks
// are loaded one ahead of the block being XORed in.  FULL: the 2048
// columns lie inside the blocks (every wave but the last one of a launch).
template <int K, int M, bool FULL>
__device__ __forceinline__ void encode_columns(const BitmatrixParams &p, uint64_t s0,
                                               uint64_t s1, uint64_t B) {
  uint32_t par[M][8];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int b = 0; b < 8; ++b) par[i][b] = 0;

  uint32_t cur[8], nxt[8];
  load16<FULL>(p.data[0], s0, B, cur);
  load16<FULL>(p.data[0], s1, B, cur + 4);
  unroll<K>([&](auto J) {
    constexpr int j = decltype(J)::value;
    if constexpr (j + 1 < K) {
      load16<FULL>(p.data[j + 1], s0, B, nxt);
      load16<FULL>(p.data[j + 1], s1, B, nxt + 4);
    }
    // keep the scheduler from hoisting later blocks' loads above this
    // block's work (their registers would not fit)
    __builtin_amdgcn_sched_barrier(0);
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
    if constexpr (j + 1 < K) {
#pragma unroll
      for (int d = 0; d < 8; ++d) cur[d] = nxt[d];
    }
  });

#pragma unroll
  for (int i = 0; i < M; ++i) {
    bit_transpose(par[i]);
    store16<FULL>(p.parity[i], s0, B, par[i]);
    store16<FULL>(p.parity[i], s1, B, par[i] + 4);
  }
}

// Register budget: M parity x 8 planes, two blocks of 8 dwords, temporaries.
template <int M>
constexpr int bitmatrix_waves_per_eu() { return M <= 4 ? 6 : 4; }

template <int K, int M>
__global__ void __launch_bounds__(kBitmatrixThreads)
__attribute__((amdgpu_waves_per_eu(bitmatrix_waves_per_eu<M>()))) bitmatrix_kernel(BitmatrixParams p) {
  const uint64_t B = p.block_bytes;
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wave = ((uint64_t)blockIdx.x * kBitmatrixThreads + threadIdx.x) >> 6;
  const uint64_t c = wave * kWaveCols;
  if (c >= B) return;
  const uint64_t s0 = c + 16 * lane, s1 = s0 + 1024;
  if (c + kWaveCols <= B)
    encode_columns<K, M, true>(p, s0, s1, B);
  else
    encode_columns<K, M, false>(p, s0, s1, B);
}

using BitmatrixFn = void (*)(BitmatrixParams);

// The codes compiled in (GF(2^8), polynomial 0x11D).
BitmatrixFn pick_bitmatrix(int k, int m) {
  if (k == 6 && m == 3) return bitmatrix_kernel<6, 3>;
  if (k == 10 && m == 4) return bitmatrix_kernel<10, 4>;
  if (k == 12 && m == 4) return bitmatrix_kernel<12, 4>;
  if (k == 32 && m == 8) return bitmatrix_kernel<32, 8>;
  return nullptr;
}

}  // namespace

bool bitmatrix_supported(int k, int m, int w, unsigned poly) {
  return w == 8 && poly == kPoly && pick_bitmatrix(k, m) != nullptr;
}

int launch_bitmatrix(int k, int m, const uint8_t *const *data, uint8_t *const *parity,
                     uint64_t offset, uint64_t block_bytes, void *stream) {
  const BitmatrixFn fn = pick_bitmatrix(k, m);
  if (!fn || block_bytes == 0 || block_bytes > kMaxPieceBytes) return (int)hipErrorInvalidValue;
  BitmatrixParams p{};
  for (int j = 0; j < k; ++j) p.data[j] = data[j] + offset;
  for (int i = 0; i < m; ++i) p.parity[i] = parity[i] + offset;
  p.block_bytes = block_bytes;
  const uint64_t waves = (block_bytes + kWaveCols - 1) / kWaveCols;
  const uint64_t wgs = (waves + kBitmatrixThreads / 64 - 1) / (kBitmatrixThreads / 64);
  hipLaunchKernelGGL(fn, dim3((uint32_t)wgs), dim3(kBitmatrixThreads), 0,
                     (hipStream_t)stream, p);
  return (int)hipGetLastError();
}

}  // namespace rsp
