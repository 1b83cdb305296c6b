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
//     (the extra term clears the consumed byte).  The rotated copies of T'
//     are separate LDS tables; for M = 8 rotations by 4 bytes are free (swap
//     the two dwords), so 4 copies serve 8 positions.
// k is padded at the top to a multiple of M with zero symbols (leading zeros
// leave a zero remainder unchanged), so the rotation is back at 0 at the end.
//
// Decode = Sec. 3.3 in remainder form.  The same LFSR over the symbols read
// (erased or unread ones are zero and never loaded: Opt2 of Sec. 4), XOR the
// parity read, gives r(x) = received word mod g(x), whose values at the roots
// alpha^i are the paper's step-1 values D(alpha^i).  The erased symbols are
// then C * r for a small per-pattern matrix C = V^-1 W (Vandermonde inverse
// computed once per pattern on the host: Opt3), applied as m packed product
// lookups, one per remainder byte (region-level multiply-XOR: Opt4).
//
// LDS tables.  Each table is a GF(2)-linear map of one byte, expanded by
// every workgroup from 8 basis values passed in the kernel arguments.  Entry
// e of every table sits at byte e*256 (plus a per-table offset and a
// per-lane replica), so v_perm_b32(state, lane_offset) yields the address
// directly; replicas spread the 16 lanes of a quarter-wave over distinct
// banks.
#include <hip/hip_runtime.h>

#include "rs_internal.h"

namespace rsp {
namespace {

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

__device__ __forceinline__ uint32_t rotl32(uint32_t x, int s) {
  s &= 31;
  return s ? (x << s) | (x >> (32 - s)) : x;
}

__device__ __forceinline__ uint64_t rotl64(uint64_t x, int s) {
  s &= 63;
  return s ? (x << s) | (x >> (64 - s)) : x;
}

// 4x4 byte transpose: o_b = (i0.byte b, i1.byte b, i2.byte b, i3.byte b).
__device__ __forceinline__ void transpose4(uint32_t i0, uint32_t i1, uint32_t i2, uint32_t i3,
                                           uint32_t &o0, uint32_t &o1, uint32_t &o2,
                                           uint32_t &o3) {
  const uint32_t lo01 = perm(i1, i0, 0x05010400u);  // i0.b0 i1.b0 i0.b1 i1.b1
  const uint32_t hi01 = perm(i1, i0, 0x07030602u);  // i0.b2 i1.b2 i0.b3 i1.b3
  const uint32_t lo23 = perm(i3, i2, 0x05010400u);
  const uint32_t hi23 = perm(i3, i2, 0x07030602u);
  o0 = perm(lo23, lo01, 0x05040100u);
  o1 = perm(lo23, lo01, 0x07060302u);
  o2 = perm(hi23, hi01, 0x05040100u);
  o3 = perm(hi23, hi01, 0x07060302u);
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

// Expands the LFSR tables: 4 rotated copies of T', each 16 (M=4, 4-byte
// values) or 8 (M=8, 8-byte values) replicas wide, 64 bytes per copy per row.
template <int M>
__device__ void build_lfsr_tables(uint8_t *lds, const uint32_t *basis) {
  for (uint32_t idx = threadIdx.x; idx < 1024; idx += blockDim.x) {
    const uint32_t f = idx >> 2, v = idx & 3;
    const uint32_t base = f * kRowBytes + v * 64;
    if constexpr (M == 4) {
      const uint32_t x = rotl32(lin32(f, basis), 8 * (v + 1));
#pragma unroll
      for (int r = 0; r < 4; ++r) st4(lds, base + 16 * r, x, x, x, x);
    } else {
      const uint64_t x = rotl64(lin64(f, basis), 8 * (v + 1));
      const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
#pragma unroll
      for (int r = 0; r < 4; ++r) st4(lds, base + 16 * r, lo, hi, lo, hi);
    }
  }
}

// Expands the decode apply tables U'_b (one per remainder byte b < m): for
// M=4, 4 tables x 16 replicas; for M=8, 8 tables x 4 replicas.
template <int M>
__device__ void build_apply_tables(uint8_t *lds, const CodecParams &p) {
  constexpr uint32_t kTables = M;
  for (uint32_t idx = threadIdx.x; idx < 256 * kTables; idx += blockDim.x) {
    const uint32_t f = idx / kTables, b = idx % kTables;
    const bool used = (int)b < p.m;
    if constexpr (M == 4) {
      const uint32_t base = kApplyRegion + f * kRowBytes + b * 64;
      const uint32_t x = used ? lin32(f, p.apply_basis[b]) : 0u;
#pragma unroll
      for (int r = 0; r < 4; ++r) st4(lds, base + 16 * r, x, x, x, x);
    } else {
      const uint32_t base = kApplyRegion + f * kRowBytes + b * 32;
      const uint64_t x = used ? lin64(f, p.apply_basis[b]) : 0ull;
      const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
      st4(lds, base, lo, hi, lo, hi);
      st4(lds, base + 16, lo, hi, lo, hi);
    }
  }
}

// Loads W dwords (4*W byte columns starting at col) of one block; columns
// past the end of the block read as zero.
template <int W, bool BYTEWISE>
__device__ __forceinline__ void load_cols(const uint8_t *ptr, uint64_t col, uint64_t B,
                                          uint32_t (&a)[W]) {
  if (!BYTEWISE && col + 4 * W <= B) {
    const uint8_t *q = ptr + col;
    if constexpr (W == 4) {
      const uint4 v = *reinterpret_cast<const uint4 *>(q);
      a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
    } else if constexpr (W == 2) {
      const uint2 v = *reinterpret_cast<const uint2 *>(q);
      a[0] = v.x; a[1] = v.y;
    } else {
      a[0] = *reinterpret_cast<const uint32_t *>(q);
    }
  } else {
#pragma unroll
    for (int d = 0; d < W; ++d) {
      uint32_t v = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint64_t c = col + 4 * d + i;
        if (c < B) v |= (uint32_t)ptr[c] << (8 * i);
      }
      a[d] = v;
    }
  }
}

template <int W, bool BYTEWISE>
__device__ __forceinline__ void store_cols(uint8_t *ptr, uint64_t col, uint64_t B,
                                           const uint32_t (&a)[W]) {
  if (!BYTEWISE && col + 4 * W <= B) {
    uint8_t *q = ptr + col;
    if constexpr (W == 4) {
      *reinterpret_cast<uint4 *>(q) = make_uint4(a[0], a[1], a[2], a[3]);
    } else if constexpr (W == 2) {
      *reinterpret_cast<uint2 *>(q) = make_uint2(a[0], a[1]);
    } else {
      *reinterpret_cast<uint32_t *>(q) = a[0];
    }
  } else {
#pragma unroll
    for (int d = 0; d < W; ++d) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint64_t c = col + 4 * d + i;
        if (c < B) ptr[c] = (uint8_t)(a[d] >> (8 * i));
      }
    }
  }
}

// One LFSR step at window position q (compile time) for one column.
template <int M>
__device__ __forceinline__ void lfsr_step(uint32_t (&s)[M / 4], const uint8_t *lds,
                                          uint32_t loff, int q) {
  const int bp = q & 3;
  if constexpr (M == 4) {
    const uint32_t addr = perm(s[0], loff, 0x0C0C0400u | ((uint32_t)bp << 8));
    s[0] ^= *reinterpret_cast<const uint32_t *>(lds + addr + bp * 64);
  } else {
    const int half = q >> 2;
    const uint32_t addr = perm(s[half], loff, 0x0C0C0400u | ((uint32_t)bp << 8));
    const uint2 v = *reinterpret_cast<const uint2 *>(lds + addr + bp * 64);
    if (half == 0) {
      s[0] ^= v.x;
      s[1] ^= v.y;
    } else {
      s[0] ^= v.y;
      s[1] ^= v.x;
    }
  }
}

template <int M, int W, int MODE, bool BYTEWISE>
__global__ void __launch_bounds__(1024) codec_kernel(CodecParams p) {
  constexpr int NQ = M / 4;   // dwords of state per column
  constexpr int NC = 4 * W;   // columns per lane
  __shared__ __attribute__((aligned(16))) uint8_t lds[MODE == kDecode ? 131072 : 65536];

  build_lfsr_tables<M>(lds, p.lfsr_basis);
  if constexpr (MODE == kDecode) build_apply_tables<M>(lds, p);
  __syncthreads();

  const uint32_t lane = threadIdx.x & 63;
  const uint32_t loff = M == 4 ? (lane & 15) * 4 : (lane & 7) * 8;
  const uint64_t B = p.block_bytes;
  const uint64_t nchunks = (B + NC - 1) / NC;
  const int groups = p.k_pad / M;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;

  for (uint64_t ch = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; ch < nchunks;
       ch += stride) {
    const uint64_t col = ch * NC;
    uint32_t s[NC][NQ];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int h = 0; h < NQ; ++h) s[c][h] = 0;

    for (int g = 0; g < groups; ++g) {
      // M symbols per column: window position q takes block k_pad-1-(g*M+q).
      uint32_t a[M][W];
#pragma unroll
      for (int q = 0; q < M; ++q) {
        const int j = p.k_pad - 1 - (g * M + q);
        const uint8_t *ptr = j < p.k ? p.data[j] : nullptr;
        if (ptr) {
          load_cols<W, BYTEWISE>(ptr, col, B, a[q]);
        } else {
#pragma unroll
          for (int w = 0; w < W; ++w) a[q][w] = 0;
        }
      }
      // Transpose so that each column's M symbols fill its state window.
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int h = 0; h < NQ; ++h) {
          uint32_t d0, d1, d2, d3;
          transpose4(a[4 * h][w], a[4 * h + 1][w], a[4 * h + 2][w], a[4 * h + 3][w], d0, d1,
                     d2, d3);
          s[4 * w + 0][h] ^= d0;
          s[4 * w + 1][h] ^= d1;
          s[4 * w + 2][h] ^= d2;
          s[4 * w + 3][h] ^= d3;
        }
#pragma unroll
      for (int q = 0; q < M; ++q)
#pragma unroll
        for (int c = 0; c < NC; ++c) lfsr_step<M>(s[c], lds, loff, q);
    }
    // k_pad is a multiple of M: the rotation is back at 0 and byte b of the
    // state is remainder coefficient r_(m-1-b).

    if constexpr (MODE == kDecode) {
      // Add the parity symbols read: p_i is coefficient i of the received
      // word, i.e. byte m-1-i of the state.
#pragma unroll
      for (int h = 0; h < NQ; ++h) {
        uint32_t a[4][W];
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
          const int i = p.m - 1 - (4 * h + bb);
          const uint8_t *ptr = i >= 0 ? p.par_in[i] : nullptr;
          if (ptr) {
            load_cols<W, BYTEWISE>(ptr, col, B, a[bb]);
          } else {
#pragma unroll
            for (int w = 0; w < W; ++w) a[bb][w] = 0;
          }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
          uint32_t d0, d1, d2, d3;
          transpose4(a[0][w], a[1][w], a[2][w], a[3][w], d0, d1, d2, d3);
          s[4 * w + 0][h] ^= d0;
          s[4 * w + 1][h] ^= d1;
          s[4 * w + 2][h] ^= d2;
          s[4 * w + 3][h] ^= d3;
        }
      }
      // Rebuilt symbol e = byte e of sum_b U'_b[byte b of the remainder].
      const uint32_t aoff = (M == 4 ? (lane & 15) * 4 : (lane & 3) * 8) | kApplyRegion;
      uint32_t L[NC][NQ];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int h = 0; h < NQ; ++h) L[c][h] = 0;
#pragma unroll
      for (int b = 0; b < M; ++b) {
        if (b < p.m) {
          const uint32_t sel = 0x0C020400u | ((uint32_t)(b & 3) << 8);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const uint32_t addr = perm(s[c][b >> 2], aoff, sel);
            if constexpr (M == 4) {
              L[c][0] ^= *reinterpret_cast<const uint32_t *>(lds + addr + b * 64);
            } else {
              const uint2 v = *reinterpret_cast<const uint2 *>(lds + addr + b * 32);
              L[c][0] ^= v.x;
              L[c][1] ^= v.y;
            }
          }
        }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int h = 0; h < NQ; ++h) s[c][h] = L[c][h];
    }

    // Byte b of s[c] goes to column c of output o, where o = m-1-b for
    // encode (parity p_o) and o = b for decode (erased block o).
#pragma unroll
    for (int h = 0; h < NQ; ++h) {
      uint32_t o[4][W];
#pragma unroll
      for (int w = 0; w < W; ++w)
        transpose4(s[4 * w][h], s[4 * w + 1][h], s[4 * w + 2][h], s[4 * w + 3][h], o[0][w],
                   o[1][w], o[2][w], o[3][w]);
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const int b = 4 * h + bb;
        const int oi = MODE == kEncode ? p.m - 1 - b : b;
        if (oi >= 0 && oi < p.n_out) store_cols<W, BYTEWISE>(p.out[oi], col, B, o[bb]);
      }
    }
  }
}

using KernelFn = void (*)(CodecParams);

template <int MODE>
KernelFn pick(int sb, int w, bool bytewise) {
  if (bytewise) return sb == 4 ? codec_kernel<4, 1, MODE, true> : codec_kernel<8, 1, MODE, true>;
  if (sb == 4) {
    if (w == 4) return codec_kernel<4, 4, MODE, false>;
    if (w == 2) return codec_kernel<4, 2, MODE, false>;
    return codec_kernel<4, 1, MODE, false>;
  }
  if (w == 4) return codec_kernel<8, 4, MODE, false>;
  if (w == 2) return codec_kernel<8, 2, MODE, false>;
  return codec_kernel<8, 1, MODE, false>;
}

}  // namespace

int codec_wgs_per_cu(Mode mode) { return mode == kDecode ? 1 : 2; }

int launch_codec(Mode mode, int sb, const CodecParams &p, const LaunchCfg &cfg, void *stream) {
  KernelFn fn = mode == kEncode ? pick<kEncode>(sb, cfg.dwords_per_lane, cfg.bytewise)
                                : pick<kDecode>(sb, cfg.dwords_per_lane, cfg.bytewise);
  hipLaunchKernelGGL(fn, dim3(cfg.grid), dim3(cfg.threads), 0,
                     reinterpret_cast<hipStream_t>(stream), p);
  return (int)hipGetLastError();
}

}  // namespace rsp
