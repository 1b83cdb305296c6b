// Delta-parity update with register-resident split-nibble products: the
// fast region multiply by a constant that Sec. 6 points to, with no LDS.
//
// The update adds sum_j P[:, j] * delta_j to the parity (the update property
// of Sec. 3.2 with the generator-matrix columns of Sec. 6).  Each product
// c * x of a byte x by a constant c = P[i][j] is split by nibbles,
//     c * x = c * (x & 15)  ^  c * (x & 0xF0),
// and each half is a 16-entry byte table (16 bytes = 4 dwords) held in
// registers.  v_perm_b32 looks up 4 bytes at once in an 8-byte window
// (entries 0-7 or 8-15 of a table), so one nibble lookup of a dword of 4
// columns is two v_perm_b32 and one v_bfi_b32 that keeps, per byte, the
// window its index's bit 3 names.  The per-dword index and mask work is
// shared by all the constants a changed block meets; a dword of 4 parity
// columns then costs 7 VALU operations per constant (two lookups and one
// 3-input XOR), with no transposes: the data, parity and results stay in
// block order.  With C changed blocks and m parity blocks the C * m tables
// take 8 * C * m VGPRs, so the kernel is built for C <= 2 and C * m <= 8.
#include <hip/hip_runtime.h>

#include "batch_tiles.h"
#include "rs_internal.h"

namespace rsp {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <class T>
using global_ptr = __attribute__((address_space(1))) T *;

__device__ __forceinline__ u32x4 load16(const uint8_t *p) {
  return __builtin_nontemporal_load((const global_ptr<const u32x4>)(uintptr_t)p);
}

__device__ __forceinline__ void store16(uint8_t *p, u32x4 v) {
  __builtin_nontemporal_store(v, (global_ptr<u32x4>)(uintptr_t)p);
}

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// Nibble indices of a dword of 4 symbols, ready for lookups: the low 3 bits
// of each nibble (v_perm_b32 selectors) and, per byte, all ones where the
// nibble's bit 3 is set (v_bfi_b32 mask choosing entries 8-15).
struct Nibbles {
  uint32_t sel_lo, mask_lo, sel_hi, mask_hi;
};

__device__ __forceinline__ Nibbles nibbles(uint32_t x) {
  Nibbles n;
  const uint32_t lo = x & 0x0F0F0F0Fu, hi = (x >> 4) & 0x0F0F0F0Fu;
  n.sel_lo = lo & 0x07070707u;
  n.sel_hi = hi & 0x07070707u;
  // bit 3 of each nibble spread over its byte: (b3 << 8) - b3 = 0xFF or 0
  const uint32_t b_lo = (lo >> 3) & 0x01010101u, b_hi = (hi >> 3) & 0x01010101u;
  n.mask_lo = (b_lo << 8) - b_lo;
  n.mask_hi = (b_hi << 8) - b_hi;
  return n;
}

// acc ^ c * x for the 4 bytes of x, with c's tables t[0..3] (c * n for
// n < 16, entry n at byte n of the 16 bytes) and t[4..7] (c * (n << 4)).
__device__ __forceinline__ uint32_t add_product(uint32_t acc, const uint32_t (&t)[8],
                                                const Nibbles &n) {
  const uint32_t lo = (perm(t[3], t[2], n.sel_lo) & n.mask_lo) |
                      (perm(t[1], t[0], n.sel_lo) & ~n.mask_lo);
  const uint32_t hi = (perm(t[7], t[6], n.sel_hi) & n.mask_hi) |
                      (perm(t[5], t[4], n.sel_hi) & ~n.mask_hi);
  return __builtin_amdgcn_bitop3_b32(acc, lo, hi, 0x96);   // acc ^ lo ^ hi
}

// One table entry by its byte index, for the byte-wise tail (read from
// memory, the kernel arguments or the batch arena: a dynamic index into the
// register copy would put it in scratch memory).
template <class P>
__device__ __forceinline__ uint32_t entry(P t, int half, uint32_t n) {
  return (t[4 * half + (n >> 2)] >> (8 * (n & 3))) & 0xFFu;
}

// Columns [c0, c1) of one stripe (c0 a multiple of 16): parity[i] ^= the
// products of the C changed blocks.  The C * MM tables come from `src`
// (entry q at src + 8 q, q = t * MM + i) into registers; thread `me` of
// `count` takes the 16-byte chunks me, me + count, ...; the thread with
// `tail` set does the last (c1 - c0) mod 16 bytes byte by byte.
template <int C, int MM, class P>
__device__ __forceinline__ void nibble_columns(const uint8_t *const (&delta)[C],
                                               uint8_t *const (&parity)[MM], P src,
                                               uint64_t c0, uint64_t c1, uint64_t me,
                                               uint64_t count, bool tail) {
  uint32_t tab[C * MM][8];
#pragma unroll
  for (int q = 0; q < C * MM; ++q)
#pragma unroll
    for (int d = 0; d < 8; ++d) tab[q][d] = src[8 * q + d];
  const uint64_t chunks = (c1 - c0) / 16;
  for (uint64_t ch = me; ch < chunks; ch += count) {
    const uint64_t col = c0 + ch * 16;
    u32x4 acc[MM];
#pragma unroll
    for (int i = 0; i < MM; ++i) acc[i] = load16(parity[i] + col);
#pragma unroll
    for (int t = 0; t < C; ++t) {
      const u32x4 x = load16(delta[t] + col);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const Nibbles n = nibbles(x[w]);
#pragma unroll
        for (int i = 0; i < MM; ++i) acc[i][w] = add_product(acc[i][w], tab[t * MM + i], n);
      }
    }
#pragma unroll
    for (int i = 0; i < MM; ++i) store16(parity[i] + col, acc[i]);
  }
  if (tail) {
    for (uint64_t col = c0 + chunks * 16; col < c1; ++col) {
#pragma unroll
      for (int i = 0; i < MM; ++i) {
        uint32_t v = parity[i][col];
#pragma unroll
        for (int t = 0; t < C; ++t) {
          const uint32_t x = delta[t][col];
          v ^= entry(src + 8 * (t * MM + i), 0, x & 15) ^ entry(src + 8 * (t * MM + i), 1, x >> 4);
        }
        parity[i][col] = (uint8_t)v;
      }
    }
  }
}

// One stripe per launch: grid-stride over its 16-byte chunks.
template <int C, int MM>
__global__ void __launch_bounds__(512) nibble_update_kernel(NibbleParams p) {
  const uint8_t *delta[C];
  uint8_t *parity[MM];
#pragma unroll
  for (int t = 0; t < C; ++t) delta[t] = p.delta[t];
#pragma unroll
  for (int i = 0; i < MM; ++i) parity[i] = p.parity[i];
  nibble_columns<C, MM>(delta, parity, &p.tab[0][0], 0, p.block_bytes,
                        (uint64_t)blockIdx.x * blockDim.x + threadIdx.x,
                        (uint64_t)gridDim.x * blockDim.x, blockIdx.x == 0 && threadIdx.x == 0);
}

// Batched updates: persistent workgroups claim tiles of all the stripes of
// a group.  A stripe's descriptor holds its changed-block count c (field k)
// and m; its pointer table starts with the c changed delta blocks, then the
// m parity blocks (read and written in place); its tables are the apply
// set apply_set of the arena (c * m x 8 dwords).
template <int C, int MM>
__device__ __forceinline__ void nibble_tile(tiles::cptr<uint64_t> ptrs, tiles::cptr<uint32_t> tab,
                                            uint64_t c0, uint64_t c1) {
  const uint8_t *delta[C];
  uint8_t *parity[MM];
#pragma unroll
  for (int t = 0; t < C; ++t) delta[t] = reinterpret_cast<const uint8_t *>(ptrs[t]);
#pragma unroll
  for (int i = 0; i < MM; ++i) parity[i] = reinterpret_cast<uint8_t *>(ptrs[C + i]);
  nibble_columns<C, MM>(delta, parity, tab, c0, c1, threadIdx.x, blockDim.x, threadIdx.x == 0);
}

__global__ void __launch_bounds__(1024) nibble_batch_kernel(BatchGroup g) {
  const BatchHeader *hdr = reinterpret_cast<const BatchHeader *>(g.arena);
  const tiles::cptr<uint32_t> sets =
      (tiles::cptr<uint32_t>)(uintptr_t)(g.arena + ((tiles::cptr<BatchHeader>)(uintptr_t)hdr)->off_apply);
  tiles::run(g, [&](tiles::cptr<StripeDesc> d, tiles::cptr<uint64_t> ptrs, uint64_t c0,
                    uint64_t c1) {
    const tiles::cptr<uint32_t> tab = sets + (uint64_t)d->apply_set * (kMaxM * 16);
    switch (d->k * 16 + d->m) {   // (c, m), uniform
      case 0x11: nibble_tile<1, 1>(ptrs, tab, c0, c1); break;
      case 0x12: nibble_tile<1, 2>(ptrs, tab, c0, c1); break;
      case 0x13: nibble_tile<1, 3>(ptrs, tab, c0, c1); break;
      case 0x14: nibble_tile<1, 4>(ptrs, tab, c0, c1); break;
      case 0x15: nibble_tile<1, 5>(ptrs, tab, c0, c1); break;
      case 0x16: nibble_tile<1, 6>(ptrs, tab, c0, c1); break;
      case 0x17: nibble_tile<1, 7>(ptrs, tab, c0, c1); break;
      case 0x18: nibble_tile<1, 8>(ptrs, tab, c0, c1); break;
      case 0x21: nibble_tile<2, 1>(ptrs, tab, c0, c1); break;
      case 0x22: nibble_tile<2, 2>(ptrs, tab, c0, c1); break;
      case 0x23: nibble_tile<2, 3>(ptrs, tab, c0, c1); break;
      case 0x24: nibble_tile<2, 4>(ptrs, tab, c0, c1); break;
      default: break;   // not planned for this kernel
    }
  });
}

using NibbleFn = void (*)(NibbleParams);

template <int C>
NibbleFn pick_nibble(int m) {
  switch (m) {
    case 1: return nibble_update_kernel<C, 1>;
    case 2: return nibble_update_kernel<C, 2>;
    case 3: return nibble_update_kernel<C, 3>;
    case 4: return nibble_update_kernel<C, 4>;
    default: break;
  }
  if constexpr (C == 1) {
    switch (m) {
      case 5: return nibble_update_kernel<1, 5>;
      case 6: return nibble_update_kernel<1, 6>;
      case 7: return nibble_update_kernel<1, 7>;
      case 8: return nibble_update_kernel<1, 8>;
      default: break;
    }
  }
  return nullptr;
}

}  // namespace

bool nibble_supported(int c, int m) {
  return c >= 1 && c <= kNibbleMaxBlocks && m >= 1 && c * m <= kNibbleMaxProducts;
}

int launch_nibble_batch(const BatchGroup &g, int grid, int threads, void *stream) {
  if (threads < 64 || threads > 1024 || threads % 64 || grid < 1) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(nibble_batch_kernel, dim3(grid), dim3(threads), 0,
                     reinterpret_cast<hipStream_t>(stream), g);
  return (int)hipGetLastError();
}

int launch_nibble_update(const NibbleParams &p, int grid, void *stream) {
  const NibbleFn fn = p.c == 1 ? pick_nibble<1>(p.m) : p.c == 2 ? pick_nibble<2>(p.m) : nullptr;
  if (!fn) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(512), 0, reinterpret_cast<hipStream_t>(stream), p);
  return (int)hipGetLastError();
}

}  // namespace rsp
