// Tile loop of the persistent batch kernels other than the table-driven
// codec kernel (the bit-sliced encode, the split-nibble update): the same
// arena, tile map, claim counter and tile orders as batch_kernel.  Every
// thread of the workgroup calls tile(descriptor, pointer table, c0, c1) for
// each tile the workgroup claims: columns [c0, c1) of that stripe's blocks.
#pragma once

#include <hip/hip_runtime.h>

#include "rs_internal.h"

namespace rsp {
namespace tiles {

template <class T>
using cptr = const __attribute__((address_space(4))) T *;

__device__ __forceinline__ uint32_t uniform32(uint32_t x) {
  return __builtin_amdgcn_readfirstlane(x);
}

template <class Tile>
__device__ __forceinline__ void run(const BatchGroup &g, Tile &&tile) {
  __shared__ uint64_t next_claim;
  BatchHeader *hdr = reinterpret_cast<BatchHeader *>(g.arena);
  const cptr<BatchHeader> chdr = (cptr<BatchHeader>)(uintptr_t)hdr;
  const uint64_t total = chdr->total_tiles;
  const cptr<StripeDesc> descs = (cptr<StripeDesc>)(uintptr_t)(g.arena + chdr->off_descs);
  const cptr<uint64_t> ptr_table = (cptr<uint64_t>)(uintptr_t)(g.arena + chdr->off_ptrs);
  const cptr<uint32_t> tile_stripe = (cptr<uint32_t>)(uintptr_t)g.tile_stripe;
  unsigned long long *counter = reinterpret_cast<unsigned long long *>(&hdr->counter);
  const uint32_t tile_cols = chdr->tile_cols;

  // claim c -> tile: in order (0) or runs of neighbouring tiles per
  // workgroup (1), as in the table-driven batch kernel
  const bool runs = chdr->tile_order != 0;
  const uint64_t P = gridDim.x;
  const uint64_t run_len = (total + P - 1) / P;
  const uint64_t claims = runs ? run_len * P : total;
  if (threadIdx.x == 0) next_claim = atomicAdd(counter, 1ull);
  __syncthreads();
  for (;;) {
    const uint64_t c = (uint64_t)uniform32((uint32_t)(next_claim >> 32)) << 32 |
                       uniform32((uint32_t)next_claim);
    __syncthreads();   // every thread has read next_claim
    if (c >= claims) break;
    if (threadIdx.x == 0) next_claim = atomicAdd(counter, 1ull);
    const uint64_t t = runs ? (c % P) * run_len + c / P : c;
    if (t < total) {
      const uint32_t s = tile_stripe[t];
      const uint64_t bytes = descs[s].block_bytes;
      const uint64_t c0 = (t - descs[s].tile_begin) * tile_cols;
      const uint64_t c1 = bytes - c0 > tile_cols ? c0 + tile_cols : bytes;
      tile(descs + s, ptr_table + descs[s].ptr_off, c0, c1);
    }
    __syncthreads();   // next_claim is about to change
  }
}

}  // namespace tiles
}  // namespace rsp
