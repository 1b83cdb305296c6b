// Streaming probe: the achievable HBM rate for a codec's read:write mix.
//
// A stripe here is n_in input blocks and n_out output blocks of B bytes each,
// laid out at base + s * stripe_stride + b * block_stride.  The probe reads
// every input byte once and writes every output byte once -- each output is
// the XOR of the inputs, so no load can be dropped -- with the same 16-byte
// non-temporal accesses and the same walk over column tiles as the batch
// codec kernels, but with no coding arithmetic and no LDS.  Its bytes per
// second bound what a codec kernel moving the same blocks can reach on this
// part; measuring it beside the codec kernels gives their distance to the
// achievable rate as well as to the nominal peak.
#include <hip/hip_runtime.h>

#include "rs_internal.h"

namespace rsp {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <class T>
using global_ptr = __attribute__((address_space(1))) T *;

struct ProbeArgs {
  uint8_t *base;
  uint64_t stripe_stride, block_stride;
  uint32_t stripes, n_in, n_out;
  uint32_t block_bytes;   // multiple of 16
  uint32_t tile_cols;     // multiple of 16
  uint32_t tiles_per_stripe;
};

__device__ __forceinline__ u32x4 load16(const uint8_t *p) {
  return __builtin_nontemporal_load((const global_ptr<const u32x4>)(uintptr_t)p);
}

__device__ __forceinline__ void store16(uint8_t *p, u32x4 v) {
  __builtin_nontemporal_store(v, (global_ptr<u32x4>)(uintptr_t)p);
}

// Tiles are handed out statically: workgroup w takes tiles w, w + grid, ...
// (a tile is tile_cols columns of one stripe, as in the batch kernels).  A
// lane covers 16 columns per round; the inputs of a round are loaded eight
// at a time, all issued before the first is used.
__global__ void __launch_bounds__(512) stream_probe_kernel(ProbeArgs a) {
  const uint64_t total = (uint64_t)a.stripes * a.tiles_per_stripe;
  for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const uint32_t s = (uint32_t)(t / a.tiles_per_stripe);
    const uint32_t c0 = (uint32_t)(t % a.tiles_per_stripe) * a.tile_cols;
    const uint32_t c1 = min(c0 + a.tile_cols, a.block_bytes);
    uint8_t *stripe = a.base + s * a.stripe_stride;
    for (uint32_t col = c0 + 16 * threadIdx.x; col < c1; col += 16 * blockDim.x) {
      u32x4 acc = {0u, 0u, 0u, 0u};
      for (uint32_t b0 = 0; b0 < a.n_in; b0 += 8) {
        u32x4 v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (b0 + i < a.n_in) v[i] = load16(stripe + (b0 + i) * a.block_stride + col);
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (b0 + i < a.n_in) acc ^= v[i];
      }
      for (uint32_t o = 0; o < a.n_out; ++o)
        store16(stripe + (a.n_in + o) * a.block_stride + col, acc);
    }
  }
}

}  // namespace

int launch_stream_probe(uint8_t *base, uint64_t stripe_stride, uint64_t block_stride,
                        uint32_t stripes, uint32_t n_in, uint32_t n_out, uint32_t block_bytes,
                        uint32_t tile_cols, int grid, void *stream) {
  ProbeArgs a{base, stripe_stride, block_stride, stripes, n_in, n_out, block_bytes, tile_cols,
              (block_bytes + tile_cols - 1) / tile_cols};
  hipLaunchKernelGGL(stream_probe_kernel, dim3(grid), dim3(512), 0,
                     reinterpret_cast<hipStream_t>(stream), a);
  return (int)hipGetLastError();
}

}  // namespace rsp
