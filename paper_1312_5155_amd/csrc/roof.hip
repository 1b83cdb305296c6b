// Streaming probe: the achievable HBM rate for a codec's read:write mix.
//
// A stripe here is n_in input blocks and n_out output blocks of B bytes each,
// laid out at base + s * stripe_stride + b * block_stride.  The probe reads
// every input byte once and writes every output byte once -- each output is
// the XOR of the inputs, so no load can be dropped -- with the same 16-byte
// non-temporal accesses and the same two walks over column tiles as the
// batch codec kernels, but with no coding arithmetic and no LDS.  Its bytes
// per second bound what a codec kernel moving the same blocks can reach on
// this part; measuring it beside the codec kernels gives their distance to
// the achievable rate as well as to the nominal peak.
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
  uint32_t tile_order;    // 0: tiles round robin over workgroups; 1: runs
};

__device__ __forceinline__ u32x4 load16(const uint8_t *p) {
  return __builtin_nontemporal_load((const global_ptr<const u32x4>)(uintptr_t)p);
}

__device__ __forceinline__ void store16(uint8_t *p, u32x4 v) {
  __builtin_nontemporal_store(v, (global_ptr<u32x4>)(uintptr_t)p);
}

// Tiles are handed out statically: with order 0 workgroup w takes tiles w,
// w + grid, ... (at any moment the workgroups work on neighbouring tiles);
// with order 1 it takes its own run of consecutive tiles.  A lane covers 32
// columns per round (two 16-byte accesses per block, 512 bytes apart in a
// wave); the inputs of a round are loaded eight blocks at a time, all
// issued before the first is used.
__global__ void __launch_bounds__(512) stream_probe_kernel(ProbeArgs a) {
  const uint64_t total = (uint64_t)a.stripes * a.tiles_per_stripe;
  const uint64_t run = (total + gridDim.x - 1) / gridDim.x;
  const uint64_t first = a.tile_order ? blockIdx.x * run : blockIdx.x;
  const uint64_t last = a.tile_order ? min(total, first + run) : total;
  const uint64_t step = a.tile_order ? 1 : gridDim.x;
  for (uint64_t t = first; t < last; t += step) {
    const uint32_t s = (uint32_t)(t / a.tiles_per_stripe);
    const uint32_t c0 = (uint32_t)(t % a.tiles_per_stripe) * a.tile_cols;
    const uint32_t c1 = min(c0 + a.tile_cols, a.block_bytes);
    uint8_t *stripe = a.base + s * a.stripe_stride;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = threadIdx.x >> 6;
    for (uint32_t w0 = c0 + 2048 * wave; w0 < c1; w0 += 2048 * (blockDim.x >> 6)) {
      // this wave's 2 KiB: lane columns w0 + 16 lane and w0 + 1024 + 16 lane
      const uint32_t col[2] = {w0 + 16 * lane, w0 + 1024 + 16 * lane};
      const bool ok[2] = {col[0] < c1, col[1] < c1};
      u32x4 acc[2] = {{0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}};
      for (uint32_t b0 = 0; b0 < a.n_in; b0 += 8) {
        u32x4 v[8][2];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            if (b0 + i < a.n_in && ok[h])
              v[i][h] = load16(stripe + (b0 + i) * a.block_stride + col[h]);
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            if (b0 + i < a.n_in && ok[h]) acc[h] ^= v[i][h];
      }
      for (uint32_t o = 0; o < a.n_out; ++o)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (ok[h]) store16(stripe + (a.n_in + o) * a.block_stride + col[h], acc[h]);
    }
  }
}

}  // namespace

int launch_stream_probe(uint8_t *base, uint64_t stripe_stride, uint64_t block_stride,
                        uint32_t stripes, uint32_t n_in, uint32_t n_out, uint32_t block_bytes,
                        uint32_t tile_cols, uint32_t tile_order, int grid, void *stream) {
  ProbeArgs a{base, stripe_stride, block_stride, stripes, n_in, n_out, block_bytes, tile_cols,
              (block_bytes + tile_cols - 1) / tile_cols, tile_order};
  hipLaunchKernelGGL(stream_probe_kernel, dim3(grid), dim3(512), 0,
                     reinterpret_cast<hipStream_t>(stream), a);
  return (int)hipGetLastError();
}

}  // namespace rsp
