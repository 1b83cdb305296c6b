// Allocation-free batch entry point: the batch kernels of rs_poly_batch_* with
// their scratch memory (zero page, descriptor arena, tile map and tile
// counter) in one file-scope device array instead of library allocations.
//
// Layout of `scratch` (per device, found with hipGetSymbolAddress):
//   [0, 64 KiB)                       zero page (stands in for absent blocks)
//   arena of width w (m <= 4: w = 0; 4 < m <= 8: w = 1), kArenaBytes each:
//                                     header, descriptors, pointer table,
//                                     table bases; the header holds the tile
//                                     counter, which the prepare kernel clears
//   tile map of width w, kTileCap entries of 4 bytes each
// Nothing here calls hipMalloc, hipFree, hipHostMalloc or creates streams,
// events or graphs; the descriptors reach the arena by hipMemcpyAsync from
// a static host buffer (pageable: the runtime stages it, so the buffer may
// be reused as soon as the call returns).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/rs_poly.h"
#include "batch_plan.h"
#include "runtime.h"

namespace rsp {
namespace {

constexpr size_t kZeroBytes = kZeroPageBytes;               // 64 KiB
constexpr size_t kArenaBytes = RS_POLY_NOALLOC_ARENA_BYTES;  // per width
constexpr size_t kTileCap = RS_POLY_NOALLOC_MAX_TILES;       // per width
constexpr size_t kArenaOff[2] = {kZeroBytes, kZeroBytes + kArenaBytes};
constexpr size_t kTilesOff[2] = {kZeroBytes + 2 * kArenaBytes,
                                 kZeroBytes + 2 * kArenaBytes + 4 * kTileCap};
constexpr size_t kScratchBytes = kZeroBytes + 2 * kArenaBytes + 2 * 4 * kTileCap;
static_assert(kScratchBytes == RS_POLY_NOALLOC_SCRATCH_BYTES, "header and layout agree");
static_assert(kArenaBytes % 256 == 0 && kZeroBytes % 256 == 0, "regions stay 256-byte aligned");

__device__ __align__(256) uint8_t scratch[kScratchBytes];

// Clears `bytes` (a multiple of 16) at p; a kernel rather than a memset.
__global__ void clear_scratch_kernel(uint8_t *p, size_t bytes) {
  uint4 *q = reinterpret_cast<uint4 *>(p);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < bytes / 16;
       i += (size_t)gridDim.x * blockDim.x)
    q[i] = make_uint4(0, 0, 0, 0);
}

std::mutex g_mu;                      // host staging and per-device set-up
uint8_t *g_scratch[64] = {};          // device address of `scratch`, per device
alignas(256) uint8_t g_host[kArenaBytes];   // packed upload of one width

// Once per device, with it current: the array's device address, and the
// whole array cleared (the zero page must read as zeros; the rest is
// rewritten by every call).  Called with g_mu held.
int setup(int dev, hipStream_t st, uint8_t **out) {
  if (dev < 0 || dev >= 64) return RS_EDEVICE;
  if (!g_scratch[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RS_EDEVICE;
    hipLaunchKernelGGL(clear_scratch_kernel, dim3(256), dim3(256), 0, st,
                       static_cast<uint8_t *>(p), kScratchBytes);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
      return RS_EDEVICE;
    g_scratch[dev] = static_cast<uint8_t *>(p);
  }
  *out = g_scratch[dev];
  return RS_OK;
}

}  // namespace
}  // namespace rsp

using namespace rsp;

extern "C" int rs_poly_batch_noalloc(int op, const rs_poly_stripe_t *stripes, int count,
                                     void *stream) {
  if (op != RS_POLY_OP_ENCODE && op != RS_POLY_OP_DECODE && op != RS_POLY_OP_UPDATE)
    return RS_EINVAL;
  if (count < 0) return RS_EINVAL;
  if (count > 0 && !stripes) return RS_ENULL;
  if (count == 0) return RS_OK;
  const int ncu = device_cu_count();
  if (ncu <= 0) return RS_EDEVICE;
  rs_poly_launch_t launch[kBatchWidths];
  for (int w = 0; w < kBatchWidths; ++w) launch[w] = default_launch(op, w);
  GroupPlan plan[kBatchWidths];
  size_t upload_len[kBatchWidths] = {0, 0};
  size_t offs[kBatchWidths][4];
  size_t total = 0;
  int rc = plan_batch(op, stripes, count, launch, ncu, plan, upload_len, offs, &total);
  if (rc != RS_OK) return rc;
  if (total == 0) return RS_OK;
  for (int w = 0; w < kBatchWidths; ++w)
    if (!plan[w].descs.empty() && (upload_len[w] > kArenaBytes || plan[w].tiles > kTileCap))
      return RS_EINVAL;   // beyond the scratch array's capacity

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RS_EDEVICE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_mu);
  uint8_t *base = nullptr;
  rc = setup(dev, st, &base);
  if (rc != RS_OK) return rc;
  for (int w = 0; w < kBatchWidths; ++w) {
    const GroupPlan &gp = plan[w];
    if (gp.descs.empty()) continue;
    pack_group(gp, upload_len[w], offs[w], (uint32_t)launch[w].tile_order, g_host);
    uint8_t *arena = base + kArenaOff[w];
    if (hipMemcpyAsync(arena, g_host, upload_len[w], hipMemcpyHostToDevice, st) != hipSuccess)
      return RS_EDEVICE;
    const BatchGroup g{arena, reinterpret_cast<uint32_t *>(base + kTilesOff[w]), base, nullptr};
    LaunchCfg lc{};
    lc.dwords_per_lane = launch[w].bytes_per_lane / 4;
    lc.threads = launch[w].threads;
    lc.grid = ncu * launch[w].wgs_per_cu;
    lc.nibble = launch[w].table_placement == RS_POLY_TABLES_NIBBLE;
    lc.bm = gp.bm;
    lc.nibble_update = gp.nibble;
    const Mode mode = op == RS_POLY_OP_DECODE   ? kDecode
                      : op == RS_POLY_OP_UPDATE ? (gp.matrix ? kUpdateMatrix : kUpdate)
                                                : kEncode;
    rc = hip_status(launch_batch(mode, w ? 8 : 4, g, gp.tiles, lc, stream, /*pull=*/false));
    if (rc != RS_OK) return rc;
  }
  return RS_OK;
}
