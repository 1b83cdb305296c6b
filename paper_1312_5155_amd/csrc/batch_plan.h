// Host planning of a batch call, shared by the batch object (batch.cpp) and
// the allocation-free entry point (noalloc.hip): validation, the per-width
// descriptor / pointer / table-basis regions, the tile split, and the
// packed upload.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <map>
#include <memory>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/rs_poly.h"
#include "gf.h"
#include "rs_internal.h"

namespace rsp {

constexpr int kBatchWidths = 2;  // state width 4 bytes (m <= 4), 8 bytes (m <= 8)

inline size_t plan_align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Per-call host view of one group before upload.
struct GroupPlan {
  std::vector<StripeDesc> descs;
  std::vector<uint64_t> ptrs;
  std::vector<uint32_t> lfsr;   // 16 per set
  std::vector<uint32_t> apply;  // kMaxM*16 per set
  std::unordered_map<const Code *, uint32_t> lfsr_index;
  std::unordered_map<const DecodePlan *, uint32_t> apply_index;
  // matrix-form update: table bases per (code, changed-block set); the set
  // is packed one index per byte (at most 8 indices below 255, count apart)
  struct MatrixKey {
    const Code *code;
    uint64_t packed;
    int n;
    bool operator<(const MatrixKey &o) const {
      return std::tie(code, packed, n) < std::tie(o.code, o.packed, o.n);
    }
  };
  std::map<MatrixKey, uint32_t> matrix_index;
  bool matrix = false;   // update group in the generator-matrix form
  bool nibble = false;   // update group in the register split-nibble form
  const BitmatrixCode *bm = nullptr;  // encode group of one code, bit-sliced
  std::vector<std::shared_ptr<const DecodePlan>> keep;  // plans alive during the call
  uint64_t tiles = 0;
  uint32_t tile_cols = 0;
  uint64_t bytes = 0;   // user bytes (k * B summed), for tuning choices

  size_t layout(size_t *o_descs, size_t *o_ptrs, size_t *o_lfsr, size_t *o_apply) const {
    size_t off = plan_align_up(sizeof(BatchHeader), 256);
    *o_descs = off;
    off = plan_align_up(off + descs.size() * sizeof(StripeDesc), 256);
    *o_ptrs = off;
    off = plan_align_up(off + ptrs.size() * sizeof(uint64_t), 256);
    *o_lfsr = off;
    off = plan_align_up(off + lfsr.size() * sizeof(uint32_t), 256);
    *o_apply = off;
    off = plan_align_up(off + apply.size() * sizeof(uint32_t), 256);
    return off;
  }
};


// Launch shape the library uses for (op, width) until it is set or tuned.
rs_poly_launch_t default_launch(int op, int wide);

// Validates every stripe of a call (any error rejects the whole call) and
// fills the plan of each state width: descriptors, pointer table, table
// bases, tiles (sized from launch[width] and num_cu) and the layout of its
// upload (upload_len[w] bytes, region offsets offs[w]).  total_upload is 0
// when there is nothing to run.
int plan_batch(int op, const rs_poly_stripe_t *stripes, int count,
               const rs_poly_launch_t *launch, int num_cu, GroupPlan *plan,
               size_t *upload_len, size_t (*offs)[4], size_t *total_upload);

// Writes a width's upload (header, then the regions) into h.
void pack_group(const GroupPlan &gp, size_t upload_len, const size_t *offs, uint32_t tile_order,
                uint8_t *h);

}  // namespace rsp
