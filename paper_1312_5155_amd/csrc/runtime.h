// Helpers shared by the C-ABI entry points: validation, kernel-argument
// filling and default launch shapes.
#pragma once

#include <stdint.h>

#include <mutex>

#include "gf.h"
#include "rs_internal.h"

// The opaque code handle of the C ABI.
struct rs_poly {
  rsp::Code code;
  std::mutex mu;
};

namespace rsp {

// CUs of the current device (cached); -1 on a HIP error.
int device_cu_count();
// Largest of 16, 8, 4, 1 that divides the address.
int pointer_alignment(const void *p);
// Launch shape for one stripe of B-byte blocks whose pointers are all
// aligned to min_align bytes.
LaunchCfg default_cfg(Mode mode, int state_bytes, uint64_t B, int min_align, int num_cu);
// hipError_t -> RS_OK / RS_EDEVICE.
int hip_status(int err);

// Checks flags and an erasure list against the code; on success writes the
// list sorted increasingly to sorted_out (capacity kMaxM).
int validate_erasures(const Code &c, const int *e, int t, unsigned flags, int *sorted_out);

// Kernel arguments for the column range [offset, offset + B) of a stripe.
void fill_encode_params(const Code &c, const uint8_t *const *data, uint8_t *const *parity,
                        uint64_t offset, uint64_t B, CodecParams *p);
// Delta-parity update: data slots j < span (one past the highest changed
// block) hold the delta blocks or nullptr, parity is read and written in
// place.
int update_span(const Code &c, const uint8_t *const *delta);
// Number of changed blocks; the first kMatrixMaxBlocks indices go to which.
int update_changed(const Code &c, const uint8_t *const *delta, int *which);
// Matrix-form update (n <= kMatrixMaxBlocks changed blocks which[0..n)):
// data slot t holds the delta of block which[t], apply basis t its
// generator-matrix column table.
void fill_matrix_update_params(const Code &c, const uint8_t *const *delta,
                               uint8_t *const *parity, const int *which, int n,
                               uint64_t offset, uint64_t B, CodecParams *p);
void fill_update_params(const Code &c, const uint8_t *const *delta, uint8_t *const *parity,
                        int span, uint64_t offset, uint64_t B, CodecParams *p);
void fill_decode_params(const Code &c, const DecodePlan &plan, uint8_t *const *blocks,
                        const int *sorted, int t, uint64_t offset, uint64_t B,
                        CodecParams *p);

}  // namespace rsp
