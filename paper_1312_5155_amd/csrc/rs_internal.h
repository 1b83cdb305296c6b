// Internal interface between the host library (api.cpp, gf.cpp) and the HIP
// kernels (codec.hip).  Not installed; the public ABI is include/rs_poly.h.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace rsp {

constexpr int kMaxN = 255;
constexpr int kMaxM = 8;

// ---------------------------------------------------------------- tables --
//
// Every table the kernels look up is a GF(2)-linear map of one byte, so it
// is fully described by the images of the 8 unit bytes 1, 2, 4, ..., 128
// ("basis").  The host computes basis values; each workgroup expands them
// into 256-entry tables in LDS.  A value is 4 bytes (codes with m <= 4) or 8
// bytes (m <= 8), stored as 1 or 2 dwords.
//
// LDS layout: entry e of every table starts at byte e * 256, so a single
// v_perm_b32 turns (index byte, lane offset byte) into an LDS address.  Each
// 256-byte entry row holds several tables side by side, each replicated so
// that lanes of a wave spread over banks.
constexpr uint32_t kRowBytes = 256;
constexpr uint32_t kApplyRegion = 65536;     // decode apply tables start here

// State width in bytes for a code with m parity symbols.
inline int state_bytes(int m) { return m <= 4 ? 4 : 8; }

// Kernel arguments, passed by value (about 2.8 KiB, within the kernarg limit).
struct CodecParams {
  const uint8_t *data[kMaxN];     // d_j; nullptr = symbol 0, not read
  const uint8_t *par_in[kMaxM];   // decode: parity p_i read back, or nullptr
  uint8_t *out[kMaxM];            // encode: p_i; decode: i-th erased block
  uint64_t block_bytes;
  int32_t k;                      // data blocks
  int32_t m;                      // parity symbols (remainder bytes)
  int32_t k_pad;                  // k rounded up to the state width
  int32_t n_out;                  // blocks written
  uint32_t lfsr_basis[16];        // 8 values of T'(2^b), 1 or 2 dwords each
  uint32_t apply_basis[kMaxM][16];// decode: per remainder byte, 8 values
};

enum Mode : int { kEncode = 0, kDecode = 1 };

// A launch configuration of the codec kernel.
struct LaunchCfg {
  int dwords_per_lane;   // 1, 2 or 4: bytes per lane per block = 4x this
  int threads;           // workgroup size, multiple of 64, <= 1024
  int grid;              // workgroups; 0 = pick from the size
  bool bytewise;         // byte loads/stores (for misaligned blocks)
};

// Launches the codec kernel for one stripe.  Returns a hipError_t as int.
int launch_codec(Mode mode, int state_bytes, const CodecParams &p,
                 const LaunchCfg &cfg, void *stream);

// Resident workgroups per CU the kernel is sized for (LDS bound).
int codec_wgs_per_cu(Mode mode);

}  // namespace rsp
