// C ABI of librs_poly.so: code handles, plain (one stripe per launch)
// encode and decode.  Validation happens here, on the host, before any HIP
// call.
#include <hip/hip_runtime_api.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "../../include/rs_poly.h"
#include "gf.h"
#include "rs_internal.h"
#include "runtime.h"

namespace rsp {

int device_cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  static std::mutex mu;
  static int cache[64] = {};
  std::lock_guard<std::mutex> lock(mu);
  if (dev < 0 || dev >= 64) return -1;
  if (cache[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return -1;
    cache[dev] = n;
  }
  return cache[dev];
}

const uint8_t *device_zero_page() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  static std::mutex mu;
  static uint8_t *pages[64] = {};
  std::lock_guard<std::mutex> lock(mu);
  if (!pages[dev]) {
    void *p = nullptr;
    if (hipMalloc(&p, kZeroPageBytes) != hipSuccess) return nullptr;
    if (hipMemset(p, 0, kZeroPageBytes) != hipSuccess) {
      (void)hipFree(p);
      return nullptr;
    }
    pages[dev] = static_cast<uint8_t *>(p);
  }
  return pages[dev];
}

int pointer_alignment(const void *p) {
  const uintptr_t v = reinterpret_cast<uintptr_t>(p);
  if ((v & 15) == 0) return 16;
  if ((v & 7) == 0) return 8;
  if ((v & 3) == 0) return 4;
  return 1;
}

LaunchCfg default_cfg(Mode mode, int sb, uint64_t B, int min_align, int num_cu) {
  LaunchCfg cfg{};
  if (min_align < 4) {
    cfg.bytewise = true;
    cfg.dwords_per_lane = 1;
  } else {
    // Widest loads that still give every CU a few thousand lanes of work.
    const uint64_t want_lanes = (uint64_t)num_cu * 1024;
    int w = std::min(codec_plain_max_dwords(sb), min_align / 4);
    while (w > 1 && (B + 4 * w - 1) / (4 * w) < want_lanes) w /= 2;
    cfg.dwords_per_lane = w;
  }
  // Wide codes: 1024 threads, so that a kernel that runs one workgroup per
  // CU (the decode's 128 KiB of tables; every 16-byte-per-lane kernel's
  // 128-144 KiB in the interleaved layout) still has four waves per SIMD.
  const int tmax = codec_max_threads(mode, sb, cfg.dwords_per_lane);
  cfg.threads = sb == 8 ? tmax : std::min(512, tmax);
  const uint64_t cols = 4ull * cfg.dwords_per_lane;
  const uint64_t chunks = (B + cols - 1) / cols;
  const uint64_t wgs = (chunks + cfg.threads - 1) / cfg.threads;
  const uint64_t resident = (uint64_t)num_cu * codec_wgs_per_cu(mode);
  cfg.grid = (int)std::max<uint64_t>(1, std::min(wgs, resident));
  return cfg;
}

int hip_status(int err) { return err == 0 ? RS_OK : RS_EDEVICE; }

int validate_erasures(const Code &c, const int *e, int t, unsigned flags, int *sorted_out) {
  if (flags & ~RS_POLY_FLAG_ALL_SURVIVORS) return RS_EINVAL;
  if (t < 0) return RS_EINVAL;
  if (t > c.m()) return RS_ETOOMANY;
  if (t > 0 && !e) return RS_ENULL;
  for (int i = 0; i < t; ++i) {
    if (e[i] < 0 || e[i] >= c.n()) return RS_ERANGE;
    sorted_out[i] = e[i];
  }
  std::sort(sorted_out, sorted_out + t);
  for (int i = 1; i < t; ++i)
    if (sorted_out[i] == sorted_out[i - 1]) return RS_ERANGE;
  return RS_OK;
}

static int round_up(int x, int to) { return (x + to - 1) / to * to; }

void fill_encode_params(const Code &c, const uint8_t *const *data, uint8_t *const *parity,
                        uint64_t offset, uint64_t B, CodecParams *p) {
  for (int j = 0; j < c.k(); ++j) p->data[j] = data[j] + offset;
  for (int i = 0; i < c.m(); ++i) p->out[i] = parity[i] + offset;
  p->block_bytes = B;
  p->k = c.k();
  p->m = c.m();
  p->k_pad = round_up(c.k(), c.state_bytes());
  p->n_out = c.m();
  memcpy(p->lfsr_basis, c.lfsr_basis(), sizeof(p->lfsr_basis));
}

int update_span(const Code &c, const uint8_t *const *delta) {
  int span = 0;
  for (int j = 0; j < c.k(); ++j)
    if (delta[j]) span = j + 1;
  return span;
}

int update_changed(const Code &c, const uint8_t *const *delta, int *which) {
  int n = 0;
  for (int j = 0; j < c.k(); ++j)
    if (delta[j]) {
      if (n < kMatrixMaxBlocks) which[n] = j;
      ++n;
    }
  return n;
}

void fill_matrix_update_params(const Code &c, const uint8_t *const *delta,
                               uint8_t *const *parity, const int *which, int n,
                               uint64_t offset, uint64_t B, CodecParams *p) {
  for (int t = 0; t < n; ++t) {
    p->data[t] = delta[which[t]] + offset;
    c.column_basis(which[t], p->apply_basis[t]);
  }
  for (int i = 0; i < c.m(); ++i) {
    p->par_in[i] = parity[i] + offset;
    p->out[i] = parity[i] + offset;
  }
  p->block_bytes = B;
  p->k = n;
  p->m = c.m();
  p->k_pad = round_up(n, c.state_bytes());
  p->n_out = c.m();
}

void fill_update_params(const Code &c, const uint8_t *const *delta, uint8_t *const *parity,
                        int span, uint64_t offset, uint64_t B, CodecParams *p) {
  for (int j = 0; j < span; ++j) p->data[j] = delta[j] ? delta[j] + offset : nullptr;
  for (int i = 0; i < c.m(); ++i) {
    p->par_in[i] = parity[i] + offset;
    p->out[i] = parity[i] + offset;
  }
  p->block_bytes = B;
  p->k = span;
  p->m = c.m();
  p->k_pad = round_up(span, c.state_bytes());
  p->n_out = c.m();
  memcpy(p->lfsr_basis, c.lfsr_basis(), sizeof(p->lfsr_basis));
}

// Per (changed block t, parity i) the two 16-entry tables of the constant
// P[i][j], column j = which[t] of the generator matrix (Sec. 6): the
// products by the low nibbles n and by the high nibbles n << 4, entry n in
// byte n (zero for w = 4, whose symbols have no high nibble).
void nibble_tables(const Code &c, const int *which, int changed, uint32_t (*out)[8]) {
  const Field &f = c.field();
  for (int t = 0; t < changed; ++t) {
    const uint8_t *col = c.column(which[t]);
    for (int i = 0; i < c.m(); ++i) {
      uint8_t lo[16], hi[16];
      for (int n = 0; n < 16; ++n) {
        lo[n] = f.mul(col[i], (uint8_t)n);
        hi[n] = f.w() == 8 ? f.mul(col[i], (uint8_t)(n << 4)) : 0;
      }
      memcpy(&out[t * c.m() + i][0], lo, 16);
      memcpy(&out[t * c.m() + i][4], hi, 16);
    }
  }
}

void fill_decode_params(const Code &c, const DecodePlan &plan, uint8_t *const *blocks,
                        const int *sorted, int t, uint64_t offset, uint64_t B,
                        CodecParams *p) {
  for (int b : plan.read) {
    if (b < c.k())
      p->data[b] = blocks[b] + offset;
    else
      p->par_in[b - c.k()] = blocks[b] + offset;
  }
  for (int r = 0; r < t; ++r) p->out[r] = blocks[sorted[r]] + offset;
  p->block_bytes = B;
  p->k = plan.span;   // data blocks above the span are unread
  p->m = c.m();
  p->k_pad = round_up(plan.span, c.state_bytes());
  p->n_out = t;
  memcpy(p->lfsr_basis, c.lfsr_basis(), sizeof(p->lfsr_basis));
  memcpy(p->apply_basis, plan.apply_basis, sizeof(p->apply_basis));
}

}  // namespace rsp

using namespace rsp;

extern "C" {

int rs_poly_init(int k, int m, int w, unsigned prim_poly, rs_poly_t **out) {
  if (!out) return RS_ENULL;
  *out = nullptr;
  rs_poly_t *h = new (std::nothrow) rs_poly_t;
  if (!h) return RS_ENOMEM;
  const int rc = h->code.init(k, m, w, prim_poly);
  if (rc != RS_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return RS_OK;
}

void rs_poly_free(rs_poly_t *h) { delete h; }

const char *rs_poly_strerror(int err) {
  switch (err) {
    case RS_OK: return "success";
    case RS_EINVAL: return "invalid argument (code parameters, flags or size)";
    case RS_ERANGE: return "erasure index out of range or repeated";
    case RS_ETOOMANY: return "more erasures than parity blocks";
    case RS_ENULL: return "required pointer is NULL";
    case RS_EDEVICE: return "HIP runtime error";
    case RS_ENOMEM: return "out of memory";
    case RS_EBUSY: return "resource busy";
    default: return "unknown status";
  }
}

int rs_poly_generator(const rs_poly_t *h, uint8_t *g) {
  if (!h || !g) return RS_ENULL;
  memcpy(g, h->code.generator(), (size_t)h->code.m() + 1);
  return RS_OK;
}

int rs_poly_encode(rs_poly_t *h, const uint8_t *const *data, uint8_t *const *parity,
                   size_t block_bytes, void *stream) {
  if (!h || !data || !parity) return RS_ENULL;
  const Code &c = h->code;
  int align = 16;
  for (int j = 0; j < c.k(); ++j) {
    if (!data[j]) return RS_ENULL;
    align = std::min(align, pointer_alignment(data[j]));
  }
  for (int i = 0; i < c.m(); ++i) {
    if (!parity[i]) return RS_ENULL;
    align = std::min(align, pointer_alignment(parity[i]));
  }
  if (block_bytes == 0) return RS_OK;

  std::lock_guard<std::mutex> lock(h->mu);
  const int ncu = device_cu_count();
  const uint8_t *zp = device_zero_page();
  if (ncu <= 0 || !zp) return RS_EDEVICE;
  // One launch per column range of at most kMaxPieceBytes.
  for (uint64_t off = 0; off < block_bytes; off += kMaxPieceBytes) {
    const uint64_t piece = std::min<uint64_t>(kMaxPieceBytes, block_bytes - off);
    CodecParams p;
    memset(&p, 0, sizeof(p));
    fill_encode_params(c, data, parity, off, piece, &p);
    p.zero_page = zp;
    const LaunchCfg cfg = default_cfg(kEncode, c.state_bytes(), piece, align, ncu);
    const int rc = hip_status(launch_codec(kEncode, c.state_bytes(), p, cfg, stream));
    if (rc != RS_OK) return rc;
  }
  return RS_OK;
}

int rs_poly_bitmatrix_supported(int k, int m, int w, unsigned poly) {
  Code c;
  return k <= kBitmatrixMaxK && c.init(k, m, w, poly) == RS_OK && c.bitmatrix() ? 1 : 0;
}

int rs_poly_encode_bitmatrix(rs_poly_t *h, const uint8_t *const *data, uint8_t *const *parity,
                             size_t block_bytes, void *stream) {
  if (!h || !data || !parity) return RS_ENULL;
  const Code &c = h->code;
  const BitmatrixCode *bc = c.bitmatrix();
  if (!bc) return RS_EINVAL;   // k above kBitmatrixMaxK
  for (int j = 0; j < c.k(); ++j) {
    if (!data[j]) return RS_ENULL;
    if (pointer_alignment(data[j]) < 16) return RS_EINVAL;
  }
  for (int i = 0; i < c.m(); ++i) {
    if (!parity[i]) return RS_ENULL;
    if (pointer_alignment(parity[i]) < 16) return RS_EINVAL;
  }
  if (block_bytes == 0) return RS_OK;

  std::lock_guard<std::mutex> lock(h->mu);
  for (uint64_t off = 0; off < block_bytes; off += kMaxPieceBytes) {
    const uint64_t piece = std::min<uint64_t>(kMaxPieceBytes, block_bytes - off);
    const int rc = hip_status(launch_bitmatrix(*bc, data, parity, off, piece, stream));
    if (rc != RS_OK) return rc;
  }
  return RS_OK;
}

int rs_poly_encode_matrix(rs_poly_t *h, const uint8_t *const *data, uint8_t *const *parity,
                          size_t block_bytes, void *stream) {
  if (!h || !data || !parity) return RS_ENULL;
  const Code &c = h->code;
  if (c.k() > kMatrixWideMaxBlocks) return RS_EINVAL;
  int align = 16;
  for (int j = 0; j < c.k(); ++j) {
    if (!data[j]) return RS_ENULL;
    align = std::min(align, pointer_alignment(data[j]));
  }
  for (int i = 0; i < c.m(); ++i) {
    if (!parity[i]) return RS_ENULL;
    align = std::min(align, pointer_alignment(parity[i]));
  }
  if (block_bytes == 0) return RS_OK;
  // The matrix-form update of every data block from zero parity: the same
  // kernel, with the old-parity reads sent to the zero page.  Up to 8
  // blocks the tables share one LDS row set (the kernel of rs_poly_update);
  // more take the wide form, 32 tables in two LDS regions, built in the
  // kernel from the column coefficients.
  int which[kMatrixMaxBlocks];
  for (int j = 0; j < c.k() && j < kMatrixMaxBlocks; ++j) which[j] = j;
  const Mode mode = c.k() <= kMatrixMaxBlocks ? kUpdateMatrix : kUpdateMatrixWide;

  std::lock_guard<std::mutex> lock(h->mu);
  const int ncu = device_cu_count();
  const uint8_t *zp = device_zero_page();
  if (ncu <= 0 || !zp) return RS_EDEVICE;
  const int sb = c.state_bytes();
  for (uint64_t off = 0; off < block_bytes; off += kMaxPieceBytes) {
    const uint64_t piece = std::min<uint64_t>(kMaxPieceBytes, block_bytes - off);
    CodecParams p;
    memset(&p, 0, sizeof(p));
    if (mode == kUpdateMatrix) {
      fill_matrix_update_params(c, data, parity, which, c.k(), off, piece, &p);
      for (int i = 0; i < c.m(); ++i) p.par_in[i] = nullptr;
    } else {
      for (int j = 0; j < c.k(); ++j) {
        p.data[j] = data[j] + off;
        memcpy(p.mat_coef[j], c.column(j), (size_t)c.m());
      }
      for (int i = 0; i < c.m(); ++i) p.out[i] = parity[i] + off;
      p.block_bytes = piece;
      p.k = c.k();
      p.m = c.m();
      p.k_pad = (c.k() + sb - 1) / sb * sb;
      p.n_out = c.m();
      p.field_poly = c.field().poly();
      p.field_w = c.field().w();
    }
    p.zero_page = zp;
    const LaunchCfg cfg = default_cfg(mode, sb, piece, align, ncu);
    const int rc = hip_status(launch_codec(mode, sb, p, cfg, stream));
    if (rc != RS_OK) return rc;
  }
  return RS_OK;
}

int rs_poly_update(rs_poly_t *h, const uint8_t *const *delta, uint8_t *const *parity,
                   size_t block_bytes, void *stream) {
  if (!h || !delta || !parity) return RS_ENULL;
  const Code &c = h->code;
  int align = 16;
  for (int j = 0; j < c.k(); ++j)
    if (delta[j]) align = std::min(align, pointer_alignment(delta[j]));
  for (int i = 0; i < c.m(); ++i) {
    if (!parity[i]) return RS_ENULL;
    align = std::min(align, pointer_alignment(parity[i]));
  }
  // Blocks above the highest changed one contribute nothing: the LFSR
  // starts there.  No changed block at all leaves the parity as it is.
  const int span = update_span(c, delta);
  if (block_bytes == 0 || span == 0) return RS_OK;
  // Up to kMatrixMaxBlocks changed blocks: the generator-matrix form, one
  // lookup per changed block (Sec. 6); more: the LFSR form.
  int which[kMatrixMaxBlocks];
  const int changed = update_changed(c, delta, which);
  const Mode mode = changed <= kMatrixMaxBlocks ? kUpdateMatrix : kUpdate;

  std::lock_guard<std::mutex> lock(h->mu);
  const int ncu = device_cu_count();
  const uint8_t *zp = device_zero_page();
  if (ncu <= 0 || !zp) return RS_EDEVICE;
  const int sb = c.state_bytes();
  for (uint64_t off = 0; off < block_bytes; off += kMaxPieceBytes) {
    const uint64_t piece = std::min<uint64_t>(kMaxPieceBytes, block_bytes - off);
    CodecParams p;
    memset(&p, 0, sizeof(p));
    if (mode == kUpdateMatrix)
      fill_matrix_update_params(c, delta, parity, which, changed, off, piece, &p);
    else
      fill_update_params(c, delta, parity, span, off, piece, &p);
    p.zero_page = zp;
    const LaunchCfg cfg = default_cfg(mode, sb, piece, align, ncu);
    const int rc = hip_status(launch_codec(mode, sb, p, cfg, stream));
    if (rc != RS_OK) return rc;
  }
  return RS_OK;
}

int rs_poly_update_nibble(rs_poly_t *h, const uint8_t *const *delta, uint8_t *const *parity,
                          size_t block_bytes, void *stream) {
  if (!h || !delta || !parity) return RS_ENULL;
  const Code &c = h->code;
  int which[kMatrixMaxBlocks];
  const int changed = update_changed(c, delta, which);
  for (int i = 0; i < c.m(); ++i)
    if (!parity[i]) return RS_ENULL;
  if (changed == 0) return RS_OK;
  if (!nibble_supported(changed, c.m())) return RS_EINVAL;
  for (int t = 0; t < changed; ++t)
    if (pointer_alignment(delta[which[t]]) < 16) return RS_EINVAL;
  for (int i = 0; i < c.m(); ++i)
    if (pointer_alignment(parity[i]) < 16) return RS_EINVAL;
  if (block_bytes == 0) return RS_OK;
  NibbleParams p;
  memset(&p, 0, sizeof(p));
  nibble_tables(c, which, changed, p.tab);
  for (int t = 0; t < changed; ++t) p.delta[t] = delta[which[t]];
  for (int i = 0; i < c.m(); ++i) p.parity[i] = parity[i];
  p.block_bytes = block_bytes;
  p.c = changed;
  p.m = c.m();
  std::lock_guard<std::mutex> lock(h->mu);
  const int ncu = device_cu_count();
  if (ncu <= 0) return RS_EDEVICE;
  const uint64_t chunks = std::max<uint64_t>(1, block_bytes / 16);
  const int grid = (int)std::min<uint64_t>((chunks + 511) / 512, (uint64_t)ncu * 8);
  return hip_status(launch_nibble_update(p, grid, stream));
}

int rs_poly_decode(rs_poly_t *h, uint8_t *const *blocks, size_t block_bytes,
                   const int *erasures, int n_erasures, unsigned flags, void *stream) {
  if (!h) return RS_ENULL;
  int sorted[kMaxM];
  const int rc = validate_erasures(h->code, erasures, n_erasures, flags, sorted);
  if (rc != RS_OK) return rc;
  if (n_erasures == 0) return RS_OK;
  if (!blocks) return RS_ENULL;
  auto plan = h->code.plan(sorted, n_erasures, flags);
  int align = 16;
  for (int b : plan->read) {
    if (!blocks[b]) return RS_ENULL;
    align = std::min(align, pointer_alignment(blocks[b]));
  }
  for (int i = 0; i < n_erasures; ++i) {
    if (!blocks[sorted[i]]) return RS_ENULL;
    align = std::min(align, pointer_alignment(blocks[sorted[i]]));
  }
  if (block_bytes == 0) return RS_OK;

  std::lock_guard<std::mutex> lock(h->mu);
  const int ncu = device_cu_count();
  const uint8_t *zp = device_zero_page();
  if (ncu <= 0 || !zp) return RS_EDEVICE;
  const int sb = h->code.state_bytes();
  for (uint64_t off = 0; off < block_bytes; off += kMaxPieceBytes) {
    const uint64_t piece = std::min<uint64_t>(kMaxPieceBytes, block_bytes - off);
    CodecParams p;
    memset(&p, 0, sizeof(p));
    fill_decode_params(h->code, *plan, blocks, sorted, n_erasures, off, piece, &p);
    p.zero_page = zp;
    const LaunchCfg cfg = default_cfg(kDecode, sb, piece, align, ncu);
    const int rc = hip_status(launch_codec(kDecode, sb, p, cfg, stream));
    if (rc != RS_OK) return rc;
  }
  return RS_OK;
}

int rs_poly_stream_probe(uint8_t *base, size_t stripe_stride, size_t block_stride, int stripes,
                        int n_in, int n_out, size_t block_bytes, int tile_bytes, int tile_order,
                        void *stream) {
  if (!base) return RS_ENULL;
  if (stripes < 0 || n_in < 0 || n_in > RS_POLY_MAX_N || n_out < 0 || n_out > RS_POLY_MAX_M ||
      n_in + n_out == 0)
    return RS_EINVAL;
  if (pointer_alignment(base) < 16 || stripe_stride % 16 || block_stride % 16 ||
      block_bytes % 16 || block_bytes > kMaxPieceBytes || block_bytes > block_stride ||
      (uint64_t)(n_in + n_out) * block_stride > stripe_stride || tile_bytes < 4096 ||
      tile_bytes % 16 || (tile_order != 0 && tile_order != 1))
    return RS_EINVAL;
  if (stripes == 0 || block_bytes == 0) return RS_OK;
  const int ncu = device_cu_count();
  if (ncu <= 0) return RS_EDEVICE;
  return hip_status(launch_stream_probe(base, stripe_stride, block_stride, (uint32_t)stripes,
                                        (uint32_t)n_in, (uint32_t)n_out, (uint32_t)block_bytes,
                                        (uint32_t)tile_bytes, (uint32_t)tile_order, 2 * ncu,
                                        stream));
}

int rs_poly_decode_plan(rs_poly_t *h, const int *erasures, int n_erasures, unsigned flags,
                        int *read_set, int *n_read, uint8_t *coeffs) {
  if (!h) return RS_ENULL;
  int sorted[kMaxM];
  const int rc = validate_erasures(h->code, erasures, n_erasures, flags, sorted);
  if (rc != RS_OK) return rc;
  auto plan = h->code.plan(sorted, n_erasures, flags);
  if (read_set)
    for (size_t i = 0; i < plan->read.size(); ++i) read_set[i] = plan->read[i];
  if (n_read) *n_read = (int)plan->read.size();
  if (coeffs) {
    // Rows in the caller's order of the erasure list.
    const int m = h->code.m();
    for (int i = 0; i < n_erasures; ++i) {
      const int r = (int)(std::find(sorted, sorted + n_erasures, erasures[i]) - sorted);
      memcpy(coeffs + (size_t)i * m, plan->coeffs.data() + (size_t)r * m, (size_t)m);
    }
  }
  return RS_OK;
}

}  // extern "C"
