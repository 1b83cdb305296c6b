// Host-side GF(2^w) arithmetic and per-code / per-erasure-pattern
// coefficient preparation for the codec kernels.
#pragma once

#include <stdint.h>

#include <array>
#include <list>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "rs_internal.h"

namespace rsp {

// GF(2^w), w in {4, 8}, built from a primitive polynomial with alpha = 2.
class Field {
 public:
  // Returns false if poly does not have degree w or x is not primitive.
  bool init(int w, unsigned poly);
  uint8_t mul(uint8_t a, uint8_t b) const {
    if (a == 0 || b == 0) return 0;
    return exp_[log_[a] + log_[b]];
  }
  uint8_t inv(uint8_t a) const { return exp_[order_ - log_[a]]; }
  uint8_t alpha_pow(long e) const {
    long r = e % order_;
    if (r < 0) r += order_;
    return exp_[r];
  }
  int order() const { return order_; }
  int w() const { return w_; }
  unsigned poly() const { return poly_; }

 private:
  int w_ = 0, order_ = 0;
  unsigned poly_ = 0;
  uint8_t exp_[512] = {};  // doubled so that exp_[log a + log b] needs no mod
  int log_[256] = {};
};

// Byte-linear packed table described by the images of 1, 2, ..., 128.
struct Basis {
  uint32_t v[16];  // value of 2^b in v[b] (4-byte state) or v[2b], v[2b+1]
};

// A decode plan: which blocks are read and the packed apply-table bases.
struct DecodePlan {
  std::vector<int> read;          // API indices read, increasing
  int span = 1;                   // 1 + highest data index read (at least 1):
                                  // the LFSR starts at data block span - 1
  std::vector<uint8_t> coeffs;    // t x m, row e = rebuilt symbol e
  uint32_t apply_basis[kMaxM][16];
};

// Code description shared by every call on one handle.
class Code {
 public:
  int init(int k, int m, int w, unsigned poly);  // 0 or an RS_E* code
  int k() const { return k_; }
  int m() const { return m_; }
  int n() const { return k_ + m_; }
  int state_bytes() const { return sb_; }
  const uint8_t *generator() const { return g_; }
  const uint32_t *lfsr_basis() const { return lfsr_basis_; }
  const Field &field() const { return F_; }
  // Degree of API block b in the codeword polynomial (eq. (2)).
  int position(int b) const { return b < k_ ? m_ + b : b - k_; }
  // Packed-table basis of the generator-matrix column of data block j
  // (Sec. 6): byte x maps to the remainder of x * x^(m+j) mod g(x), byte b
  // holding coefficient m-1-b.  16 dwords, as lfsr_basis().
  void column_basis(int j, uint32_t *basis) const;
  // The m coefficients of x^(m+j) mod g(x), low degree first (column j of
  // the generator matrix, Sec. 6).
  const uint8_t *column(int j) const { return &pcol_[(size_t)j * m_]; }
  // The bit-sliced form of the code (k <= kBitmatrixMaxK), else nullptr.
  const BitmatrixCode *bitmatrix() const { return bm_rows_ ? &bm_ : nullptr; }
  // Plan for the erasure list e[0..t), validated and sorted increasingly by
  // the caller; rebuilt symbol i is block e[i].  Cached (Opt3 of Sec. 4).
  std::shared_ptr<const DecodePlan> plan(const int *e, int t, unsigned flags);

 private:
  std::shared_ptr<DecodePlan> build_plan(const int *e, int t, unsigned flags) const;

  int k_ = 0, m_ = 0, sb_ = 4;
  Field F_;
  uint8_t g_[kMaxM + 1] = {};
  uint32_t lfsr_basis_[16] = {};
  std::vector<uint8_t> pcol_;   // k x m: row j = coefficients of x^(m+j) mod g
  std::unique_ptr<BitRows> bm_rows_;
  BitmatrixCode bm_;

  // LRU cache of plans keyed by (erased-block bitmap, flags).
  struct Key {
    std::array<uint64_t, 4> mask;
    unsigned flags;
    bool operator==(const Key &o) const { return mask == o.mask && flags == o.flags; }
  };
  struct KeyHash {
    size_t operator()(const Key &k) const;
  };
  static constexpr size_t kCacheCap = 4096;
  std::mutex mu_;
  std::list<std::pair<Key, std::shared_ptr<DecodePlan>>> lru_;
  std::unordered_map<Key, decltype(lru_)::iterator, KeyHash> index_;
};

}  // namespace rsp
