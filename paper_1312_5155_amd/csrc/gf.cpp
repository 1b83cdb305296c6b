// Host-side field arithmetic, generator polynomial, LFSR table bases and
// per-erasure-pattern decode coefficients.
#include "gf.h"

#include <string.h>

#include <algorithm>

#include "../../include/rs_poly.h"

namespace rsp {

bool Field::init(int w, unsigned poly) {
  if (w != 4 && w != 8) return false;
  const int q = 1 << w;
  if ((poly >> w) != 1u) return false;
  w_ = w;
  poly_ = poly;
  order_ = q - 1;
  for (int i = 0; i < 256; ++i) log_[i] = -1;
  // Successive powers of alpha = x; a power seen twice before q-1 steps
  // means x is not a generator.
  unsigned x = 1;
  for (int e = 0; e < order_; ++e) {
    if (log_[x] >= 0) return false;
    log_[x] = e;
    exp_[e] = (uint8_t)x;
    exp_[e + order_] = (uint8_t)x;
    x <<= 1;
    if (x & (unsigned)q) x ^= poly;
  }
  return x == 1;
}

static void invert(const Field &F, int t, uint8_t *a /* t x t, destroyed */,
                   uint8_t *out /* t x t */) {
  // Gauss-Jordan on [a | I].  a is a Vandermonde matrix over distinct
  // points, hence nonsingular: a pivot always exists.
  for (int i = 0; i < t; ++i)
    for (int j = 0; j < t; ++j) out[i * t + j] = (uint8_t)(i == j);
  for (int c = 0; c < t; ++c) {
    int piv = c;
    while (a[piv * t + c] == 0) ++piv;
    if (piv != c)
      for (int j = 0; j < t; ++j) {
        std::swap(a[piv * t + j], a[c * t + j]);
        std::swap(out[piv * t + j], out[c * t + j]);
      }
    const uint8_t s = F.inv(a[c * t + c]);
    for (int j = 0; j < t; ++j) {
      a[c * t + j] = F.mul(a[c * t + j], s);
      out[c * t + j] = F.mul(out[c * t + j], s);
    }
    for (int r = 0; r < t; ++r) {
      const uint8_t f = a[r * t + c];
      if (r == c || f == 0) continue;
      for (int j = 0; j < t; ++j) {
        a[r * t + j] ^= F.mul(f, a[c * t + j]);
        out[r * t + j] ^= F.mul(f, out[c * t + j]);
      }
    }
  }
}

// Packs the images of the unit bytes 1, 2, ..., 128 of a byte-linear map
// whose value for byte x is sum_b coef[b](x) << 8b.
template <typename ValueOf>
static void make_basis(int sb, int w, ValueOf value_of, uint32_t *basis) {
  memset(basis, 0, 16 * sizeof(uint32_t));
  for (int bit = 0; bit < w; ++bit) {
    const uint64_t v = value_of((uint8_t)(1u << bit));
    if (sb == 4) {
      basis[bit] = (uint32_t)v;
    } else {
      basis[2 * bit] = (uint32_t)v;
      basis[2 * bit + 1] = (uint32_t)(v >> 32);
    }
  }
}

int Code::init(int k, int m, int w, unsigned poly) {
  if (w != 4 && w != 8) return RS_EINVAL;
  if (k < 1 || m < 1 || m > kMaxM) return RS_EINVAL;
  if (k + m > (1 << w) - 1) return RS_EINVAL;
  if (!F_.init(w, poly)) return RS_EINVAL;
  k_ = k;
  m_ = m;
  sb_ = rsp::state_bytes(m);

  // g(x) = prod_{i<m} (x + alpha^i), low degree first (Sec. 3.1).
  memset(g_, 0, sizeof(g_));
  g_[0] = 1;
  for (int i = 0; i < m; ++i) {
    const uint8_t r = F_.alpha_pow(i);
    for (int d = i + 1; d >= 1; --d) g_[d] = g_[d - 1] ^ F_.mul(g_[d], r);
    g_[0] = F_.mul(g_[0], r);
  }

  // T'[f] = sum_b (g_(m-1-b) f) << 8b  ^  f << 8(sb-1): the LFSR feedback
  // value plus the term that clears the consumed window byte.
  const int sb = sb_;
  auto tval = [this, sb](uint8_t f) -> uint64_t {
    uint64_t v = 0;
    for (int b = 0; b < m_; ++b) v |= (uint64_t)F_.mul(g_[m_ - 1 - b], f) << (8 * b);
    return v ^ ((uint64_t)f << (8 * (sb - 1)));
  };
  make_basis(sb, w, tval, lfsr_basis_);

  // Generator-matrix columns (Sec. 6): x^m mod g = g_0 + ... + g_(m-1)
  // x^(m-1) (characteristic 2), then one multiplication by x mod g per data
  // block.
  pcol_.assign((size_t)k * m, 0);
  std::vector<uint8_t> r(g_, g_ + m);
  for (int j = 0; j < k; ++j) {
    memcpy(&pcol_[(size_t)j * m], r.data(), (size_t)m);
    const uint8_t top = r[m - 1];
    for (int i = m - 1; i >= 1; --i) r[i] = r[i - 1] ^ F_.mul(top, g_[i]);
    r[0] = F_.mul(top, g_[0]);
  }

  // Bit-sliced form (k <= kBitmatrixMaxK): row b of the product by c_ij has
  // bit b' set when bit b of c_ij * 2^b' is.
  bm_ = BitmatrixCode{};
  if (k <= kBitmatrixMaxK) {
    bm_rows_ = std::make_unique<BitRows>();
    memset(bm_rows_.get(), 0, sizeof(BitRows));
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < m; ++i) {
        const uint8_t c = pcol_[(size_t)j * m + i];
        for (int bi = 0; bi < w; ++bi) {
          const uint8_t prod = F_.mul(c, (uint8_t)(1u << bi));
          for (int b = 0; b < w; ++b)
            if ((prod >> b) & 1) bm_rows_->r[j][i][b] |= (uint8_t)(1u << bi);
        }
      }
    bm_.k = k;
    bm_.m = m;
    bm_.builtin = bitmatrix_builtin(k, m, w, poly);
    bm_.rows = bm_rows_.get();
    bm_.key = (int)(poly << 12) | (k << 4) | m;
  }
  return RS_OK;
}

void Code::column_basis(int j, uint32_t *basis) const {
  const uint8_t *col = &pcol_[(size_t)j * m_];
  auto val = [this, col](uint8_t x) -> uint64_t {
    uint64_t v = 0;
    for (int b = 0; b < m_; ++b) v |= (uint64_t)F_.mul(col[m_ - 1 - b], x) << (8 * b);
    return v;
  };
  make_basis(sb_, F_.w(), val, basis);
}

size_t Code::KeyHash::operator()(const Key &k) const {
  uint64_t h = 0x9E3779B97F4A7C15ull ^ k.flags;
  for (uint64_t x : k.mask) {
    h ^= x + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
  }
  return (size_t)h;
}

std::shared_ptr<DecodePlan> Code::build_plan(const int *e, int t, unsigned flags) const {
  auto plan = std::make_shared<DecodePlan>();
  const int n = k_ + m_;
  std::vector<char> erased(n, 0);
  for (int i = 0; i < t; ++i) erased[e[i]] = 1;

  // Blocks read: every survivor, or (default) the k survivors of lowest
  // degree in the code polynomial -- the surviving parity blocks (degrees
  // 0..m-1), then the surviving data blocks from d_0 up.  The LFSR then
  // starts at the highest data block read, so the unread top data blocks
  // cost no steps.
  std::vector<int> by_degree;
  for (int i = 0; i < m_; ++i) by_degree.push_back(k_ + i);
  for (int j = 0; j < k_; ++j) by_degree.push_back(j);
  const int want = (flags & RS_POLY_FLAG_ALL_SURVIVORS) ? n : k_;
  std::vector<int> unknown(e, e + t);  // erased first, in output order
  for (int b : by_degree) {
    if (erased[b]) continue;
    if ((int)plan->read.size() < want)
      plan->read.push_back(b);
    else
      unknown.push_back(b);  // survivor left unread: solved for, discarded
  }
  std::sort(plan->read.begin(), plan->read.end());
  plan->span = 1;
  for (int b : plan->read)
    if (b < k_) plan->span = std::max(plan->span, b + 1);
  const int u = (int)unknown.size();

  // V[i][j] = alpha^(i pos(U_j)), i, j < u, over the unknown positions; the
  // values r(alpha^i) = sum_l r_l alpha^(i l) of the reduced received word
  // equal V * (unknown symbols).  C = V^-1 W with W[i][l] = alpha^(i l).
  std::vector<uint8_t> V(u * u), Vi(u * u);
  for (int i = 0; i < u; ++i)
    for (int j = 0; j < u; ++j) V[i * u + j] = F_.alpha_pow((long)i * position(unknown[j]));
  invert(F_, u, V.data(), Vi.data());
  plan->coeffs.assign((size_t)t * m_, 0);
  for (int r = 0; r < t; ++r)
    for (int l = 0; l < m_; ++l) {
      uint8_t acc = 0;
      for (int i = 0; i < u; ++i) acc ^= F_.mul(Vi[r * u + i], F_.alpha_pow((long)i * l));
      plan->coeffs[r * m_ + l] = acc;
    }

  // Apply table for state byte b (remainder coefficient r_(m-1-b)): packed
  // over the rebuilt symbols r < t at byte r.
  memset(plan->apply_basis, 0, sizeof(plan->apply_basis));
  for (int b = 0; b < m_; ++b) {
    const int l = m_ - 1 - b;
    auto uval = [&](uint8_t x) -> uint64_t {
      uint64_t v = 0;
      for (int r = 0; r < t; ++r) v |= (uint64_t)F_.mul(plan->coeffs[r * m_ + l], x) << (8 * r);
      return v;
    };
    make_basis(sb_, F_.w(), uval, plan->apply_basis[b]);
  }
  return plan;
}

std::shared_ptr<const DecodePlan> Code::plan(const int *e, int t, unsigned flags) {
  Key key{};
  for (int i = 0; i < t; ++i) key.mask[e[i] >> 6] |= 1ull << (e[i] & 63);
  key.flags = flags;
  std::lock_guard<std::mutex> lock(mu_);
  auto it = index_.find(key);
  if (it != index_.end()) {
    lru_.splice(lru_.begin(), lru_, it->second);
    return it->second->second;
  }
  auto plan = build_plan(e, t, flags);
  lru_.emplace_front(key, plan);
  index_[key] = lru_.begin();
  if (lru_.size() > kCacheCap) {
    index_.erase(lru_.back().first);
    lru_.pop_back();
  }
  return plan;
}

}  // namespace rsp
