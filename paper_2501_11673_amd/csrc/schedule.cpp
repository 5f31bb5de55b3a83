// Block schedule generator; see schedule.hpp for the exact draw order.
#include "schedule.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <stdexcept>

namespace kpp {

double online_rate(int32_t kind, int64_t m, int64_t n, int32_t s) {
  if (kind == 1) return (static_cast<double>(n) / static_cast<double>(s)) * std::log(static_cast<double>(n));
  return (static_cast<double>(std::min(m, n)) / static_cast<double>(s)) *
         std::log(static_cast<double>(m));
}

BlockSchedule::BlockSchedule(MemoMode mode, int64_t N, int32_t s, uint64_t seed, double B0,
                             int32_t num_blocks, bool partition)
    : mode_(mode), N_(N), s_(s), B0_(B0), g_(seed) {
  if (s < 1 || N < s) throw std::invalid_argument("block size must satisfy 1 <= s <= rows");
  perm_.resize(static_cast<size_t>(N));
  if (N <= kBitmapMaxRows) bits_.assign(static_cast<size_t>((N + 63) / 64), 0);
  if (mode_ == MemoMode::Fixed) {
    if (partition) {
      std::iota(perm_.begin(), perm_.end(), 0);
      // the swap targets depend on the draws alone: each batch is drawn first
      // and its targets prefetched, then swapped in order
      constexpr int64_t kBatch = 32;
      int64_t kb[kBatch];
      for (int64_t j0 = 0; j0 + 1 < N; j0 += kBatch) {
        const int64_t nj = std::min<int64_t>(kBatch, N - 1 - j0);
        for (int64_t u = 0; u < nj; ++u) {
          kb[u] = j0 + u + static_cast<int64_t>(g_.bounded(static_cast<uint64_t>(N - j0 - u)));
          __builtin_prefetch(&perm_[kb[u]], 1);
        }
        for (int64_t u = 0; u < nj; ++u) std::swap(perm_[j0 + u], perm_[kb[u]]);
      }
      // chunk c is positions c s .. c s + l - 1 of the permutation, its rows in
      // ascending order: one pass over the rows, each to the chunk of its position
      const int64_t nchunks = (N + s - 1) / s;
      rows_.assign(static_cast<size_t>(nchunks * s), -1);
      len_.resize(static_cast<size_t>(nchunks));
      for (int64_t c = 0; c < nchunks; ++c) len_[c] = static_cast<int32_t>(std::min<int64_t>(s, N - c * s));
      std::vector<int32_t> chunk_of(static_cast<size_t>(N));
      for (int64_t c = 0; c < nchunks; ++c)
        for (int64_t j = c * s; j < c * s + len_[c]; ++j) chunk_of[perm_[j]] = static_cast<int32_t>(c);
      std::vector<int32_t> fill(static_cast<size_t>(nchunks), 0);
      for (int64_t r = 0; r < N; ++r) {
        const int64_t c = chunk_of[r];
        rows_[static_cast<size_t>(c * s + fill[c]++)] = static_cast<int32_t>(r);
      }
    } else {
      if (num_blocks < 1) throw std::invalid_argument("fixed collection needs num_blocks >= 1");
      std::iota(perm_.begin(), perm_.end(), 0);
      for (int32_t b = 0; b < num_blocks; ++b) add_subset();
    }
    used_.assign(len_.size(), 0);
  } else {
    std::iota(perm_.begin(), perm_.end(), 0);
  }
}

// Partial Fisher-Yates on the identity permutation (perm_ is the identity on
// entry and on exit: only the positions the draws touched are put back, so a
// subset costs O(s log s), or O(s + N / 64) with the bitmap, not O(N)).
void BlockSchedule::add_subset() {
  touched_.clear();
  for (int32_t j = 0; j < s_; ++j) {
    int64_t k = j + static_cast<int64_t>(g_.bounded(static_cast<uint64_t>(N_ - j)));
    std::swap(perm_[j], perm_[k]);
    touched_.push_back(k);
  }
  size_t base = rows_.size();
  rows_.resize(base + s_);
  int32_t* out = rows_.data() + base;
  if (!bits_.empty()) {
    // the rows are distinct: set their bits, then read them back in order
    for (int32_t j = 0; j < s_; ++j) {
      const int32_t r = perm_[j];
      bits_[static_cast<size_t>(r) >> 6] |= uint64_t{1} << (r & 63);
    }
    int32_t o = 0;
    for (size_t w = 0; o < s_; ++w) {
      uint64_t v = bits_[w];
      if (v == 0) continue;
      bits_[w] = 0;
      do {
        out[o++] = static_cast<int32_t>(w * 64 + static_cast<size_t>(__builtin_ctzll(v)));
        v &= v - 1;
      } while (v != 0);
    }
  } else {
    std::copy(perm_.begin(), perm_.begin() + s_, out);
    std::sort(out, out + s_);
  }
  len_.push_back(s_);
  for (int32_t j = 0; j < s_; ++j) perm_[j] = static_cast<int32_t>(j);
  for (int64_t k : touched_) perm_[k] = static_cast<int32_t>(k);
}

BlockSchedule::BlockSchedule(int64_t N, int32_t s, const int32_t* table, int32_t B, const int32_t* seq, int64_t L)
    : mode_(MemoMode::Fixed), N_(N), s_(s), B0_(0.0), g_(0), explicit_(true) {
  if (s < 1 || N < s) throw std::invalid_argument("block size must satisfy 1 <= s <= rows");
  if (B < 1 || table == nullptr) throw std::invalid_argument("an explicit schedule needs a table of at least one block");
  if (L < 0 || (L > 0 && seq == nullptr)) throw std::invalid_argument("explicit schedule: bad step sequence");
  rows_.assign(table, table + static_cast<size_t>(B) * s);
  for (int32_t b = 0; b < B; ++b) {
    const int32_t* r = table + static_cast<size_t>(b) * s;
    int32_t l = 0;
    while (l < s && r[l] >= 0) ++l;
    if (l == 0) throw std::invalid_argument("explicit schedule: empty block");
    for (int32_t j = l; j < s; ++j)
      if (r[j] != -1) throw std::invalid_argument("explicit schedule: rows after the padding of a block");
    for (int32_t j = 0; j < l; ++j) {
      if (r[j] >= N) throw std::invalid_argument("explicit schedule: row index out of range");
      if (j > 0 && r[j] <= r[j - 1]) throw std::invalid_argument("explicit schedule: rows of a block must ascend");
    }
    len_.push_back(l);
  }
  seq_.assign(seq, seq + L);
  for (int32_t b : seq_)
    if (b < 0 || b >= B) throw std::invalid_argument("explicit schedule: block id out of range");
  used_.assign(len_.size(), 0);
}

int32_t BlockSchedule::next(bool* is_new) {
  int32_t b;
  bool fresh = false;
  if (explicit_) {
    if (t_ >= static_cast<int64_t>(seq_.size())) throw std::out_of_range("explicit schedule exhausted");
    b = seq_[static_cast<size_t>(t_)];
    fresh = !used_[b];
    used_[b] = 1;
    ++t_;
    if (is_new) *is_new = fresh;
    return b;
  }
  switch (mode_) {
    case MemoMode::Fixed: {
      b = static_cast<int32_t>(g_.bounded(len_.size()));
      fresh = !used_[b];
      used_[b] = 1;
      break;
    }
    case MemoMode::Online: {
      double u = g_.uniform();
      if (t_ == 0 || u < B0_ / static_cast<double>(t_)) {
        add_subset();
        b = static_cast<int32_t>(len_.size()) - 1;
        fresh = true;
      } else {
        b = static_cast<int32_t>(g_.bounded(len_.size()));
      }
      break;
    }
    case MemoMode::Off:
    default: {
      add_subset();
      b = static_cast<int32_t>(len_.size()) - 1;
      fresh = true;
      break;
    }
  }
  ++t_;
  if (is_new) *is_new = fresh;
  return b;
}

namespace {
template <typename T>
void put(std::vector<uint8_t>* out, const T& v) {
  const uint8_t* p = reinterpret_cast<const uint8_t*>(&v);
  out->insert(out->end(), p, p + sizeof(T));
}
template <typename T>
void put_vec(std::vector<uint8_t>* out, const std::vector<T>& v) {
  put<uint64_t>(out, v.size());
  if (v.empty()) return;
  const uint8_t* p = reinterpret_cast<const uint8_t*>(v.data());
  out->insert(out->end(), p, p + v.size() * sizeof(T));
}
struct Reader {
  const uint8_t* p;
  size_t left;
  template <typename T>
  T get() {
    if (left < sizeof(T)) throw std::invalid_argument("schedule state is truncated");
    T v;
    std::memcpy(&v, p, sizeof(T));
    p += sizeof(T);
    left -= sizeof(T);
    return v;
  }
  template <typename T>
  std::vector<T> get_vec(uint64_t max_len) {
    const uint64_t len = get<uint64_t>();
    if (len > max_len || len * sizeof(T) > left) throw std::invalid_argument("schedule state is malformed");
    std::vector<T> v(len);
    if (len > 0) std::memcpy(v.data(), p, len * sizeof(T));
    p += len * sizeof(T);
    left -= len * sizeof(T);
    return v;
  }
};
constexpr uint32_t kScheduleStateTag = 0x4b505353u;   // "KPSS"
}  // namespace

void BlockSchedule::save(std::vector<uint8_t>* out) const {
  put<uint32_t>(out, kScheduleStateTag);
  put<int32_t>(out, static_cast<int32_t>(mode_));
  put<int64_t>(out, N_);
  put<int32_t>(out, s_);
  put<double>(out, B0_);
  put<uint64_t>(out, g_.state());
  put<int64_t>(out, t_);
  put<uint8_t>(out, explicit_ ? 1 : 0);
  put_vec(out, rows_);
  put_vec(out, len_);
  put_vec(out, used_);
  put_vec(out, seq_);
}

BlockSchedule BlockSchedule::load(const uint8_t* data, size_t bytes) {
  Reader r{data, bytes};
  if (r.get<uint32_t>() != kScheduleStateTag) throw std::invalid_argument("not a schedule state");
  const int32_t mode = r.get<int32_t>();
  const int64_t N = r.get<int64_t>();
  const int32_t s = r.get<int32_t>();
  const double B0 = r.get<double>();
  const uint64_t state = r.get<uint64_t>();
  const int64_t t = r.get<int64_t>();
  const bool expl = r.get<uint8_t>() != 0;
  if (mode < 0 || mode > 2 || s < 1 || N < s || t < 0) throw std::invalid_argument("schedule state is malformed");
  const uint64_t cap = uint64_t{1} << 40;
  std::vector<int32_t> rows = r.get_vec<int32_t>(cap);
  std::vector<int32_t> len = r.get_vec<int32_t>(cap);
  std::vector<uint8_t> used = r.get_vec<uint8_t>(cap);
  std::vector<int32_t> seq = r.get_vec<int32_t>(cap);
  if (rows.size() != len.size() * static_cast<size_t>(s) || (!used.empty() && used.size() != len.size()))
    throw std::invalid_argument("schedule state is malformed");
  for (size_t b = 0; b < len.size(); ++b) {
    if (len[b] < 1 || len[b] > s) throw std::invalid_argument("schedule state is malformed");
    for (int32_t j = 0; j < len[b]; ++j) {
      const int32_t v = rows[b * s + j];
      if (v < 0 || v >= N) throw std::invalid_argument("schedule state is malformed");
    }
  }
  for (int32_t b : seq)
    if (b < 0 || static_cast<size_t>(b) >= len.size()) throw std::invalid_argument("schedule state is malformed");
  if (expl && t > static_cast<int64_t>(seq.size())) throw std::invalid_argument("schedule state is malformed");
  // a generator of the right shape, then the saved state in place of its draws
  BlockSchedule out(MemoMode::Online, N, s, 0, B0, 0, true);
  out.mode_ = static_cast<MemoMode>(mode);
  out.g_ = SplitMix64(state);
  out.t_ = t;
  out.explicit_ = expl;
  out.rows_ = std::move(rows);
  out.len_ = std::move(len);
  out.used_ = std::move(used);
  out.seq_ = std::move(seq);
  return out;
}

}  // namespace kpp
