// Block schedule generator; see schedule.hpp for the exact draw order.
#include "schedule.hpp"

#include <algorithm>
#include <cmath>
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
  if (mode_ == MemoMode::Fixed) {
    if (partition) {
      std::iota(perm_.begin(), perm_.end(), 0);
      for (int64_t j = 0; j + 1 < N; ++j) {
        int64_t k = j + static_cast<int64_t>(g_.bounded(static_cast<uint64_t>(N - j)));
        std::swap(perm_[j], perm_[k]);
      }
      for (int64_t lo = 0; lo < N; lo += s) {
        int32_t l = static_cast<int32_t>(std::min<int64_t>(s, N - lo));
        size_t base = rows_.size();
        rows_.resize(base + s, -1);
        std::copy(perm_.begin() + lo, perm_.begin() + lo + l, rows_.begin() + base);
        std::sort(rows_.begin() + base, rows_.begin() + base + l);
        len_.push_back(l);
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
// subset costs O(s log s), not O(N)).
void BlockSchedule::add_subset() {
  touched_.clear();
  for (int32_t j = 0; j < s_; ++j) {
    int64_t k = j + static_cast<int64_t>(g_.bounded(static_cast<uint64_t>(N_ - j)));
    std::swap(perm_[j], perm_[k]);
    touched_.push_back(k);
  }
  size_t base = rows_.size();
  rows_.resize(base + s_);
  std::copy(perm_.begin(), perm_.begin() + s_, rows_.begin() + base);
  std::sort(rows_.begin() + base, rows_.end());
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

}  // namespace kpp
