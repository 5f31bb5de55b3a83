// Block schedule of the Kaczmarz++ / CD++ solver (host side).
//
// The paper's block selection (Section 5.2 "simplified block memoization",
// Algorithm 2 for CD++, Algorithm 5 for Kaczmarz++, and the fixed collection
// of Algorithm 1) never looks at the iterate, so the whole sequence of blocks
// depends on the seed alone and can be produced ahead of the device work.
//
// Random numbers: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): a Weyl
// counter advanced by 0x9E3779B97F4A7C15 and the published 64-bit mixer.
//   uniform()  = (next() >> 11) * 2^-53
//   bounded(k) = ((next() >> 11) * k) >> 53        (128-bit product)
//   subset     = sorted first s entries of a partial Fisher-Yates shuffle of
//                0..N-1 that swaps position j with j + bounded(N - j)
// Modes:
//   ONLINE: step 0 takes a new block; step t >= 1 draws u = uniform() and
//           takes a new block iff u < B0 / t, else reuses block bounded(|B|).
//           B0 = (rows/s) ln(rows) for CD++, (min(m, n)/s) ln(m) for K++.
//   FIXED:  the collection is drawn first -- a random partition (Fisher-Yates
//           over all rows, positions 0..N-2, then consecutive chunks of s, the
//           last chunk possibly shorter) or num_blocks subsets -- and each
//           step uses block bounded(B).
//   OFF:    a new subset at every step; its factor is not kept.
//   Explicit (caller-given): a table of blocks (rows ascending, -1 after the
//           last row of a shorter block) and the block id of every step; each
//           block is factored on first use and kept, as in FIXED.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace kpp {

class SplitMix64 {
 public:
  explicit SplitMix64(uint64_t seed) : state_(seed) {}
  uint64_t state() const { return state_; }
  uint64_t next() {
    state_ += 0x9E3779B97F4A7C15ull;
    uint64_t z = state_;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return static_cast<double>(next() >> 11) * (1.0 / 9007199254740992.0); }
  uint64_t bounded(uint64_t k) {
    unsigned __int128 p = static_cast<unsigned __int128>(next() >> 11) * k;
    return static_cast<uint64_t>(p >> 53);
  }

 private:
  uint64_t state_;
};

enum class MemoMode : int32_t { Off = 0, Online = 1, Fixed = 2 };

// Row counts up to this order a new subset's rows through a bitmap of all rows
// (a scan of N / 64 words) instead of a comparison sort.
constexpr int64_t kBitmapMaxRows = int64_t{1} << 18;

// Sequential schedule generator: next() yields the block of step 0, 1, 2, ...
class BlockSchedule {
 public:
  BlockSchedule(MemoMode mode, int64_t N, int32_t s, uint64_t seed, double B0,
                int32_t num_blocks, bool partition);
  // Explicit schedule: table holds B x s row indices, seq the block of each of
  // L steps.  Throws std::invalid_argument on a malformed table or sequence.
  BlockSchedule(int64_t N, int32_t s, const int32_t* table, int32_t B, const int32_t* seq, int64_t L);

  // Block id of the next step; *is_new is set when that block is used for the
  // first time (its factor has to be computed).
  int32_t next(bool* is_new);

  int64_t steps_done() const { return t_; }
  int32_t num_blocks() const { return static_cast<int32_t>(len_.size()); }
  int32_t block_size() const { return s_; }
  const int32_t* rows(int32_t b) const { return rows_.data() + static_cast<size_t>(b) * s_; }
  int32_t len(int32_t b) const { return len_[b]; }
  // For OFF mode the table only needs the latest block: callers may drop old ones.
  MemoMode mode() const { return mode_; }
  bool is_explicit() const { return explicit_; }
  int64_t length() const { return static_cast<int64_t>(seq_.size()); }

  // The generator's whole state (draws made, collection, step count) as
  // bytes, and a generator that continues exactly where the saved one stopped.
  void save(std::vector<uint8_t>* out) const;
  static BlockSchedule load(const uint8_t* data, size_t bytes);  // throws std::invalid_argument

 private:
  void add_subset();
  MemoMode mode_;
  int64_t N_;
  int32_t s_;
  double B0_;
  SplitMix64 g_;
  int64_t t_ = 0;
  std::vector<int32_t> rows_;  // num_blocks x s (entries past len are -1)
  std::vector<int32_t> len_;
  std::vector<uint8_t> used_;
  std::vector<int32_t> perm_;
  std::vector<int64_t> touched_;
  std::vector<uint64_t> bits_;   // one bit per row (N <= kBitmapMaxRows): a subset's rows in order
  bool explicit_ = false;
  std::vector<int32_t> seq_;
};

// B0 of the Bernoulli(min(1, B0 / t)) rule.
double online_rate(int32_t kind, int64_t m, int64_t n, int32_t s);

}  // namespace kpp
