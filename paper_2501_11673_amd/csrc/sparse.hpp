// Sparse systems: the block step with A in compressed sparse rows (CSR).
//
// The paper's cost statement for inputs that are sparse and already incoherent
// (Section 1, limitations; RHT dropped as Section 3 allows) replaces the n-wide
// block products by products over the block's nonzeros.  The step here keeps
// that cost per step:
//
//   block rows     r = A_S x - b_S from the CSR rows of S (one wave per row)
//   back-projection  w = A_S^T y from a column-compressed copy of A_S that is
//                  built once per memoized block, next to its factor
//   momentum       m <- c (m - w), x <- x - w + eta m in a deferred form:
//                  x = u + t01 v, m = t11 v with (t01, t11) kept on the host,
//                  so a step touches only the block's columns; u, v are folded
//                  back into x, m (one pass over n) at a window's end or when
//                  the coefficients grow past a bound
//
// A step of the deferred form: with w the back-projection and (t01, t11)
// before the step, u -= (1 - t01 / t11) w and v -= w / t11, then
// t01 += eta c t11 and t11 *= c.  (Expanding u + t01' v and t11' v gives
// x - w + eta c (m - w) and c (m - w).)
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "kernels.hpp"

namespace kpp {

// Column-compressed copies of the memoized Kaczmarz++ blocks, one arena.  A
// block with z nonzeros owns entries [off, off + z + 1) of each array:
//   val[off + p], row[off + p]  the p-th nonzero in (column, row) order and
//                               its row within the block
//   col[off + q]                the q-th distinct column (q < nu)
//   ptr[off + q]                first nonzero of that column (ptr[off + nu] = z)
// and the block's slot holds nu in a per-slot array.
struct CscArena {
  double* val = nullptr;
  int32_t* row = nullptr;
  int32_t* col = nullptr;
  int32_t* ptr = nullptr;
};

// Blocks up to this many nonzeros are built in LDS; larger ones use a global
// workspace of csr_build_ws_doubles(z) doubles.
constexpr int32_t kCsrLdsEntries = 4096;
// A block holds at most this many nonzeros (the sort key keeps 20 bits of
// the nonzero's index within the block).
constexpr int64_t kCsrMaxBlockNnz = int64_t{1} << 20;
// Staging per new block: arena offset (two words), z, workspace offset (two
// words, negative: LDS).
constexpr int32_t kCsrMetaInts = 5;

// A signed 64-bit value as two staged words (low, high) and back.
inline void csr_meta_put(int32_t* w, int64_t v) {
  const uint64_t u = static_cast<uint64_t>(v);
  w[0] = static_cast<int32_t>(static_cast<uint32_t>(u & 0xffffffffu));
  w[1] = static_cast<int32_t>(static_cast<uint32_t>(u >> 32));
}

inline size_t csr_build_ws_doubles(int64_t z) {
  int64_t P2 = 1;   // sort keys (a power of two), values, densified row, compressed ids
  while (P2 < z) P2 <<= 1;
  const int64_t d = P2 + 2 * z + (z + 1) / 2;
  return static_cast<size_t>((d + 1) & ~int64_t{1});
}

// flag |= 1 bad row pointers, 2 a column out of range or not increasing in
// its row, 4 a NaN or Inf in the values or in b
void launch_csr_check(const int64_t* rp, const int32_t* ci, const double* cv, const double* b, int64_t m,
                      int64_t n, int64_t nnz, int32_t* flag, hipStream_t st);

// out[i] = sum_k A[rows[i], k] (u[k] + t01 v[k]) for i < sb (v unread when t01 = 0)
void launch_csr_rows_dot(const int64_t* rp, const int32_t* ci, const double* cv, const int32_t* rows, int32_t sb,
                         const double* u, const double* v, double t01, double* out, hipStream_t st);

// w = A_S^T y over slot q's column-compressed block (at off, z nonzeros, nu[q]
// columns); u -= au w, v -= av w on those columns
void launch_csc_apply(const CscArena& ar, int64_t off, int32_t z, const int32_t* nu, int32_t q, const double* y,
                      int32_t sb, double au, double av, double* u, double* v, hipStream_t st);

// CD++: w = I_S^T y; u[rows[i]] -= au y[i], v[rows[i]] -= av y[i]
void launch_rows_apply(const int32_t* rows, int32_t sb, const double* y, double au, double av, double* u, double* v,
                       hipStream_t st);

// u <- u + t01 v, v <- t11 v over n entries (the deferred iterate made explicit)
void launch_lazy_fold(double* u, double* v, int64_t n, double t01, double t11, hipStream_t st);

// Memo miss of nb Kaczmarz++ blocks (staged rows[k * s], lens[k], slot_of[k],
// meta[kCsrMetaInts * k]): the column-compressed copy into the arena, nu into
// nu[slot], and the regularized Gram A_S A_S^T + lambda I into the slot's
// lower part (column-major s x s), in fixed summation order.  err |= 4 when
// a block's nonzero count differs from the staged z.
void launch_csr_block_build(const int64_t* rp, const int32_t* ci, const double* cv, const int32_t* rows,
                            const int32_t* lens, const int32_t* slot_of, const int32_t* meta, int32_t nb, int32_t s,
                            double lambda, double* G, int64_t stride, const CscArena& ar, int32_t* nu, double* ws,
                            bool any_lds, bool any_global, int32_t* err, hipStream_t st);

// Memo miss of nb CD++ blocks: G = A_SS + lambda I from the CSR rows.
void launch_csr_gram_cd(const int64_t* rp, const int32_t* ci, const double* cv, const int32_t* rows,
                        const int32_t* lens, const int32_t* slot_of, int32_t nb, int32_t s, double lambda, double* G,
                        int64_t stride, hipStream_t st);

// A run of sparse steps in one launch of a team of G workgroups
// (kSparseTeamThreads threads each).  Workgroup g owns the column slice
// [g n / G, (g + 1) n / G) of u and v.  Per step: partial r over the slice
// (block rows from the CSR arrays, the slice's part of each row from the
// block's team table), all-gather of the partials, the workgroup's rows of
// y = G^{-1} r, all-gather of y, back-projection on the slice (Kaczmarz++:
// the block's compressed columns in the slice; CD++: the block rows in the
// slice).  Only the two all-gathers cross workgroups: no workgroup writes
// another's slice.  coef holds (t01, au, av) of each step; step_info
// kSparseStepInts words per step: slot, block length, nonzeros z, and
// (Kaczmarz++) the arena offset as two words.  Workgroup 0 keeps the
// DevState on chip and writes it back at the end.  Flags: r round at
// flags[g * kSparseFlagStride], y round at flags[kYFlagOffset + g *
// kSparseFlagStride], raised to epoch + k + 1 at step k; every wait is
// bounded by spin_limit polls (then err |= 2 and the team leaves).
constexpr int kSparseTeamThreads = 256;
constexpr int kSparseTeamMax = 16;
constexpr int kSparseStepInts = 5;
constexpr int kSparseFlagStride = 32;
// Team table of a slot (int32): row-relative start of each slice in each
// block row, (s x (G + 1), row-major), then the slice boundaries among the
// block's compressed columns (Kaczmarz++) or block rows (CD++) (G + 1).
__host__ __device__ inline int64_t csr_team_stride(int32_t s, int32_t G) { return static_cast<int64_t>(s + 1) * (G + 1); }
__host__ __device__ inline int64_t csr_slice_lo(int64_t n, int32_t G, int32_t g) { return (static_cast<int64_t>(g) * n) / G; }
struct SparseTeamArgs {
  const int64_t* rp = nullptr;
  const int32_t* ci = nullptr;
  const double* cv = nullptr;
  const double* b = nullptr;
  const int32_t* rows = nullptr;
  const double* L = nullptr;   // memo slots (G^{-1} at +s*s)
  int64_t slot_stride = 0;
  const int32_t* team = nullptr;
  int64_t team_stride = 0;
  const int32_t* step_info = nullptr;
  const double* coef = nullptr;
  CscArena ar;
  double* u = nullptr;
  double* v = nullptr;
  DevState* ds = nullptr;
  double* xr = nullptr;   // r partials, [2][G][s]
  double* xy = nullptr;   // y, [2][s]
  uint32_t* flags = nullptr;
  uint32_t epoch = 0;
  int64_t spin_limit = 0;
  int32_t* err = nullptr;
  uint64_t* phase_ticks = nullptr;   // optional profile: workgroup 0's wall-clock ticks per phase
  int32_t s = 0, W = 0, zeta = 0, adaptive = 0, G = 1;
};
void launch_sparse_team(int32_t kind, const SparseTeamArgs& a, hipStream_t st);

// Team tables of nb new blocks (staged rows, lens, slot_of; Kaczmarz++: the
// arena offsets in meta, after launch_csr_block_build) into team[slot *
// csr_team_stride(s, G)].
void launch_csr_team_tables(int32_t kind, const int64_t* rp, const int32_t* ci, const int32_t* rows,
                            const int32_t* lens, const int32_t* slot_of, const int32_t* meta, const CscArena& ar,
                            const int32_t* nu, int32_t nb, int32_t s, int64_t n, int32_t G, int32_t* team,
                            hipStream_t st);

// ||A x - b||^2 into *out (partial sums per workgroup in part, then one
// workgroup adds them in order); part holds csr_residual_parts(m) doubles.
constexpr int kCsrResidRowsPerGroup = 32;   // 4 waves of 8 rows
inline int64_t csr_residual_parts(int64_t m) { return (m + kCsrResidRowsPerGroup - 1) / kCsrResidRowsPerGroup; }
void launch_csr_residual_sq(const int64_t* rp, const int32_t* ci, const double* cv, const double* b, int64_t m,
                            const double* x, double* part, double* out, hipStream_t st);

}  // namespace kpp
