// HIP kernels (gfx950) of the sparse (CSR) block step; the deferred momentum
// form and the arena layout are described in sparse.hpp.
//
// Every reduction runs in a fixed order, so a run is bitwise repeatable: the
// block Gram and the back-projection sum each column's nonzeros in row order
// from the column-compressed copy instead of scattering with atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels.hpp"
#include "exchange.hpp"
#include "lanes.hpp"
#include "sparse.hpp"
#include "step_state.hpp"

namespace kpp {
namespace {

constexpr int kST = 256;   // threads of the step kernels (4 waves)
constexpr int kBT = 512;   // threads of the block-build kernel (8 waves)
constexpr int kKeyBits = 20;
constexpr uint64_t kKeyMask = (uint64_t{1} << kKeyBits) - 1;
constexpr int kRowsPerWave = 8;   // rows a wave sums in the true-residual kernel
static_assert((kST / 64) * kRowsPerWave == kCsrResidRowsPerGroup, "residual partial layout");
constexpr size_t kBuildLds = static_cast<size_t>(kCsrLdsEntries) * (3 * sizeof(double) + sizeof(int32_t));

__device__ __forceinline__ int64_t meta_i64(const int32_t* p) {
  return static_cast<int64_t>((static_cast<uint64_t>(static_cast<uint32_t>(p[1])) << 32) |
                              static_cast<uint64_t>(static_cast<uint32_t>(p[0])));
}

// --------------------------------------------------------------------------
// structure check: one thread per row
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kST) void k_csr_check(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                   const double* __restrict__ cv, const double* __restrict__ b,
                                                   int64_t m, int64_t n, int64_t nnz, int32_t* flag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kST + threadIdx.x;
  if (i >= m) return;
  int bad = 0;
  const int64_t a = rp[i], e = rp[i + 1];
  if ((i == 0 && a != 0) || (i == m - 1 && e != nnz) || a < 0 || e < a || e > nnz) {
    bad |= 1;
  } else {
    int64_t prev = -1;
    for (int64_t k = a; k < e; ++k) {
      const int64_t c = ci[k];
      if (c <= prev || c >= n) {
        bad |= 2;
        break;
      }
      prev = c;
      if (!isfinite(cv[k])) bad |= 4;
    }
  }
  if (!isfinite(b[i])) bad |= 4;
  if (bad) atomicOr(flag, bad);
}

// --------------------------------------------------------------------------
// step: block rows (one wave per row of S)
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kST) void k_csr_rows_dot(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                      const double* __restrict__ cv, const int32_t* __restrict__ rows,
                                                      int32_t sb, const double* __restrict__ u,
                                                      const double* __restrict__ v, double t01,
                                                      double* __restrict__ out) {
  const int w = blockIdx.x * (kST / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (w >= sb) return;
  const int64_t r = rows[w];
  const int64_t a = rp[r], e = rp[r + 1];
  double acc = 0.0;
  if (t01 != 0.0) {
    for (int64_t k = a + lane; k < e; k += 64) {
      const int32_t c = ci[k];
      acc = fma(cv[k], fma(t01, v[c], u[c]), acc);
    }
  } else {
    for (int64_t k = a + lane; k < e; k += 64) acc = fma(cv[k], u[ci[k]], acc);
  }
  acc = wave_sum(acc);
  if (lane == 0) out[w] = acc;
}

// --------------------------------------------------------------------------
// step: back-projection and deferred momentum update
// --------------------------------------------------------------------------
// One thread per distinct column of the block: w_j = sum over the column's
// nonzeros in row order of A_ij y_i.
__global__ __launch_bounds__(kST) void k_csc_apply(const double* __restrict__ cval, const int32_t* __restrict__ crow,
                                                   const int32_t* __restrict__ ccol,
                                                   const int32_t* __restrict__ cptr, const int32_t* __restrict__ nu,
                                                   int32_t q, const double* __restrict__ y, int32_t sb, double au,
                                                   double av, double* __restrict__ u, double* __restrict__ v) {
  __shared__ double ys[kMaxBlock];
  for (int i = threadIdx.x; i < sb; i += kST) ys[i] = y[i];
  __syncthreads();
  const int32_t k = blockIdx.x * kST + threadIdx.x;
  if (k >= nu[q]) return;
  const int32_t p0 = cptr[k], p1 = cptr[k + 1];
  double w = 0.0;
  for (int32_t p = p0; p < p1; ++p) w = fma(cval[p], ys[crow[p]], w);
  const int64_t j = ccol[k];
  u[j] = fma(-au, w, u[j]);
  v[j] = fma(-av, w, v[j]);
}

__global__ __launch_bounds__(kST) void k_rows_apply(const int32_t* __restrict__ rows, int32_t sb,
                                                    const double* __restrict__ y, double au, double av,
                                                    double* __restrict__ u, double* __restrict__ v) {
  const int i = blockIdx.x * kST + threadIdx.x;
  if (i >= sb) return;
  const int64_t j = rows[i];
  const double yi = y[i];
  u[j] = fma(-au, yi, u[j]);
  v[j] = fma(-av, yi, v[j]);
}

__global__ __launch_bounds__(kST) void k_lazy_fold(double* __restrict__ u, double* __restrict__ v, int64_t n,
                                                   double t01, double t11) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kST;
  for (int64_t j = static_cast<int64_t>(blockIdx.x) * kST + threadIdx.x; j < n; j += stride) {
    const double vj = v[j];
    u[j] = fma(t01, vj, u[j]);
    v[j] = t11 * vj;
  }
}

// --------------------------------------------------------------------------
// memo miss, Kaczmarz++: column-compressed copy and regularized Gram
// --------------------------------------------------------------------------
// One workgroup per new block.  The block's nonzeros are numbered e = 0..z-1
// in row order; key (column << 20 | e) sorts them into (column, row) order
// (bitonic sort), heads of equal columns give the compressed column ids q,
// and the arena receives values, rows, columns and column starts.  The Gram
// then densifies one row i at a time over the compressed columns and every
// row k >= i takes its dot product with it (nonzeros of k in column order).
// Blocks with z <= kCsrLdsEntries work in LDS, larger ones in the global
// workspace (the GLOBAL instantiation); each launch skips the other kind.
__device__ void block_incl_scan(int32_t* scan, int tid) {
  __syncthreads();
  for (int o = 1; o < kBT; o <<= 1) {
    const int32_t a = tid >= o ? scan[tid - o] : 0;
    __syncthreads();
    scan[tid] += a;
    __syncthreads();
  }
}

template <bool GLOBAL>
__global__ __launch_bounds__(kBT) void k_csr_block_build(
    const int64_t* __restrict__ rp, const int32_t* __restrict__ ci, const double* __restrict__ cv,
    const int32_t* __restrict__ rows, const int32_t* __restrict__ lens, const int32_t* __restrict__ slot_of,
    const int32_t* __restrict__ meta, int32_t s, double lambda, double* __restrict__ G, int64_t stride,
    CscArena ar, int32_t* __restrict__ nu, double* __restrict__ ws, int32_t* __restrict__ err) {
  extern __shared__ __align__(16) unsigned char dyn[];
  __shared__ int32_t rowoff[kMaxBlock + 1];
  __shared__ int64_t rowbase[kMaxBlock];
  __shared__ int32_t scan[kBT];
  const int blk = blockIdx.x, tid = threadIdx.x;
  const int32_t* M = meta + static_cast<int64_t>(kCsrMetaInts) * blk;
  const int64_t off = meta_i64(M);
  const int32_t z = M[2];
  const int64_t wso = meta_i64(M + 3);
  if (GLOBAL != (wso >= 0)) return;
  const int sb = lens[blk];
  const int32_t* R = rows + static_cast<int64_t>(blk) * s;
  double* Gb = G + static_cast<int64_t>(slot_of[blk]) * stride;
  int32_t P2 = 1;
  while (P2 < z) P2 <<= 1;
  uint64_t* keys;
  double *ev, *dense;
  int32_t* qid;
  if (GLOBAL) {
    double* w = ws + wso;
    keys = reinterpret_cast<uint64_t*>(w);
    ev = w + P2;
    dense = ev + z;
    qid = reinterpret_cast<int32_t*>(dense + z);
  } else {
    keys = reinterpret_cast<uint64_t*>(dyn);
    ev = reinterpret_cast<double*>(dyn) + kCsrLdsEntries;
    dense = ev + kCsrLdsEntries;
    qid = reinterpret_cast<int32_t*>(dense + kCsrLdsEntries);
  }
  // row lengths and offsets within the block (s <= kBT: one row a thread)
  int32_t len = 0;
  if (tid < sb) {
    const int64_t r = R[tid];
    const int64_t a = rp[r];
    len = static_cast<int32_t>(rp[r + 1] - a);
    rowbase[tid] = a;
  }
  scan[tid] = len;
  block_incl_scan(scan, tid);
  if (tid < sb) rowoff[tid] = scan[tid] - len;
  if (tid == 0) rowoff[sb] = scan[kBT - 1];
  __syncthreads();
  if (rowoff[sb] != z) {
    if (tid == 0) atomicOr(err, 4);
    return;
  }
  // sort keys, values in row order
  const int wv = tid >> 6, lane = tid & 63;
  for (int i = wv; i < sb; i += kBT / 64) {
    const int32_t o = rowoff[i], l = rowoff[i + 1] - o;
    const int64_t g = rowbase[i];
    for (int32_t j = lane; j < l; j += 64) {
      const int32_t e = o + j;
      keys[e] = (static_cast<uint64_t>(static_cast<uint32_t>(ci[g + j])) << kKeyBits) | static_cast<uint64_t>(e);
      ev[e] = cv[g + j];
    }
  }
  for (int32_t e = z + tid; e < P2; e += kBT) keys[e] = ~uint64_t{0};
  __syncthreads();
  for (int32_t k = 2; k <= P2; k <<= 1) {
    for (int32_t j = k >> 1; j > 0; j >>= 1) {
      for (int32_t t = tid; t < (P2 >> 1); t += kBT) {
        const int32_t a = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const int32_t c = a + j;
        const uint64_t ka = keys[a], kc = keys[c];
        if ((ka > kc) == ((a & k) == 0)) {
          keys[a] = kc;
          keys[c] = ka;
        }
      }
      __syncthreads();
    }
  }
  // compressed column ids: thread tid owns sorted positions [p0, p1)
  const int32_t C = (z + kBT - 1) / kBT;
  const int32_t p0 = min(z, tid * C), p1 = min(z, p0 + C);
  int32_t heads = 0;
  for (int32_t p = p0; p < p1; ++p)
    heads += (p == 0 || (keys[p] >> kKeyBits) != (keys[p - 1] >> kKeyBits)) ? 1 : 0;
  scan[tid] = heads;
  block_incl_scan(scan, tid);
  const int32_t nuv = scan[kBT - 1];
  int32_t q = scan[tid] - heads - 1;
  for (int32_t p = p0; p < p1; ++p) {
    const uint64_t key = keys[p];
    const int32_t col = static_cast<int32_t>(key >> kKeyBits);
    if (p == 0 || col != static_cast<int32_t>(keys[p - 1] >> kKeyBits)) {
      ++q;
      ar.col[off + q] = col;
      ar.ptr[off + q] = p;
    }
    const int32_t e = static_cast<int32_t>(key & kKeyMask);
    int lo = 0, hi = sb - 1;   // the row holding e: the last i with rowoff[i] <= e
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rowoff[mid] <= e)
        lo = mid;
      else
        hi = mid - 1;
    }
    ar.val[off + p] = ev[e];
    ar.row[off + p] = lo;
    qid[e] = q;
  }
  if (tid == 0) {
    ar.ptr[off + nuv] = z;
    nu[slot_of[blk]] = nuv;
  }
  for (int32_t k = tid; k < nuv; k += kBT) dense[k] = 0.0;
  __syncthreads();
  // Gram, lower part, column i at a time
  for (int i = 0; i < sb; ++i) {
    const int32_t oi = rowoff[i], li = rowoff[i + 1] - oi;
    for (int32_t j = tid; j < li; j += kBT) dense[qid[oi + j]] = ev[oi + j];
    __syncthreads();
    for (int k = i + tid; k < sb; k += kBT) {
      const int32_t ok = rowoff[k], lk = rowoff[k + 1] - ok;
      double g = 0.0;
      for (int32_t j = 0; j < lk; ++j) g = fma(ev[ok + j], dense[qid[ok + j]], g);
      Gb[static_cast<int64_t>(i) * s + k] = g + (k == i ? lambda : 0.0);
    }
    __syncthreads();
    for (int32_t j = tid; j < li; j += kBT) dense[qid[oi + j]] = 0.0;
    __syncthreads();
  }
}

// --------------------------------------------------------------------------
// memo miss, CD++: G = A_SS + lambda I from the rows of S
// --------------------------------------------------------------------------
// The lower part is cleared, then one wave per row i looks each nonzero's
// column up among the (ascending) rows of S and keeps those at k <= i.
__global__ __launch_bounds__(kST) void k_csr_gram_cd(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                     const double* __restrict__ cv, const int32_t* __restrict__ rows,
                                                     const int32_t* __restrict__ lens,
                                                     const int32_t* __restrict__ slot_of, int32_t s, double lambda,
                                                     double* __restrict__ G, int64_t stride) {
  __shared__ int32_t rs[kMaxBlock];
  const int blk = blockIdx.x, tid = threadIdx.x;
  const int sb = lens[blk];
  const int32_t* R = rows + static_cast<int64_t>(blk) * s;
  double* Gb = G + static_cast<int64_t>(slot_of[blk]) * stride;
  for (int i = tid; i < sb; i += kST) rs[i] = R[i];
  for (int32_t e = tid; e < sb * sb; e += kST) {
    const int32_t k = e / sb, i = e - k * sb;
    if (i >= k) Gb[static_cast<int64_t>(k) * s + i] = (i == k) ? lambda : 0.0;
  }
  __syncthreads();
  const int wv = tid >> 6, lane = tid & 63;
  for (int i = wv; i < sb; i += kST / 64) {
    const int64_t r = rs[i];
    const int64_t a = rp[r], e = rp[r + 1];
    for (int64_t kk = a + lane; kk < e; kk += 64) {
      const int32_t c = ci[kk];
      if (c > r) continue;
      int lo = 0, hi = i;   // c among rs[0..i]
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rs[mid] < c)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (rs[lo] == c) Gb[static_cast<int64_t>(lo) * s + i] = cv[kk] + (lo == i ? lambda : 0.0);
    }
  }
}

// --------------------------------------------------------------------------
// a run of steps in one launch of a team
// --------------------------------------------------------------------------
// Phases of a step in workgroup g (layout and protocol in sparse.hpp):
//   1. p_g[i] = A_i[slice] (u + t01 v)[slice]: one thread per block row over
//      the slice's nonzeros of the row (a contiguous range: columns ascend);
//      published, then the r round: r_i = sum_h p_h[i] - b_i, partials added
//      in team order (the same values in every workgroup)
//   2. the workgroup's rows of y = G^{-1} r (a wave per row, lanes over k,
//      the lane sums added by a fixed butterfly); published, then the y round;
//      workgroup 0 keeps the step's bookkeeping from ||r||^2
//   3. back-projection on the slice: one thread per compressed column
//      (Kaczmarz++) or block row (CD++) in the slice, u -= au w, v -= av w
// The exchange buffers alternate between steps (epoch parity): a workgroup
// can be at most one step ahead of the slowest (it needs every workgroup's y
// of the current step to go on), so it never overwrites data still read.
constexpr int kTT = kSparseTeamThreads;

// What a thread loads ahead for one step (none of it depends on x): the
// step's slot, length and arena offset; the thread's block row (row tid: its
// start in the CSR arrays, its b entry and its slice's range, the first
// kRowPre nonzeros);
// G^{-1} entries of the workgroup's first rows of y (rows y0 + wave and
// y0 + wave + 4, lanes over k < 128); and the thread's first compressed
// column (Kaczmarz++: bounds, column, first nonzero) or block row in the slice
// (CD++).
constexpr int kRowPre = 2;
struct TeamPre {
  int32_t q, sb, z;
  int64_t off;
  int64_t base;
  double bi;
  int32_t j0, j1;
  int32_t ci[kRowPre];
  double cv[kRowPre];
  double gi[4];
  int32_t c0, c1;
  int32_t p0, p1, col, crow;
  double cval;
};

template <int KIND>
__device__ __forceinline__ void team_pre_a(const SparseTeamArgs& a, int32_t k, TeamPre& n) {
  const int32_t* in = a.step_info + kSparseStepInts * k;
  n.q = in[0];
  n.sb = in[1];
  n.z = in[2];
  n.off = meta_i64(in + 3);
}

// second level: the thread's row index (kept in base until the row pointer
// arrives) and the slice's column (or row) bounds
template <int KIND>
__device__ __forceinline__ void team_pre_b(const SparseTeamArgs& a, int tid, int g, TeamPre& n) {
  const int32_t* TT = a.team + static_cast<int64_t>(n.q) * a.team_stride;
  const int T1 = a.G + 1;
  n.base = tid < n.sb ? a.rows[static_cast<int64_t>(n.q) * a.s + tid] : -1;
  n.c0 = TT[a.s * T1 + g];
  n.c1 = TT[a.s * T1 + g + 1];
}

// third level: row start and slice range, G^{-1} rows, column bounds (or the
// CD++ row of the slice)
template <int KIND>
__device__ __forceinline__ void team_pre_c(const SparseTeamArgs& a, int tid, int g, TeamPre& n) {
  const int32_t* TT = a.team + static_cast<int64_t>(n.q) * a.team_stride;
  const int T1 = a.G + 1;
  if (n.base >= 0) {
    const int64_t row = n.base;
    n.base = a.rp[row];
    n.bi = a.b[row];
    n.j0 = TT[tid * T1 + g];
    n.j1 = TT[tid * T1 + g + 1];
  } else {
    n.base = 0;
    n.bi = 0.0;
    n.j0 = n.j1 = 0;
  }
  const int lane = tid & 63, wv = tid >> 6;
  const int y0 = (g * n.sb) / a.G, y1 = ((g + 1) * n.sb) / a.G;
  const double* Gb = a.L + static_cast<int64_t>(n.q) * a.slot_stride + static_cast<int64_t>(a.s) * a.s;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int i = y0 + wv + 4 * t;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int kk = lane + 64 * u;
      n.gi[2 * t + u] = (i < y1 && kk < n.sb) ? Gb[static_cast<int64_t>(i) * a.s + kk] : 0.0;
    }
  }
  const int32_t c = n.c0 + tid;
  n.p0 = n.p1 = n.col = 0;
  if (c < n.c1) {
    if (KIND == 0) {
      n.p0 = a.ar.ptr[n.off + c];
      n.p1 = a.ar.ptr[n.off + c + 1];
      n.col = a.ar.col[n.off + c];
    } else {
      n.col = a.rows[static_cast<int64_t>(n.q) * a.s + c];
    }
  }
}

// fourth level: the row's first nonzeros in the slice and the column's first
// nonzero
template <int KIND>
__device__ __forceinline__ void team_pre_d(const SparseTeamArgs& a, int tid, TeamPre& n) {
#pragma unroll
  for (int t = 0; t < kRowPre; ++t) {
    n.ci[t] = 0;
    n.cv[t] = 0.0;
    if (n.j0 + t < n.j1) {
      n.ci[t] = a.ci[n.base + n.j0 + t];
      n.cv[t] = a.cv[n.base + n.j0 + t];
    }
  }
  n.crow = 0;
  n.cval = 0.0;
  if (KIND == 0 && n.c0 + tid < n.c1) {
    n.crow = a.ar.row[n.off + n.p0];
    n.cval = a.ar.val[n.off + n.p0];
  }
}

template <int KIND>
__global__ __launch_bounds__(kTT) void k_sparse_team(SparseTeamArgs a) {
  __shared__ double r[kMaxBlock];
  __shared__ double y[kMaxBlock];
  __shared__ double red[kTT / 64];
  __shared__ DevState st;
  __shared__ int abort_flag;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int g = blockIdx.x, G = a.G, s = a.s, T1 = G + 1;
  if (tid == 0) {
    abort_flag = 0;
    if (g == 0) st = *a.ds;
  }
  // optional phase profile (workgroup 0, thread 0): ticks[p] accumulates the
  // wall-clock time from mark p-1 to mark p
  const bool prof = a.phase_ticks != nullptr && g == 0 && tid == 0;
  uint64_t tick_last = 0, ticks[kFusedPhases];
#pragma unroll
  for (int p = 0; p < kFusedPhases; ++p) ticks[p] = 0;
#define KPP_MARK(p)                   \
  if (prof) {                         \
    const uint64_t now_ = wall_clock64(); \
    ticks[p] += now_ - tick_last;     \
    tick_last = now_;                 \
  }
  TeamPre cur;
  team_pre_a<KIND>(a, 0, cur);
  team_pre_b<KIND>(a, tid, g, cur);
  team_pre_c<KIND>(a, tid, g, cur);
  team_pre_d<KIND>(a, tid, cur);
  __syncthreads();
  if (prof) tick_last = wall_clock64();
  for (int32_t k = 0; k < a.W; ++k) {
    const uint32_t ep = a.epoch + static_cast<uint32_t>(k) + 1u;
    const int32_t q = cur.q, sb = cur.sb;
    const int64_t off = cur.off;
    const double t01 = a.coef[3 * k], au = a.coef[3 * k + 1], av = a.coef[3 * k + 2];
    const int32_t* R = a.rows + static_cast<int64_t>(q) * s;
    const int32_t* TT = a.team + static_cast<int64_t>(q) * a.team_stride;
    double* Pb = a.xr + static_cast<size_t>(ep & 1u) * G * s;
    double* Yb = a.xy + static_cast<size_t>(ep & 1u) * s;
    const bool more = k + 1 < a.W;
    TeamPre nx = cur;
    if (more) team_pre_a<KIND>(a, k + 1, nx);
    // 1. partial r over the slice: the thread's row (prefetched), then rows
    //    past kTT (blocks of more than kTT rows)
    if (tid < sb) {
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < kRowPre; ++t) {
        if (cur.j0 + t < cur.j1) {
          const uint32_t c = static_cast<uint32_t>(cur.ci[t]);
          acc = fma(cur.cv[t], t01 != 0.0 ? fma(t01, a.v[c], a.u[c]) : a.u[c], acc);
        }
      }
      for (int64_t e = cur.base + cur.j0 + kRowPre; e < cur.base + cur.j1; ++e) {
        const uint32_t c = static_cast<uint32_t>(a.ci[e]);
        acc = fma(a.cv[e], t01 != 0.0 ? fma(t01, a.v[c], a.u[c]) : a.u[c], acc);
      }
      r[tid] = acc;
    }
    for (int i = tid + kTT; i < sb; i += kTT) {
      const int64_t base = a.rp[R[i]];
      double acc = 0.0;
      for (int64_t e = base + TT[i * T1 + g]; e < base + TT[i * T1 + g + 1]; ++e) {
        const uint32_t c = static_cast<uint32_t>(a.ci[e]);
        acc = fma(a.cv[e], t01 != 0.0 ? fma(t01, a.v[c], a.u[c]) : a.u[c], acc);
      }
      r[i] = acc;
    }
    __syncthreads();
    KPP_MARK(0)
    if (wv == 0) {
      for (int i = lane; i < sb; i += 64) st_coherent(&Pb[static_cast<size_t>(g) * s + i], r[i]);
      if (lane == 0) st_flag_after_stores(&a.flags[g * kSparseFlagStride], ep);
    }
    if (more) team_pre_b<KIND>(a, tid, g, nx);
    if (tid < G) {
      int64_t spins = 0;
      while (static_cast<int32_t>(ld_flag(&a.flags[tid * kSparseFlagStride]) - ep) < 0) {
        if (++spins > a.spin_limit) {
          atomicOr(a.err, 2);
          abort_flag = 1;
          break;
        }
      }
    }
    __syncthreads();
    KPP_MARK(1)
    if (abort_flag) break;
    // the team's partials of row i in one batch of loads, added in team order
    for (int i = tid; i < sb; i += kTT) {
      double pv[kSparseTeamMax];
#pragma unroll
      for (int h = 0; h < kSparseTeamMax; ++h) pv[h] = h < G ? ld_coherent(&Pb[static_cast<size_t>(h) * s + i]) : 0.0;
      double acc = 0.0;
#pragma unroll
      for (int h = 0; h < kSparseTeamMax; ++h)
        if (h < G) acc += pv[h];
      r[i] = acc - (i == tid ? cur.bi : a.b[R[i]]);
    }
    __syncthreads();
    KPP_MARK(2)
    // 2. this workgroup's rows of y (the first two of each wave from the
    //    prefetched entries)
    const int y0 = (g * sb) / G, y1 = ((g + 1) * sb) / G;
    const double* Gb = a.L + static_cast<int64_t>(q) * a.slot_stride + static_cast<int64_t>(s) * s;
    {
      // rows y0 + wv and y0 + wv + 4 from the prefetched entries, summed over
      // the lanes together (one butterfly for the pair)
      const int i0 = y0 + wv, i1 = i0 + kTT / 64;
      double acc0 = 0.0, acc1 = 0.0;
      const double r0 = lane < sb ? r[lane] : 0.0, r1 = lane + 64 < sb ? r[lane + 64] : 0.0;
      acc0 = fma(cur.gi[1], r1, cur.gi[0] * r0);
      acc1 = fma(cur.gi[3], r1, cur.gi[2] * r0);
      for (int kk = lane + 128; kk < sb; kk += 64) {
        if (i0 < y1) acc0 = fma(Gb[static_cast<int64_t>(i0) * s + kk], r[kk], acc0);
        if (i1 < y1) acc1 = fma(Gb[static_cast<int64_t>(i1) * s + kk], r[kk], acc1);
      }
      double v = fold(acc0, acc1, 32, (lane & 32) != 0);
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) v = fold(v, v, o, false);
      if (lane == 0 && i0 < y1) y[i0] = v;
      if (lane == 32 && i1 < y1) y[i1] = v;
      for (int i = i1 + kTT / 64; i < y1; i += kTT / 64) {   // rows past two a wave
        double acc = 0.0;
        for (int kk = lane; kk < sb; kk += 64) acc = fma(Gb[static_cast<int64_t>(i) * s + kk], r[kk], acc);
        acc = wave_sum(acc);
        if (lane == 0) y[i] = acc;
      }
    }
    if (g == 0) {
      double rr = 0.0;
      for (int i = tid; i < sb; i += kTT) rr = fma(r[i], r[i], rr);
      rr = wave_sum(rr);
      if (lane == 0) red[wv] = rr;
    }
    __syncthreads();
    KPP_MARK(3)
    if (wv == 0) {
      for (int i = y0 + lane; i < y1; i += 64) st_coherent(&Yb[i], y[i]);
      if (lane == 0) st_flag_after_stores(&a.flags[kYFlagOffset + g * kSparseFlagStride], ep);
    }
    if (g == 0 && tid == 0) {
      double rr = 0.0;
      for (int w = 0; w < kTT / 64; ++w) rr += red[w];
      step_state_update(st, rr, a.zeta, a.adaptive);
    }
    if (more) team_pre_c<KIND>(a, tid, g, nx);
    if (tid < G) {
      int64_t spins = 0;
      while (static_cast<int32_t>(ld_flag(&a.flags[kYFlagOffset + tid * kSparseFlagStride]) - ep) < 0) {
        if (++spins > a.spin_limit) {
          atomicOr(a.err, 2);
          abort_flag = 1;
          break;
        }
      }
    }
    __syncthreads();
    KPP_MARK(4)
    if (abort_flag) break;
    for (int i = tid; i < sb; i += kTT) y[i] = ld_coherent(&Yb[i]);
    __syncthreads();
    KPP_MARK(5)
    // 3. back-projection on the slice (the thread's first column or row from
    //    the prefetched entries)
    if (KIND == 0) {
      const int32_t* __restrict__ bptr = a.ar.ptr + off;
      const int32_t* __restrict__ bcol = a.ar.col + off;
      const int32_t* __restrict__ brow = a.ar.row + off;
      const double* __restrict__ bval = a.ar.val + off;
      if (cur.c0 + tid < cur.c1) {
        double w = fma(cur.cval, y[cur.crow], 0.0);
        for (int32_t p = cur.p0 + 1; p < cur.p1; ++p) w = fma(bval[p], y[brow[p]], w);
        const uint32_t j = static_cast<uint32_t>(cur.col);
        a.u[j] = fma(-au, w, a.u[j]);
        a.v[j] = fma(-av, w, a.v[j]);
      }
      for (int32_t c = cur.c0 + tid + kTT; c < cur.c1; c += kTT) {
        const int32_t p0 = bptr[c], p1 = bptr[c + 1];
        double w = 0.0;
        for (int32_t p = p0; p < p1; ++p) w = fma(bval[p], y[brow[p]], w);
        const uint32_t j = static_cast<uint32_t>(bcol[c]);
        a.u[j] = fma(-au, w, a.u[j]);
        a.v[j] = fma(-av, w, a.v[j]);
      }
    } else {
      if (cur.c0 + tid < cur.c1) {
        const uint32_t j = static_cast<uint32_t>(cur.col);
        const double yi = y[cur.c0 + tid];
        a.u[j] = fma(-au, yi, a.u[j]);
        a.v[j] = fma(-av, yi, a.v[j]);
      }
      for (int i = cur.c0 + tid + kTT; i < cur.c1; i += kTT) {
        const uint32_t j = static_cast<uint32_t>(R[i]);
        a.u[j] = fma(-au, y[i], a.u[j]);
        a.v[j] = fma(-av, y[i], a.v[j]);
      }
    }
    if (more) team_pre_d<KIND>(a, tid, nx);
    __syncthreads();
    KPP_MARK(6)
    cur = nx;
  }
#undef KPP_MARK
  if (prof) {
#pragma unroll
    for (int p = 0; p < kFusedPhases; ++p)
      atomicAdd(reinterpret_cast<unsigned long long*>(&a.phase_ticks[p]), static_cast<unsigned long long>(ticks[p]));
  }
  if (g == 0 && tid == 0) *a.ds = st;
}

// Team tables of new blocks: one workgroup per block.  Row i's slice starts
// by binary search of each slice's first column among the row's (ascending)
// columns; the slice boundaries among the compressed columns (Kaczmarz++) or
// the block rows (CD++, ascending) likewise.
__global__ __launch_bounds__(kST) void k_csr_team_tables(int32_t kind, const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         const int32_t* __restrict__ rows,
                                                         const int32_t* __restrict__ lens,
                                                         const int32_t* __restrict__ slot_of,
                                                         const int32_t* __restrict__ meta, CscArena ar,
                                                         const int32_t* __restrict__ nu, int32_t s, int64_t n,
                                                         int32_t G, int32_t* __restrict__ team) {
  const int blk = blockIdx.x, tid = threadIdx.x;
  const int sb = lens[blk];
  const int32_t* R = rows + static_cast<int64_t>(blk) * s;
  const int T1 = G + 1;
  int32_t* TT = team + static_cast<int64_t>(slot_of[blk]) * csr_team_stride(s, G);
  for (int e = tid; e < sb * T1; e += kST) {
    const int i = e / T1, g = e - i * T1;
    const int64_t a0 = rp[R[i]], a1 = rp[R[i] + 1];
    int64_t lo = a0, hi = a1;   // first nonzero of row i with column >= the slice's first column
    if (g == G) {
      lo = a1;
    } else if (g > 0) {
      const int64_t c = csr_slice_lo(n, G, g);
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ci[mid] < c)
          lo = mid + 1;
        else
          hi = mid;
      }
    }
    TT[e] = static_cast<int32_t>(lo - a0);
  }
  for (int g = tid; g < T1; g += kST) {
    int32_t lo = 0, hi;
    const int64_t c = g == G ? n : csr_slice_lo(n, G, g);
    if (kind == 0) {
      const int64_t off = meta_i64(meta + static_cast<int64_t>(kCsrMetaInts) * blk);
      const int32_t* col = ar.col + off;
      hi = nu[slot_of[blk]];
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (col[mid] < c)
          lo = mid + 1;
        else
          hi = mid;
      }
    } else {
      hi = sb;
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (R[mid] < c)
          lo = mid + 1;
        else
          hi = mid;
      }
    }
    TT[s * T1 + g] = lo;
  }
}

// --------------------------------------------------------------------------
// true residual ||A x - b||^2
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kST) void k_csr_resid_part(const int64_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci,
                                                        const double* __restrict__ cv, const double* __restrict__ b,
                                                        int64_t m, const double* __restrict__ x,
                                                        double* __restrict__ part) {
  __shared__ double red[kST / 64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r0 = (static_cast<int64_t>(blockIdx.x) * (kST / 64) + wv) * kRowsPerWave;
  double acc = 0.0;
  for (int t = 0; t < kRowsPerWave; ++t) {
    const int64_t r = r0 + t;
    if (r >= m) break;
    const int64_t a = rp[r], e = rp[r + 1];
    double d = 0.0;
    for (int64_t k = a + lane; k < e; k += 64) d = fma(cv[k], x[ci[k]], d);
    d = wave_sum(d) - b[r];
    acc = fma(d, d, acc);
  }
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(kST) void k_sum_parts(const double* __restrict__ part, int64_t np,
                                                   double* __restrict__ out) {
  __shared__ double red[kST];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += kST) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kST / 2; o > 0; o >>= 1) {
    if (static_cast<int>(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

unsigned grid_of(int64_t work, int per) { return static_cast<unsigned>((work + per - 1) / per); }

}  // namespace

void launch_csr_check(const int64_t* rp, const int32_t* ci, const double* cv, const double* b, int64_t m, int64_t n,
                      int64_t nnz, int32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_csr_check, dim3(grid_of(m, kST)), dim3(kST), 0, st, rp, ci, cv, b, m, n, nnz, flag);
}

void launch_csr_rows_dot(const int64_t* rp, const int32_t* ci, const double* cv, const int32_t* rows, int32_t sb,
                         const double* u, const double* v, double t01, double* out, hipStream_t st) {
  if (sb <= 0) return;
  hipLaunchKernelGGL(k_csr_rows_dot, dim3(grid_of(sb, kST / 64)), dim3(kST), 0, st, rp, ci, cv, rows, sb, u, v, t01,
                     out);
}

void launch_csc_apply(const CscArena& ar, int64_t off, int32_t z, const int32_t* nu, int32_t q, const double* y,
                      int32_t sb, double au, double av, double* u, double* v, hipStream_t st) {
  if (z <= 0) return;
  hipLaunchKernelGGL(k_csc_apply, dim3(grid_of(z, kST)), dim3(kST), 0, st, ar.val + off, ar.row + off,
                     ar.col + off, ar.ptr + off, nu, q, y, sb, au, av, u, v);
}

void launch_rows_apply(const int32_t* rows, int32_t sb, const double* y, double au, double av, double* u, double* v,
                       hipStream_t st) {
  if (sb <= 0) return;
  hipLaunchKernelGGL(k_rows_apply, dim3(grid_of(sb, kST)), dim3(kST), 0, st, rows, sb, y, au, av, u, v);
}

void launch_lazy_fold(double* u, double* v, int64_t n, double t01, double t11, hipStream_t st) {
  const unsigned g = static_cast<unsigned>(std::min<int64_t>(grid_of(n, kST), 8192));
  hipLaunchKernelGGL(k_lazy_fold, dim3(g), dim3(kST), 0, st, u, v, n, t01, t11);
}

void launch_csr_block_build(const int64_t* rp, const int32_t* ci, const double* cv, const int32_t* rows,
                            const int32_t* lens, const int32_t* slot_of, const int32_t* meta, int32_t nb, int32_t s,
                            double lambda, double* G, int64_t stride, const CscArena& ar, int32_t* nu, double* ws,
                            bool any_lds, bool any_global, int32_t* err, hipStream_t st) {
  if (nb <= 0) return;
  if (any_lds) {
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_csr_block_build<false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kBuildLds));
      attr_set = true;
    }
    hipLaunchKernelGGL(k_csr_block_build<false>, dim3(nb), dim3(kBT), kBuildLds, st, rp, ci, cv, rows, lens, slot_of,
                       meta, s, lambda, G, stride, ar, nu, ws, err);
  }
  if (any_global)
    hipLaunchKernelGGL(k_csr_block_build<true>, dim3(nb), dim3(kBT), 0, st, rp, ci, cv, rows, lens, slot_of, meta, s,
                       lambda, G, stride, ar, nu, ws, err);
}

void launch_csr_gram_cd(const int64_t* rp, const int32_t* ci, const double* cv, const int32_t* rows,
                        const int32_t* lens, const int32_t* slot_of, int32_t nb, int32_t s, double lambda, double* G,
                        int64_t stride, hipStream_t st) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_csr_gram_cd, dim3(nb), dim3(kST), 0, st, rp, ci, cv, rows, lens, slot_of, s, lambda, G,
                     stride);
}

void launch_sparse_team(int32_t kind, const SparseTeamArgs& a, hipStream_t st) {
  if (a.W <= 0) return;
  if (kind == 0)
    hipLaunchKernelGGL(k_sparse_team<0>, dim3(a.G), dim3(kTT), 0, st, a);
  else
    hipLaunchKernelGGL(k_sparse_team<1>, dim3(a.G), dim3(kTT), 0, st, a);
}

void launch_csr_team_tables(int32_t kind, const int64_t* rp, const int32_t* ci, const int32_t* rows,
                            const int32_t* lens, const int32_t* slot_of, const int32_t* meta, const CscArena& ar,
                            const int32_t* nu, int32_t nb, int32_t s, int64_t n, int32_t G, int32_t* team,
                            hipStream_t st) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_csr_team_tables, dim3(nb), dim3(kST), 0, st, kind, rp, ci, rows, lens, slot_of, meta, ar, nu,
                     s, n, G, team);
}

void launch_csr_residual_sq(const int64_t* rp, const int32_t* ci, const double* cv, const double* b, int64_t m,
                            const double* x, double* part, double* out, hipStream_t st) {
  const int64_t np = csr_residual_parts(m);
  hipLaunchKernelGGL(k_csr_resid_part, dim3(static_cast<unsigned>(np)), dim3(kST), 0, st, rp, ci, cv, b, m, x, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kST), 0, st, part, np, out);
}

}  // namespace kpp
