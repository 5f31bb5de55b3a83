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
#include "sparse.hpp"

namespace kpp {
namespace {

constexpr int kST = 256;   // threads of the step kernels (4 waves)
constexpr int kBT = 512;   // threads of the block-build kernel (8 waves)
constexpr int kKeyBits = 20;
constexpr uint64_t kKeyMask = (uint64_t{1} << kKeyBits) - 1;
constexpr int kRowsPerWave = 8;   // rows a wave sums in the true-residual kernel
static_assert((kST / 64) * kRowsPerWave == kCsrResidRowsPerGroup, "residual partial layout");
constexpr size_t kBuildLds = static_cast<size_t>(kCsrLdsEntries) * (3 * sizeof(double) + sizeof(int32_t));

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

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

void launch_csr_residual_sq(const int64_t* rp, const int32_t* ci, const double* cv, const double* b, int64_t m,
                            const double* x, double* part, double* out, hipStream_t st) {
  const int64_t np = csr_residual_parts(m);
  hipLaunchKernelGGL(k_csr_resid_part, dim3(static_cast<unsigned>(np)), dim3(kST), 0, st, rp, ci, cv, b, m, x, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kST), 0, st, part, np, out);
}

}  // namespace kpp
