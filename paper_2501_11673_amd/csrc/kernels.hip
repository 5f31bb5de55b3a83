// HIP kernels (gfx950) of the block step: one launch per phase.
//
//   block gemv        r = A_S x - b_S                    (Algorithm 5 / 2: "r_t <- A_S x_t - b_S")
//   block project     y = (L L^T)^{-1} r, window sums, checkpoint (Section 5.4)
//   update            m <- c (m - w), x <- x - w + eta m  (eq. (momentum)) with
//                     w = A_S^T y (eq. (bk)) or I_S^T y (eq. (cd-update))
//   gram / cholesky   memo miss: G = A_S A_S^T + lam I or A_SS + lam I, L = chol(G)
//   residual          ||A x - b||^2 (eq. (residual-error))
//
// Every reduction runs in a fixed order so that a run is bitwise repeatable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels.hpp"
#include "step_state.hpp"
#include "lsqr.hpp"
#include "multi.hpp"

namespace kpp {
namespace {

constexpr int kT = 256;  // threads per workgroup (4 waves of 64)

// Sum over the 256 threads of a workgroup; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
  return r;
}


// --------------------------------------------------------------------------
// r-partials: grid (P, sb); workgroup (p, i) sums columns [p*chunk, (p+1)*chunk)
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kT) void k_block_gemv_partial(
    const double* __restrict__ A, int64_t lda, int64_t n, const int32_t* __restrict__ rows,
    const double* __restrict__ x, double* __restrict__ rpart, int32_t P, int64_t chunk) {
  __shared__ double red[4];
  const int i = blockIdx.y;
  const int p = blockIdx.x;
  const double* Ai = A + static_cast<int64_t>(rows[i]) * lda;
  const int64_t j0 = static_cast<int64_t>(p) * chunk;
  const int64_t j1 = min(n, j0 + chunk);
  double acc = 0.0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += kT) acc = fma(Ai[j], x[j], acc);
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) rpart[static_cast<int64_t>(i) * P + p] = acc;
}

// --------------------------------------------------------------------------
// projection through the memoized inverse and checkpoint bookkeeping: one workgroup
// --------------------------------------------------------------------------
__device__ void step_state(DevState* ds, double rr, int32_t zeta, int32_t adaptive) {
  DevState s = *ds;
  step_state_update(s, rr, zeta, adaptive);
  *ds = s;
}

__global__ __launch_bounds__(kT) void k_block_project(
    const double* __restrict__ rpart, int32_t P, const double* __restrict__ b,
    const int32_t* __restrict__ rows, int32_t sb, const double* __restrict__ Ginv, int32_t ldl,
    double* __restrict__ y, DevState* __restrict__ ds, int32_t zeta, int32_t adaptive) {
  __shared__ double r[kMaxBlock];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  double part = 0.0;
  for (int i = tid; i < sb; i += kT) {
    const double* rp = rpart + static_cast<int64_t>(i) * P;
    double acc = 0.0;
    for (int p = 0; p < P; ++p) acc += rp[p];
    const double ri = acc - b[rows[i]];
    r[i] = ri;
    part = fma(ri, ri, part);
  }
  const double rr = block_sum(part, red);
  __syncthreads();
  // y = G^{-1} r with the memoized inverse (symmetric: column i = row i)
  for (int i = tid; i < sb; i += kT) {
    double acc = 0.0;
    for (int k = 0; k < sb; ++k) acc = fma(Ginv[static_cast<int64_t>(k) * ldl + i], r[k], acc);
    y[i] = acc;
  }
  if (tid == 0) step_state(ds, rr, zeta, adaptive);
}

// The same for large blocks: y's rows split over workgroups of 16 (thread
// (i mod 16, kk) sums k = kk, kk + 16, ...; the 16 partial sums of a row are
// added in a fixed order).  Every workgroup forms r the same way; workgroup 0
// alone does the step's bookkeeping.
constexpr int kProjRows = 16;
__global__ __launch_bounds__(kT) void k_block_project_rows(
    const double* __restrict__ rpart, int32_t P, const double* __restrict__ b,
    const int32_t* __restrict__ rows, int32_t sb, const double* __restrict__ Ginv, int32_t ldl,
    double* __restrict__ y, DevState* __restrict__ ds, int32_t zeta, int32_t adaptive) {
  __shared__ double r[kMaxBlock];
  __shared__ double red[4];
  __shared__ double pr[kT / kProjRows][kProjRows + 1];
  const int tid = threadIdx.x;
  double part = 0.0;
  for (int i = tid; i < sb; i += kT) {
    const double* rp = rpart + static_cast<int64_t>(i) * P;
    double acc = 0.0;
    for (int p = 0; p < P; ++p) acc += rp[p];
    const double ri = acc - b[rows[i]];
    r[i] = ri;
    part = fma(ri, ri, part);
  }
  const double rr = block_sum(part, red);
  __syncthreads();
  const int ri = tid & (kProjRows - 1), kk = tid / kProjRows;
  const int i = blockIdx.x * kProjRows + ri;
  double acc = 0.0;
  if (i < sb)
    for (int k = kk; k < sb; k += kT / kProjRows) acc = fma(Ginv[static_cast<int64_t>(k) * ldl + i], r[k], acc);
  pr[kk][ri] = acc;
  __syncthreads();
  if (tid < kProjRows && i < sb) {
    double v = 0.0;
    for (int q = 0; q < kT / kProjRows; ++q) v += pr[q][tid];
    y[i] = v;
  }
  if (blockIdx.x == 0 && tid == 0) step_state(ds, rr, zeta, adaptive);
}

// --------------------------------------------------------------------------
// momentum + iterate update over all n coordinates
// --------------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(kT) void k_update(const double* __restrict__ A, int64_t lda,
                                               int64_t n, const int32_t* __restrict__ rows,
                                               int32_t sb, const double* __restrict__ y,
                                               const DevState* __restrict__ ds, double eta,
                                               double* __restrict__ x, double* __restrict__ mom) {
  __shared__ double ys[kMaxBlock];
  __shared__ int32_t rs[kMaxBlock];
  for (int i = threadIdx.x; i < sb; i += kT) {
    ys[i] = y[i];
    rs[i] = rows[i];
  }
  __syncthreads();
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
  if (j >= n) return;
  double w = 0.0;
  if (KIND == 0) {
    for (int i = 0; i < sb; ++i) w = fma(A[static_cast<int64_t>(rs[i]) * lda + j], ys[i], w);
  } else {
    int lo = 0, hi = sb;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (rs[mid] < j)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo < sb && rs[lo] == j) w = ys[lo];
  }
  const double c = ds->c;
  const double mn = __dmul_rn(c, __dsub_rn(mom[j], w));
  mom[j] = mn;
  x[j] = __dadd_rn(__dsub_rn(x[j], w), __dmul_rn(eta, mn));
}

// --------------------------------------------------------------------------
// several right-hand sides: the same three phases, every A_S element used for
// all k columns (registers hold k sums per thread)
// --------------------------------------------------------------------------
// R = A_S X on the matrix cores (FP64 16x16x4): workgroup (p, ti) forms the
// 16-row tile ti of R over column chunk p of A, each wave a quarter of the
// chunk; the four wave tiles are summed in a fixed order.  Operands of the
// MFMA: lane l supplies A[row ti 16 + l % 16][k + l / 16] and
// X[k + l / 16][c0 + l % 16]; register r of lane l returns R[l / 16 + 4 r][c0 + l % 16]
// (the layout the Gram kernels use).  NT tiles of 16 right-hand sides.
typedef double v4d_m __attribute__((ext_vector_type(4)));
template <int NT>
__global__ __launch_bounds__(kT) void k_block_gemm_mfma(const double* __restrict__ A, int64_t lda, int64_t n,
                                                        const int32_t* __restrict__ rows, int32_t sb,
                                                        const double* __restrict__ X, int64_t ldx, int32_t k,
                                                        double* __restrict__ rpart, int32_t P) {
  __shared__ double red[4][NT][4][64];
  const int p = blockIdx.x, i0 = blockIdx.y * 16;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const bool rok = i0 + li < sb;
  const double* Arow = A + static_cast<int64_t>(rows[rok ? i0 + li : 0]) * lda;
  const int64_t kb = static_cast<int64_t>(p) * kGemmChunk + w * (kGemmChunk / 4);
  const int64_t ke = min(n, kb + kGemmChunk / 4);
  v4d_m acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = v4d_m{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int64_t k0 = kb; k0 < ke; k0 += 4) {
    const int64_t kk = k0 + lk;
    const bool kok = kk < ke;
    const double a = (rok && kok) ? Arow[kk] : 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int c = 16 * t + li;
      const double b = (kok && c < k) ? X[kk * ldx + c] : 0.0;
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) red[w][t][r][lane] = acc[t][r];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double v = (red[0][t][r][lane] + red[1][t][r][lane]) + (red[2][t][r][lane] + red[3][t][r][lane]);
        const int i = i0 + lk + 4 * r, c = 16 * t + li;
        if (i < sb && c < k) rpart[(static_cast<int64_t>(i) * P + p) * k + c] = v;
      }
  }
}

__global__ __launch_bounds__(kT) void k_block_project_multi(
    const double* __restrict__ rpart, int32_t P, int32_t k, const double* __restrict__ B, int64_t ldb,
    const int32_t* __restrict__ rows, int32_t sb, const double* __restrict__ Ginv, int32_t ldl,
    double* __restrict__ Y, DevState* __restrict__ ds, const int32_t* __restrict__ frozen, int32_t zeta,
    int32_t adaptive) {
  __shared__ double r[kMaxBlock];
  __shared__ double red[4];
  const int c = blockIdx.x;
  if (frozen[c]) return;   // uniform over the workgroup
  const int tid = threadIdx.x;
  double part = 0.0;
  for (int i = tid; i < sb; i += kT) {
    double acc = 0.0;
    for (int p = 0; p < P; ++p) acc += rpart[(static_cast<int64_t>(i) * P + p) * k + c];
    const double ri = acc - B[static_cast<int64_t>(rows[i]) * ldb + c];
    r[i] = ri;
    part = fma(ri, ri, part);
  }
  const double rr = block_sum(part, red);
  __syncthreads();
  for (int i = tid; i < sb; i += kT) {
    double acc = 0.0;
    for (int q = 0; q < sb; ++q) acc = fma(Ginv[static_cast<int64_t>(q) * ldl + i], r[q], acc);
    Y[static_cast<int64_t>(c) * ldl + i] = acc;
  }
  if (tid == 0) step_state(ds + c, rr, zeta, adaptive);
}

template <int KIND, int KM>
__global__ __launch_bounds__(kT) void k_update_multi(const double* __restrict__ A, int64_t lda, int64_t n,
                                                     const int32_t* __restrict__ rows, int32_t sb,
                                                     const double* __restrict__ Y, int32_t s, int32_t k,
                                                     const DevState* __restrict__ ds,
                                                     const int32_t* __restrict__ frozen, double eta,
                                                     double* __restrict__ X, int64_t ldx, double* __restrict__ M) {
  __shared__ int32_t rs[kMaxBlock];
  __shared__ double cc[kMaxRhs];
  __shared__ int32_t fz[kMaxRhs];
  for (int i = threadIdx.x; i < sb; i += kT) rs[i] = rows[i];
  if (threadIdx.x < k) {
    cc[threadIdx.x] = ds[threadIdx.x].c;
    fz[threadIdx.x] = frozen[threadIdx.x];
  }
  __syncthreads();
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
  if (j >= n) return;
  double w[KM];
#pragma unroll
  for (int c = 0; c < KM; ++c) w[c] = 0.0;
  if (KIND == 0) {
    for (int i = 0; i < sb; ++i) {
      const double a = A[static_cast<int64_t>(rs[i]) * lda + j];
#pragma unroll
      for (int c = 0; c < KM; ++c)
        if (c < k) w[c] = fma(a, Y[static_cast<int64_t>(c) * s + i], w[c]);
    }
  } else {
    int lo = 0, hi = sb;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (rs[mid] < j)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo < sb && rs[lo] == j) {
#pragma unroll
      for (int c = 0; c < KM; ++c)
        if (c < k) w[c] = Y[static_cast<int64_t>(c) * s + lo];
    }
  }
  double* xr = X + j * ldx;
  double* mr = M + j * k;
#pragma unroll
  for (int c = 0; c < KM; ++c) {
    if (c < k && !fz[c]) {
      const double mn = __dmul_rn(cc[c], __dsub_rn(mr[c], w[c]));
      mr[c] = mn;
      xr[c] = __dadd_rn(__dsub_rn(xr[c], w[c]), __dmul_rn(eta, mn));
    }
  }
}

// CD++ update with one thread per (coordinate j, right-hand side c): w is
// y_c at j's position in the block, or 0
__global__ __launch_bounds__(kT) void k_update_multi_cd(int64_t n, const int32_t* __restrict__ rows, int32_t sb,
                                                        const double* __restrict__ Y, int32_t s, int32_t k,
                                                        const DevState* __restrict__ ds,
                                                        const int32_t* __restrict__ frozen, double eta,
                                                        double* __restrict__ X, int64_t ldx, double* __restrict__ M) {
  __shared__ int32_t rs[kMaxBlock];
  for (int i = threadIdx.x; i < sb; i += kT) rs[i] = rows[i];
  __syncthreads();
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
  if (e >= n * k) return;
  const int64_t j = e / k;
  const int c = static_cast<int>(e - j * k);
  if (frozen[c]) return;
  int lo = 0, hi = sb;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (rs[mid] < j)
      lo = mid + 1;
    else
      hi = mid;
  }
  const double w = (lo < sb && rs[lo] == j) ? Y[static_cast<int64_t>(c) * s + lo] : 0.0;
  const double mn = __dmul_rn(ds[c].c, __dsub_rn(M[e], w));
  M[e] = mn;
  double* xe = X + j * ldx + c;
  *xe = __dadd_rn(__dsub_rn(*xe, w), __dmul_rn(eta, mn));
}

__global__ __launch_bounds__(kT) void k_column(const double* __restrict__ X, int64_t ldx, int64_t n, int32_t c,
                                               double* __restrict__ out) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
  if (j < n) out[j] = X[j * ldx + c];
}

// --------------------------------------------------------------------------
// memo miss: regularized Grams (lower part, column-major slots)
// --------------------------------------------------------------------------
template <typename TA>
__global__ __launch_bounds__(kT) void k_gram_cd(const TA* __restrict__ A, int64_t lda,
                                                const int32_t* __restrict__ rows,
                                                const int32_t* __restrict__ lens, int32_t s,
                                                double lambda, double* __restrict__ G, int64_t stride,
                                                const int32_t* __restrict__ slot_of,
                                                const int32_t* __restrict__ only) {
  const int blk = blockIdx.x;
  if (only && !only[blk]) return;
  const int sb = lens[blk];
  const int32_t* R = rows + static_cast<int64_t>(blk) * s;
  double* Gb = G + static_cast<int64_t>(slot_of[blk]) * stride;
  for (int e = threadIdx.x; e < sb * sb; e += kT) {
    const int k = e / sb, i = e - k * sb;
    if (i >= k) Gb[static_cast<int64_t>(k) * s + i] = static_cast<double>(A[static_cast<int64_t>(R[i]) * lda + R[k]]) + (i == k ? lambda : 0.0);
  }
}

// --------------------------------------------------------------------------
// memo miss: Cholesky, one workgroup per block (right-looking, column by column)
// --------------------------------------------------------------------------
// Low-precision pass: a block whose Frobenius condition number
// ||G||_F ||G^{-1}||_F (at least kappa_2(G), at most s kappa_2(G)) exceeds
// chk.kappa_max is marked for the FP64 Gram and factor.
__device__ __forceinline__ void flag_ill_conditioned(const FactorCheck& chk, int blk, double norm_g2,
                                                     double norm_gi2) {
  const double kf = sqrt(norm_g2 * norm_gi2);
  if (!(kf <= chk.kappa_max)) {
    chk.flag[blk] = 1;
    atomicAdd(chk.counter, 1);
  }
}

template <bool IN_LDS>
__global__ __launch_bounds__(kT) void k_cholesky(double* __restrict__ G, int32_t s, int64_t stride,
                                                 const int32_t* __restrict__ lens,
                                                 const int32_t* __restrict__ slot_of,
                                                 int32_t* __restrict__ err, FactorCheck chk) {
  extern __shared__ double lds[];
  const int blk = blockIdx.x;
  if (chk.only && !chk.only[blk]) return;
  const int sb = lens[blk];
  double* Gb = G + static_cast<int64_t>(slot_of[blk]) * stride;
  double* M;
  int ld;
  if (IN_LDS) {
    M = lds;
    ld = sb;
    for (int e = threadIdx.x; e < sb * sb; e += kT) {
      const int k = e / sb, i = e - k * sb;
      M[k * sb + i] = (i >= k) ? Gb[static_cast<int64_t>(k) * s + i] : 0.0;
    }
  } else {
    M = Gb;
    ld = s;
  }
  if (chk.flag) {
    // ||G||_F^2 of the symmetric Gram, kept for the condition test made once
    // G^{-1} exists: in the last entry of the inverse's region, which is
    // neither read nor written before the inverse is stored
    __shared__ double red4[4];
    double acc = 0.0;
    for (int e = threadIdx.x; e < sb * sb; e += kT) {
      const int k = e / sb, i = e - k * sb;
      if (i >= k) {
        const double v = Gb[static_cast<int64_t>(k) * s + i];
        acc += (i == k ? 1.0 : 2.0) * v * v;
      }
    }
    acc = block_sum(acc, red4);
    if (threadIdx.x == 0) Gb[2 * static_cast<int64_t>(s) * s - 1] = acc;
  }
  int bad = 0;
  for (int j = 0; j < sb; ++j) {
    __syncthreads();
    double d = M[static_cast<int64_t>(j) * ld + j];
    if (!(d > 0.0)) bad = 1;
    d = sqrt(d);
    for (int i = j + 1 + threadIdx.x; i < sb; i += kT) M[static_cast<int64_t>(j) * ld + i] /= d;
    __syncthreads();
    if (threadIdx.x == 0) M[static_cast<int64_t>(j) * ld + j] = d;
    // trailing update, one row per thread: M(i, k) -= L(i, j) L(k, j), j < k <= i
    for (int i = j + 1 + threadIdx.x; i < sb; i += kT) {
      const double lij = M[static_cast<int64_t>(j) * ld + i];
      for (int k = j + 1; k <= i; ++k)
        M[static_cast<int64_t>(k) * ld + i] = fma(-lij, M[static_cast<int64_t>(j) * ld + k], M[static_cast<int64_t>(k) * ld + i]);
    }
  }
  __shared__ int bad_any;
  if (threadIdx.x == 0) bad_any = 0;
  __syncthreads();
  if (bad) atomicOr(&bad_any, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    double lo = 1.0 / 0.0, hi = 0.0;
    for (int i = 0; i < sb; ++i) {
      const double d = M[static_cast<int64_t>(i) * ld + i];
      lo = fmin(lo, d);
      hi = fmax(hi, d);
    }
    const double ratio = hi / lo;
    const bool ill = !(ratio * ratio <= chk.kappa_max);
    if (chk.flag) {
      const int f = (bad_any || ill) ? 1 : 0;
      chk.flag[blk] = f;
      if (f) atomicAdd(chk.counter, 1);
    } else if (bad_any) {
      atomicOr(err, 1);
    }
  }
  // write back L with zero strict upper triangle and zero padding
  for (int e = threadIdx.x; e < s * s; e += kT) {
    const int k = e / s, i = e - k * s;
    double v = 0.0;
    if (i < sb && k < sb && i >= k) v = IN_LDS ? M[k * sb + i] : Gb[static_cast<int64_t>(k) * s + i];
    if (IN_LDS || !(i < sb && k < sb && i >= k)) Gb[static_cast<int64_t>(k) * s + i] = v;
  }
}

// --------------------------------------------------------------------------
// ||A x - b||^2: one wave per row, 4 rows per workgroup; then a fixed-order sum
// --------------------------------------------------------------------------
// sum_j A_i[j] x[j] over this lane's entries j = lane, lane + 64, ... in that
// order (one FMA chain), with eight entries of each operand in flight
__device__ __forceinline__ double row_dot_lane(const double* __restrict__ Ai, const double* __restrict__ x, int64_t n,
                                               int lane) {
  double acc = 0.0;
  int64_t j = lane;
  for (; j + 7 * 64 < n; j += 8 * 64) {
    double a[8], v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = Ai[j + 64 * u];
      v[u] = x[j + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = fma(a[u], v[u], acc);
  }
  for (; j < n; j += 64) acc = fma(Ai[j], x[j], acc);
  return acc;
}

__global__ __launch_bounds__(kT) void k_residual_rows(const double* __restrict__ A, int64_t lda,
                                                      int64_t m, int64_t n,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ b,
                                                      double* __restrict__ rowsq) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= m) return;
  double acc = row_dot_lane(A + i * lda, x, n, lane);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) {
    const double r = acc - b[i];
    rowsq[i] = r * r;
  }
}

__global__ __launch_bounds__(kT) void k_sum(const double* __restrict__ v, int64_t len,
                                            double* __restrict__ out) {
  __shared__ double red[4];
  // thread t adds v[t], v[t + kT], ... in order, eight loads in flight
  double acc = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 7 * kT < len; i += 8 * kT) {
    double w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) w[u] = v[i + static_cast<int64_t>(kT) * u];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += w[u];
  }
  for (; i < len; i += kT) acc += v[i];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) *out = acc;
}

__global__ __launch_bounds__(kT) void k_check_finite(const double* __restrict__ A, int64_t lda,
                                                     int64_t m, int64_t n,
                                                     const double* __restrict__ b,
                                                     int32_t* __restrict__ flag) {
  const int64_t i = blockIdx.x;
  int bad = 0;
  for (int64_t j = threadIdx.x; j < n; j += kT) bad |= !isfinite(A[i * lda + j]);
  if (threadIdx.x == 0) bad |= !isfinite(b[i]);
  if (bad) atomicOr(flag, 1);
  (void)m;
}

__global__ __launch_bounds__(kT) void k_convert_f32(const double* __restrict__ A, int64_t lda, int64_t m,
                                                    int64_t n, float* __restrict__ out) {
  const int64_t total = m * n;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * kT) {
    const int64_t i = e / n, j = e - i * n;
    out[e] = static_cast<float>(A[i * lda + j]);
  }
}

__global__ __launch_bounds__(kT) void k_convert_bf16(const double* __restrict__ A, int64_t lda, int64_t m,
                                                     int64_t n, uint16_t* __restrict__ out) {
  const int64_t total = m * n;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * kT) {
    const int64_t i = e / n, j = e - i * n;
    const uint32_t f = __float_as_uint(static_cast<float>(A[i * lda + j]));
    out[e] = static_cast<uint16_t>((f + 0x7fffu + ((f >> 16) & 1u)) >> 16);   // A is finite
  }
}

// r = b - A x, one wave per row
__global__ __launch_bounds__(kT) void k_residual_vec(const double* __restrict__ A, int64_t lda, int64_t m,
                                                     int64_t n, const double* __restrict__ x,
                                                     const double* __restrict__ b, double* __restrict__ r,
                                                     double* __restrict__ rowsq) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= m) return;
  double acc = row_dot_lane(A + i * lda, x, n, lane);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) {
    const double ri = b[i] - acc;
    r[i] = ri;
    rowsq[i] = ri * ri;
  }
}

__global__ __launch_bounds__(kT) void k_axpy1(double* __restrict__ x, const double* __restrict__ d, int64_t n) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
  if (j < n) x[j] += d[j];
}

// A run's starting state (rho = rho0, c from rho0, the stop threshold), its
// error flag cleared and its momentum zeroed, in one launch.
__global__ __launch_bounds__(kT) void k_state_init(DevState* __restrict__ ds, double rho0, double thr,
                                                   int32_t* __restrict__ err, double* __restrict__ mom, int64_t n) {
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
  for (int64_t i = i0; i < n; i += static_cast<int64_t>(gridDim.x) * kT) mom[i] = 0.0;
  if (i0 == 0) {
    DevState s{};
    s.rho = rho0;
    s.c = (1.0 - rho0) / (1.0 + rho0);
    s.thr = thr;
    s.rho_before = rho0;
    *ds = s;
    *err = 0;
  }
}

// Up to three vectors zeroed in one launch (length 0 skips one).
__global__ __launch_bounds__(kT) void k_zero3(double* __restrict__ a, int64_t na, double* __restrict__ b, int64_t nb,
                                              double* __restrict__ c, int64_t nc) {
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x, step = static_cast<int64_t>(gridDim.x) * kT;
  for (int64_t i = i0; i < na; i += step) a[i] = 0.0;
  for (int64_t i = i0; i < nb; i += step) b[i] = 0.0;
  for (int64_t i = i0; i < nc; i += step) c[i] = 0.0;
}


// --------------------------------------------------------------------------
// memo miss, after the factor: G^{-1} = L^{-T} L^{-1} of the block (stored
// after L in the slot, full symmetric, row = column).  L^{-1} comes from an
// in-place triangular inversion (column j from the right: the inverse's column
// j is -(1/L_jj) times the already inverted trailing triangle applied to
// L's column j below the diagonal); then G^{-1}(i, k) = sum_{r >= max(i,k)}
// L^{-1}(r, i) L^{-1}(r, k).  Blocks up to kLdsCholMax rows work in LDS
// (leading dimension sb + 1 against bank conflicts), larger ones in the
// slot's scratch third.  One workgroup per slot.
// --------------------------------------------------------------------------
// L^{-T} column-major (entry (i, k) = L^{-1}(k, i) at k * s + i) in the slot's
// last third, from L^{-1} column-major in its second third
__device__ void write_linv_transpose(double* base, int32_t s, int32_t sb) {
  const int64_t ss = static_cast<int64_t>(s) * s;
  const double* Li = base + ss;
  double* Lt = base + 2 * ss;
  for (int e = threadIdx.x; e < sb * sb; e += kT) {
    const int k = e / sb, i = e - k * sb;
    Lt[static_cast<int64_t>(k) * s + i] = (k >= i) ? Li[static_cast<int64_t>(i) * s + k] : 0.0;
  }
}

template <bool IN_LDS, bool LINV = false>
__global__ __launch_bounds__(kT) void k_factor_inverse(double* __restrict__ slots, int64_t stride,
                                                       int32_t s, const int32_t* __restrict__ lens,
                                                       const int32_t* __restrict__ slot_of,
                                                       FactorCheck chk,
                                                       const int32_t* __restrict__ skip) {
  extern __shared__ double lds[];
  __shared__ double red4[4];
  __shared__ double norm_g2;
  const int blk = blockIdx.x;
  if ((chk.only && !chk.only[blk]) || (skip && skip[blk])) return;
  const int sb = lens[blk];
  double* base = slots + static_cast<int64_t>(slot_of[blk]) * stride;
  const double* Lc = base;
  double* Gi = base + static_cast<int64_t>(s) * s;
  if (chk.flag && threadIdx.x == 0) norm_g2 = Gi[static_cast<int64_t>(s) * s - 1];  // left by k_cholesky
  double* M;
  double* tmp;
  int64_t ld;
  if (IN_LDS) {
    M = lds;
    ld = sb + 1;
    tmp = lds + static_cast<int64_t>(sb) * ld;
  } else {
    M = base + 2 * static_cast<int64_t>(s) * s;
    ld = s;
    tmp = Gi;  // G^{-1} is written only after the inversion; its first column is free until then
  }
  // M = L (column-major, lower)
  for (int e = threadIdx.x; e < sb * sb; e += kT) {
    const int k = e / sb, i = e - k * sb;
    M[k * ld + i] = (i >= k) ? Lc[static_cast<int64_t>(k) * s + i] : 0.0;
  }
  for (int j = sb - 1; j >= 0; --j) {
    __syncthreads();
    const double d = 1.0 / M[static_cast<int64_t>(j) * ld + j];
    for (int i = j + 1 + threadIdx.x; i < sb; i += kT) {
      double acc = 0.0;
      for (int k = j + 1; k <= i; ++k) acc = fma(M[static_cast<int64_t>(k) * ld + i], M[static_cast<int64_t>(j) * ld + k], acc);
      tmp[i] = acc;
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < sb; i += kT) M[static_cast<int64_t>(j) * ld + i] = -d * tmp[i];
    if (threadIdx.x == 0) M[static_cast<int64_t>(j) * ld + j] = d;
  }
  __syncthreads();
  if constexpr (LINV) {
    // keep L^{-1} itself, column-major (entry (i, k) at k * s + i), zero above
    // the diagonal, and L^{-T} the same way in the slot's last third
    for (int e = threadIdx.x; e < sb * sb; e += kT) {
      const int k = e / sb, i = e - k * sb;
      Gi[static_cast<int64_t>(k) * s + i] = (i >= k) ? M[static_cast<int64_t>(k) * ld + i] : 0.0;
    }
    __syncthreads();
    write_linv_transpose(base, s, sb);
    return;
  }
  // G^{-1} = M^T M; thread owns column k, entries i >= k, mirrored to (k, i)
  for (int k = threadIdx.x; k < sb; k += kT) {
    for (int i = k; i < sb; ++i) {
      double acc = 0.0;
      for (int r = i; r < sb; ++r) acc = fma(M[static_cast<int64_t>(i) * ld + r], M[static_cast<int64_t>(k) * ld + r], acc);
      Gi[static_cast<int64_t>(i) * s + k] = acc;
      Gi[static_cast<int64_t>(k) * s + i] = acc;
    }
  }
  if (chk.flag) {
    __syncthreads();
    double acc = 0.0;
    for (int e = threadIdx.x; e < sb * sb; e += kT) {
      const int k = e / sb, i = e - k * sb;
      const double v = Gi[static_cast<int64_t>(k) * s + i];
      acc = fma(v, v, acc);
    }
    acc = block_sum(acc, red4);
    if (threadIdx.x == 0) flag_ill_conditioned(chk, blk, norm_g2, acc);
  }
}

// --------------------------------------------------------------------------
// memo miss for blocks of kLdsCholMax+1 .. kFusedMaxBlock rows, blocked in LDS.
//
// k_cholesky_panel: left-looking Cholesky in panels of kPanel columns.  The
// panel (rows p0 .. sb-1 of columns p0 .. p0+pw-1) sits in LDS; the matrix
// cores bring it up to date with the finished columns of L (read from the
// slot), then the panel is factored column by column in LDS and written back.
// With chk.flag it leaves ||G||_F^2 in the first entry of the slot's last
// third.
// --------------------------------------------------------------------------
constexpr int kPanel = 32;
constexpr int kPanelLd = kPanel + 1;

constexpr size_t kCholPanelLds = static_cast<size_t>(kFusedMaxBlock) * kPanelLd * sizeof(double);
// diagonal blocks of L in LDS for the inverse, 32 x 32 each, two doubles of
// padding between blocks so that the two blocks a wave reads sit in different banks
constexpr int kLdBlock = kPanel * kPanel + 2;
static_assert(kPanel == 32, "the inverse's LDS staging indexes blocks of 32 x 32 with shifts");
constexpr size_t kInverseBlockedLds = static_cast<size_t>(kFusedMaxBlock / kPanel) * kLdBlock * sizeof(double);

// The panel update of the Cholesky on the matrix cores (FP64 16x16x4, the
// operand layout of k_block_gemm_mfma): P(i, c) -= sum_{k < p0} L(p0 + i, k)
// L(p0 + c, k) for the R rows and pw columns of the panel, both operands read
// from the finished columns of L in the slot (column-major, 16 consecutive
// rows a lane group), the sums started from the panel in LDS.  Wave wv owns
// row tiles wv, wv + 4, ... (at most four: R <= kFusedMaxBlock - kPanel) and
// both column tiles; k advances 16 at a time with the next 16 in flight.
__device__ __forceinline__ void chol_panel_update(double* P, const double* Gb, int32_t s, int p0, int R, int pw,
                                                  int lane, int wv) {
  const int cl = lane & 15, kq = lane >> 4;
  const int NTr = (R + 15) >> 4;
  v4d_m acc[4][2];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int tc = 0; tc < 2; ++tc)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * (wv + 4 * t) + 4 * r + kq, c = 16 * tc + cl;
        acc[t][tc][r] = (i < R && c < pw) ? P[i * kPanelLd + c] : 0.0;
      }
  double av[2][4][4], bv[2][4][2];
  auto fetch = [&](int b, int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double* Lk = Gb + static_cast<int64_t>(k0 + 4 * q + kq) * s + p0;   // L(p0 + i, k) at Lk[i]
#pragma unroll
      for (int tc = 0; tc < 2; ++tc) bv[b][q][tc] = 16 * tc + cl < pw ? Lk[16 * tc + cl] : 0.0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = 16 * (wv + 4 * t) + cl;
        av[b][q][t] = i < R ? -Lk[i] : 0.0;
      }
    }
  };
  fetch(0, 0);
  for (int k0 = 0; k0 < p0; k0 += 32) {   // p0 is a multiple of kPanel
    if (k0 + 16 < p0) fetch(1, k0 + 16);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (wv + 4 * t < NTr)
#pragma unroll
          for (int tc = 0; tc < 2; ++tc)
            acc[t][tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0][q][t], bv[0][q][tc], acc[t][tc], 0, 0, 0);
    if (k0 + 32 < p0) fetch(0, k0 + 32);
    if (k0 + 16 < p0) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (wv + 4 * t < NTr)
#pragma unroll
            for (int tc = 0; tc < 2; ++tc)
              acc[t][tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1][q][t], bv[1][q][tc], acc[t][tc], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int tc = 0; tc < 2; ++tc)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * (wv + 4 * t) + 4 * r + kq, c = 16 * tc + cl;
        if (i < R && c < pw) P[i * kPanelLd + c] = acc[t][tc][r];
      }
}

__global__ __launch_bounds__(kT) void k_cholesky_panel(double* __restrict__ G, int32_t s, int64_t stride,
                                                       const int32_t* __restrict__ lens,
                                                       const int32_t* __restrict__ slot_of,
                                                       int32_t* __restrict__ err, FactorCheck chk) {
  extern __shared__ double lds[];
  double* P = lds;                                  // P[i * kPanelLd + c] = G(p0 + i, p0 + c)
  __shared__ double red4[4];
  __shared__ double diag_hi[4];
  __shared__ double colbuf[kPanel];
  __shared__ double piv;
  __shared__ int bad_any;
  const int blk = blockIdx.x;
  if (chk.only && !chk.only[blk]) return;
  const int sb = lens[blk];
  const int tid = threadIdx.x;
  const int64_t ss = static_cast<int64_t>(s) * s;
  double* Gb = G + static_cast<int64_t>(slot_of[blk]) * stride;
  if (chk.flag) {
    double acc = 0.0;
    for (int e = tid; e < sb * sb; e += kT) {
      const int k = e / sb, i = e - k * sb;
      if (i >= k) {
        const double v = Gb[static_cast<int64_t>(k) * s + i];
        acc += (i == k ? 1.0 : 2.0) * v * v;
      }
    }
    acc = block_sum(acc, red4);
    if (tid == 0) Gb[2 * ss] = acc;
  }
  if (tid == 0) bad_any = 0;
  __syncthreads();
  int bad = 0;
  for (int p0 = 0; p0 < sb; p0 += kPanel) {
    const int pw = min(kPanel, sb - p0), R = sb - p0;
    if (tid < R) {
      // panel row tid, its loads all in flight (coalesced over the threads)
      double v[kPanel];
#pragma unroll
      for (int c = 0; c < kPanel; ++c) v[c] = c < pw ? Gb[static_cast<int64_t>(p0 + c) * s + p0 + tid] : 0.0;
#pragma unroll
      for (int c = 0; c < kPanel; ++c) P[tid * kPanelLd + c] = v[c];
    }
    __syncthreads();
    if (p0 > 0) chol_panel_update(P, Gb, s, p0, R, pw, tid & 63, tid >> 6);
    __syncthreads();
    // factor the panel with row tid in registers: per column, the pivot and
    // the column's entries in the panel's first rows go through LDS
    double prow[kPanel];
#pragma unroll
    for (int c = 0; c < kPanel; ++c) prow[c] = (tid < R && c < pw) ? P[tid * kPanelLd + c] : 0.0;
#pragma unroll
    for (int c = 0; c < kPanel; ++c) {
      if (c < pw) {
        if (tid == c) piv = prow[c];
        __syncthreads();
        const double d2 = piv;
        if (!(d2 > 0.0)) bad = 1;
        const double d = sqrt(d2);
        if (tid == c) prow[c] = d;
        if (tid > c) prow[c] /= d;
        if (tid < pw) colbuf[tid] = prow[c];
        __syncthreads();
        if (tid > c && tid < R) {
#pragma unroll
          for (int c2 = c + 1; c2 < kPanel; ++c2)
            if (c2 < pw && c2 <= tid) prow[c2] = fma(-prow[c], colbuf[c2], prow[c2]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kPanel; ++c)
      if (c < pw && tid < R && tid >= c) Gb[static_cast<int64_t>(p0 + c) * s + p0 + tid] = prow[c];
    __syncthreads();
  }
  if (bad) atomicOr(&bad_any, 1);
  // smallest and largest diagonal entry of L (fmin / fmax: any order gives the same result)
  double lo = 1.0 / 0.0, hi = 0.0;
  if (tid < sb) {
    const double d = Gb[static_cast<int64_t>(tid) * s + tid];
    lo = d;
    hi = d;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_down(lo, off, 64));
    hi = fmax(hi, __shfl_down(hi, off, 64));
  }
  if ((tid & 63) == 0) {
    red4[tid >> 6] = lo;
    diag_hi[tid >> 6] = hi;
  }
  __syncthreads();
  if (tid == 0) {
    lo = fmin(fmin(red4[0], red4[1]), fmin(red4[2], red4[3]));
    hi = fmax(fmax(diag_hi[0], diag_hi[1]), fmax(diag_hi[2], diag_hi[3]));
    const double ratio = hi / lo;
    const bool ill = !(ratio * ratio <= chk.kappa_max);
    if (chk.flag) {
      const int f = (bad_any || ill) ? 1 : 0;
      chk.flag[blk] = f;
      if (f) atomicAdd(chk.counter, 1);
    } else if (bad_any) {
      atomicOr(err, 1);
    }
  }
  // zero strict upper triangle and padding: thread i clears row i (s <= kT)
  if (tid < s)
    for (int k = 0; k < s; ++k)
      if (tid >= sb || k >= sb || k > tid) Gb[static_cast<int64_t>(k) * s + tid] = 0.0;
}

// --------------------------------------------------------------------------
// G^{-1} = L^{-T} L^{-1} of a block of kLdsCholMax+1 .. kFusedMaxBlock rows.
// X = L^{-1}: first the diagonal blocks X_rr = L_rr^{-1} of kPanel rows, all
// at once by substitution (thread (r, c) forms column c of block r from the
// block staged in LDS); then one block row at a time the columns to the left,
// X_rq = -X_rr T with T = sum_k L_rk X_kq, on the matrix cores (FP64
// 16x16x4, the operand layout of k_block_gemm_mfma).  X is kept row-major in
// the slot's last third.  Then G^{-1}(i, j) = sum_{k >= max(i, j)}
// X(k, i) X(k, j), the 16 x 16 tiles of the lower triangle on the matrix cores
// and each stored with its mirror image, so the inverse is exactly symmetric.
// The diagonal blocks of X are written whole (zeros above their diagonal);
// other entries above the diagonal, and entries past the block, are never
// read (the loads are masked).  With chk.flag the Frobenius condition number
// is tested as in k_factor_inverse.
// --------------------------------------------------------------------------

// Column tile jt of X_rq (rows r0 .. r0 + w - 1, columns 16 jt .. 16 jt + 15,
// r0 > 0 a multiple of kPanel).  T(a, j) = sum_{k = j}^{r0 - 1} L(r0 + a, k)
// X(k, j) for the block row's two 16-row tiles, k advancing 16 at a time with
// the next 16 in flight; then X(r0 + a, j) = -sum_b X_rr(a, b) T(b, j), where
// register q of T's tile is the 4 x 16 operand of the q-th k step as it stands.
__device__ __forceinline__ void inv_xrq_tile(double* X, const double* Lc, int32_t s, int r0, int w, int jt,
                                             int lane) {
  const int cl = lane & 15, kq = lane >> 4;
  const int cb = 16 * jt + cl;
  v4d_m t0 = {0.0, 0.0, 0.0, 0.0}, t1 = {0.0, 0.0, 0.0, 0.0};
  double a0[2][4], a1[2][4], bx[2][4];
  auto fetch = [&](int b, int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 4 * q + kq;
      const double* Lk = Lc + static_cast<int64_t>(k) * s + r0;   // L(r0 + a, k) at Lk[a]
      a0[b][q] = cl < w ? Lk[cl] : 0.0;
      a1[b][q] = 16 + cl < w ? Lk[16 + cl] : 0.0;
      bx[b][q] = cb <= k ? X[static_cast<int64_t>(k) * s + cb] : 0.0;
    }
  };
  auto mma = [&](int b) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      t0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[b][q], bx[b][q], t0, 0, 0, 0);
      t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[b][q], bx[b][q], t1, 0, 0, 0);
    }
  };
  // r0 - 16 jt is a multiple of 16
  int k0 = 16 * jt;
  fetch(0, k0);
  for (; k0 + 16 < r0; k0 += 32) {
    fetch(1, k0 + 16);
    mma(0);
    if (k0 + 32 < r0) fetch(0, k0 + 32);
    mma(1);
  }
  if (k0 < r0) mma(0);
  v4d_m o0 = {0.0, 0.0, 0.0, 0.0}, o1 = {0.0, 0.0, 0.0, 0.0};
  const double* Xr0 = X + static_cast<int64_t>(r0 + cl) * s + r0;        // X(r0 + a, r0 + b) at Xr0[b], a = cl
  const double* Xr1 = X + static_cast<int64_t>(r0 + 16 + cl) * s + r0;   // a = 16 + cl
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b0 = 4 * q + kq, b1 = 16 + 4 * q + kq;
    const double x00 = cl < w && b0 < w ? Xr0[b0] : 0.0;
    const double x10 = 16 + cl < w && b0 < w ? Xr1[b0] : 0.0;
    const double x01 = cl < w && b1 < w ? Xr0[b1] : 0.0;
    const double x11 = 16 + cl < w && b1 < w ? Xr1[b1] : 0.0;
    o0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x00, t0[q], o0, 0, 0, 0);
    o1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x10, t0[q], o1, 0, 0, 0);
    o0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x01, t1[q], o0, 0, 0, 0);
    o1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x11, t1[q], o1, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int a = 4 * r + kq;
    if (a < w) X[static_cast<int64_t>(r0 + a) * s + cb] = -o0[r];
    if (16 + a < w) X[static_cast<int64_t>(r0 + 16 + a) * s + cb] = -o1[r];
  }
}

// Tiles (ti, tj0 .. tj0 + CNT - 1), tj0 + CNT - 1 <= ti, of G^{-1} = X^T X:
// sum over k = 16 ti .. sb - 1 of X(k, 16 ti + a) X(k, 16 tj + b) (the terms
// with k < 16 ti vanish: X is lower triangular), k advancing 16 at a time with
// the next 16 in flight.  Lower entries and their mirror images are stored;
// on a diagonal tile only a >= b.
template <int CNT>
__device__ __forceinline__ void ginv_tiles(double* Gi, const double* X, int32_t s, int sb, int ti, int tj0, int lane) {
  const int cl = lane & 15, kq = lane >> 4;
  const int ca = 16 * ti + cl;
  v4d_m acc[CNT];
#pragma unroll
  for (int t = 0; t < CNT; ++t) acc[t] = v4d_m{0.0, 0.0, 0.0, 0.0};
  double av[2][4], bv[2][4][CNT];
  auto fetch = [&](int b, int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 4 * q + kq;
      const bool kin = k < sb;
      const double* Xk = X + static_cast<int64_t>(k) * s;
      av[b][q] = kin && ca <= k ? Xk[ca] : 0.0;
#pragma unroll
      for (int t = 0; t < CNT; ++t) {
        const int cb = 16 * (tj0 + t) + cl;
        bv[b][q][t] = kin && cb <= k ? Xk[cb] : 0.0;
      }
    }
  };
  auto mma = [&](int b) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < CNT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[b][q], bv[b][q][t], acc[t], 0, 0, 0);
  };
  int k0 = 16 * ti;
  fetch(0, k0);
  for (; k0 + 16 < sb; k0 += 32) {
    fetch(1, k0 + 16);
    mma(0);
    if (k0 + 32 < sb) fetch(0, k0 + 32);
    mma(1);
  }
  if (k0 < sb) mma(0);
#pragma unroll
  for (int t = 0; t < CNT; ++t) {
    const int tj = tj0 + t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = 4 * r + kq;
      const int i = 16 * ti + a, j = 16 * tj + cl;
      if (i < sb && j < sb && (tj < ti || a >= cl)) {
        Gi[static_cast<int64_t>(i) * s + j] = acc[t][r];
        Gi[static_cast<int64_t>(j) * s + i] = acc[t][r];
      }
    }
  }
}

template <bool LINV = false>
__global__ __launch_bounds__(kT) void k_inverse_blocked(double* __restrict__ slots, int64_t stride, int32_t s,
                                                        const int32_t* __restrict__ lens,
                                                        const int32_t* __restrict__ slot_of, FactorCheck chk,
                                                        const int32_t* __restrict__ skip) {
  extern __shared__ double lds[];                   // diagonal blocks of L, kLdBlock doubles apart
  __shared__ double red4[4];
  const int blk = blockIdx.x;
  if ((chk.only && !chk.only[blk]) || (skip && skip[blk])) return;
  const int sb = lens[blk];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t ss = static_cast<int64_t>(s) * s;
  double* base = slots + static_cast<int64_t>(slot_of[blk]) * stride;
  const double* Lc = base;                          // L(i, k) at Lc[k * s + i]
  double* Gi = base + ss;
  double* X = base + 2 * ss;                        // X(i, j) at X[i * s + j]
  const double norm_g2 = chk.flag ? X[0] : 0.0;     // left by the Cholesky, overwritten below
  const int npan = (sb + kPanel - 1) / kPanel;
  // block r of LDS: Ld[k * kPanel + a] = L(32 r + a, 32 r + k), zero past the block
  for (int e = tid; e < npan * kPanel * kPanel; e += kT) {
    const int r = e >> 10, k = (e >> 5) & 31, a = e & 31;
    const int r0 = r * kPanel, w = min(kPanel, sb - r0);
    lds[r * kLdBlock + k * kPanel + a] = (a < w && k < w) ? Lc[static_cast<int64_t>(r0 + k) * s + r0 + a] : 0.0;
  }
  __syncthreads();
  {
    // X_rr = L_rr^{-1}: column c of diagonal block r in registers, rows i > c
    // by substitution; the block row's w x w corner of X is written whole
    const int r = tid >> 5, c = tid & 31;
    const int r0 = r * kPanel, w = min(kPanel, sb - r0);
    const double* Ld = lds + r * kLdBlock;
    if (r < npan && c < w) {
      double xc[kPanel];
#pragma unroll
      for (int i = 0; i < kPanel; ++i) {
        double v = 0.0;
        if (i == c) {
          v = 1.0 / Ld[i * kPanel + i];
        } else if (i > c && i < w) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < i; ++k)
            if (k >= c) acc = fma(Ld[k * kPanel + i], xc[k], acc);
          v = -acc / Ld[i * kPanel + i];
        }
        xc[i] = v;
      }
#pragma unroll
      for (int i = 0; i < kPanel; ++i)
        if (i < w) X[static_cast<int64_t>(r0 + i) * s + r0 + c] = xc[i];
    }
  }
  __syncthreads();
  for (int r0 = kPanel; r0 < sb; r0 += kPanel) {
    const int w = min(kPanel, sb - r0);
    // column tiles of X_rq, four to a wave in the order that evens out their lengths
    const int ntc = r0 >> 4;
#pragma unroll 1
    for (int u = 0; u < 4; ++u) {
      const int jt = (u & 1) ? 8 * ((u + 1) >> 1) - 1 - wv : 8 * (u >> 1) + wv;
      if (jt < ntc) inv_xrq_tile(X, Lc, s, r0, w, jt, lane);
    }
    __syncthreads();
  }
  if constexpr (LINV) {
    // X = L^{-1} row-major is L^{-T} column-major already: copy L^{-1}
    // column-major into the second third, then clear X above the diagonal
    for (int e = tid; e < sb * sb; e += kT) {
      const int k = e / sb, i = e - k * sb;
      Gi[static_cast<int64_t>(k) * s + i] = (i >= k) ? X[static_cast<int64_t>(i) * s + k] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < sb * sb; e += kT) {
      const int k = e / sb, i = e - k * sb;
      if (i > k) X[static_cast<int64_t>(k) * s + i] = 0.0;
    }
    return;
  }
  // G^{-1}: jobs of up to four tiles of one tile row, dealt to the waves by the
  // same greedy rule in every wave (the least loaded wave takes the next job)
  {
    const int nt = (sb + 15) >> 4;
    int l0 = 0, l1 = 0, l2 = 0, l3 = 0;   // work dealt to each wave so far
#pragma unroll 1
    for (int ti = 0; ti < nt; ++ti) {
#pragma unroll 1
      for (int tj0 = 0; tj0 <= ti; tj0 += 4) {
        const int cnt = min(4, ti + 1 - tj0);
        int who = 0, lw = l0;
        if (l1 < lw) { who = 1; lw = l1; }
        if (l2 < lw) { who = 2; lw = l2; }
        if (l3 < lw) who = 3;
        const int cost = (nt - ti) * (cnt + 1);
        l0 += who == 0 ? cost : 0;
        l1 += who == 1 ? cost : 0;
        l2 += who == 2 ? cost : 0;
        l3 += who == 3 ? cost : 0;
        if (who != wv) continue;
        switch (cnt) {
          case 1: ginv_tiles<1>(Gi, X, s, sb, ti, tj0, lane); break;
          case 2: ginv_tiles<2>(Gi, X, s, sb, ti, tj0, lane); break;
          case 3: ginv_tiles<3>(Gi, X, s, sb, ti, tj0, lane); break;
          default: ginv_tiles<4>(Gi, X, s, sb, ti, tj0, lane); break;
        }
      }
    }
  }
  // padding: thread j clears column j past the block (s <= kT)
  if (tid < s)
    for (int i = 0; i < s; ++i)
      if (i >= sb || tid >= sb) Gi[static_cast<int64_t>(i) * s + tid] = 0.0;
  if (chk.flag) {
    __syncthreads();
    double acc = 0.0;
    for (int e = tid; e < sb * sb; e += kT) {
      const int i = e / sb, jj = e - i * sb;
      const double v = Gi[static_cast<int64_t>(i) * s + jj];
      acc = fma(v, v, acc);
    }
    acc = block_sum(acc, red4);
    if (tid == 0) flag_ill_conditioned(chk, blk, norm_g2, acc);
  }
}

// --------------------------------------------------------------------------
// memo miss for blocks of up to 128 rows (one workgroup per block): the
// regularized Gram is cut into 16 x 16 tiles of its lower triangle, held in
// LDS (column-major tiles, column stride 17 so that the matrix-core operand
// and result patterns hit distinct banks).
//   Cholesky, right-looking over tile columns p: wave 0 factors the diagonal
//   tile in registers (lane r holds row r; each column's entries are
//   broadcast with readlane) and inverts it (lane k forms column k of the
//   inverse by forward substitution); the tiles below are L_ip = A_ip
//   L_pp^{-T}, and the trailing tiles are updated A_ij -= L_ip L_jp^T, each
//   tile product on the FP64 16x16x4 matrix cores, tiles spread over waves.
//   L^{-1} in place, tile column j from the last to the first:
//   X_ij = -(sum_{k=j+1..i} X_ik L_kj) X_jj (the X_ik are the columns already
//   inverted, X_jj the diagonal inverse kept from the factorization).
//   G^{-1} = X^T X tile by tile (G^{-1}_ij = sum_{k>=i} X_ki^T X_kj), stored
//   with its mirror image so the result is exactly symmetric.
// Ragged blocks are padded with the identity up to the next tile edge.
// Matrix-core layouts (16x16x4 FP64): lane l supplies X[l % 16][l / 16] of
// the 16 x 4 operand and Y[l / 16][l % 16] of the 4 x 16 one; register q of
// lane l receives D[l / 16 + 4 q][l % 16].
// --------------------------------------------------------------------------
constexpr int kFT = 16;                          // tile edge
constexpr int kFLd = 17;                         // LDS column stride inside a tile
constexpr int kFTile = kFT * kFLd;               // doubles per LDS tile
constexpr int kFMaxT = kFactorSmallMax / kFT;    // tiles per block edge (8)
constexpr int kFLower = kFMaxT * (kFMaxT + 1) / 2;
constexpr int kFLdsDoubles = (kFLower + kFMaxT + 4) * kFTile;   // tiles, diagonal inverses, wave scratch
constexpr size_t kFactorTiledLds = static_cast<size_t>(kFLdsDoubles) * sizeof(double);

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int ftix(int i, int j) { return i * (i + 1) / 2 + j; }
__device__ __forceinline__ double rdlane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ f64x4 mma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// acc += sign * Xt Yt over the tile's 16 columns, where lane l reads operand
// entries at xa + (kk + l/16) * kFLd + l%16 ("n": X = the tile itself) or
// xa + (l%16) * kFLd + kk + l/16 ("t": X = the tile transposed).
template <bool XT, bool YT>
__device__ __forceinline__ f64x4 tile_mma(const double* xa, const double* yb, f64x4 acc, int lane, double sign) {
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < kFT; kk += 4) {
    const double a = XT ? xa[lr * kFLd + kk + lk] : xa[(kk + lk) * kFLd + lr];
    const double b = YT ? yb[lr * kFLd + kk + lk] : yb[(kk + lk) * kFLd + lr];
    acc = mma(sign * a, b, acc);
  }
  return acc;
}
__device__ __forceinline__ f64x4 tile_load_d(const double* t, int lane) {
  const int c = lane & 15, r = lane >> 4;
  return f64x4{t[c * kFLd + r], t[c * kFLd + r + 4], t[c * kFLd + r + 8], t[c * kFLd + r + 12]};
}
__device__ __forceinline__ void tile_store_d(double* t, f64x4 v, int lane) {
  const int c = lane & 15, r = lane >> 4;
  t[c * kFLd + r] = v[0];
  t[c * kFLd + r + 4] = v[1];
  t[c * kFLd + r + 8] = v[2];
  t[c * kFLd + r + 12] = v[3];
}

__global__ __launch_bounds__(kT) void k_factor_small(double* __restrict__ slots, int64_t stride,
                                                     int32_t s, const int32_t* __restrict__ lens,
                                                     const int32_t* __restrict__ slot_of,
                                                     int32_t want_inverse, int32_t* __restrict__ err,
                                                     FactorCheck chk) {
  extern __shared__ double fl[];
  double* T = fl;                                  // lower tiles, tile (i, j) at ftix(i, j) * kFTile
  double* Dv = fl + kFLower * kFTile;              // inverses of the diagonal tiles of L
  double* Sc = Dv + kFMaxT * kFTile;               // one scratch tile per wave
  __shared__ double red4[4];
  __shared__ double rdiag[kFT];   // 1 / L_jj of the diagonal tile being inverted
  __shared__ double norm_g2;
  __shared__ int flag_blk;
  const int blk = blockIdx.x;
  if (chk.only && !chk.only[blk]) return;
  const int sb = lens[blk];
  double* Lc = slots + static_cast<int64_t>(slot_of[blk]) * stride;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nt = (sb + kFT - 1) / kFT;
  const int nlow = nt * (nt + 1) / 2;
  // G (lower triangle of the slot) into the tiles, identity past the block:
  // thread tid holds entry (r, c) = (tid % 16, tid / 16) of every tile; the
  // loads of kGB tiles go out together (one after the other they are a chain
  // of global round trips)
  double g2 = 0.0;
  {
    constexpr int kGB = 12;
    const int c = tid >> 4, r = tid & 15;
    for (int t0 = 0; t0 < nlow; t0 += kGB) {
      double v[kGB];
      int ti = 0;
      while ((ti + 1) * (ti + 2) / 2 <= t0) ++ti;
      int tj = t0 - ti * (ti + 1) / 2;
#pragma unroll
      for (int u = 0; u < kGB; ++u) {
        const int i = ti * kFT + r, k = tj * kFT + c;
        const bool in = t0 + u < nlow && i < sb && k < sb;
        v[u] = (in && i >= k) ? Lc[static_cast<int64_t>(k) * s + i] : ((i == k && !(i < sb && k < sb)) ? 1.0 : 0.0);
        if (++tj > ti) {
          ++ti;
          tj = 0;
        }
      }
      ti = 0;
      while ((ti + 1) * (ti + 2) / 2 <= t0) ++ti;
      tj = t0 - ti * (ti + 1) / 2;
#pragma unroll
      for (int u = 0; u < kGB; ++u) {
        const int i = ti * kFT + r, k = tj * kFT + c;
        if (t0 + u < nlow) {
          if (i < sb && k < sb) g2 += (i == k ? 1.0 : 2.0) * v[u] * v[u];
          T[(t0 + u) * kFTile + c * kFLd + r] = v[u];
        }
        if (++tj > ti) {
          ++ti;
          tj = 0;
        }
      }
    }
  }
  if (chk.flag) {
    g2 = block_sum(g2, red4);
    if (tid == 0) norm_g2 = g2;
  }
  __syncthreads();

  int bad = 0;
  for (int p = 0; p < nt; ++p) {
    double* Tp = T + ftix(p, p) * kFTile;
    double* Dp = Dv + p * kFTile;
    if (wv == 0) {
      // the diagonal tile: lane r (mod 16) holds row r
      const int r = lane & 15;
      double a[kFT];
#pragma unroll
      for (int c = 0; c < kFT; ++c) a[c] = Tp[c * kFLd + r];
#pragma unroll
      for (int j = 0; j < kFT; ++j) {
        const double d = rdlane(a[j], j);
        bad |= !(d > 0.0);
        const double ljj = sqrt(d);
        const double rl = 1.0 / ljj;
        if (lane == 0) rdiag[j] = rl;
        a[j] = r > j ? a[j] * rl : (r == j ? ljj : a[j]);
#pragma unroll
        for (int k = j + 1; k < kFT; ++k) {
          const double lk = rdlane(a[j], k);
          a[k] = r >= k ? fma(-a[j], lk, a[k]) : a[k];
        }
      }
      if (lane < kFT) {
#pragma unroll
        for (int c = 0; c < kFT; ++c)
          if (c <= r) Tp[c * kFLd + r] = a[c];
      }
      // its inverse: lane k forms column k by forward substitution, reading
      // the factor back from LDS (the same address in every lane)
      const int kc = lane & 15;
      double x[kFT];
#pragma unroll
      for (int i = 0; i < kFT; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < i; ++m) acc = fma(Tp[m * kFLd + i], x[m], acc);
        const double inv = rdiag[i];   // the same 1 / L_ii the factorization formed
        x[i] = i == kc ? inv : (i > kc ? -acc * inv : 0.0);
      }
      if (lane < kFT) {
#pragma unroll
        for (int i = 0; i < kFT; ++i) Dp[kc * kFLd + i] = x[i];
      }
    }
    __syncthreads();
    // tiles below the diagonal: L_ip = A_ip L_pp^{-T}
    for (int i = p + 1 + wv; i < nt; i += 4) {
      double* Ti = T + ftix(i, p) * kFTile;
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
      acc = tile_mma<false, false>(Ti, Dp, acc, lane, 1.0);
      tile_store_d(Ti, acc, lane);
    }
    __syncthreads();
    // trailing tiles: A_ij -= L_ip L_jp^T
    const int mrem = nt - p - 1;
    for (int u = wv; u < mrem * (mrem + 1) / 2; u += 4) {
      int ii = 0;
      while ((ii + 1) * (ii + 2) / 2 <= u) ++ii;
      const int i = p + 1 + ii, j = p + 1 + (u - ii * (ii + 1) / 2);
      double* Tij = T + ftix(i, j) * kFTile;
      f64x4 acc = tile_load_d(Tij, lane);
      acc = tile_mma<false, false>(T + ftix(i, p) * kFTile, T + ftix(j, p) * kFTile, acc, lane, -1.0);
      tile_store_d(Tij, acc, lane);
    }
    __syncthreads();
  }

  // breakdown, and kappa(G) >= (max L_ii / min L_ii)^2 from the factor's diagonal
  if (wv == 0) {
    double lo = 1.0 / 0.0, hi = 0.0;
    for (int i = lane; i < sb; i += 64) {
      const double d = T[ftix(i >> 4, i >> 4) * kFTile + (i & 15) * kFLd + (i & 15)];
      lo = fmin(lo, d);
      hi = fmax(hi, d);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, off, 64));
      hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    if (lane == 0) {
      const double ratio = hi / lo;
      const bool ill = !(ratio * ratio <= chk.kappa_max);
      if (chk.flag) {
        // low-precision pass: mark the block for an FP64 redo instead of failing
        const int f = (bad || ill) ? 1 : 0;
        chk.flag[blk] = f;
        if (f) atomicAdd(chk.counter, 1);
        flag_blk = f;
      } else {
        if (bad) atomicOr(err, 1);
        flag_blk = 0;
      }
    }
  }
  __syncthreads();
  // L to the slot (column-major, zero outside the block's lower triangle)
#pragma unroll 8
  for (int e = tid; e < s * s; e += kT) {
    const int i = e % s, k = e / s;
    Lc[static_cast<int64_t>(k) * s + i] =
        (i < sb && k < sb && i >= k) ? T[ftix(i >> 4, k >> 4) * kFTile + (k & 15) * kFLd + (i & 15)] : 0.0;
  }
  if (flag_blk || !want_inverse) return;   // uniform: the FP64 pass recomputes a flagged block

  // L^{-1} in place, tile columns from the last to the first
  double* Sw = Sc + wv * kFTile;
  for (int j = nt - 2; j >= 0; --j) {
    // X_ij for i = j + 1 + wv and i = j + 5 + wv (a tile column has at most 7)
    auto column_tile = [&](int i) {
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int k = j + 1; k <= i; ++k) {
        const double* Xik = k == i ? Dv + i * kFTile : T + ftix(i, k) * kFTile;
        acc = tile_mma<false, true>(Xik, T + ftix(k, j) * kFTile, acc, lane, 1.0);
      }
      tile_store_d(Sw, acc, lane);
      const f64x4 zero = {0.0, 0.0, 0.0, 0.0};
      return tile_mma<false, true>(Sw, Dv + j * kFTile, zero, lane, -1.0);
    };
    const int i0 = j + 1 + wv, i1 = j + 5 + wv;
    f64x4 res0 = {0.0, 0.0, 0.0, 0.0}, res1 = {0.0, 0.0, 0.0, 0.0};
    if (i0 < nt) res0 = column_tile(i0);
    if (i1 < nt) res1 = column_tile(i1);
    __syncthreads();
    if (i0 < nt) tile_store_d(T + ftix(i0, j) * kFTile, res0, lane);
    if (i1 < nt) tile_store_d(T + ftix(i1, j) * kFTile, res1, lane);
    __syncthreads();
  }
  // G^{-1} = X^T X, lower tiles, stored with their mirror images
  double* Gi = Lc + static_cast<int64_t>(s) * s;
  double gi2 = 0.0;
  for (int u = wv; u < nlow; u += 4) {
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= u) ++i;
    const int j = u - i * (i + 1) / 2;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k = i; k < nt; ++k) {
      const double* Xki = k == i ? Dv + i * kFTile : T + ftix(k, i) * kFTile;
      const double* Xkj = k == j ? Dv + j * kFTile : T + ftix(k, j) * kFTile;
      acc = tile_mma<true, true>(Xki, Xkj, acc, lane, 1.0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = i * kFT + (lane >> 4) + 4 * q, col = j * kFT + (lane & 15);
      if (row < sb && col < sb && (i != j || row >= col)) {
        const double v = acc[q];
        Gi[static_cast<int64_t>(col) * s + row] = v;
        Gi[static_cast<int64_t>(row) * s + col] = v;
        gi2 += (row == col ? 1.0 : 2.0) * v * v;
      }
    }
  }
  if (chk.flag) {
    gi2 = block_sum(gi2, red4);
    if (tid == 0) flag_ill_conditioned(chk, blk, norm_g2, gi2);
  }
}

// d_j = sum_i A_ij z_i in two passes: workgroup (c, r) owns 256 consecutive
// columns and the r-th of `splits` consecutive row ranges, walks its rows in
// order with eight loads in flight (coalesced row segments) and writes a
// partial sum; the second pass adds the partials in split order
// (deterministic).  One split writes d directly.
__global__ __launch_bounds__(kT) void k_gemv_t_part(const double* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                    const double* __restrict__ z, int32_t splits,
                                                    double* __restrict__ out) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
  if (j >= n) return;
  const int64_t per = (m + splits - 1) / splits;
  const int64_t r0 = static_cast<int64_t>(blockIdx.y) * per, r1 = min(m, r0 + per);
  double acc = 0.0;
  int64_t i = r0;
  for (; i + 8 <= r1; i += 8) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = A[(i + u) * lda + j];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = fma(a[u], z[i + u], acc);
  }
  for (; i < r1; ++i) acc = fma(A[i * lda + j], z[i], acc);
  out[static_cast<int64_t>(blockIdx.y) * n + j] = acc;
}

__global__ __launch_bounds__(kT) void k_gemv_t_sum(const double* __restrict__ part, int64_t n, int32_t splits,
                                                   double* __restrict__ d) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
  if (j >= n) return;
  double acc = 0.0;
  for (int32_t r = 0; r < splits; ++r) acc += part[static_cast<int64_t>(r) * n + j];
  d[j] = acc;
}

// Block rows and lengths from a staging area into their slots.
__global__ __launch_bounds__(kT) void k_scatter_rows(const int32_t* __restrict__ stage_rows,
                                                     const int32_t* __restrict__ stage_lens,
                                                     const int32_t* __restrict__ slot_of, int32_t s,
                                                     int32_t* __restrict__ rows, int32_t* __restrict__ lens) {
  const int k = blockIdx.x;
  const int q = slot_of[k];
  for (int i = threadIdx.x; i < s; i += kT) rows[static_cast<int64_t>(q) * s + i] = stage_rows[static_cast<int64_t>(k) * s + i];
  if (threadIdx.x == 0) lens[q] = stage_lens[k];
}

__global__ __launch_bounds__(kT) void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t base, int32_t step) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; i < n; i += static_cast<int64_t>(gridDim.x) * kT)
    p[i] = base + step * static_cast<int32_t>(i);
}

__global__ __launch_bounds__(kT) void k_zero_f64(double* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kT) + threadIdx.x; i < n; i += static_cast<int64_t>(gridDim.x) * kT)
    p[i] = 0.0;
}

}  // namespace

void launch_fill_i32(int32_t* p, int64_t n, int32_t base, int32_t step, hipStream_t st) {
  if (n <= 0) return;
  const int64_t g = std::min<int64_t>((n + kT - 1) / kT, 4096);
  hipLaunchKernelGGL(k_fill_i32, dim3(static_cast<unsigned>(g)), dim3(kT), 0, st, p, n, base, step);
}

void launch_zero_f64(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  const int64_t g = std::min<int64_t>((n + kT - 1) / kT, 4096);
  hipLaunchKernelGGL(k_zero_f64, dim3(static_cast<unsigned>(g)), dim3(kT), 0, st, p, n);
}

void launch_block_gemv_partial(const double* A, int64_t lda, int64_t n, const int32_t* rows,
                               int32_t sb, const double* x, double* rpart, int32_t P,
                               int64_t chunk, hipStream_t st) {
  dim3 grid(P, sb);
  hipLaunchKernelGGL(k_block_gemv_partial, grid, dim3(kT), 0, st, A, lda, n, rows, x, rpart, P,
                     chunk);
}

void launch_block_project(const double* rpart, int32_t P, const double* b, const int32_t* rows,
                          int32_t sb, const double* L, int32_t ldl, double* y, DevState* ds,
                          int32_t zeta, int32_t adaptive, hipStream_t st) {
  if (ldl > 128) {   // large blocks: rows of y over workgroups
    const unsigned g = static_cast<unsigned>((sb + kProjRows - 1) / kProjRows);
    hipLaunchKernelGGL(k_block_project_rows, dim3(g), dim3(kT), 0, st, rpart, P, b, rows, sb, L, ldl, y, ds, zeta,
                       adaptive);
    return;
  }
  hipLaunchKernelGGL(k_block_project, dim3(1), dim3(kT), 0, st, rpart, P, b, rows, sb, L, ldl, y,
                     ds, zeta, adaptive);
}

void launch_update(int32_t kind, const double* A, int64_t lda, int64_t n, const int32_t* rows,
                   int32_t sb, const double* y, const DevState* ds, double eta, double* x,
                   double* mom, hipStream_t st) {
  dim3 grid(static_cast<unsigned>((n + kT - 1) / kT));
  if (kind == 0)
    hipLaunchKernelGGL(k_update<0>, grid, dim3(kT), 0, st, A, lda, n, rows, sb, y, ds, eta, x, mom);
  else
    hipLaunchKernelGGL(k_update<1>, grid, dim3(kT), 0, st, A, lda, n, rows, sb, y, ds, eta, x, mom);
}

void launch_block_gemm_partial(const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb,
                               const double* X, int64_t ldx, int32_t k, double* rpart, int32_t P, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(P), static_cast<unsigned>((sb + 15) / 16));
  if (k <= 16)
    hipLaunchKernelGGL(k_block_gemm_mfma<1>, grid, dim3(kT), 0, st, A, lda, n, rows, sb, X, ldx, k, rpart, P);
  else
    hipLaunchKernelGGL(k_block_gemm_mfma<2>, grid, dim3(kT), 0, st, A, lda, n, rows, sb, X, ldx, k, rpart, P);
}

void launch_block_project_multi(const double* rpart, int32_t P, int32_t k, const double* B, int64_t ldb,
                                const int32_t* rows, int32_t sb, const double* Ginv, int32_t s, double* Y,
                                DevState* ds, const int32_t* frozen, int32_t zeta, int32_t adaptive, hipStream_t st) {
  hipLaunchKernelGGL(k_block_project_multi, dim3(k), dim3(kT), 0, st, rpart, P, k, B, ldb, rows, sb, Ginv, s, Y, ds,
                     frozen, zeta, adaptive);
}

void launch_update_multi(int32_t kind, const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb,
                         const double* Y, int32_t s, int32_t k, const DevState* ds, const int32_t* frozen, double eta,
                         double* X, int64_t ldx, double* M, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n + kT - 1) / kT));
#define KPP_UPDATE_MULTI(KIND, KM)                                                                               \
  hipLaunchKernelGGL((k_update_multi<KIND, KM>), grid, dim3(kT), 0, st, A, lda, n, rows, sb, Y, s, k, ds, frozen, \
                     eta, X, ldx, M)
  if (kind == 1) {
    const int64_t total = n * k;
    hipLaunchKernelGGL(k_update_multi_cd, dim3(static_cast<unsigned>((total + kT - 1) / kT)), dim3(kT), 0, st, n,
                       rows, sb, Y, s, k, ds, frozen, eta, X, ldx, M);
    return;
  }
  if (k <= 4) KPP_UPDATE_MULTI(0, 4);
  else if (k <= 8) KPP_UPDATE_MULTI(0, 8);
  else if (k <= 16) KPP_UPDATE_MULTI(0, 16);
  else KPP_UPDATE_MULTI(0, 32);
#undef KPP_UPDATE_MULTI
}

void launch_column(const double* X, int64_t ldx, int64_t n, int32_t c, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_column, dim3(static_cast<unsigned>((n + kT - 1) / kT)), dim3(kT), 0, st, X, ldx, n, c, out);
}

void launch_gram(int32_t kind, const double* A, int64_t lda, int64_t n, const int32_t* rows,
                 const int32_t* lens, int32_t s, int32_t nb, double lambda, double* G, int64_t stride,
                 const int32_t* slot_of, double* ws, hipStream_t st, const int32_t* only) {
  if (nb <= 0) return;
  if (kind == 0) {
    launch_gram_syrk(A, lda, n, rows, lens, s, nb, lambda, G, stride, slot_of, only, ws, st);
  } else {
    hipLaunchKernelGGL(k_gram_cd<double>, dim3(nb), dim3(kT), 0, st, A, lda, rows, lens, s, lambda, G,
                       stride, slot_of, only);
  }
}

void launch_cholesky(double* G, int32_t s, int64_t stride, const int32_t* lens, int32_t nb,
                     const int32_t* slot_of, int32_t* err, hipStream_t st, FactorCheck chk) {
  if (nb <= 0) return;
  if (s > kLdsCholMax && s <= kFusedMaxBlock) {
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cholesky_panel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kCholPanelLds));
      attr_set = true;
    }
    hipLaunchKernelGGL(k_cholesky_panel, dim3(nb), dim3(kT), kCholPanelLds, st, G, s, stride, lens, slot_of, err,
                       chk);
    return;
  }
  if (s <= kLdsCholMax) {
    const size_t lds = static_cast<size_t>(s) * s * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cholesky<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>(kLdsCholMax * kLdsCholMax * sizeof(double)));
      attr_set = true;
    }
    hipLaunchKernelGGL(k_cholesky<true>, dim3(nb), dim3(kT), lds, st, G, s, stride, lens, slot_of, err, chk);
  } else {
    hipLaunchKernelGGL(k_cholesky<false>, dim3(nb), dim3(kT), 0, st, G, s, stride, lens, slot_of, err, chk);
  }
}

void launch_residual_sq(const double* A, int64_t lda, int64_t m, int64_t n, const double* x,
                        const double* b, double* part, int32_t nparts, double* out,
                        hipStream_t st) {
  (void)nparts;
  const unsigned g = static_cast<unsigned>((m + 3) / 4);
  hipLaunchKernelGGL(k_residual_rows, dim3(g), dim3(kT), 0, st, A, lda, m, n, x, b, part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kT), 0, st, part, m, out);
}

void launch_check_finite(const double* A, int64_t lda, int64_t m, int64_t n, const double* b,
                         int32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_check_finite, dim3(static_cast<unsigned>(m)), dim3(kT), 0, st, A, lda, m, n,
                     b, flag);
}

void launch_factor_inverse(double* slots, int64_t stride, int32_t s, const int32_t* lens, int32_t nb,
                           const int32_t* slot_of, hipStream_t st, FactorCheck chk, const int32_t* skip) {
  if (nb <= 0) return;
  if (s > kLdsCholMax && s <= kFusedMaxBlock) {
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_inverse_blocked<false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kInverseBlockedLds));
      attr_set = true;
    }
    hipLaunchKernelGGL(k_inverse_blocked<false>, dim3(nb), dim3(kT), kInverseBlockedLds, st, slots, stride, s, lens,
                       slot_of, chk, skip);
    return;
  }
  if (s <= kLdsCholMax) {
    const size_t lds = (static_cast<size_t>(s) * (s + 1) + s) * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_factor_inverse<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>((kLdsCholMax * (kLdsCholMax + 1) + kLdsCholMax) * sizeof(double)));
      attr_set = true;
    }
    hipLaunchKernelGGL(k_factor_inverse<true>, dim3(nb), dim3(kT), lds, st, slots, stride, s, lens, slot_of, chk, skip);
  } else {
    hipLaunchKernelGGL(k_factor_inverse<false>, dim3(nb), dim3(kT), 0, st, slots, stride, s, lens, slot_of, chk, skip);
  }
}

void launch_factor_linv(double* slots, int64_t stride, int32_t s, const int32_t* lens, int32_t nb,
                        const int32_t* slot_of, hipStream_t st) {
  if (nb <= 0) return;
  if (s > kLdsCholMax && s <= kFusedMaxBlock) {
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_inverse_blocked<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kInverseBlockedLds));
      attr_set = true;
    }
    hipLaunchKernelGGL(k_inverse_blocked<true>, dim3(nb), dim3(kT), kInverseBlockedLds, st, slots, stride, s, lens,
                       slot_of, FactorCheck(), nullptr);
    return;
  }
  if (s <= kLdsCholMax) {
    const size_t lds = (static_cast<size_t>(s) * (s + 1) + s) * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_factor_inverse<true, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>((kLdsCholMax * (kLdsCholMax + 1) + kLdsCholMax) * sizeof(double)));
      attr_set = true;
    }
    hipLaunchKernelGGL((k_factor_inverse<true, true>), dim3(nb), dim3(kT), lds, st, slots, stride, s, lens, slot_of,
                       FactorCheck(), nullptr);
  } else {
    hipLaunchKernelGGL((k_factor_inverse<false, true>), dim3(nb), dim3(kT), 0, st, slots, stride, s, lens, slot_of,
                       FactorCheck(), nullptr);
  }
}

void launch_factor_small(double* slots, int64_t stride, int32_t s, const int32_t* lens, int32_t nb,
                         const int32_t* slot_of, int32_t want_inverse, int32_t* err, hipStream_t st,
                         FactorCheck chk) {
  if (nb <= 0) return;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_factor_small),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kFactorTiledLds));
    attr_set = true;
  }
  hipLaunchKernelGGL(k_factor_small, dim3(nb), dim3(kT), kFactorTiledLds, st, slots, stride, s, lens, slot_of,
                     want_inverse, err, chk);
}

void launch_scatter_rows(const int32_t* stage_rows, const int32_t* stage_lens, const int32_t* slot_of,
                         int32_t nb, int32_t s, int32_t* rows, int32_t* lens, hipStream_t st) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_scatter_rows, dim3(nb), dim3(kT), 0, st, stage_rows, stage_lens, slot_of, s, rows, lens);
}

void launch_gram_f32(int32_t kind, const float* A, int64_t lda, int64_t n, const int32_t* rows,
                     const int32_t* lens, int32_t s, int32_t nb, double lambda, double* G, int64_t stride,
                     const int32_t* slot_of, double* ws, hipStream_t st) {
  if (nb <= 0) return;
  if (kind == 0) {
    launch_gram_syrk_f32(A, lda, n, rows, lens, s, nb, lambda, G, stride, slot_of, ws, st);
  } else {
    const int32_t* only = nullptr;
    hipLaunchKernelGGL(k_gram_cd<float>, dim3(nb), dim3(kT), 0, st, A, lda, rows, lens, s, lambda, G,
                       stride, slot_of, only);
  }
}

void launch_convert_f32(const double* A, int64_t lda, int64_t m, int64_t n, float* out, hipStream_t st) {
  const int64_t total = m * n;
  const unsigned g = static_cast<unsigned>(std::min<int64_t>((total + kT - 1) / kT, 65536));
  hipLaunchKernelGGL(k_convert_f32, dim3(g), dim3(kT), 0, st, A, lda, m, n, out);
}

void launch_convert_bf16(const double* A, int64_t lda, int64_t m, int64_t n, uint16_t* out, hipStream_t st) {
  const int64_t total = m * n;
  const unsigned g = static_cast<unsigned>(std::min<int64_t>((total + kT - 1) / kT, 65536));
  hipLaunchKernelGGL(k_convert_bf16, dim3(g), dim3(kT), 0, st, A, lda, m, n, out);
}

void launch_residual_vec(const double* A, int64_t lda, int64_t m, int64_t n, const double* x,
                         const double* b, double* r, double* rowsq, double* out, hipStream_t st) {
  const unsigned g = static_cast<unsigned>((m + 3) / 4);
  hipLaunchKernelGGL(k_residual_vec, dim3(g), dim3(kT), 0, st, A, lda, m, n, x, b, r, rowsq);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kT), 0, st, rowsq, m, out);
}

int32_t gemv_t_splits(int64_t m, int64_t n) {
  const int64_t cols = (n + kT - 1) / kT;
  int64_t s = std::max<int64_t>(1, (2048 + cols - 1) / cols);   // about 2048 workgroups
  s = std::min<int64_t>(s, std::max<int64_t>(1, m / 64));          // at least 64 rows each
  return static_cast<int32_t>(std::min<int64_t>(s, 64));
}

void launch_gemv_t(const double* A, int64_t lda, int64_t m, int64_t n, const double* z, double* d, double* ws,
                   hipStream_t st) {
  if (n <= 0) return;
  const int32_t splits = gemv_t_splits(m, n);
  const unsigned cols = static_cast<unsigned>((n + kT - 1) / kT);
  if (splits == 1) {
    hipLaunchKernelGGL(k_gemv_t_part, dim3(cols, 1), dim3(kT), 0, st, A, lda, m, n, z, 1, d);
    return;
  }
  hipLaunchKernelGGL(k_gemv_t_part, dim3(cols, static_cast<unsigned>(splits)), dim3(kT), 0, st, A, lda, m, n, z,
                     splits, ws);
  hipLaunchKernelGGL(k_gemv_t_sum, dim3(cols), dim3(kT), 0, st, ws, n, splits, d);
}

void launch_axpy1(double* x, const double* d, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy1, dim3(static_cast<unsigned>((n + kT - 1) / kT)), dim3(kT), 0, st, x, d, n);
}

void launch_state_init(DevState* ds, double rho0, double thr, int32_t* err, double* mom, int64_t n, hipStream_t st) {
  const int64_t g = std::max<int64_t>(1, std::min<int64_t>((n + kT - 1) / kT, 1024));
  hipLaunchKernelGGL(k_state_init, dim3(static_cast<unsigned>(g)), dim3(kT), 0, st, ds, rho0, thr, err, mom, n);
}

void launch_zero3(double* a, int64_t na, double* b, int64_t nb, double* c, int64_t nc, hipStream_t st) {
  const int64_t n = std::max(na, std::max(nb, nc));
  if (n <= 0) return;
  const int64_t g = std::min<int64_t>((n + kT - 1) / kT, 1024);
  hipLaunchKernelGGL(k_zero3, dim3(static_cast<unsigned>(g)), dim3(kT), 0, st, a, na, b, nb, c, nc);
}

}  // namespace kpp
