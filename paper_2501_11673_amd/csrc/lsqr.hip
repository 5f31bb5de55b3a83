// Sketch-preconditioned LSQR projection of Kaczmarz++ (Section 4.1; the Proj
// routine of Algorithm 5), carried in the s coordinates described in
// lsqr.hpp.  LSQR is Paige and Saunders' algorithm (Golub-Kahan
// bidiagonalization with one plane rotation per iteration).  For s above 128
// the products with L^{-1} and L^{-T} split the s rows over workgroups of 16
// rows each (below, one workgroup does them); the rotation runs in one
// workgroup; the two products with A_S per
// iteration run across the device (k_lsqr_at here, the block gemv of the
// exact path for A_S p).
#include <cstddef>

#include "lsqr.hpp"

namespace kpp {
namespace {

constexpr int kL = 256;        // threads per workgroup of the column kernels
constexpr int kS = 1024;       // threads of the one-workgroup kernels on s-vectors
constexpr int kSRows = 256;    // output rows per pass of those kernels (4 threads each)
constexpr int kAtRows = 16;    // block rows per workgroup of the A_S^T z pass
constexpr int kMidRows = 16;   // rows per workgroup of the L^{-1} and L^{-T} products (16 k-lanes each)
constexpr int kMidOneGroup = 128;   // largest s whose products stay in one workgroup

// sum over the workgroup of NT threads, in every thread (fixed order)
template <int NT>
__device__ double wg_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < NT / 64; ++i) t += red[i];
  return t;
}

// out_i = sum_k B[k s + i] v_k for i < sb (B column-major, s x s): thread
// (i mod 256, part) sums k = part, part + 4, ..., the four parts are added in
// a fixed order.  v and out in LDS; ends with a barrier.
__device__ void mv_colmajor(const double* __restrict__ B, int32_t s, int32_t sb, const double* v, double* out,
                            double* part4) {
  const int i0 = threadIdx.x & (kSRows - 1), pt = threadIdx.x / kSRows;
  for (int ib = 0; ib < sb; ib += kSRows) {
    const int i = ib + i0;
    double a0 = 0.0, a1 = 0.0;
    if (i < sb) {
      int k = pt;
      for (; k + 4 < sb; k += 8) {
        a0 = fma(B[static_cast<int64_t>(k) * s + i], v[k], a0);
        a1 = fma(B[static_cast<int64_t>(k + 4) * s + i], v[k + 4], a1);
      }
      if (k < sb) a0 = fma(B[static_cast<int64_t>(k) * s + i], v[k], a0);
    }
    part4[pt * kSRows + i0] = a0 + a1;
    __syncthreads();
    if (pt == 0 && i < sb)
      out[i] = (part4[i0] + part4[kSRows + i0]) + (part4[2 * kSRows + i0] + part4[3 * kSRows + i0]);
    __syncthreads();
  }
}

// Xt[j s + i] = A[rows[i], j] (0 for i >= sb): a 64 x 64 tile (columns j0..,
// block rows i0..) is read along A's rows and written along Xt's rows through
// LDS, so both sides are coalesced
constexpr int kGatherTile = 64;
__global__ __launch_bounds__(kL) void k_sketch_gather(const double* __restrict__ A, int64_t lda, int64_t n,
                                                      const int32_t* __restrict__ rows, int32_t sb, int32_t s,
                                                      double* __restrict__ Xt) {
  __shared__ double tile[kGatherTile][kGatherTile + 1];
  const int64_t j0 = static_cast<int64_t>(blockIdx.x) * kGatherTile;
  const int i0 = blockIdx.y * kGatherTile;
  const int tx = threadIdx.x & (kGatherTile - 1), ty = threadIdx.x / kGatherTile;
  for (int r = ty; r < kGatherTile; r += kL / kGatherTile) {
    const int i = i0 + r;
    const int64_t j = j0 + tx;
    tile[r][tx] = (i < sb && j < n) ? A[static_cast<int64_t>(rows[i]) * lda + j] : 0.0;
  }
  __syncthreads();
  for (int c = ty; c < kGatherTile; c += kL / kGatherTile) {
    const int64_t j = j0 + c;
    const int i = i0 + tx;
    if (j < n && i < s) Xt[j * s + i] = tile[tx][c];
  }
}

__global__ __launch_bounds__(kL) void k_sketch_select(const double* __restrict__ Y, int32_t s,
                                                      const int32_t* __restrict__ T, int32_t tau, int32_t sb,
                                                      double scale, double* __restrict__ Ahat) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kL + threadIdx.x;
  if (e >= static_cast<int64_t>(s) * tau) return;
  const int i = static_cast<int>(e / tau), k = static_cast<int>(e % tau);
  Ahat[e] = i < sb ? scale * Y[static_cast<int64_t>(T[k]) * s + i] : 0.0;
}

__global__ __launch_bounds__(kS) void k_lsqr_start(const double* __restrict__ y, const double* __restrict__ Lt,
                                                   int32_t s, int32_t sb, LsqrState* __restrict__ L) {
  __shared__ double red[kS / 64];
  __shared__ double u[kMaxBlock];
  __shared__ double zt[kMaxBlock];
  __shared__ double part4[4 * kSRows];
  double acc = 0.0;
  for (int i = threadIdx.x; i < sb; i += kS) acc = fma(y[i], y[i], acc);
  const double beta = sqrt(wg_sum<kS>(acc, red));
  for (int i = threadIdx.x; i < sb; i += kS) {
    L->zx[i] = 0.0;
    u[i] = beta > 0.0 ? y[i] / beta : 0.0;
    L->u[i] = u[i];
  }
  __syncthreads();
  mv_colmajor(Lt, s, sb, u, zt, part4);   // z~ = L^{-T} u
  for (int i = threadIdx.x; i < sb; i += kS) L->zt[i] = zt[i];
  if (threadIdx.x == 0) {
    L->beta = beta;
    L->phibar = beta;
    L->live = beta > 0.0 ? 1 : 0;
  }
}

// p_part[c n + j] = sum over block rows 16 c .. 16 c + 15 of A[rows[i], j] z~_i
__global__ __launch_bounds__(kL) void k_lsqr_at(const double* __restrict__ A, int64_t lda, int64_t n,
                                                const int32_t* __restrict__ rows, int32_t sb,
                                                const LsqrState* __restrict__ L, double* __restrict__ ppart) {
  if (!L->live) return;   // uniform over the grid
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kL + threadIdx.x;
  const int i0 = blockIdx.y * kAtRows;
  const int i1 = min(sb, i0 + kAtRows);
  if (j >= n) return;
  double acc = 0.0;
  for (int i = i0; i < i1; ++i) acc = fma(A[static_cast<int64_t>(rows[i]) * lda + j], L->zt[i], acc);
  ppart[static_cast<int64_t>(blockIdx.y) * n + j] = acc;
}

// p = the sum of the row-chunk parts (fixed order), and the workgroup partial
// sums of ||p||^2
__global__ __launch_bounds__(kL) void k_lsqr_at_sum(const double* __restrict__ ppart, int32_t nchunks, int64_t n,
                                                    const LsqrState* __restrict__ L, double* __restrict__ p,
                                                    double* __restrict__ partsq) {
  __shared__ double red[kL / 64];
  if (!L->live) return;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kL + threadIdx.x;
  double acc = 0.0;
  if (j < n) {
    for (int c = 0; c < nchunks; ++c) acc += ppart[static_cast<int64_t>(c) * n + j];
    p[j] = acc;
  }
  const double sq = wg_sum<kL>(acc * acc, red);
  if (threadIdx.x == 0) partsq[blockIdx.x] = sq;
}

__global__ __launch_bounds__(kL) void k_lsqr_post(const double* __restrict__ partsq, int32_t ngroups, int32_t sb,
                                                  double lambda, int32_t first, LsqrState* __restrict__ L) {
  __shared__ double red[kL / 64];
  __shared__ double sh[4];
  if (!L->live) return;
  double zz = 0.0;
  for (int i = threadIdx.x; i < sb; i += kL) zz = fma(L->zt[i], L->zt[i], zz);
  zz = wg_sum<kL>(zz, red);
  if (threadIdx.x == 0) {
    double pp = 0.0;
    for (int g = 0; g < ngroups; ++g) pp += partsq[g];
    const double alpha = sqrt(pp + lambda * zz);
    double coef_x = 0.0, coef_w = 0.0;
    int live = 1;
    if (first) {
      if (!(alpha > 0.0)) live = 0;
      L->rhobar = alpha;
    } else {
      const double rho = hypot(L->rhobar, L->beta);
      if (rho == 0.0) {
        live = 0;
      } else {
        const double c = L->rhobar / rho, sn = L->beta / rho;
        const double theta = sn * alpha;
        L->rhobar = -c * alpha;
        const double phi = c * L->phibar;
        L->phibar = sn * L->phibar;
        coef_x = phi / rho;
        coef_w = theta / rho;
      }
    }
    L->alpha = alpha;
    L->pscale = alpha > 0.0 ? 1.0 / alpha : 0.0;
    sh[0] = alpha;
    sh[1] = coef_x;
    sh[2] = coef_w;
    sh[3] = live;
  }
  __syncthreads();
  const double alpha = sh[0], coef_x = sh[1], coef_w = sh[2];
  const bool live = sh[3] != 0.0;
  if (!live) {
    if (threadIdx.x == 0) L->live = 0;
    return;
  }
  for (int i = threadIdx.x; i < sb; i += kL) {
    const double v = alpha > 0.0 ? L->zt[i] / alpha : L->zt[i];
    if (first) {
      L->zw[i] = v;
    } else {
      // x <- x + (phi / rho) w with the old w, then w <- v - (theta / rho) w
      const double w = L->zw[i];
      L->zx[i] = fma(coef_x, w, L->zx[i]);
      L->zw[i] = v - coef_w * w;
    }
    L->zv[i] = v;
  }
}

// M v = L^{-1} (A_S p pscale + lambda v) from the partial sums of A_S p,
// u = (M v - alpha u) / beta, z~ = L^{-T} u - beta v, in one workgroup (the
// form for s <= kMidOneGroup, where a second launch costs more than the
// products save when split)
__global__ __launch_bounds__(kS) void k_lsqr_mid(const double* __restrict__ rpart, int32_t P,
                                                 const double* __restrict__ Li, const double* __restrict__ Lt,
                                                 int32_t s, int32_t sb, double lambda, LsqrState* __restrict__ L) {
  __shared__ double red[kS / 64];
  __shared__ double t[kMaxBlock];
  __shared__ double u[kMaxBlock];
  __shared__ double part4[4 * kSRows];
  if (!L->live) return;
  const double pscale = L->pscale, alpha = L->alpha;
  for (int i = threadIdx.x; i < sb; i += kS) {
    double q = 0.0;
    for (int k = 0; k < P; ++k) q += rpart[static_cast<int64_t>(i) * P + k];
    t[i] = fma(lambda, L->zv[i], q * pscale);
  }
  __syncthreads();
  mv_colmajor(Li, s, sb, t, u, part4);   // L^{-1} t
  double acc = 0.0;
  for (int i = threadIdx.x; i < sb; i += kS) {
    const double ui = u[i] - alpha * L->u[i];   // u~ = M v - alpha u
    u[i] = ui;
    acc = fma(ui, ui, acc);
  }
  const double beta = sqrt(wg_sum<kS>(acc, red));
  for (int i = threadIdx.x; i < sb; i += kS) {
    if (beta > 0.0) u[i] /= beta;
    L->u[i] = u[i];
  }
  __syncthreads();
  mv_colmajor(Lt, s, sb, u, t, part4);   // L^{-T} u
  for (int i = threadIdx.x; i < sb; i += kS) L->zt[i] = t[i] - beta * L->zv[i];
  if (threadIdx.x == 0) L->beta = beta;
}


// Rows 16 b .. 16 b + 15 of B v (B column-major, s x s; v in LDS): thread
// (r, kk) = (tid mod 16, tid / 16) sums k = kk, kk + 16, ..., and the 16
// partial sums of a row are added in a fixed order by thread r.  Returns the
// row's value in threads 0..15 (0 elsewhere); ends with a barrier.
__device__ double mv_rows16(const double* __restrict__ B, int32_t s, int32_t sb, const double* v,
                            double (*part)[kMidRows + 1]) {
  const int r = threadIdx.x & (kMidRows - 1), kk = threadIdx.x / kMidRows;
  const int i = blockIdx.x * kMidRows + r;
  double acc = 0.0;
  if (i < sb)
    for (int k = kk; k < sb; k += kL / kMidRows) acc = fma(B[static_cast<int64_t>(k) * s + i], v[k], acc);
  part[kk][r] = acc;
  __syncthreads();
  double y = 0.0;
  if (threadIdx.x < kMidRows)
    for (int q = 0; q < kL / kMidRows; ++q) y += part[q][threadIdx.x];
  __syncthreads();
  return y;
}

// u~ = M v - alpha u = L^{-1} (A_S p pscale + lambda v) - alpha u, its rows
// of this workgroup, from the partial sums of A_S p (every workgroup forms
// the whole s-vector it multiplies)
__global__ __launch_bounds__(kL) void k_lsqr_mid_a(const double* __restrict__ rpart, int32_t P,
                                                   const double* __restrict__ Li, int32_t s, int32_t sb,
                                                   double lambda, LsqrState* __restrict__ L) {
  __shared__ double t[kMaxBlock];
  __shared__ double part[kL / kMidRows][kMidRows + 1];
  if (!L->live) return;   // uniform over the grid
  const double pscale = L->pscale, alpha = L->alpha;
  for (int k = threadIdx.x; k < sb; k += kL) {
    double q = 0.0;
    for (int c = 0; c < P; ++c) q += rpart[static_cast<int64_t>(k) * P + c];
    t[k] = fma(lambda, L->zv[k], q * pscale);
  }
  __syncthreads();
  const double y = mv_rows16(Li, s, sb, t, part);
  const int i = blockIdx.x * kMidRows + threadIdx.x;
  if (threadIdx.x < kMidRows && i < sb) L->ut[i] = y - alpha * L->u[i];
}

// beta = ||u~||, u = u~ / beta, and this workgroup's rows of
// z~ = L^{-T} u - beta v (every workgroup forms beta and u the same way).
// START: the first LSQR iteration from z = 0 with u~ = src = L^{-1} r, so
// z~ = L^{-T} u, x = 0, and the recurrences start (as k_lsqr_start).
template <bool START>
__global__ __launch_bounds__(kL) void k_lsqr_mid_b(const double* __restrict__ src, const double* __restrict__ Lt,
                                                   int32_t s, int32_t sb, LsqrState* __restrict__ L) {
  __shared__ double red[kL / 64];
  __shared__ double u[kMaxBlock];
  __shared__ double part[kL / kMidRows][kMidRows + 1];
  if (!START && !L->live) return;
  double acc = 0.0;
  for (int k = threadIdx.x; k < sb; k += kL) acc = fma(src[k], src[k], acc);
  const double beta = sqrt(wg_sum<kL>(acc, red));
  for (int k = threadIdx.x; k < sb; k += kL) u[k] = beta > 0.0 ? src[k] / beta : (START ? 0.0 : src[k]);
  __syncthreads();
  const double y = mv_rows16(Lt, s, sb, u, part);
  const int i = blockIdx.x * kMidRows + threadIdx.x;
  if (threadIdx.x < kMidRows && i < sb) {
    L->u[i] = u[i];
    if (START) {
      L->zt[i] = y;
      L->zx[i] = 0.0;
    } else {
      L->zt[i] = y - beta * L->zv[i];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    L->beta = beta;
    if (START) {
      L->phibar = beta;
      L->live = beta > 0.0 ? 1 : 0;
    }
  }
}

}  // namespace

void launch_sketch_gather(const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb, int32_t s,
                          double* Xt, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n + kGatherTile - 1) / kGatherTile),
                  static_cast<unsigned>((s + kGatherTile - 1) / kGatherTile));
  hipLaunchKernelGGL(k_sketch_gather, grid, dim3(kL), 0, st, A, lda, n, rows, sb, s, Xt);
}

void launch_sketch_select(const double* Y, int32_t s, const int32_t* T, int32_t tau, int32_t sb, double scale,
                          double* Ahat, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(s) * tau;
  hipLaunchKernelGGL(k_sketch_select, dim3(static_cast<unsigned>((total + kL - 1) / kL)), dim3(kL), 0, st, Y, s, T,
                     tau, sb, scale, Ahat);
}

void launch_lsqr_start(const double* y, const double* Linv, int32_t s, int32_t sb, LsqrState* L, hipStream_t st) {
  const double* Lt = Linv + static_cast<int64_t>(s) * s;
  if (s <= kMidOneGroup) {
    hipLaunchKernelGGL(k_lsqr_start, dim3(1), dim3(kS), 0, st, y, Lt, s, sb, L);
    return;
  }
  const unsigned g = static_cast<unsigned>((sb + kMidRows - 1) / kMidRows);
  hipLaunchKernelGGL(k_lsqr_mid_b<true>, dim3(g), dim3(kL), 0, st, y, Lt, s, sb, L);
}

int32_t lsqr_at_groups(int64_t n) { return static_cast<int32_t>((n + kL - 1) / kL); }

int32_t lsqr_at_chunks(int32_t s) { return (s + kAtRows - 1) / kAtRows; }

void launch_lsqr_at(const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb, const LsqrState* L,
                    double* ppart, double* p, double* partsq, hipStream_t st) {
  const int32_t nch = lsqr_at_chunks(sb);
  const unsigned gx = static_cast<unsigned>(lsqr_at_groups(n));
  hipLaunchKernelGGL(k_lsqr_at, dim3(gx, static_cast<unsigned>(nch)), dim3(kL), 0, st, A, lda, n, rows, sb, L, ppart);
  hipLaunchKernelGGL(k_lsqr_at_sum, dim3(gx), dim3(kL), 0, st, ppart, nch, n, L, p, partsq);
}

void launch_lsqr_post(const double* partsq, int32_t ngroups, int32_t sb, double lambda, int32_t first, LsqrState* L,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_lsqr_post, dim3(1), dim3(kL), 0, st, partsq, ngroups, sb, lambda, first, L);
}

void launch_lsqr_mid(const double* rpart, int32_t P, const double* Linv, int32_t s, int32_t sb, double lambda,
                     LsqrState* L, hipStream_t st) {
  const double* Lt = Linv + static_cast<int64_t>(s) * s;
  if (s <= kMidOneGroup) {
    hipLaunchKernelGGL(k_lsqr_mid, dim3(1), dim3(kS), 0, st, rpart, P, Linv, Lt, s, sb, lambda, L);
    return;
  }
  const unsigned g = static_cast<unsigned>((sb + kMidRows - 1) / kMidRows);
  hipLaunchKernelGGL(k_lsqr_mid_a, dim3(g), dim3(kL), 0, st, rpart, P, Linv, s, sb, lambda, L);
  const double* ut = reinterpret_cast<const double*>(reinterpret_cast<const char*>(L) + offsetof(LsqrState, ut));
  hipLaunchKernelGGL(k_lsqr_mid_b<false>, dim3(g), dim3(kL), 0, st, ut, Lt, s, sb, L);
}

}  // namespace kpp
