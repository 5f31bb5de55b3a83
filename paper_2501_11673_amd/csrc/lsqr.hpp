// Internal launchers of the sketch-preconditioned LSQR projection of
// Kaczmarz++ (Section 4.1; the Proj routine of Algorithm 5).  Not part of the
// C ABI.
//
// With L the lower Cholesky factor of A_hat A_hat^T + lambda I (A_hat = A_S
// Pi^T, the SRHT sketch), Proj runs LSQR on M = L^{-1} [A_S, sqrt(lambda) I].
// Every vector LSQR forms in the column space of M, v = M^T u - beta v, has
// the form [A_S^T z; sqrt(lambda) z] for some z in R^s, so the iteration is
// carried in those s coordinates: a v is its z, ||v||^2 = ||A_S^T z||^2 +
// lambda ||z||^2, M v = L^{-1} (A_S (A_S^T z) + lambda z), M^T u = the z
// L^{-T} u.  The n-vectors are never stored beyond p = A_S^T z of the current
// iteration, and the result w = A_S^T z_x is formed by the step's update
// kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace kpp {

// Device state of one LSQR solve (one step).  Vectors are indexed by block row.
struct LsqrState {
  double alpha, beta, phibar, rhobar, pscale;
  int32_t live;   // 0 once the iteration has stopped (a zero norm or rotation)
  int32_t pad;
  double u[kMaxBlock];
  double zv[kMaxBlock];   // current v
  double zw[kMaxBlock];   // LSQR's search direction w
  double zx[kMaxBlock];   // the iterate x (its first n entries are A_S^T zx)
  double zt[kMaxBlock];   // M^T u - beta v before normalisation
  double ut[kMaxBlock];   // M v - alpha u before normalisation
};

// L^{-1} of each slot's factor at +s*s, column-major (entry (i, k) at k s + i),
// zero above the diagonal, so y_i = sum_k slot[s s + k s + i] r_k is L^{-1} r;
// and L^{-T} the same way at +2 s*s.
void launch_factor_linv(double* slots, int64_t stride, int32_t s, const int32_t* lens, int32_t nb,
                        const int32_t* slot_of, hipStream_t st);

// Xt (n x s, row-major) = A_S^T for the sb rows of one block (columns past sb: 0).
void launch_sketch_gather(const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb, int32_t s,
                          double* Xt, hipStream_t st);
// Ahat (s x tau, row-major) = scale * Y[T[k], i] for i < sb (rows past sb: 0),
// Y (N x s) = H D [A_S, 0]^T.
void launch_sketch_select(const double* Y, int32_t s, const int32_t* T, int32_t tau, int32_t sb, double scale,
                          double* Ahat, hipStream_t st);

// LSQR from z = 0 on M z = y, y = L^{-1} r (left in y by the projection
// kernel): beta_1, u_1, and z~ = L^{-T} u_1.  Linv points at the slot's
// L^{-1}; L^{-T} follows it.
void launch_lsqr_start(const double* y, const double* Linv, int32_t s, int32_t sb, LsqrState* L, hipStream_t st);
// p = A_S^T z~ (n entries) and the lsqr_at_groups(n) workgroup partial sums
// of ||p||^2; ppart holds lsqr_at_chunks(sb) x n partial products.
int32_t lsqr_at_groups(int64_t n);
int32_t lsqr_at_chunks(int32_t s);
void launch_lsqr_at(const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb, const LsqrState* L,
                    double* ppart, double* p, double* partsq, hipStream_t st);
// alpha = sqrt(||p||^2 + lambda ||z~||^2), v = z~ / alpha; first: set up the
// recurrences, else: one plane rotation and the updates of x and w.
void launch_lsqr_post(const double* partsq, int32_t ngroups, int32_t sb, double lambda, int32_t first, LsqrState* L,
                      hipStream_t st);
// M v = L^{-1} (A_S p pscale + lambda v) from the partial sums of A_S p,
// u = (M v - alpha u) / beta, z~ = L^{-T} u - beta v.
void launch_lsqr_mid(const double* rpart, int32_t P, const double* Linv, int32_t s, int32_t sb, double lambda,
                     LsqrState* L, hipStream_t st);

}  // namespace kpp
