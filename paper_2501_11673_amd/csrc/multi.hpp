// Internal launchers of the several-right-hand-side solve (kpp_solve_multi):
// k systems A x_c = b_c on one A share the block schedule, the memoized
// factors and every pass over A_S; each keeps its own momentum, window sums
// and adaptive rho (Algorithms 2 and 5 run k times in lockstep).  X, M and B
// are row-major with k values per row (leading dimension ld >= k).  Not part
// of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace kpp {

constexpr int kMaxRhs = 32;
constexpr int64_t kGemmChunk = 256;   // columns of A per partial of the block product
inline int32_t gemm_parts(int64_t n) { return static_cast<int32_t>((n + kGemmChunk - 1) / kGemmChunk); }

// rpart[(i P + p) k + c] = sum_{j in chunk p} A[rows[i], j] X[j, c], P = gemm_parts(n)
// (FP64 matrix cores)
void launch_block_gemm_partial(const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb,
                               const double* X, int64_t ldx, int32_t k, double* rpart, int32_t P, hipStream_t st);
// per right-hand side c with frozen[c] == 0: r_c = sum_p rpart - B[rows, c],
// the step's bookkeeping in ds[c], and Y[c s + i] = (G^{-1} r_c)_i
void launch_block_project_multi(const double* rpart, int32_t P, int32_t k, const double* B, int64_t ldb,
                                const int32_t* rows, int32_t sb, const double* Ginv, int32_t s, double* Y,
                                DevState* ds, const int32_t* frozen, int32_t zeta, int32_t adaptive, hipStream_t st);
// per c with frozen[c] == 0: w = A_S^T y_c (Kaczmarz++) or I_S^T y_c (CD++),
// M[:, c] <- c_c (M[:, c] - w), X[:, c] <- X[:, c] - w + eta M[:, c]
void launch_update_multi(int32_t kind, const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb,
                         const double* Y, int32_t s, int32_t k, const DevState* ds, const int32_t* frozen, double eta,
                         double* X, int64_t ldx, double* M, hipStream_t st);
// out[j] = X[j * ldx + c] for j < n (a column into a contiguous vector)
void launch_column(const double* X, int64_t ldx, int64_t n, int32_t c, double* out, hipStream_t st);

}  // namespace kpp
