// Regularized block Grams of Kaczmarz++ on the matrix cores (memo miss path,
// Algorithm 1 and Section 5.2): G = A_S A_S^T + lambda I for nb blocks at once.
//
// The s x s lower triangle is cut into 64 x 64 tiles and the n columns into
// chunks; one workgroup forms one tile over one chunk with 16 x 16 x 4 MFMA
// products (FP64, or FP32 inputs with FP32 accumulation for the mixed-precision
// path), staging 64 x 32 panels of both row groups in LDS.  The per-chunk
// partial tiles go to a workspace in FP64 and a second kernel sums them in
// chunk order (deterministic), adds lambda on the diagonal and writes the
// lower triangle of the column-major slot.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace kpp {
namespace {

constexpr int kGT = kGramTile;    // output tile edge
constexpr int kKc = kGramPanel;   // columns per LDS panel
constexpr int kGThreads = 256;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename TA>
struct Mfma;
// D = X Y with X 16 x 4 (lane l holds X[l % 16][l / 16]) and Y 4 x 16 (lane l
// holds Y[l / 16][l % 16]); register r of lane l holds D[row(l, r)][l % 16],
// where the row order differs between the two instructions (measured on gfx950).
template <>
struct Mfma<double> {
  using acc_t = v4d;
  static __device__ __forceinline__ v4d step(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
  using acc_t = v4f;
  static __device__ __forceinline__ v4f step(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// t-th tile of the lower triangle in row order -> (ti, tj), ti >= tj
__device__ __forceinline__ void tile_coords(int t, int& ti, int& tj) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  ti = i;
  tj = t - i * (i + 1) / 2;
}

// Partial tile P[i][j] = sum_{k in chunk} A[r_i, k] A[r_j, k] for block rows
// i in tile row ti, j in tile column tj.  The MFMA takes rows of tile tj as
// its first operand and rows of tile ti as its second, so lane l, register r
// holds P[i0 + 16x + l % 16][j0 + 16y + row(l, r)] and the column-major tile
// store is contiguous across lanes.
template <typename TA>
__global__ __launch_bounds__(kGThreads) void k_gram_syrk(const TA* __restrict__ A, int64_t lda, int64_t n,
                                                         const int32_t* __restrict__ rows,
                                                         const int32_t* __restrict__ lens, int32_t s,
                                                         const int32_t* __restrict__ only, int32_t nchunks,
                                                         int64_t chunk, int32_t ntiles, double* __restrict__ ws) {
  using Acc = typename Mfma<TA>::acc_t;
  __shared__ TA Ps[kGT][kKc + 1];   // rows of tile ti
  __shared__ TA Qs[kGT][kKc + 1];   // rows of tile tj (unused on diagonal tiles)
  __shared__ int32_t ri[kGT], rj[kGT];
  const int ch = blockIdx.x, t = blockIdx.y, blk = blockIdx.z;
  if (only && !only[blk]) return;
  const int sb = lens[blk];
  int ti, tj;
  tile_coords(t, ti, tj);
  const int i0 = ti * kGT, j0 = tj * kGT;
  if (i0 >= sb) return;  // uniform over the workgroup
  const bool diag = ti == tj;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int32_t* R = rows + static_cast<int64_t>(blk) * s;
  if (tid < kGT) {
    ri[tid] = R[min(i0 + tid, sb - 1)];
    rj[tid] = R[min(j0 + tid, sb - 1)];
  }
  __syncthreads();
  const int64_t k_begin = static_cast<int64_t>(ch) * chunk;
  const int64_t k_end = min(n, k_begin + chunk);

  // panel element e = tid + 256 q: row e / 32, column e % 32 (a wave reads two
  // contiguous row segments per load)
  TA pv[8], qv[8];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + kGThreads * q;
      const int r = e >> 5, c = e & 31;
      const int64_t k = k0 + c;
      const bool ok_k = k < k_end;
      pv[q] = (ok_k && i0 + r < sb) ? A[static_cast<int64_t>(ri[r]) * lda + k] : TA(0);
      if (!diag) qv[q] = (ok_k && j0 + r < sb) ? A[static_cast<int64_t>(rj[r]) * lda + k] : TA(0);
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + kGThreads * q;
      const int r = e >> 5, c = e & 31;
      Ps[r][c] = pv[q];
      if (!diag) Qs[r][c] = qv[q];
    }
  };

  // wave wv forms the 32 x 32 quadrant (rows 32 (wv >> 1), columns 32 (wv & 1));
  // on a diagonal tile the strictly upper quadrant is not needed
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
  const bool active = !(diag && wr < wc);
  TA(*Qp)[kKc + 1] = diag ? Ps : Qs;
  Acc acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = Acc{0, 0, 0, 0};

  fetch(k_begin);
  for (int64_t k0 = k_begin; k0 < k_end; k0 += kKc) {
    __syncthreads();  // the previous panel is consumed
    stash();
    __syncthreads();
    if (k0 + kKc < k_end) fetch(k0 + kKc);
    if (active) {
      const int li = lane & 15, lk = lane >> 4;
#pragma unroll
      for (int kk = 0; kk < kKc; kk += 4) {
        const TA a0 = Qp[wc + li][kk + lk], a1 = Qp[wc + 16 + li][kk + lk];
        const TA b0 = Ps[wr + li][kk + lk], b1 = Ps[wr + 16 + li][kk + lk];
        acc[0][0] = Mfma<TA>::step(a0, b0, acc[0][0]);
        acc[0][1] = Mfma<TA>::step(a1, b0, acc[0][1]);
        acc[1][0] = Mfma<TA>::step(a0, b1, acc[1][0]);
        acc[1][1] = Mfma<TA>::step(a1, b1, acc[1][1]);
      }
    }
  }
  if (!active) return;
  // acc[x][y]: rows wr + 16x + (lane % 16), columns wc + 16y + row(lane, r)
  double* W = ws + ((static_cast<int64_t>(blk) * ntiles + t) * nchunks + ch) * (kGT * kGT);
  const int li = lane & 15;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wr + 16 * x + li, j = wc + 16 * y + Mfma<TA>::row(lane, r);
        W[j * kGT + i] = static_cast<double>(acc[x][y][r]);
      }
}

// G[slot][j * s + i] = sum over chunks of the partial tiles (+ lambda on the
// diagonal), lower triangle only
__global__ __launch_bounds__(kGThreads) void k_gram_reduce(const double* __restrict__ ws, const int32_t* __restrict__ lens,
                                                           int32_t s, const int32_t* __restrict__ only,
                                                           int32_t nchunks, int32_t ntiles, double lambda,
                                                           double* __restrict__ G, int64_t stride,
                                                           const int32_t* __restrict__ slot_of) {
  const int t = blockIdx.x, blk = blockIdx.y;
  if (only && !only[blk]) return;
  const int sb = lens[blk];
  int ti, tj;
  tile_coords(t, ti, tj);
  const int i0 = ti * kGT, j0 = tj * kGT;
  if (i0 >= sb) return;
  const double* W = ws + (static_cast<int64_t>(blk) * ntiles + t) * nchunks * (kGT * kGT);
  double* Gb = G + static_cast<int64_t>(slot_of[blk]) * stride;
  for (int e = threadIdx.x; e < kGT * kGT; e += kGThreads) {
    const int i = i0 + (e & (kGT - 1)), j = j0 + (e >> 6);
    if (i >= sb || j >= sb || i < j) continue;
    double acc = 0.0;
    for (int c = 0; c < nchunks; ++c) acc += W[static_cast<int64_t>(c) * kGT * kGT + e];
    Gb[static_cast<int64_t>(j) * s + i] = acc + (i == j ? lambda : 0.0);
  }
}

}  // namespace

template <typename TA>
static void launch_syrk(const TA* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens, int32_t s,
                        int32_t nb, double lambda, double* G, int64_t stride, const int32_t* slot_of,
                        const int32_t* only, double* ws, hipStream_t st) {
  int32_t nc, nt;
  int64_t chunk;
  gram_syrk_plan(s, n, nb, &nc, &chunk, &nt);
  hipLaunchKernelGGL(k_gram_syrk<TA>, dim3(nc, nt, nb), dim3(kGThreads), 0, st, A, lda, n, rows, lens, s, only, nc,
                     chunk, nt, ws);
  hipLaunchKernelGGL(k_gram_reduce, dim3(nt, nb), dim3(kGThreads), 0, st, ws, lens, s, only, nc, nt, lambda, G,
                     stride, slot_of);
}

void launch_gram_syrk(const double* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens, int32_t s,
                      int32_t nb, double lambda, double* G, int64_t stride, const int32_t* slot_of,
                      const int32_t* only, double* ws, hipStream_t st) {
  if (nb <= 0) return;
  launch_syrk<double>(A, lda, n, rows, lens, s, nb, lambda, G, stride, slot_of, only, ws, st);
}

void launch_gram_syrk_capped(const double* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens,
                             int32_t s, int32_t nb, double lambda, double* G, int64_t stride, const int32_t* slot_of,
                             double* ws, size_t max_work, hipStream_t st) {
  if (nb <= 0) return;
  int32_t nc, nt;
  int64_t chunk;
  gram_syrk_plan_capped(s, n, nb, max_work, &nc, &chunk, &nt);
  hipLaunchKernelGGL(k_gram_syrk<double>, dim3(nc, nt, nb), dim3(kGThreads), 0, st, A, lda, n, rows, lens, s,
                     nullptr, nc, chunk, nt, ws);
  hipLaunchKernelGGL(k_gram_reduce, dim3(nt, nb), dim3(kGThreads), 0, st, ws, lens, s, nullptr, nc, nt, lambda, G,
                     stride, slot_of);
}

void launch_gram_syrk_f32(const float* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens, int32_t s,
                          int32_t nb, double lambda, double* G, int64_t stride, const int32_t* slot_of,
                          double* ws, hipStream_t st) {
  if (nb <= 0) return;
  launch_syrk<float>(A, lda, n, rows, lens, s, nb, lambda, G, stride, slot_of, nullptr, ws, st);
}

}  // namespace kpp
