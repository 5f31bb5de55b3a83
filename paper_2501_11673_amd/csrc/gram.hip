// Regularized block Grams of Kaczmarz++ on the matrix cores (memo miss path,
// Algorithm 1 and Section 5.2): G = A_S A_S^T + lambda I for nb blocks at once.
//
// One workgroup forms every 16 x 16 tile of one block's lower triangle over
// one chunk of the n columns.  The block's rows are cut into NG groups of 16
// (s <= 16 NG); per chunk the rows are staged in LDS panels of KC columns
// (double-buffered: the next panel's loads are in flight while the matrix
// cores work on the current one), so every entry of A_S is read once.  Tile
// (i, j) is the 16x16x4 MFMA product of row group i with row group j (FP64,
// or FP32 inputs with FP32 accumulation for the mixed-precision path); the
// waves take the tiles round-robin.  The per-chunk partial tiles go to a
// workspace in FP64 and a second kernel sums them in chunk order
// (deterministic), adds lambda on the diagonal and writes the lower triangle
// of the column-major slot.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace kpp {
namespace {

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

// Shape of the Gram kernel for NG row groups: waves, panel width, lower tiles,
// tiles per wave and tile parts (workgroups per block and chunk).
// The 128-row shape (NG = 8) runs eight waves of 64 registers (16-column
// panels, three tiles per wave, two workgroups per block and chunk), so that
// it fits beside a resident step kernel on every SIMD: the memo-miss path
// runs concurrently with the step kernel.
template <int NG>
struct GramShape {
  static constexpr int NW = NG <= 4 ? 4 : 8;
  static constexpr int KC = NG <= 4 ? 32 : (NG <= 16 ? 16 : 8);
  static constexpr int R = 16 * NG;
  static constexpr int NTILE = NG * (NG + 1) / 2;
  static constexpr int TPW = NG == 8 ? 3 : (NG <= 16 ? (NTILE + NW - 1) / NW : 17);
  static constexpr int PARTS = (NTILE + NW * TPW - 1) / (NW * TPW);
  static constexpr int LOADS = R * KC / (NW * 64);   // panel entries per thread
};

// t-th tile of the lower triangle in row order -> (ti, tj), ti >= tj
__device__ __forceinline__ void tile_coords(int t, int& ti, int& tj) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  ti = i;
  tj = t - i * (i + 1) / 2;
}

// Partial tiles of block blockIdx.z over chunk blockIdx.x (tile part
// blockIdx.y): ws[((blk * nchunks + ch) * ntiles + t) * 256 + a * 16 + b] =
// sum_{k in chunk} A[r_{16 ti + a}, k] A[r_{16 tj + b}, k].  Rows past the
// block and columns past n enter as zeros.
template <typename TA, int NG>
__global__ __launch_bounds__(GramShape<NG>::NW * 64) void k_gram_block(
    const TA* __restrict__ A, int64_t lda, int64_t n, const int32_t* __restrict__ rows,
    const int32_t* __restrict__ lens, int32_t s, const int32_t* __restrict__ only, int32_t nchunks, int64_t chunk,
    double* __restrict__ ws) {
  using Sh = GramShape<NG>;
  using Acc = typename Mfma<TA>::acc_t;
  constexpr int NT = Sh::NW * 64, KC = Sh::KC, LD = KC + 1;
  __shared__ TA P[2][Sh::R * LD];
  __shared__ int32_t ri[Sh::R];
  const int ch = blockIdx.x, part = blockIdx.y, blk = blockIdx.z;
  if (only && !only[blk]) return;
  const int sb = lens[blk];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int32_t* Rw = rows + static_cast<int64_t>(blk) * s;
  for (int i = tid; i < Sh::R; i += NT) ri[i] = i < sb ? Rw[i] : -1;
  __syncthreads();
  const int64_t k_begin = static_cast<int64_t>(ch) * chunk;
  const int64_t k_end = min(n, k_begin + chunk);

  // panel entry e = tid + NT q: row e / KC, column e % KC (a wave reads
  // 64 / KC whole row segments per load)
  TA pv[Sh::LOADS];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < Sh::LOADS; ++q) {
      const int e = tid + NT * q;
      const int r = e / KC, c = e % KC;
      const int64_t k = k0 + c;
      const int32_t row = ri[r];
      pv[q] = (row >= 0 && k < k_end) ? A[static_cast<int64_t>(row) * lda + k] : TA(0);
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int q = 0; q < Sh::LOADS; ++q) {
      const int e = tid + NT * q;
      P[b][(e / KC) * LD + e % KC] = pv[q];
    }
  };

  // this wave's tiles: t = wv + NW (part + PARTS u); operand rows in LDS
  int aoff[Sh::TPW], boff[Sh::TPW];
  bool act[Sh::TPW];
#pragma unroll
  for (int u = 0; u < Sh::TPW; ++u) {
    const int t = wv + Sh::NW * (part + Sh::PARTS * u);
    act[u] = t < Sh::NTILE;
    int ti = 0, tj = 0;
    if (act[u]) tile_coords(t, ti, tj);
    aoff[u] = (16 * ti + (lane & 15)) * LD + (lane >> 4);
    boff[u] = (16 * tj + (lane & 15)) * LD + (lane >> 4);
  }
  Acc acc[Sh::TPW];
#pragma unroll
  for (int u = 0; u < Sh::TPW; ++u) acc[u] = Acc{0, 0, 0, 0};

  fetch(k_begin);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = k_begin; k0 < k_end; k0 += KC) {
    const bool more = k0 + KC < k_end;
    if (more) fetch(k0 + KC);
    const TA* Pb = P[buf];
#pragma unroll 1
    for (int kk = 0; kk < KC; kk += 4) {
#pragma unroll
      for (int u = 0; u < Sh::TPW; ++u)
        if (act[u]) acc[u] = Mfma<TA>::step(Pb[aoff[u] + kk], Pb[boff[u] + kk], acc[u]);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // acc[u]: entry (row(lane, r), lane % 16) of tile t
  double* W = ws + (static_cast<int64_t>(blk) * nchunks + ch) * Sh::NTILE * 256;
#pragma unroll
  for (int u = 0; u < Sh::TPW; ++u) {
    if (!act[u]) continue;
    const int t = wv + Sh::NW * (part + Sh::PARTS * u);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      W[t * 256 + Mfma<TA>::row(lane, r) * 16 + (lane & 15)] = static_cast<double>(acc[u][r]);
  }
}

// The 128-row shape in FP64 (NG = 8) as the memo-miss path runs it beside the
// resident step kernel: four waves (one per SIMD, at most 136 registers each:
// what the step kernel leaves) and every tile of the block in one workgroup,
// so each entry of A_S is read once; 8-column panels keep the loads of the
// next two panels within that budget.  The tiles go to the waves by row
// groups, nine each: wave 0 takes the lower tiles among groups 0-3 but
// (3, 3), wave 1 those among groups 4-7 but (7, 7), waves 2 and 3 the cross
// tiles of groups 4-5 and 6-7 with groups 0-3 and the tile (3, 3) or (7, 7),
// whose operand they hold.  A wave reads one operand per row group it
// touches (4 or 6 per k step) and uses it on both sides: lane l holds
// A[r_{16 g + l % 16}, k + l / 16], the X operand for g = ti and the Y
// operand for g = tj.
// Same workspace layout and arguments as k_gram_block<TA, 8> (one tile part).
template <typename TA>
__global__ __launch_bounds__(256) void k_gram_block128(const TA* __restrict__ A, int64_t lda, int64_t n,
                                                       const int32_t* __restrict__ rows,
                                                       const int32_t* __restrict__ lens, int32_t s,
                                                       const int32_t* __restrict__ only, int32_t nchunks,
                                                       int64_t chunk, double* __restrict__ ws) {
  using Acc = typename Mfma<TA>::acc_t;
  constexpr int NT = 256, KC = 8, LD = KC + 1, R = 128, NTILE = 36, LOADS = R * KC / NT;
  __shared__ TA P[2][R * LD];
  __shared__ int32_t ri[R];
  const int ch = blockIdx.x, blk = blockIdx.z;
  if (only && !only[blk]) return;
  const int sb = lens[blk];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int32_t* Rw = rows + static_cast<int64_t>(blk) * s;
  for (int i = tid; i < R; i += NT) ri[i] = i < sb ? Rw[i] : -1;
  __syncthreads();
  const int64_t k_begin = static_cast<int64_t>(ch) * chunk;
  const int64_t k_end = min(n, k_begin + chunk);

  TA pa[LOADS];
  auto fetch = [&](TA(&pv)[LOADS], int64_t k0) {
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      const int e = tid + NT * q;
      const int r = e / KC, c = e % KC;
      const int64_t k = k0 + c;
      const int32_t row = ri[r];
      pv[q] = (row >= 0 && k < k_end) ? A[static_cast<int64_t>(row) * lda + k] : TA(0);
    }
  };
  auto stash = [&](TA(&pv)[LOADS], int b) {
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      const int e = tid + NT * q;
      P[b][(e / KC) * LD + e % KC] = pv[q];
    }
  };

  // operand f of this wave: row group gof(f)
  const bool tri = wv < 2;
  int foff[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int g = tri ? (f < 4 ? 4 * wv + f : 0) : (f < 2 ? 4 + 2 * (wv - 2) + f : f - 2);
    foff[f] = (16 * g + (lane & 15)) * LD + (lane >> 4);
  }
  Acc acc[9];
#pragma unroll
  for (int u = 0; u < 9; ++u) acc[u] = Acc{0, 0, 0, 0};

  auto mma = [&](const TA* Pb) {
#pragma unroll 1
    for (int kk = 0; kk < KC; kk += 4) {
      TA F[6];
#pragma unroll
      for (int f = 0; f < 6; ++f) F[f] = Pb[foff[f] + kk];
      if (tri) {
        // (i, j), 0 <= j <= i < 4, in row order, but (3, 3)
#pragma unroll
        for (int i = 0, u = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j <= i && u < 9; ++j, ++u) acc[u] = Mfma<TA>::step(F[i], F[j], acc[u]);
      } else {
        // (i, j), i < 2 (operands 0, 1), j < 4 (operands 2..5); then group 3
        // (operand 5, wave 2) or group 7 (operand 1, wave 3) with itself
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[4 * i + j] = Mfma<TA>::step(F[i], F[2 + j], acc[4 * i + j]);
        const TA d = wv == 2 ? F[5] : F[1];
        acc[8] = Mfma<TA>::step(d, d, acc[8]);
      }
    }
  };
  // panel p (columns k_begin + KC p ...) sits in LDS buffer p % 2 while the
  // loads of panels p + 1 and p + 2 are in flight, in pa and pb by turns
  // (eight registers more than one panel ahead: 136 in all, what the step
  // kernel leaves)
  const int np = static_cast<int>((k_end - k_begin + KC - 1) / KC);
  auto col = [&](int q) { return k_begin + static_cast<int64_t>(q) * KC; };
  TA pb[LOADS];
  fetch(pa, k_begin);
  stash(pa, 0);
  if (np > 1) fetch(pa, col(1));
  __syncthreads();
  int p = 0;
  for (; p + 1 < np; p += 2) {
    if (p + 2 < np) fetch(pb, col(p + 2));
    mma(P[0]);
    stash(pa, 1);
    __syncthreads();
    if (p + 3 < np) fetch(pa, col(p + 3));
    mma(P[1]);
    if (p + 2 < np) stash(pb, 0);
    __syncthreads();
  }
  if (p < np) mma(P[0]);
  double* W = ws + (static_cast<int64_t>(blk) * nchunks + ch) * NTILE * 256;
  auto put = [&](int u, int ti, int tj) {
    const int t = ti * (ti + 1) / 2 + tj;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      W[t * 256 + Mfma<TA>::row(lane, r) * 16 + (lane & 15)] = static_cast<double>(acc[u][r]);
  };
  if (tri) {
#pragma unroll
    for (int i = 0, u = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j <= i && u < 9; ++j, ++u) put(u, 4 * wv + i, 4 * wv + j);
  } else {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) put(4 * i + j, 4 + 2 * (wv - 2) + i, j);
    const int gd = wv == 2 ? 3 : 7;
    put(8, gd, gd);
  }
}

// The 256-row shape (NG = 16): eight waves, every tile of the block in one
// workgroup, 16-column panels double-buffered in LDS.  The tiles go to the
// waves by 4 x 4 super-blocks of row groups, so that a wave reads 8 operands
// per k step for 16 or 20 products: waves 0-5 take the off-diagonal
// super-blocks (I, J) = (1, 0), (2, 0), (2, 1), (3, 0), (3, 1), (3, 2) (16
// tiles each), waves 6 and 7 the lower tiles of the diagonal super-blocks 0
// and 1, and 2 and 3 (20 each).  Same operand layout, workspace layout
// (136 tiles per block and chunk) and arguments as k_gram_block.
template <typename TA>
__global__ __launch_bounds__(512) void k_gram_block256(const TA* __restrict__ A, int64_t lda, int64_t n,
                                                       const int32_t* __restrict__ rows,
                                                       const int32_t* __restrict__ lens, int32_t s,
                                                       const int32_t* __restrict__ only, int32_t nchunks,
                                                       int64_t chunk, double* __restrict__ ws) {
  using Acc = typename Mfma<TA>::acc_t;
  constexpr int NT = 512, KC = 16, LD = KC + 1, R = 256, NTILE = 136, LOADS = R * KC / NT;
  __shared__ TA P[2][R * LD];
  __shared__ int32_t ri[R];
  const int ch = blockIdx.x, blk = blockIdx.z;
  if (only && !only[blk]) return;
  const int sb = lens[blk];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int32_t* Rw = rows + static_cast<int64_t>(blk) * s;
  for (int i = tid; i < R; i += NT) ri[i] = i < sb ? Rw[i] : -1;
  __syncthreads();
  const int64_t k_begin = static_cast<int64_t>(ch) * chunk;
  const int64_t k_end = min(n, k_begin + chunk);

  TA pa[LOADS];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      const int e = tid + NT * q;
      const int r = e / KC, c = e % KC;
      const int64_t k = k0 + c;
      const int32_t row = ri[r];
      pa[q] = (row >= 0 && k < k_end) ? A[static_cast<int64_t>(row) * lda + k] : TA(0);
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      const int e = tid + NT * q;
      P[b][(e / KC) * LD + e % KC] = pa[q];
    }
  };

  // operand f of this wave: row group gop(f)
  const bool diag = wv >= 6;
  const int I = wv < 1 ? 1 : (wv < 3 ? 2 : 3);
  const int J = wv - I * (I - 1) / 2;
  int foff[8];
#pragma unroll
  for (int f = 0; f < 8; ++f) {
    const int g = diag ? 8 * (wv - 6) + f : (f < 4 ? 4 * I + f : 4 * J + f - 4);
    foff[f] = (16 * g + (lane & 15)) * LD + (lane >> 4);
  }
  Acc acc[20];
#pragma unroll
  for (int u = 0; u < 20; ++u) acc[u] = Acc{0, 0, 0, 0};

  auto mma = [&](const TA* Pb) {
#pragma unroll 1
    for (int kk = 0; kk < KC; kk += 4) {
      TA F[8];
#pragma unroll
      for (int f = 0; f < 8; ++f) F[f] = Pb[foff[f] + kk];
      if (diag) {
        // (i, j), 0 <= j <= i < 4, of both diagonal super-blocks, in row order
#pragma unroll
        for (int h = 0, u = 0; h < 2; ++h)
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j, ++u) acc[u] = Mfma<TA>::step(F[4 * h + i], F[4 * h + j], acc[u]);
      } else {
        // (4 I + a, 4 J + b)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[4 * a + b] = Mfma<TA>::step(F[a], F[4 + b], acc[4 * a + b]);
      }
    }
  };
  const int np = static_cast<int>((k_end - k_begin + KC - 1) / KC);
  fetch(k_begin);
  stash(0);
  __syncthreads();
  for (int p = 0; p < np; ++p) {
    if (p + 1 < np) fetch(k_begin + static_cast<int64_t>(p + 1) * KC);
    mma(P[p & 1]);
    if (p + 1 < np) stash((p + 1) & 1);
    __syncthreads();
  }
  double* W = ws + (static_cast<int64_t>(blk) * nchunks + ch) * NTILE * 256;
  auto put = [&](int u, int ti, int tj) {
    const int t = ti * (ti + 1) / 2 + tj;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      W[t * 256 + Mfma<TA>::row(lane, r) * 16 + (lane & 15)] = static_cast<double>(acc[u][r]);
  };
  if (diag) {
#pragma unroll
    for (int h = 0, u = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j, ++u) {
          const int g0 = 8 * (wv - 6) + 4 * h;
          put(u, g0 + i, g0 + j);
        }
  } else {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) put(4 * a + b, 4 * I + a, 4 * J + b);
  }
}

// G[slot][j * s + i] = sum over chunks of the partial tiles (+ lambda on the
// diagonal), lower triangle of the block only; chunks summed in order, with
// eight loads in flight
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ ws, const int32_t* __restrict__ lens,
                                                     int32_t s, const int32_t* __restrict__ only, int32_t nchunks,
                                                     int32_t ntiles, double lambda, double* __restrict__ G,
                                                     int64_t stride, const int32_t* __restrict__ slot_of) {
  const int t = blockIdx.x, blk = blockIdx.y;
  if (only && !only[blk]) return;
  const int sb = lens[blk];
  int ti, tj;
  tile_coords(t, ti, tj);
  const int e = threadIdx.x;
  const int i = 16 * ti + (e >> 4), j = 16 * tj + (e & 15);
  if (i >= sb || j >= sb || i < j) return;
  const int64_t cs = static_cast<int64_t>(ntiles) * 256;
  const double* W = ws + static_cast<int64_t>(blk) * nchunks * cs + t * 256 + e;
  double acc = 0.0;
  int c = 0;
  for (; c + 8 <= nchunks; c += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = W[(c + u) * cs];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; c < nchunks; ++c) acc += W[c * cs];
  G[static_cast<int64_t>(slot_of[blk]) * stride + static_cast<int64_t>(j) * s + i] = acc + (i == j ? lambda : 0.0);
}

}  // namespace

template <typename TA, int NG>
static void launch_block_grams(const TA* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens, int32_t s,
                               int32_t nb, const int32_t* only, int32_t nc, int64_t chunk, double* ws, hipStream_t st) {
  using Sh = GramShape<NG>;
  if constexpr (NG == 8 && sizeof(TA) == 8) {
    hipLaunchKernelGGL((k_gram_block128<TA>), dim3(nc, 1, nb), dim3(256), 0, st, A, lda, n, rows, lens, s, only, nc,
                       chunk, ws);
  } else if constexpr (NG == 16) {
    hipLaunchKernelGGL((k_gram_block256<TA>), dim3(nc, 1, nb), dim3(512), 0, st, A, lda, n, rows, lens, s, only, nc,
                       chunk, ws);
  } else {
    hipLaunchKernelGGL((k_gram_block<TA, NG>), dim3(nc, Sh::PARTS, nb), dim3(Sh::NW * 64), 0, st, A, lda, n, rows,
                       lens, s, only, nc, chunk, ws);
  }
}

template <typename TA>
static void launch_syrk_planned(const TA* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens,
                                int32_t s, int32_t nb, double lambda, double* G, int64_t stride,
                                const int32_t* slot_of, const int32_t* only, double* ws, int32_t nc, int64_t chunk,
                                int32_t nt, hipStream_t st) {
  switch (gram_groups(s)) {
    case 2: launch_block_grams<TA, 2>(A, lda, n, rows, lens, s, nb, only, nc, chunk, ws, st); break;
    case 4: launch_block_grams<TA, 4>(A, lda, n, rows, lens, s, nb, only, nc, chunk, ws, st); break;
    case 8: launch_block_grams<TA, 8>(A, lda, n, rows, lens, s, nb, only, nc, chunk, ws, st); break;
    case 16: launch_block_grams<TA, 16>(A, lda, n, rows, lens, s, nb, only, nc, chunk, ws, st); break;
    default: launch_block_grams<TA, 32>(A, lda, n, rows, lens, s, nb, only, nc, chunk, ws, st); break;
  }
  hipLaunchKernelGGL(k_gram_reduce, dim3(nt, nb), dim3(256), 0, st, ws, lens, s, only, nc, nt, lambda, G, stride,
                     slot_of);
}

template <typename TA>
static void launch_syrk(const TA* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens, int32_t s,
                        int32_t nb, double lambda, double* G, int64_t stride, const int32_t* slot_of,
                        const int32_t* only, double* ws, hipStream_t st) {
  int32_t nc, nt;
  int64_t chunk;
  gram_syrk_plan(s, n, nb, &nc, &chunk, &nt);
  launch_syrk_planned<TA>(A, lda, n, rows, lens, s, nb, lambda, G, stride, slot_of, only, ws, nc, chunk, nt, st);
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
  launch_syrk_planned<double>(A, lda, n, rows, lens, s, nb, lambda, G, stride, slot_of, nullptr, ws, nc, chunk, nt, st);
}

void launch_gram_syrk_f32(const float* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens, int32_t s,
                          int32_t nb, double lambda, double* G, int64_t stride, const int32_t* slot_of,
                          double* ws, hipStream_t st) {
  if (nb <= 0) return;
  launch_syrk<float>(A, lda, n, rows, lens, s, nb, lambda, G, stride, slot_of, nullptr, ws, st);
}

}  // namespace kpp
