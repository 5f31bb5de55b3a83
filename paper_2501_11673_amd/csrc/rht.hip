// Randomized Hadamard transform on the device (Definition d:rht).
//
// One kernel family applies H_R along one digit of the row index of a
// row-major matrix: row = hi * (R sigma) + r * sigma + lo, r in [0, R).  In
// Sylvester order H_{R1 R2} = H_{R1} (x) H_{R2} with the high digit outer, so
// passes over the digits of M commute and together give H_M, the product
// Algorithm 4 forms recursively.  M up to 4096 is one pass, larger M two.
//
// Fused into the first pass: the random diagonal D on the rows (Algorithms 2
// and 5) and on the columns (the two-sided transform of Algorithm 2), and the
// zero padding to a power of two (rows and columns past the input read as 0).
// Fused into the last pass: a diagonal on the output rows (the back-transform
// x = D H xbar of Algorithm 2), truncation, and an optional transposed store:
// for symmetric A, H A H = H (H A)^T, so the two-sided transform is two
// one-sided ones with the first one's result stored transposed.  Algorithm 3
// (SymFHT) halves the additions of that route by recursing on the diagonal
// blocks; on this device the transform is bound by HBM traffic, not by
// additions, so the kernels keep the route that streams A in two passes.
//
// Tiles.  A digit with R >= 128 runs k_fht_strip: a workgroup of 16 waves holds
// R rows of an 8-column strip (64-byte row segments): r's low 3 bits are lane
// bits 3..5, the next 4 bits the wave, the rest J = R / 128 registers per lane.
// The butterflies run in registers (high bits), across lanes by DPP and the
// permlane swaps (low bits), and across waves through LDS (middle bits).  A
// digit with R < 128 runs k_fht_small: one lane per column, R registers.
#include "kernels.hpp"

namespace kpp {
namespace {

constexpr int kStripCols = 8;
constexpr int kStripWaves = 16;
constexpr int kStripThreads = 64 * kStripWaves;
constexpr int kStripLow = 8 * kStripWaves;       // rows of a digit spanned by lanes and waves
constexpr int kSmallThreads = 256;
constexpr int kVecThreads = 1024;
constexpr int kVecMax = 4096;                    // one-pass vector transforms in LDS

// Register values exchanged per LDS round (up to 16: 128 KB of LDS).  Rounds
// of 8 with two workgroups per compute unit measured slower for J = 16.
template <int J>
constexpr int lds_round() { return J < 16 ? J : 16; }
template <int J>
constexpr size_t strip_lds_bytes() { return sizeof(double) * lds_round<J>() * kStripWaves * 64; }

struct FhtPass {
  const double* in;
  int64_t ld_in;
  double* out;
  int64_t ld_out;
  int64_t rows_valid;      // input rows >= rows_valid read as 0
  int64_t cols_valid;      // input columns >= cols_valid read as 0
  int64_t ncols;           // columns produced
  int64_t rows_out;        // output rows >= rows_out are not stored
  int64_t sigma;           // row stride of the digit
  int64_t rsig;            // R * sigma
  int64_t nstrips;         // column strips
  int64_t tiles;           // nstrips * sigma * (M / (R sigma))
  const int8_t* isign;     // input row factor isign[row] * iscale (null: none)
  const int8_t* csign;     // input column factor csign[col] * cscale (null: none)
  const int8_t* osign;     // output row factor osign[row] * oscale (null: none)
  double iscale, cscale, oscale;
  int32_t transpose_out;   // store out[col * ld_out + row]
  int32_t pad;
};

__device__ __forceinline__ double load_in(const FhtPass& a, int64_t row, int64_t col) {
  if (row >= a.rows_valid || col >= a.cols_valid) return 0.0;
  double v = a.in[row * a.ld_in + col];
  if (a.isign) v *= static_cast<double>(a.isign[row]) * a.iscale;
  if (a.csign) v *= static_cast<double>(a.csign[col]) * a.cscale;
  return v;
}

__device__ __forceinline__ void store_out(const FhtPass& a, int64_t row, int64_t col, double v) {
  if (row >= a.rows_out) return;
  if (a.osign) v *= static_cast<double>(a.osign[row]) * a.oscale;
  if (a.transpose_out)
    a.out[col * a.ld_out + row] = v;
  else
    a.out[row * a.ld_out + col] = v;
}

// in-register Sylvester transform of v[0..K) (index bits of v are the digit's)
template <int K>
__device__ __forceinline__ void fwht_regs(double* v) {
#pragma unroll
  for (int h = 1; h < K; h <<= 1) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (i & h) continue;
      const double x = v[i], y = v[i + h];
      v[i] = x + y;
      v[i + h] = x - y;
    }
  }
}

template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Butterfly across lane bit 3 (partner lane ^ 8; row_ror:8 inside 16-lane rows).
__device__ __forceinline__ double bfly_lane8(double v, bool upper) {
  const double p = dpp_double<0x128>(v);
  return upper ? p - v : v + p;
}

// Butterflies across lane bit 5 (O = 32) or 4 (O = 16) for two register
// values x, y at once.  The permlane swap exchanges the upper half (row pairs
// for 16) of its first operand with the lower half of its second, so after it
// the lanes with the bit clear hold x's pair and the others y's pair; sum and
// difference, then the same swap puts every result in its lane.
template <int O>
__device__ __forceinline__ void swap2(double& x, double& y) {
  const unsigned xl = __double2loint(x), xh = __double2hiint(x);
  const unsigned yl = __double2loint(y), yh = __double2hiint(y);
  const auto sl = O == 32 ? __builtin_amdgcn_permlane32_swap(xl, yl, false, false)
                          : __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
  const auto sh = O == 32 ? __builtin_amdgcn_permlane32_swap(xh, yh, false, false)
                          : __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
  x = __hiloint2double(static_cast<int>(sh[0]), static_cast<int>(sl[0]));
  y = __hiloint2double(static_cast<int>(sh[1]), static_cast<int>(sl[1]));
}
template <int O>
__device__ __forceinline__ void bfly_pair(double& x, double& y) {
  swap2<O>(x, y);
  double s = x + y, d = x - y;
  swap2<O>(s, d);
  x = s;
  y = d;
}

// Workgroups b and b + 8 are dispatched to the same XCD one after the other;
// they take the two strips that share each 128-byte line of a row.
__device__ __forceinline__ int64_t strip_tile(int64_t b) {
  const int64_t chunk = b >> 4, within = b & 15;
  return (((chunk << 3) + (within & 7)) << 1) + (within >> 3);
}

template <int J>
__global__ __launch_bounds__(kStripThreads) void k_fht_strip(FhtPass a) {
  extern __shared__ double lds[];
  const int64_t tile = strip_tile(blockIdx.x);
  if (tile >= a.tiles) return;   // uniform over the workgroup
  const int64_t strip = tile % a.nstrips;
  const int64_t rest = tile / a.nstrips;
  const int64_t lo = rest % a.sigma;
  const int64_t hi = rest / a.sigma;
  const int w = static_cast<int>(threadIdx.x >> 6);
  const int l = static_cast<int>(threadIdx.x & 63);
  const int64_t col = strip * kStripCols + (l & 7);
  const int g = l >> 3;
  const int64_t base = hi * a.rsig + lo;
  const bool live = col < a.ncols;

  double v[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int64_t r = static_cast<int64_t>(j) * kStripLow + w * 8 + g;
    v[j] = live ? load_in(a, base + r * a.sigma, col) : 0.0;
  }
  // r bits 7.. : registers
  fwht_regs<J>(v);
  // r bit 0 : lane bit 3
  const bool up8 = (l & 8) != 0;
#pragma unroll
  for (int j = 0; j < J; ++j) v[j] = bfly_lane8(v[j], up8);
  // r bits 1, 2 : lane bits 4, 5
  if constexpr (J == 1) {
    double z = 0.0;
    bfly_pair<16>(v[0], z);
    z = 0.0;
    bfly_pair<32>(v[0], z);
  } else {
#pragma unroll
    for (int j = 0; j < J; j += 2) {
      bfly_pair<16>(v[j], v[j + 1]);
      bfly_pair<32>(v[j], v[j + 1]);
    }
  }
  // r bits 3..6 : waves, through LDS in rounds of up to 16 register values.
  // Layout [q][wave][lane]: every access below is 64 consecutive doubles.
  constexpr int JC = lds_round<J>();
#pragma unroll
  for (int j0 = 0; j0 < J; j0 += JC) {
#pragma unroll
    for (int q = 0; q < JC; ++q) lds[(q * kStripWaves + w) * 64 + l] = v[j0 + q];
    __syncthreads();
    if (w < JC) {
      double u[kStripWaves];
#pragma unroll
      for (int k = 0; k < kStripWaves; ++k) u[k] = lds[(w * kStripWaves + k) * 64 + l];
      fwht_regs<kStripWaves>(u);
#pragma unroll
      for (int k = 0; k < kStripWaves; ++k) lds[(w * kStripWaves + k) * 64 + l] = u[k];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < JC; ++q) v[j0 + q] = lds[(q * kStripWaves + w) * 64 + l];
    if (j0 + JC < J) __syncthreads();
  }
  if (!live) return;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int64_t r = static_cast<int64_t>(j) * kStripLow + w * 8 + g;
    store_out(a, base + r * a.sigma, col, v[j]);
  }
}

// One column of up to 4096 rows in one pass (the vectors b, x0, x): the
// column sits in LDS and the log2 R butterfly stages run there.
__global__ __launch_bounds__(kVecThreads) void k_fht_vec(FhtPass a) {
  __shared__ double buf[kVecMax];
  const int R = static_cast<int>(a.rsig);
  for (int i = threadIdx.x; i < R; i += kVecThreads) buf[i] = load_in(a, i, 0);
  __syncthreads();
  for (int h = 1; h < R; h <<= 1) {
    for (int k = threadIdx.x; k < R / 2; k += kVecThreads) {
      const int i = (k / h) * 2 * h + (k % h);
      const double x = buf[i], y = buf[i + h];
      buf[i] = x + y;
      buf[i + h] = x - y;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < R; i += kVecThreads) store_out(a, i, 0, buf[i]);
}

// Digits with R < 128: lane = column, R registers per lane.
template <int R>
__global__ __launch_bounds__(kSmallThreads) void k_fht_small(FhtPass a) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kSmallThreads + threadIdx.x;
  const int64_t per_tile = a.nstrips * kSmallThreads;    // columns rounded up
  const int64_t tile = t / per_tile;
  const int64_t col = t % per_tile;
  if (tile >= a.tiles || col >= a.ncols) return;
  const int64_t lo = tile % a.sigma;
  const int64_t hi = tile / a.sigma;
  const int64_t base = hi * a.rsig + lo;
  double v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = load_in(a, base + r * a.sigma, col);
  fwht_regs<R>(v);
#pragma unroll
  for (int r = 0; r < R; ++r) store_out(a, base + r * a.sigma, col, v[r]);
}

template <int J>
void launch_strip(const FhtPass& a, hipStream_t st) {
  constexpr size_t lds = strip_lds_bytes<J>();
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fht_strip<J>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    attr_set = true;
  }
  const int64_t blocks = (a.tiles + 15) / 16 * 16;
  hipLaunchKernelGGL(k_fht_strip<J>, dim3(static_cast<unsigned>(blocks)), dim3(kStripThreads), lds, st, a);
}

template <int R>
void launch_small(const FhtPass& a, hipStream_t st) {
  const int64_t threads = a.tiles * a.nstrips * kSmallThreads;
  hipLaunchKernelGGL(k_fht_small<R>, dim3(static_cast<unsigned>(threads / kSmallThreads)),
                     dim3(kSmallThreads), 0, st, a);
}

void launch_pass(FhtPass a, int log_r, hipStream_t st) {
  const int64_t R = int64_t{1} << log_r;
  a.rsig = R * a.sigma;
  if (a.ncols == 1 && a.sigma == 1 && a.tiles == 1 && R >= kSmallThreads && R <= kVecMax) {
    hipLaunchKernelGGL(k_fht_vec, dim3(1), dim3(kVecThreads), 0, st, a);
    return;
  }
  if (log_r >= 7) {
    a.nstrips = (a.ncols + kStripCols - 1) / kStripCols;
    const int64_t n_hi = a.tiles;   // caller passes M / (R sigma) here
    a.tiles = a.nstrips * a.sigma * n_hi;
    switch (log_r) {
      case 7: launch_strip<1>(a, st); break;
      case 8: launch_strip<2>(a, st); break;
      case 9: launch_strip<4>(a, st); break;
      case 10: launch_strip<8>(a, st); break;
      case 11: launch_strip<16>(a, st); break;
      default: launch_strip<32>(a, st); break;
    }
    return;
  }
  a.nstrips = (a.ncols + kSmallThreads - 1) / kSmallThreads;
  a.tiles = a.sigma * a.tiles;
  switch (log_r) {
    case 0: launch_small<1>(a, st); break;
    case 1: launch_small<2>(a, st); break;
    case 2: launch_small<4>(a, st); break;
    case 3: launch_small<8>(a, st); break;
    case 4: launch_small<16>(a, st); break;
    case 5: launch_small<32>(a, st); break;
    default: launch_small<64>(a, st); break;
  }
}

}  // namespace

void launch_fht(const FhtSpec& s, hipStream_t st) {
  int lg = 0;
  while ((int64_t{1} << lg) < s.M) ++lg;
  // digits: one of lg bits, or a high digit of lg - 12 bits and a low one of 12
  const int nd = fht_passes(s.M);
  const int dlog[2] = {nd == 1 ? lg : lg - kFhtMaxDigitLog, kFhtMaxDigitLog};
  int64_t sigma = nd == 1 ? 1 : (int64_t{1} << kFhtMaxDigitLog);
  // the intermediate: out itself when the last pass can run in place on it
  const bool mid_is_out = !s.transpose_out && s.rows_out >= s.M && s.ld_out >= s.ncols;
  double* mid = mid_is_out ? s.out : s.work;
  const int64_t ld_mid = mid_is_out ? s.ld_out : s.ncols;
  for (int p = 0; p < nd; ++p) {
    const bool first = p == 0, last = p == nd - 1;
    FhtPass a{};
    a.in = first ? s.in : mid;
    a.ld_in = first ? s.ld_in : ld_mid;
    a.out = last ? s.out : mid;
    a.ld_out = last ? s.ld_out : ld_mid;
    a.rows_valid = first ? s.rows_valid : s.M;
    a.cols_valid = first ? s.cols_valid : s.ncols;
    a.ncols = s.ncols;
    a.rows_out = last ? s.rows_out : s.M;
    a.sigma = sigma;
    a.tiles = s.M / ((int64_t{1} << dlog[p]) * sigma);   // digits above this one
    a.isign = first ? s.isign : nullptr;
    a.iscale = s.iscale;
    a.csign = first ? s.csign : nullptr;
    a.cscale = s.cscale;
    a.osign = last ? s.osign : nullptr;
    a.oscale = s.oscale;
    a.transpose_out = last ? s.transpose_out : 0;
    launch_pass(a, dlog[p], st);
    sigma = 1;
  }
}

}  // namespace kpp
