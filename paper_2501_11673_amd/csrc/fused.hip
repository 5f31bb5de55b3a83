// Fused persistent block-step engine (gfx950).
//
// One launch runs W consecutive block steps of Kaczmarz++ (Algorithm 5, exact
// projection) or CD++ (Algorithm 2) for one system.  Workgroup g owns a
// contiguous column slice J_g of x and of the momentum m (64 * CPL columns,
// CPL per lane) and keeps it in registers for the whole launch.  Per step:
//   1. the workgroup's tile A_S[:, J_g] sits in registers (wave v holds block
//      rows v, v+4, ...; the 64 lanes of a wave read consecutive columns of a
//      row, so every load is coalesced); partial residuals p_g = A_S[:, J_g]
//      x[J_g] are reduced across lanes by a butterfly (RMAX rows at once);
//   2. publish p_g; wait until every workgroup has published (one
//      all-gather through per-workgroup flags: the step's only cross-CU
//      sync); r = sum_g p_g - b_S, summed in the same order in every
//      workgroup.  CD++ loads the next step's tile, rows and b values while
//      it waits (the block sequence never depends on x): waves 1-3 issue
//      their loads before the wait, wave 0 polls the flags (a wave's loads
//      complete in order, so a polling wave must not have loads in flight)
//      and issues its share right after;
//   3. y = (A_S A_S^T + lam I)^{-1} r through the memoized inverse
//      G^{-1} = L^{-T} L^{-1} of the block's Cholesky factor: CD++ needs only
//      the rows of y whose coordinates fall into J_g (w = I_S^T y), Kaczmarz++
//      needs all of y (w = A_S^T y) and forms it in every workgroup;
//   4. w on the slice, then m <- c (m - w), x <- x - w + eta m (eq. (momentum));
//   5. window sums and the checkpoint of Section 5.4 (identical scalars in
//      every workgroup; workgroup 0 writes them back).
// Every wait is bounded; on time-out the kernel sets err bit 2 and all
// workgroups leave, so a launch always ends.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace kpp {
namespace {

#ifndef KPP_FLAG_STRIDE
#define KPP_FLAG_STRIDE 32
#endif
#ifndef KPP_POLL_SLEEP
#define KPP_POLL_SLEEP 0
#endif
#ifndef KPP_PREFETCH
#define KPP_PREFETCH 1
#endif

constexpr int kT = 256;
constexpr int kFlagStride = KPP_FLAG_STRIDE;  // uint32 words between flags
// Tile entries per lane: 64 doubles, or 128 floats (the same registers) when a
// lane holds at least four columns; a wave then still holds 32 rows or fewer.
template <typename TA, int CPL>
struct TileElems {
  static constexpr int value = (sizeof(TA) == 4 && CPL >= 4) ? 128 : 64;
};
static_assert(kFlagStride * kFusedMaxGroups <= kFlagWordsAlloc, "flag area too small");

__device__ __forceinline__ double ld_coherent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_flag(uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag_release(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double rho_from_rate(double rhat, int zeta) {
  if (!(rhat < 1.0)) return 0.0;
  double r = 1.0 - pow(rhat, 1.0 / static_cast<double>(zeta));
  return fmin(1.0, fmax(0.0, r));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Load this wave's rows of the block tile: tile[r * CPL + e] = A[rows[wv + 4r], col0 + e].
// One vector load fetches the wave's row indices (lane r holds row wv + 4r),
// read back lane by lane, so every tile load issues at once.  Row indices past
// the block and columns past the matrix are clamped, not masked: those entries
// always meet a zero (x is zero beyond n, y is zero beyond the block), and A
// is finite (checked when the system is created), so they contribute nothing.
template <int CPL, typename TA, int TE>
__device__ __forceinline__ void load_tile(TA (&tile)[TE], const TA* __restrict__ A,
                                          int64_t lda, int64_t n, const int32_t* __restrict__ rows,
                                          int sb, int wv, int lane, int64_t col0) {
  constexpr int RMAX = TE / CPL;
  const int myrow = rows[min(wv + 4 * (lane & (RMAX - 1)), sb - 1)];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    const int row = __builtin_amdgcn_readlane(myrow, r);
    const TA* Ai = A + static_cast<int64_t>(row) * lda;
#pragma unroll
    for (int e = 0; e < CPL; ++e) tile[r * CPL + e] = Ai[min(col0 + e, n - 1)];
  }
}

// TA: storage and product type of A (double; float for the mixed-precision
// inner solver: the tile, the partial residuals and the direction are formed in
// FP32 with FP32 accumulation, everything else stays FP64).
// The team of G workgroups runs a.W steps (fewer when a.stop_on_cand ends it
// at a checkpoint); wg is this workgroup's index in the team.
template <int KIND, int CPL, typename TA>
__device__ __forceinline__ void fused_body(const FusedArgs& a, const int G, const int wg) {
  const TA* __restrict__ Amat = static_cast<const TA*>(a.A);
  // optional phase profile (workgroup 0, thread 0): ticks[p] accumulates the
  // wall-clock time from mark p-1 to mark p
  uint64_t tick_last = 0, ticks[kFusedPhases];
  const bool prof = a.phase_ticks != nullptr && wg == 0 && threadIdx.x == 0;
#pragma unroll
  for (int p = 0; p < kFusedPhases; ++p) ticks[p] = 0;
#define KPP_MARK(p)                                   \
  if (prof) {                                         \
    const uint64_t now_ = wall_clock64();             \
    ticks[p] += now_ - tick_last;                     \
    tick_last = now_;                                 \
  }
  constexpr int TE = TileElems<TA, CPL>::value;
  constexpr int RMAX = TE / CPL;   // rows per wave held in registers (power of two, <= 64)
  constexpr int RSHIFT = (RMAX == 64) ? 0 : (RMAX == 32) ? 1 : (RMAX == 16) ? 2 : (RMAX == 8) ? 3 : 4;
  static_assert(RMAX >= 4 && RMAX <= 64, "rows per wave");
  __shared__ int32_t rsbuf[2][256];
  __shared__ double rv[256];
  __shared__ double yv[256];
  __shared__ double stage[256];
  __shared__ double wred[KIND == 0 ? 4 * 64 * CPL : 1];
  __shared__ double red[4];
  __shared__ double bc_c;
  __shared__ int bc_stop;
  __shared__ int abort_flag;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int64_t n = a.n;
  const int s = a.s;
  const int64_t slice0 = static_cast<int64_t>(wg) * 64 * CPL;
  const int64_t slice1 = min(n, slice0 + 64 * CPL);
  const int64_t col0 = slice0 + static_cast<int64_t>(lane) * CPL;

  double xr[CPL], mr[CPL];
#pragma unroll
  for (int e = 0; e < CPL; ++e) {
    const int64_t j = col0 + e;
    xr[e] = j < n ? a.x[j] : 0.0;
    mr[e] = j < n ? a.mom[j] : 0.0;
  }
  // dual slice (Kaczmarz++ with m < n): rows d0 + tid + 256 u of [d0, d1)
  constexpr int DU = 4;
  double zxr[DU], zmr[DU];
  const bool dual = KIND == 0 && a.zx != nullptr;
  int64_t d0 = 0, d1 = 0;
  if (dual) {
    const int64_t per = (a.mrows + G - 1) / G;   // at most 256 DU (checked by the host)
    d0 = min(a.mrows, static_cast<int64_t>(wg) * per);
    d1 = min(a.mrows, d0 + per);
  }
#pragma unroll
  for (int u = 0; u < DU; ++u) {
    const int64_t i = d0 + tid + 256 * u;
    zxr[u] = (dual && i < d1) ? a.zx[i] : 0.0;
    zmr[u] = (dual && i < d1) ? a.zm[i] : 0.0;
  }
  DevState st{};
  if (tid == 0) {
    st = *a.ds;
    abort_flag = 0;
  }
  TA tile[TE];
  int q = a.step_slot[0];
  int sb = a.lens[q];
  int cur = 0;
  load_tile<CPL>(tile, Amat, a.lda, n, a.rows + static_cast<int64_t>(q) * s, sb, wv, lane, col0);
  // thread tid forms r at block row tid: it holds b there for the current step
  double bval = 0.0;
  if (tid < sb) {
    const int32_t row = a.rows[static_cast<int64_t>(q) * s + tid];
    rsbuf[0][tid] = row;
    bval = a.b[row];
  }
  __syncthreads();

  if (prof) tick_last = wall_clock64();
  for (int k = 0; k < a.W; ++k) {
    const int32_t* rs = rsbuf[cur];
    if ((KIND == 0 || !KPP_PREFETCH) && k > 0) {
      load_tile<CPL>(tile, Amat, a.lda, n, a.rows + static_cast<int64_t>(q) * s, sb, wv, lane, col0);
    }
    const double* Ginv = a.L + static_cast<int64_t>(q) * a.slot_stride + static_cast<int64_t>(s) * s;
    KPP_MARK(0)

    // 1. partial residuals of this wave's rows, butterfly across the lanes
    TA xt[CPL];
#pragma unroll
    for (int e = 0; e < CPL; ++e) xt[e] = static_cast<TA>(xr[e]);
    // the lane's products are summed in TA, the sums across lanes in FP64.
    // The pair (v[r], v[r + cnt/2]) passes through an empty asm statement:
    // otherwise the compiler may fold the two selects into one indexed read of
    // v, which it lowers to a chain of compares over the whole array.
    double v[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      TA acc = 0;
#pragma unroll
      for (int e = 0; e < CPL; ++e) acc = fma(tile[r * CPL + e], xt[e], acc);
      v[r] = static_cast<double>(acc);
    }
#pragma unroll
    for (int cnt = RMAX, o = 32; cnt > 1; cnt >>= 1, o >>= 1) {
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int r = 0; r < cnt / 2; ++r) {
        double lo = v[r], hi = v[r + cnt / 2];
        asm("" : "+v"(lo), "+v"(hi));
        const double send = up ? lo : hi;
        const double keep = up ? hi : lo;
        v[r] = keep + __shfl_xor(send, o, 64);
      }
    }
#pragma unroll
    for (int o = 32 / RMAX; o >= 1; o >>= 1) v[0] += __shfl_xor(v[0], o, 64);
    {
      const int row = wv + 4 * (lane >> RSHIFT);
      if ((lane & ((1 << RSHIFT) - 1)) == 0 && row < sb) stage[row] = v[0];
    }
    __syncthreads();
    KPP_MARK(1)

    // 2. publish; prefetch (CD++); all-gather; reduce in a fixed order
    const uint32_t ep = a.epoch + static_cast<uint32_t>(k) + 1u;
    double* Pb = a.part + static_cast<size_t>(ep & 1u) * G * s;
    if (wv == 0) {
      for (int i = lane; i < sb; i += 64) st_coherent(&Pb[static_cast<size_t>(wg) * s + i], stage[i]);
      if (lane == 0) st_flag_release(&a.flags[wg * kFlagStride], ep);
    }
    KPP_MARK(2)
    // block rows whose coordinates fall into this slice (rows are sorted)
    int lo = 0, hi = sb;
    if (KIND == 1) {
      int l = 0, h = sb;
      while (l < h) {
        const int mid = (l + h) >> 1;
        if (rs[mid] < slice0) l = mid + 1; else h = mid;
      }
      lo = l;
      h = sb;
      while (l < h) {
        const int mid = (l + h) >> 1;
        if (rs[mid] < slice1) l = mid + 1; else h = mid;
      }
      hi = l;
    }
    const bool have_next = k + 1 < a.W;
    const int qn = have_next ? a.step_slot[k + 1] : q;
    const int sbn = a.lens[qn];
    const int32_t* Rn = a.rows + static_cast<int64_t>(qn) * s;
    // CD++: the memoized inverse's rows for this slice; slice row lo + t
    // belongs to wave 1 + t % 3 (wave 0 polls), lanes hold entries k = lane + 64 u
    double grow[4] = {0.0, 0.0, 0.0, 0.0};
    const int my_first = (KIND == 1 && wv > 0) ? lo + (wv - 1) : hi;
    if (KIND == 1 && wv > 0) {
      if (my_first < hi) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int kk = lane + 64 * u;
          grow[u] = Ginv[static_cast<int64_t>(my_first) * s + min(kk, sb - 1)];
        }
      }
      if (KPP_PREFETCH && have_next) load_tile<CPL>(tile, Amat, a.lda, n, Rn, sbn, wv, lane, col0);
    }
    if (tid < G) {
      int64_t spins = 0;
      while (static_cast<int32_t>(ld_flag(&a.flags[tid * kFlagStride]) - ep) < 0) {
        if (KPP_POLL_SLEEP > 0) __builtin_amdgcn_s_sleep(KPP_POLL_SLEEP);
        if (++spins > a.spin_limit) {
          atomicOr(a.err, 2);
          abort_flag = 1;
          break;
        }
      }
    }
    __syncthreads();
    KPP_MARK(3)
    if (abort_flag) break;
    // r = sum_g p_g - b_S: wave w sums block rows 64 w .. 64 w + 63, one row
    // per lane, so that every wave's partial loads are a single batch; then
    // the next step's rows and b values (used after this step)
    double bnext = 0.0;
    const int nu = (sb + 63) >> 6;
    if (wv < nu) {
      const int c = min(tid, sb - 1);   // rows past the block: clamped, sum dropped
      double acc = 0.0;
      int g = 0;
      for (; g + 32 <= G; g += 32) {
        double t32[32];
#pragma unroll
        for (int uu = 0; uu < 32; ++uu) t32[uu] = ld_coherent(&Pb[static_cast<size_t>(g + uu) * s + c]);
#pragma unroll
        for (int uu = 0; uu < 32; ++uu) acc += t32[uu];
      }
      for (; g + 8 <= G; g += 8) {
        double t8[8];
#pragma unroll
        for (int uu = 0; uu < 8; ++uu) t8[uu] = ld_coherent(&Pb[static_cast<size_t>(g + uu) * s + c]);
#pragma unroll
        for (int uu = 0; uu < 8; ++uu) acc += t8[uu];
      }
      for (; g < G; ++g) acc += ld_coherent(&Pb[static_cast<size_t>(g) * s + c]);
      double rr_w = 0.0;
      if (tid < sb) {
        const double ri = acc - bval;
        rv[tid] = ri;
        rr_w = ri * ri;
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) rr_w += __shfl_down(rr_w, off, 64);
      if (lane == 0) red[wv] = rr_w;
    }
    // next step's rows and b (a dependent pair: issued before wave 0's tile
    // loads so that waiting for the row indices does not wait for the tile)
    if (have_next && tid < sbn) {
      const int32_t row = Rn[tid];
      rsbuf[cur ^ 1][tid] = row;
      bnext = a.b[row];
    }
    // wave 0's share of the next tile, after its partial loads have landed
    if (wv == 0 && KIND == 1 && KPP_PREFETCH && have_next) load_tile<CPL>(tile, Amat, a.lda, n, Rn, sbn, wv, lane, col0);
    __syncthreads();
    KPP_MARK(4)

    // 3. y through the memoized inverse
    if (KIND == 1) {
      if (wv > 0) {
        for (int i = my_first; i < hi; i += 3) {
          double acc = 0.0;
          if (i == my_first) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int kk = lane + 64 * u;
              if (kk < sb) acc = fma(grow[u], rv[kk], acc);
            }
          } else {
            const double* Gi = Ginv + static_cast<int64_t>(i) * s;
            for (int kk = lane; kk < sb; kk += 64) acc = fma(Gi[kk], rv[kk], acc);
          }
          acc = wave_sum(acc);
          if (lane == 0) yv[i] = acc;
        }
      }
    } else if (tid < sb) {
      double acc = 0.0;
      int kk = 0;
      for (; kk + 16 <= sb; kk += 16) {
        double g16[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) g16[u] = Ginv[static_cast<int64_t>(kk + u) * s + tid];
#pragma unroll
        for (int u = 0; u < 16; ++u) acc = fma(g16[u], rv[kk + u], acc);
      }
      for (; kk < sb; ++kk) acc = fma(Ginv[static_cast<int64_t>(kk) * s + tid], rv[kk], acc);
      yv[tid] = acc;
    }

    // 5. scalars: c for this step, window sums, checkpoint
    if (tid == 0) {
      double rr = red[0];
      for (int w = 1; w < ((sb + 63) >> 6); ++w) rr += red[w];
      const double rho = st.rho;
      st.c = (1.0 - rho) / (1.0 + rho);
      bc_c = st.c;
      const int64_t period = 2 * static_cast<int64_t>(a.zeta);
      const int64_t ph = st.t % period;
      if (ph < a.zeta)
        st.E0 += rr;
      else
        st.E1 += rr;
      bc_stop = 0;
      if (ph == period - 1) {
        st.ckpts += 1;
        st.last_E1 = st.E1;
        st.rho_before = rho;
        st.cand = (st.E1 <= st.thr) ? 1 : 0;
        bc_stop = a.stop_on_cand && st.cand;
        if (a.adaptive && st.E0 > 0.0) {
          const double qr = st.E1 / st.E0;
          if (!st.have_rhat) {
            st.rhat = qr;
            st.have_rhat = 1;
          } else {
            const double li = log(static_cast<double>(st.ckpt));
            const double li1 = log(static_cast<double>(st.ckpt) + 1.0);
            const double wgt = exp(li * li - li1 * li1);
            st.rhat = wgt * st.rhat + (1.0 - wgt) * qr;
          }
          st.ckpt += 1;
          st.rho = rho_from_rate(st.rhat, a.zeta);
        }
        st.E0 = 0.0;
        st.E1 = 0.0;
      }
      st.t += 1;
    }
    __syncthreads();
    KPP_MARK(5)
    const double c = bc_c;
    const bool stop_now = bc_stop != 0;   // the same in every workgroup of the team

    // 4. direction on the slice and the momentum update
    double w[CPL];
#pragma unroll
    for (int e = 0; e < CPL; ++e) w[e] = 0.0;
    if (KIND == 0) {
      TA wt[CPL];
#pragma unroll
      for (int e = 0; e < CPL; ++e) wt[e] = 0;
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        const int i = wv + 4 * r;
        const TA yi = static_cast<TA>((i < sb) ? yv[i] : 0.0);
#pragma unroll
        for (int e = 0; e < CPL; ++e) wt[e] = fma(tile[r * CPL + e], yi, wt[e]);
      }
#pragma unroll
      for (int e = 0; e < CPL; ++e) wred[wv * 64 * CPL + lane * CPL + e] = static_cast<double>(wt[e]);
      __syncthreads();
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        const int o = lane * CPL + e;
        w[e] = ((wred[o] + wred[64 * CPL + o]) + wred[128 * CPL + o]) + wred[192 * CPL + o];
      }
    } else {
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        const int64_t j = col0 + e;
        int l = lo, h = hi;
        while (l < h) {
          const int mid = (l + h) >> 1;
          if (rs[mid] < j) l = mid + 1; else h = mid;
        }
        if (l < hi && rs[l] == j) w[e] = yv[l];
      }
    }
    // columns past n keep x = m = 0 (the clamped tile entries there are not A's)
#pragma unroll
    for (int e = 0; e < CPL; ++e) w[e] = (col0 + e < n) ? w[e] : 0.0;
#pragma unroll
    for (int e = 0; e < CPL; ++e) {
      const double mn = __dmul_rn(c, __dsub_rn(mr[e], w[e]));
      mr[e] = mn;
      xr[e] = __dadd_rn(__dsub_rn(xr[e], w[e]), __dmul_rn(a.eta, mn));
    }
    // the same recursion on the dual: w = A_S^T y is A^T applied to y placed
    // at the block's rows
    if (dual) {
#pragma unroll
      for (int u = 0; u < DU; ++u) {
        const int64_t i = d0 + tid + 256 * u;
        if (i < d1) {
          int l = 0, h = sb;
          while (l < h) {
            const int mid = (l + h) >> 1;
            if (rs[mid] < i) l = mid + 1; else h = mid;
          }
          const double yi = (l < sb && rs[l] == i) ? yv[l] : 0.0;
          const double mn = __dmul_rn(c, __dsub_rn(zmr[u], yi));
          zmr[u] = mn;
          zxr[u] = __dadd_rn(__dsub_rn(zxr[u], yi), __dmul_rn(a.eta, mn));
        }
      }
    }
    q = qn;
    sb = sbn;
    bval = bnext;
    cur ^= 1;
    __syncthreads();
    KPP_MARK(6)
    if (stop_now) break;
  }
#undef KPP_MARK
  if (prof) {
#pragma unroll
    for (int p = 0; p < kFusedPhases; ++p) atomicAdd(reinterpret_cast<unsigned long long*>(&a.phase_ticks[p]),
                                                    static_cast<unsigned long long>(ticks[p]));
  }

  if (wv == 0) {
#pragma unroll
    for (int e = 0; e < CPL; ++e) {
      const int64_t j = col0 + e;
      if (j < n) {
        a.x[j] = xr[e];
        a.mom[j] = mr[e];
      }
    }
  }
  if (dual) {
#pragma unroll
    for (int u = 0; u < DU; ++u) {
      const int64_t i = d0 + tid + 256 * u;
      if (i < d1) {
        a.zx[i] = zxr[u];
        a.zm[i] = zmr[u];
      }
    }
  }
  if (wg == 0 && tid == 0) *a.ds = st;
}

template <int KIND, int CPL, typename TA>
__global__ __launch_bounds__(kT) void k_fused(FusedArgs a) {
  fused_body<KIND, CPL, TA>(a, static_cast<int>(gridDim.x), static_cast<int>(blockIdx.x));
}

template <int KIND, int CPL, typename TA>
__global__ __launch_bounds__(kT) void k_fused_multi(const FusedArgs* __restrict__ args,
                                                    const int32_t* __restrict__ team_start, int32_t nteams) {
  const int g = static_cast<int>(blockIdx.x);
  int t = 0;
  while (t + 1 < nteams && team_start[t + 1] <= g) ++t;
  const FusedArgs a = args[t];
  fused_body<KIND, CPL, TA>(a, team_start[t + 1] - team_start[t], g - team_start[t]);
}

template <int KIND, typename TA>
void launch_multi_kind(const FusedArgs* args, const int32_t* team_start, int32_t nteams, int total, int cpl,
                       hipStream_t st) {
  switch (cpl) {
    case 1: hipLaunchKernelGGL((k_fused_multi<KIND, 1, TA>), dim3(total), dim3(kT), 0, st, args, team_start, nteams); break;
    case 2: hipLaunchKernelGGL((k_fused_multi<KIND, 2, TA>), dim3(total), dim3(kT), 0, st, args, team_start, nteams); break;
    case 4: hipLaunchKernelGGL((k_fused_multi<KIND, 4, TA>), dim3(total), dim3(kT), 0, st, args, team_start, nteams); break;
    case 8: hipLaunchKernelGGL((k_fused_multi<KIND, 8, TA>), dim3(total), dim3(kT), 0, st, args, team_start, nteams); break;
    default: hipLaunchKernelGGL((k_fused_multi<KIND, 16, TA>), dim3(total), dim3(kT), 0, st, args, team_start, nteams); break;
  }
}

template <int KIND, typename TA>
void launch_kind(const FusedArgs& a, int cpl, int G, hipStream_t st) {
  switch (cpl) {
    case 1: hipLaunchKernelGGL((k_fused<KIND, 1, TA>), dim3(G), dim3(kT), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_fused<KIND, 2, TA>), dim3(G), dim3(kT), 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_fused<KIND, 4, TA>), dim3(G), dim3(kT), 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_fused<KIND, 8, TA>), dim3(G), dim3(kT), 0, st, a); break;
    default: hipLaunchKernelGGL((k_fused<KIND, 16, TA>), dim3(G), dim3(kT), 0, st, a); break;
  }
}

}  // namespace

void launch_fused_multi(int32_t kind, bool a_fp32, const FusedArgs* args, const int32_t* team_start,
                        int32_t nteams, int32_t total_groups, int32_t cpl, hipStream_t st) {
  if (nteams <= 0 || total_groups <= 0) return;
  if (kind == 0) {
    if (a_fp32)
      launch_multi_kind<0, float>(args, team_start, nteams, total_groups, cpl, st);
    else
      launch_multi_kind<0, double>(args, team_start, nteams, total_groups, cpl, st);
  } else {
    if (a_fp32)
      launch_multi_kind<1, float>(args, team_start, nteams, total_groups, cpl, st);
    else
      launch_multi_kind<1, double>(args, team_start, nteams, total_groups, cpl, st);
  }
}

void launch_fused(int32_t kind, bool a_fp32, const FusedArgs& a, int32_t cpl, int32_t groups, hipStream_t st) {
  if (kind == 0) {
    if (a_fp32)
      launch_kind<0, float>(a, cpl, groups, st);
    else
      launch_kind<0, double>(a, cpl, groups, st);
  } else {
    if (a_fp32)
      launch_kind<1, float>(a, cpl, groups, st);
    else
      launch_kind<1, double>(a, cpl, groups, st);
  }
}

}  // namespace kpp
