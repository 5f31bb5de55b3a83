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
//      workgroup.  CD++ issues the loads of the next step's tile before it
//      waits, so HBM latency hides behind the sync (the block sequence never
//      depends on x);
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

constexpr int kT = 256;
constexpr int kFlagStride = 32;  // uint32 words between flags (128 bytes)
constexpr int kTileMax = 64;     // tile doubles per lane

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
template <int CPL>
__device__ __forceinline__ void load_tile(double (&tile)[kTileMax], const double* __restrict__ A,
                                          int64_t lda, int64_t n, const int32_t* __restrict__ rows,
                                          int sb, int wv, int64_t col0) {
  constexpr int RMAX = kTileMax / CPL;
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    const int i = wv + 4 * r;
    if (i < sb) {
      const double* Ai = A + static_cast<int64_t>(rows[i]) * lda;
#pragma unroll
      for (int e = 0; e < CPL; ++e) tile[r * CPL + e] = (col0 + e < n) ? Ai[col0 + e] : 0.0;
    } else {
#pragma unroll
      for (int e = 0; e < CPL; ++e) tile[r * CPL + e] = 0.0;
    }
  }
}

template <int KIND, int CPL>
__global__ __launch_bounds__(kT) void k_fused(FusedArgs a) {
  constexpr int RMAX = kTileMax / CPL;   // rows per wave held in registers (power of two)
  constexpr int RSHIFT = (RMAX == 64) ? 0 : (RMAX == 32) ? 1 : (RMAX == 16) ? 2 : (RMAX == 8) ? 3 : 4;
  __shared__ int32_t rs[256];
  __shared__ double rv[256];
  __shared__ double yv[256];
  __shared__ double stage[256];
  __shared__ double wred[KIND == 0 ? 4 * 64 * CPL : 1];
  __shared__ double red[4];
  __shared__ double bc_c;
  __shared__ int abort_flag;
  __shared__ int slice_lo, slice_hi;

  const int G = gridDim.x;
  const int wg = blockIdx.x;
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
  DevState st{};
  if (tid == 0) {
    st = *a.ds;
    abort_flag = 0;
  }
  double tile[kTileMax];
  int q = a.step_slot[0];
  int sb = a.lens[q];
  load_tile<CPL>(tile, a.A, a.lda, n, a.rows + static_cast<int64_t>(q) * s, sb, wv, col0);
  __syncthreads();

  for (int k = 0; k < a.W; ++k) {
    if (KIND == 0 && k > 0) {
      q = a.step_slot[k];
      sb = a.lens[q];
      load_tile<CPL>(tile, a.A, a.lda, n, a.rows + static_cast<int64_t>(q) * s, sb, wv, col0);
    }
    const int32_t* R = a.rows + static_cast<int64_t>(q) * s;
    const double* Ginv = a.L + static_cast<int64_t>(q) * a.slot_stride + static_cast<int64_t>(s) * s;
    if (tid < sb) rs[tid] = R[tid];

    // 1. partial residuals of this wave's rows, butterfly across the lanes
    double v[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int e = 0; e < CPL; ++e) acc = fma(tile[r * CPL + e], xr[e], acc);
      v[r] = acc;
    }
#pragma unroll
    for (int cnt = RMAX, o = 32; cnt > 1; cnt >>= 1, o >>= 1) {
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int r = 0; r < cnt / 2; ++r) {
        const double send = up ? v[r] : v[r + cnt / 2];
        const double keep = up ? v[r + cnt / 2] : v[r];
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

    // 2. publish, prefetch the next tile (CD++), all-gather, reduce in a fixed order
    const uint32_t ep = a.epoch + static_cast<uint32_t>(k) + 1u;
    double* Pb = a.part + static_cast<size_t>(ep & 1u) * G * s;
    if (wv == 0) {
      for (int i = lane; i < sb; i += 64) st_coherent(&Pb[static_cast<size_t>(wg) * s + i], stage[i]);
      if (lane == 0) st_flag_release(&a.flags[wg * kFlagStride], ep);
    }
    int qn = q, sbn = sb;
    if (KIND == 1 && k + 1 < a.W) {
      qn = a.step_slot[k + 1];
      sbn = a.lens[qn];
      load_tile<CPL>(tile, a.A, a.lda, n, a.rows + static_cast<int64_t>(qn) * s, sbn, wv, col0);
    }
    if (tid == 0) {
      // block rows whose coordinates fall into this slice (rows are sorted)
      int lo = 0, hi = sb;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rs[mid] < slice0) lo = mid + 1; else hi = mid;
      }
      int lo2 = lo, hi2 = sb;
      while (lo2 < hi2) {
        const int mid = (lo2 + hi2) >> 1;
        if (rs[mid] < slice1) lo2 = mid + 1; else hi2 = mid;
      }
      slice_lo = lo;
      slice_hi = lo2;
    }
    if (tid < G) {
      int64_t spins = 0;
      while (static_cast<int32_t>(ld_flag(&a.flags[tid * kFlagStride]) - ep) < 0) {
        if (++spins > a.spin_limit) {
          atomicOr(a.err, 2);
          abort_flag = 1;
          break;
        }
      }
    }
    __syncthreads();
    if (abort_flag) break;
    double ri = 0.0;
    if (tid < sb) {
      double acc = 0.0;
      int g = 0;
      for (; g + 8 <= G; g += 8) {
        double t8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t8[u] = ld_coherent(&Pb[static_cast<size_t>(g + u) * s + tid]);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += t8[u];
      }
      for (; g < G; ++g) acc += ld_coherent(&Pb[static_cast<size_t>(g) * s + tid]);
      ri = acc - a.b[rs[tid]];
      rv[tid] = ri;
    }
    {
      double part = fma(ri, ri, 0.0);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
      if (lane == 0) red[wv] = part;
    }
    __syncthreads();

    // 3. y through the memoized inverse
    if (KIND == 1) {
      const int lo = slice_lo, hi = slice_hi;
      for (int i = lo + wv; i < hi; i += 4) {
        const double* Gi = Ginv + static_cast<int64_t>(i) * s;
        double acc = 0.0;
        for (int kk = lane; kk < sb; kk += 64) acc = fma(Gi[kk], rv[kk], acc);
        acc = wave_sum(acc);
        if (lane == 0) yv[i] = acc;
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
      const double rr = (red[0] + red[1]) + (red[2] + red[3]);
      const double rho = st.rho;
      st.c = (1.0 - rho) / (1.0 + rho);
      bc_c = st.c;
      const int64_t period = 2 * static_cast<int64_t>(a.zeta);
      const int64_t ph = st.t % period;
      if (ph < a.zeta)
        st.E0 += rr;
      else
        st.E1 += rr;
      if (ph == period - 1) {
        st.ckpts += 1;
        st.last_E1 = st.E1;
        st.rho_before = rho;
        st.cand = (st.E1 <= st.thr) ? 1 : 0;
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
    const double c = bc_c;

    // 4. direction on the slice and the momentum update
    double w[CPL];
#pragma unroll
    for (int e = 0; e < CPL; ++e) w[e] = 0.0;
    if (KIND == 0) {
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        const int i = wv + 4 * r;
        const double yi = (i < sb) ? yv[i] : 0.0;
#pragma unroll
        for (int e = 0; e < CPL; ++e) w[e] = fma(tile[r * CPL + e], yi, w[e]);
      }
#pragma unroll
      for (int e = 0; e < CPL; ++e) wred[wv * 64 * CPL + lane * CPL + e] = w[e];
      __syncthreads();
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        const int o = lane * CPL + e;
        w[e] = ((wred[o] + wred[64 * CPL + o]) + wred[128 * CPL + o]) + wred[192 * CPL + o];
      }
    } else {
      const int lo = slice_lo, hi = slice_hi;
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
#pragma unroll
    for (int e = 0; e < CPL; ++e) {
      const double mn = __dmul_rn(c, __dsub_rn(mr[e], w[e]));
      mr[e] = mn;
      xr[e] = __dadd_rn(__dsub_rn(xr[e], w[e]), __dmul_rn(a.eta, mn));
    }
    q = qn;
    sb = sbn;
    __syncthreads();
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
  if (wg == 0 && tid == 0) *a.ds = st;
}

template <int KIND>
void launch_kind(const FusedArgs& a, int cpl, int G, hipStream_t st) {
  switch (cpl) {
    case 1: hipLaunchKernelGGL((k_fused<KIND, 1>), dim3(G), dim3(kT), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_fused<KIND, 2>), dim3(G), dim3(kT), 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_fused<KIND, 4>), dim3(G), dim3(kT), 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_fused<KIND, 8>), dim3(G), dim3(kT), 0, st, a); break;
    default: hipLaunchKernelGGL((k_fused<KIND, 16>), dim3(G), dim3(kT), 0, st, a); break;
  }
}

}  // namespace

void launch_fused(int32_t kind, const FusedArgs& a, int32_t cpl, int32_t groups, hipStream_t st) {
  if (kind == 0)
    launch_kind<0>(a, cpl, groups, st);
  else
    launch_kind<1>(a, cpl, groups, st);
}

}  // namespace kpp
