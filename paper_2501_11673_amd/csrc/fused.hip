// Fused persistent block-step engine (gfx950).
//
// One launch runs W consecutive block steps of Kaczmarz++ (Algorithm 5, exact
// projection) or CD++ (Algorithm 2) for one system.  Workgroup g owns a
// contiguous column slice of x and of the momentum m and keeps it in
// registers for the whole launch.  Per step:
//   1. partial block residual over the slice: p_g = A_S[:, J_g] x[J_g]
//      (coalesced: the 64 lanes of a wave read consecutive columns of a row);
//   2. publish p_g, then wait until every workgroup has published (one
//      all-gather through per-workgroup flags: the only cross-CU sync of the
//      step) and form r = sum_g p_g - b_S in a fixed order, identically in
//      every workgroup;
//   3. every workgroup solves y = (L L^T)^{-1} r itself with the memoized
//      factor (blocked forward/back substitution, 16 rows per step through
//      the inverted diagonal blocks), so no second sync is needed;
//   4. w on the slice: A_S[:, J_g]^T y (Kaczmarz++, the A_S tile is still in
//      L2) or the entries of y whose rows fall in the slice (CD++), then
//      m <- c (m - w), x <- x - w + eta m (eq. (momentum));
//   5. window sums and the checkpoint of Section 5.4 (identical scalars in
//      every workgroup; workgroup 0 writes them back).
// Every wait is bounded; on time-out the kernel sets err = 2 and all
// workgroups leave, so a launch always ends.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace kpp {
namespace {

constexpr int kT = 256;
constexpr int kFlagStride = 32;  // uint32 words between flags (128 bytes)

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

// y = (L L^T)^{-1} r for one block, 256 threads, thread i owns row i (sb <= 256).
// In: rv[i] = r_i.  Out: rv[i] = y_i.  zv is scratch.  Lc: column-major L,
// Lr: row-major L, D: inverses of the 16 x 16 diagonal blocks (row-major).
__device__ __forceinline__ void block_solve(double* rv, double* zv, const double* __restrict__ Lc,
                                            const double* __restrict__ Lr,
                                            const double* __restrict__ D, int s, int sb) {
  const int i = threadIdx.x;
  const int K = (sb + 15) >> 4;
  double ri = (i < sb) ? rv[i] : 0.0;
  // forward: z = L^{-1} r
  for (int k = 0; k < K; ++k) {
    const int b0 = k << 4;
    const bool mine = (i >= b0) && (i < b0 + 16);
    if (mine) zv[i] = ri;
    __syncthreads();
    if (mine) {
      const int ii = i - b0;
      const double* Dk = D + k * 256 + ii * 16;
      double acc = 0.0;
      for (int c = 0; c <= ii; ++c) acc = fma(Dk[c], zv[b0 + c], acc);
      rv[i] = acc;
    }
    __syncthreads();
    if (i >= b0 + 16 && i < sb) {
      const double* Li = Lr + static_cast<int64_t>(i) * s + b0;
      const int cmax = min(16, sb - b0);
      for (int c = 0; c < cmax; ++c) ri = fma(-Li[c], rv[b0 + c], ri);
    }
  }
  __syncthreads();
  // backward: y = L^{-T} z
  double zi = (i < sb) ? rv[i] : 0.0;
  for (int k = K - 1; k >= 0; --k) {
    const int b0 = k << 4;
    const bool mine = (i >= b0) && (i < b0 + 16);
    if (mine) zv[i] = zi;
    __syncthreads();
    if (mine) {
      const int ii = i - b0;
      const double* Dk = D + k * 256;
      double acc = 0.0;
      for (int c = 15; c >= ii; --c) acc = fma(Dk[c * 16 + ii], zv[b0 + c], acc);
      rv[i] = acc;
    }
    __syncthreads();
    if (i < b0) {
      const double* Lci = Lc + static_cast<int64_t>(i) * s + b0;
      const int cmax = min(16, sb - b0);
      for (int c = 0; c < cmax; ++c) zi = fma(-Lci[c], rv[b0 + c], zi);
    }
  }
  __syncthreads();
}

template <int KIND, int CPL>
__global__ __launch_bounds__(kT) void k_fused(FusedArgs a) {
  __shared__ int32_t rs[256];
  __shared__ double rv[256];
  __shared__ double zv[256];
  __shared__ double stage[256];
  __shared__ double wred[KIND == 0 ? 4 * 64 * CPL : 1];
  __shared__ double red[4];
  __shared__ double bc_c;
  __shared__ int abort_flag;

  const int G = gridDim.x;
  const int wg = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int64_t col0 = static_cast<int64_t>(wg) * 64 * CPL + static_cast<int64_t>(lane) * CPL;
  const int64_t n = a.n;
  const int s = a.s;

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
  __syncthreads();

  for (int k = 0; k < a.W; ++k) {
    const int q = a.step_slot[k];
    const int sb = a.lens[q];
    const int32_t* R = a.rows + static_cast<int64_t>(q) * s;
    const double* Lc = a.L + static_cast<int64_t>(q) * a.slot_stride;
    if (tid < sb) rs[tid] = R[tid];
    __syncthreads();

    // 1. partial block residual over this workgroup's columns
    for (int i = wv; i < sb; i += 4) {
      const double* Ai = a.A + static_cast<int64_t>(rs[i]) * a.lda;
      double acc = 0.0;
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        const int64_t j = col0 + e;
        if (j < n) acc = fma(Ai[j], xr[e], acc);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
      if (lane == 0) stage[i] = acc;
    }
    __syncthreads();

    // 2. publish, all-gather, reduce in a fixed order
    const uint32_t ep = a.epoch + static_cast<uint32_t>(k) + 1u;
    double* Pb = a.part + static_cast<size_t>(ep & 1u) * G * s;
    if (wv == 0) {
      for (int i = lane; i < sb; i += 64) st_coherent(&Pb[static_cast<size_t>(wg) * s + i], stage[i]);
      if (lane == 0) st_flag_release(&a.flags[wg * kFlagStride], ep);
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
      for (int g = 0; g < G; ++g) acc += ld_coherent(&Pb[static_cast<size_t>(g) * s + tid]);
      ri = acc - a.b[rs[tid]];
      rv[tid] = ri;
    }
    double part = fma(ri, ri, 0.0);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
    if (lane == 0) red[wv] = part;
    __syncthreads();

    // 3. projection solve (every workgroup, same arithmetic)
    block_solve(rv, zv, Lc, Lc + static_cast<int64_t>(s) * s, Lc + 2 * static_cast<int64_t>(s) * s, s, sb);

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
      for (int i = wv; i < sb; i += 4) {
        const double* Ai = a.A + static_cast<int64_t>(rs[i]) * a.lda;
        const double yi = rv[i];
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
          const int64_t j = col0 + e;
          if (j < n) w[e] = fma(Ai[j], yi, w[e]);
        }
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
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        const int64_t j = col0 + e;
        int lo = 0, hi = sb;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (rs[mid] < j)
            lo = mid + 1;
          else
            hi = mid;
        }
        if (lo < sb && rs[lo] == j) w[e] = rv[lo];
      }
    }
#pragma unroll
    for (int e = 0; e < CPL; ++e) {
      const double mn = __dmul_rn(c, __dsub_rn(mr[e], w[e]));
      mr[e] = mn;
      xr[e] = __dadd_rn(__dsub_rn(xr[e], w[e]), __dmul_rn(a.eta, mn));
    }
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
