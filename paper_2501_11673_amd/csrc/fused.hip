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
//      it waits (the block sequence never depends on x): every wave issues
//      its loads before the wait, so the partial-residual loads after it do
//      not queue behind a tile (a wave's loads complete in order);
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
#include <type_traits>

#include "exchange.hpp"
#include "lanes.hpp"
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
// Storage of A as the kernel reads it (TS) and the type its tile and products
// use (TC): FP64 and FP32 as they are; Bf16 reads bfloat16 (the high 16 bits
// of an FP32) and widens it to FP32 as the tile is loaded.
struct Bf16 {};
template <typename TA>
struct AStore {
  using TC = TA;
  using TS = TA;
};
template <>
struct AStore<Bf16> {
  using TC = float;
  using TS = uint16_t;
};
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ float widen(uint16_t v) { return __uint_as_float(static_cast<uint32_t>(v) << 16); }
static_assert(kFlagStride * kFusedMaxGroups <= kYFlagOffset, "flag area too small");
static_assert(kYFlagOffset + 2 * kFlagStride * kFusedMaxGroups <= kFlagWordsAlloc, "flag area too small");
static_assert(4 * kTwoMaxBlock <= 2 * kFusedMaxBlock, "exchange buffer too small for r and y");

// Spin until a flag reaches epoch ep (agent-scope loads); false once the
// bound is exceeded.
__device__ __forceinline__ bool wait_flag(uint32_t* f, uint32_t ep, int64_t limit) {
  int64_t spins = 0;
  while (static_cast<int32_t>(ld_flag(f) - ep) < 0) {
    if (KPP_POLL_SLEEP > 0) __builtin_amdgcn_s_sleep(KPP_POLL_SLEEP);
    if (++spins > limit) return false;
  }
  return true;
}

__device__ __forceinline__ double rho_from_rate(double rhat, int zeta) {
  if (!(rhat < 1.0)) return 0.0;
  double r = 1.0 - pow(rhat, 1.0 / static_cast<double>(zeta));
  return fmin(1.0, fmax(0.0, r));
}

// Row index that lane r of wave wv contributes to a tile: block row wv + 4r
// (clamped to the block).  It is loaded a step ahead of the tile, so that the
// tile's loads wait for no dependent round trip.
template <int CPL, typename TA, int TE>
__device__ __forceinline__ int32_t tile_row_index(const int32_t* __restrict__ rows, int sb, int wv, int lane) {
  constexpr int RMAX = TE / CPL;
  return rows[min(wv + 4 * (lane & (RMAX - 1)), sb - 1)];
}

// Load this wave's rows of the block tile: tile[r * CPL + e] = A[rows[wv + 4r], col0 + e].
// Lane r holds the row index of row wv + 4r (tile_row_index), read back lane
// by lane, so every tile load issues at once.  When rows start
// 16-byte aligned and the whole slice lies inside the matrix (vec, the same
// for every lane of the workgroup) a lane fetches its CPL columns in loads of
// up to 16 bytes.  The choice must not differ between lanes: readlane takes
// the row index from lanes that a divergent branch would leave inactive, and
// the compiler may reuse those lanes' registers in the other branch.  The
// element path clamps row indices past the block and columns past the matrix
// instead of masking them: those entries always meet a zero (x is zero beyond
// n, y is zero beyond the block), and A is finite (checked when the system is
// created), so they contribute nothing.
template <int CPL, typename TC, typename TS, int TE>
__device__ __forceinline__ void load_tile(TC (&tile)[TE], const TS* __restrict__ A, int64_t lda, int64_t n,
                                          int32_t myrow, int64_t col0, bool vec) {
  constexpr int RMAX = TE / CPL;
  constexpr int V = (CPL < 16 / static_cast<int>(sizeof(TS))) ? CPL : 16 / static_cast<int>(sizeof(TS));
  if constexpr (V > 1) {
    if (vec) {
      typedef TS vec_t __attribute__((ext_vector_type(V)));
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        const int row = __builtin_amdgcn_readlane(myrow, r);
        const vec_t* Ai = reinterpret_cast<const vec_t*>(A + static_cast<int64_t>(row) * lda + col0);
#pragma unroll
        for (int e = 0; e < CPL / V; ++e) {
          const vec_t t = Ai[e];
#pragma unroll
          for (int j = 0; j < V; ++j) tile[r * CPL + e * V + j] = widen(t[j]);
        }
      }
      return;
    }
  }
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    const int row = __builtin_amdgcn_readlane(myrow, r);
    const TS* Ai = A + static_cast<int64_t>(row) * lda;
#pragma unroll
    for (int e = 0; e < CPL; ++e) tile[r * CPL + e] = widen(Ai[min(col0 + e, n - 1)]);
  }
}

// The launch's end state to the host mirror: the state, then the error words,
// then the sequence number (a release at system scope orders the stores
// before it).  One thread.
__device__ __forceinline__ void publish_mirror(const FusedArgs& a, const DevState& st) {
  static_assert(sizeof(DevState) % 8 == 0, "DevState in 8-byte words");
  uint64_t wds[sizeof(DevState) / 8];
  __builtin_memcpy(wds, &st, sizeof(DevState));
  uint64_t* hw = reinterpret_cast<uint64_t*>(&a.mirror->ds);
#pragma unroll
  for (int i = 0; i < static_cast<int>(sizeof(DevState) / 8); ++i)
    __hip_atomic_store(&hw[i], wds[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  const uint32_t e = __hip_atomic_load(reinterpret_cast<uint32_t*>(a.err), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t f = a.fp64_count ? __hip_atomic_load(const_cast<uint32_t*>(reinterpret_cast<const uint32_t*>(a.fp64_count)),
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                  : 0u;
  __hip_atomic_store(reinterpret_cast<uint64_t*>(&a.mirror->err), static_cast<uint64_t>(e) | (static_cast<uint64_t>(f) << 32),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(&a.mirror->seq, a.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// TA: storage and product type of A (double; float for the mixed-precision
// inner solver: the tile, the partial residuals and the direction are formed in
// FP32 with FP32 accumulation, everything else stays FP64).
// The team of G workgroups runs a.W steps (fewer when a.stop_on_cand ends it
// at a checkpoint); wg is this workgroup's index in the team.
template <int KIND, int CPL, typename TA>
__device__ __forceinline__ void fused_body(const FusedArgs& a, const int G, const int wg) {
  using TC = typename AStore<TA>::TC;
  using TS = typename AStore<TA>::TS;
  const TS* __restrict__ Amat = static_cast<const TS*>(a.A);
  // a launch enqueued ahead runs nothing after a checkpoint whose stop test
  // passed (every workgroup reads the same word, written by the previous
  // launch); a launch of no step reads nothing (the first step's slot is read
  // before the step loop)
  if (a.W <= 0 || (a.skip_on_cand &&
                   __hip_atomic_load(&a.ds->cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
    if (wg == 0 && threadIdx.x == 0 && a.mirror) {
      DevState st0;
      __builtin_memcpy(&st0, a.ds, sizeof(DevState));
      publish_mirror(a, st0);
    }
    return;
  }
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
  constexpr int TE = TileElems<TC, CPL>::value;
  constexpr int RMAX = TE / CPL;   // rows per wave held in registers (power of two, <= 64)
  constexpr int RSHIFT = (RMAX == 64) ? 0 : (RMAX == 32) ? 1 : (RMAX == 16) ? 2 : (RMAX == 8) ? 3 : 4;
  static_assert(RMAX >= 4 && RMAX <= 64, "rows per wave");
  __shared__ int32_t rsbuf[2][256];
  __shared__ double rv[256];
  __shared__ double yv[256];
  __shared__ double stage[256];
  __shared__ double wred[KIND == 0 ? 4 * 64 * CPL : 1];
  __shared__ double red[4];
  __shared__ double wpart[4 * kOwnRows];   // two-round exchange: the owner's wave sums,
  __shared__ double rloc[kOwnRows];        // its rows of r,
  __shared__ double rrk[kOwnMax];          // every owner's ||r_{R_k}||^2,
  __shared__ double yh[kTwoMaxBlock];      // and the sum of the later owners' parts of y
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
  const bool vec = a.vec_rows != 0 && slice1 == slice0 + 64 * CPL;   // uniform over the workgroup
  // Kaczmarz++, large team: exchange through row owners in two rounds (every
  // workgroup then sums the owners' parts of y; no y split)
  const bool two = KIND == 0 && a.xchg2 != 0;
  // Kaczmarz++ with y split across the team
  const bool ysplit = KIND == 0 && a.ysplit != 0 && !two;

  double xr[CPL], mr[CPL];
#pragma unroll
  for (int e = 0; e < CPL; ++e) {
    const int64_t j = col0 + e;
    xr[e] = j < n ? a.x[j] : 0.0;
    mr[e] = j < n ? a.mom[j] : 0.0;
  }
  // dual slice (Kaczmarz++ with m < n, the low-precision inner solver only):
  // rows d0 + tid + 256 u of [d0, d1)
  constexpr int DU = 4;
  double zxr[DU], zmr[DU];
  const bool dual = KIND == 0 && !std::is_same<TA, double>::value && a.zx != nullptr;
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
  TC tile[TE];
  int q = a.step_slot[0];
  int sb = a.lens[q];
  int cur = 0;
  // row indices run ahead of their use: myrow_c / myrow_n are this lane's
  // tile row index for the current and the next step, rown_n thread tid's
  // block row of the next step
  int32_t myrow_c = tile_row_index<CPL, TC, TE>(a.rows + static_cast<int64_t>(q) * s, sb, wv, lane);
  int32_t myrow_n = 0, rown_n = 0;
  if (a.W > 1) {
    const int q1 = a.step_slot[1];
    const int sb1 = a.lens[q1];
    myrow_n = tile_row_index<CPL, TC, TE>(a.rows + static_cast<int64_t>(q1) * s, sb1, wv, lane);
    if (tid < sb1) rown_n = a.rows[static_cast<int64_t>(q1) * s + tid];
  }
  load_tile<CPL>(tile, Amat, a.lda, n, myrow_c, col0, vec);
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
    if ((KIND == 0 || !KPP_PREFETCH) && k > 0) load_tile<CPL>(tile, Amat, a.lda, n, myrow_c, col0, vec);
    const double* Ginv = a.L + static_cast<int64_t>(q) * a.slot_stride + static_cast<int64_t>(s) * s;
    KPP_MARK(0)

    // 1. partial residuals of this wave's rows, butterfly across the lanes
    TC xt[CPL];
#pragma unroll
    for (int e = 0; e < CPL; ++e) xt[e] = static_cast<TC>(xr[e]);
    // the lane's products are summed in TC, the sums across lanes in FP64:
    // each butterfly stage halves the rows a lane holds, until lane l holds
    // row l >> RSHIFT of the wave (summed over lanes with the same row)
    double v[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      TC acc = 0;
#pragma unroll
      for (int e = 0; e < CPL; ++e) acc = fma(tile[r * CPL + e], xt[e], acc);
      v[r] = static_cast<double>(acc);
    }
#pragma unroll
    for (int cnt = RMAX, o = 32; cnt > 1; cnt >>= 1, o >>= 1) {
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int r = 0; r < cnt / 2; ++r) v[r] = fold(v[r], v[r + cnt / 2], o, up);
    }
#pragma unroll
    for (int o = 32 / RMAX; o >= 1; o >>= 1) v[0] = fold(v[0], v[0], o, false);
    {
      const int row = wv + 4 * (lane >> RSHIFT);
      if ((lane & ((1 << RSHIFT) - 1)) == 0 && row < sb) stage[row] = v[0];
    }
    if (two && tid < sb) rv[tid] = bval;
    __syncthreads();
    KPP_MARK(1)

    // 2. publish; prefetch (CD++); all-gather; reduce in a fixed order
    const uint32_t ep = a.epoch + static_cast<uint32_t>(k) + 1u;
    double* Pb = a.part + static_cast<size_t>(ep & 1u) * G * s;
    if (wv == 0) {
      for (int i = lane; i < sb; i += 64) st_coherent(&Pb[static_cast<size_t>(wg) * s + i], stage[i]);
      if (lane == 0) st_flag_after_stores(&a.flags[wg * kFlagStride], ep);
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
    // split Kaczmarz++: this workgroup's rows of y
    const int yper = (sb + G - 1) / G;
    if (ysplit) {
      lo = min(sb, wg * yper);
      hi = min(sb, lo + yper);
    }
    const bool have_next = k + 1 < a.W;
    const int qn = have_next ? a.step_slot[k + 1] : q;
    const int sbn = a.lens[qn];
    // Loads that do not depend on r go out before the wait, in this order: the
    // memoized inverse's rows for this slice (CD++), the next tile (CD++,
    // every wave), the next b values, the row indices of step k + 2 (last: their
    // addresses come from a chain of dependent scalar loads).  A wave's
    // loads complete in order, so the wave that polls the flags sees its first
    // flag only once these have landed, and the partial-residual loads after
    // the wait do not queue behind a tile.
    // CD++: slice rows lo + wv and lo + wv + 4 (lanes hold entries kk = lane + 64 u)
    double grow0[4] = {0.0, 0.0, 0.0, 0.0}, grow1[4] = {0.0, 0.0, 0.0, 0.0};
    const int own0 = wg * kOwnRows, own1 = min(sb, own0 + kOwnRows);
    if (two && own0 < sb && tid < sb) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (own0 + u < own1) grow0[u] = Ginv[static_cast<int64_t>(own0 + u) * s + tid];
        if (own0 + 4 + u < own1) grow1[u] = Ginv[static_cast<int64_t>(own0 + 4 + u) * s + tid];
      }
    }
    if (KIND == 1 || ysplit) {
      const int i0 = lo + wv, i1 = lo + wv + 4;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = min(lane + 64 * u, sb - 1);
        if (i0 < hi && 64 * u < sb) grow0[u] = Ginv[static_cast<int64_t>(i0) * s + kk];
        if (i1 < hi && 64 * u < sb) grow1[u] = Ginv[static_cast<int64_t>(i1) * s + kk];
      }
    }
    if (KIND == 1 && KPP_PREFETCH && have_next) load_tile<CPL>(tile, Amat, a.lda, n, myrow_n, col0, vec);
    double bnext = 0.0;
    if (have_next && tid < sbn) {
      rsbuf[cur ^ 1][tid] = rown_n;
      bnext = a.b[rown_n];
    }
    int32_t myrow_nn = 0, rown_nn = 0;
    if (k + 2 < a.W) {
      const int q2 = a.step_slot[k + 2];
      const int sb2 = a.lens[q2];
      const int32_t* R2 = a.rows + static_cast<int64_t>(q2) * s;
      myrow_nn = tile_row_index<CPL, TC, TE>(R2, sb2, wv, lane);
      if (tid < sb2) rown_nn = R2[tid];
    }
    const int nu = (sb + 63) >> 6;
    if (two) {
      // round 1: owner k waits for every partial, sums those of its rows R_k
      // (thread g < G loads workgroup g's, an 8-row butterfly per wave, the
      // four waves in order), subtracts b, and publishes c_k = G^{-1}[:, R_k]
      // r_{R_k} (thread j forms entry j from the G^{-1} column it prefetched)
      // and ||r_{R_k}||^2.  Round 2: every workgroup waits for the owners and
      // sums the c_k in owner order: the same y everywhere.  Each flag is
      // polled by a thread of its own.
      const int nown = (sb + kOwnRows - 1) / kOwnRows;
      double* Cb = a.ypart + kOwnOffset + static_cast<size_t>(ep & 1u) * kOwnMax * kOwnStride;
      uint32_t* f2 = a.flags + kYFlagOffset;
      const bool owner = own0 < sb;
      if (owner && tid < G && !wait_flag(&a.flags[tid * kFlagStride], ep, a.spin_limit)) {
        atomicOr(a.err, 2);
        abort_flag = 1;
      }
      __syncthreads();
      if (abort_flag) break;
      if (owner) {
        double pv[kOwnRows];
#pragma unroll
        for (int u = 0; u < kOwnRows; ++u)
          pv[u] = (tid < G && own0 + u < own1) ? ld_coherent(&Pb[static_cast<size_t>(tid) * s + own0 + u]) : 0.0;
#pragma unroll
        for (int cnt = kOwnRows, o = 32; cnt > 1; cnt >>= 1, o >>= 1) {
          const bool up = (lane & o) != 0;
#pragma unroll
          for (int r = 0; r < cnt / 2; ++r) pv[r] = fold(pv[r], pv[r + cnt / 2], o, up);
        }
#pragma unroll
        for (int o = 32 / kOwnRows; o >= 1; o >>= 1) pv[0] = fold(pv[0], pv[0], o, false);
        if ((lane & (64 / kOwnRows - 1)) == 0) wpart[wv * kOwnRows + lane / (64 / kOwnRows)] = pv[0];
        __syncthreads();
        if (tid < kOwnRows) {
          const int i = own0 + tid;
          rloc[tid] = (i < own1) ? (((wpart[tid] + wpart[kOwnRows + tid]) + wpart[2 * kOwnRows + tid]) +
                                    wpart[3 * kOwnRows + tid]) - rv[i]
                                 : 0.0;
        }
        __syncthreads();
        if (tid < sb) {
          double acc = 0.0;
#pragma unroll
          for (int u = 0; u < 4; ++u) acc = fma(grow0[u], rloc[u], acc);
#pragma unroll
          for (int u = 0; u < 4; ++u) acc = fma(grow1[u], rloc[4 + u], acc);
          st_coherent(&Cb[static_cast<size_t>(wg) * kOwnStride + tid], acc);
        }
        if (tid == kT - 1) {
          double q2 = 0.0;
#pragma unroll
          for (int u = 0; u < kOwnRows; ++u) q2 = fma(rloc[u], rloc[u], q2);
          st_coherent(&Cb[static_cast<size_t>(wg) * kOwnStride + kTwoMaxBlock], q2);
        }
        // every wave's stores complete before the flag
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) st_flag_after_stores(&f2[wg * kFlagStride], ep);
      }
      if (tid < nown && !wait_flag(&f2[tid * kFlagStride], ep, a.spin_limit)) {
        atomicOr(a.err, 2);
        abort_flag = 1;
      }
      __syncthreads();
      KPP_MARK(3)
      if (abort_flag) break;
      // entry j: threads j and j + 128 sum owners 0..7 and 8..15 (added
      // after the barrier below)
      static_assert(kT == 2 * kTwoMaxBlock && kOwnMax == 16, "two-round exchange layout");
      const int j = tid & (kTwoMaxBlock - 1), h = tid >> 7;
      if (j < sb) {
        double cv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k2 = 8 * h + u;
          cv[u] = (k2 < nown) ? ld_coherent(&Cb[static_cast<size_t>(k2) * kOwnStride + j]) : 0.0;
        }
        double acc = cv[0];
#pragma unroll
        for (int u = 1; u < 8; ++u) acc += cv[u];
        if (h == 0) yv[j] = acc; else yh[j] = acc;
      }
      if (tid < nown) rrk[tid] = ld_coherent(&Cb[static_cast<size_t>(tid) * kOwnStride + kTwoMaxBlock]);
    } else {
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
      rr_w = wave_sum(rr_w);
      if (lane == 0) red[wv] = rr_w;
    }
    }
    __syncthreads();
    KPP_MARK(4)

    // 3. y through the memoized inverse
    if (KIND == 1 || ysplit) {
      // CD++: the rows of y whose coordinates fall into the slice; split
      // Kaczmarz++: this workgroup's share of y.  Row lo + t belongs to wave
      // t % 4; the first two rows of a wave were loaded before the wait
      for (int i = lo + wv, j = 0; i < hi; i += 4, ++j) {
        double acc = 0.0;
        if (j < 2) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int kk = lane + 64 * u;
            if (kk < sb) acc = fma(j == 0 ? grow0[u] : grow1[u], rv[kk], acc);
          }
        } else {
          const double* Gi = Ginv + static_cast<int64_t>(i) * s;
          for (int kk = lane; kk < sb; kk += 64) acc = fma(Gi[kk], rv[kk], acc);
        }
        acc = wave_sum(acc);
        if (lane == 0) yv[i] = acc;
      }
      if (ysplit) {
        // all-gather of y: publish this workgroup's rows, wait for every
        // workgroup that owns rows, read all of y (the same values everywhere)
        __syncthreads();
        // (after a two-level exchange of r, the y all-gather has buffers and
        // flags of its own: r's occupy the first ones)
        double* Yb = a.ypart + (two ? 2 * kTwoMaxBlock : 0) + static_cast<size_t>(ep & 1u) * s;
        uint32_t* yflags = a.flags + kYFlagOffset + (two ? kFusedMaxGroups * kFlagStride : 0);
        if (wv == 0) {
          for (int i = lo + lane; i < hi; i += 64) st_coherent(&Yb[i], yv[i]);
          if (lane == 0) st_flag_after_stores(&yflags[wg * kFlagStride], ep);
        }
        const int nown = (sb + yper - 1) / yper;
        if (tid < nown) {
          int64_t spins = 0;
          while (static_cast<int32_t>(ld_flag(&yflags[tid * kFlagStride]) - ep) < 0) {
            if (++spins > a.spin_limit) {
              atomicOr(a.err, 2);
              abort_flag = 1;
              break;
            }
          }
        }
        __syncthreads();
        if (abort_flag) break;
        if (tid < sb) yv[tid] = ld_coherent(&Yb[tid]);
      }
    } else if (two) {
      if (tid < sb) yv[tid] += yh[tid];
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
      double rr = 0.0;
      if (two) {
        for (int k2 = 0; k2 < (sb + kOwnRows - 1) / kOwnRows; ++k2) rr += rrk[k2];
      } else {
        rr = red[0];
        for (int w = 1; w < ((sb + 63) >> 6); ++w) rr += red[w];
      }
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
      TC wt[CPL];
#pragma unroll
      for (int e = 0; e < CPL; ++e) wt[e] = 0;
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        const int i = wv + 4 * r;
        const TC yi = static_cast<TC>((i < sb) ? yv[i] : 0.0);
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
    myrow_c = myrow_n;
    myrow_n = myrow_nn;
    rown_n = rown_nn;
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
  if (wg == 0 && tid == 0) {
    *a.ds = st;
    if (a.mirror) publish_mirror(a, st);
  }
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
const void* fused_kernel_ptr(int cpl) {
  switch (cpl) {
    case 1: return reinterpret_cast<const void*>(&k_fused<KIND, 1, TA>);
    case 2: return reinterpret_cast<const void*>(&k_fused<KIND, 2, TA>);
    case 4: return reinterpret_cast<const void*>(&k_fused<KIND, 4, TA>);
    case 8: return reinterpret_cast<const void*>(&k_fused<KIND, 8, TA>);
    default: return reinterpret_cast<const void*>(&k_fused<KIND, 16, TA>);
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

int32_t fused_blocks_per_cu(int32_t kind, int32_t prec, int32_t cpl) {
  const void* f = nullptr;
  if (kind == 0)
    f = prec == 2 ? fused_kernel_ptr<0, Bf16>(cpl) : prec == 1 ? fused_kernel_ptr<0, float>(cpl) : fused_kernel_ptr<0, double>(cpl);
  else
    f = prec == 2 ? fused_kernel_ptr<1, Bf16>(cpl) : prec == 1 ? fused_kernel_ptr<1, float>(cpl) : fused_kernel_ptr<1, double>(cpl);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kT, 0) != hipSuccess) return 0;
  return nb;
}

void launch_fused(int32_t kind, int32_t prec, const FusedArgs& a, int32_t cpl, int32_t groups, hipStream_t st) {
  if (kind == 0) {
    if (prec == 2)
      launch_kind<0, Bf16>(a, cpl, groups, st);
    else if (prec == 1)
      launch_kind<0, float>(a, cpl, groups, st);
    else
      launch_kind<0, double>(a, cpl, groups, st);
  } else {
    if (prec == 2)
      launch_kind<1, Bf16>(a, cpl, groups, st);
    else if (prec == 1)
      launch_kind<1, float>(a, cpl, groups, st);
    else
      launch_kind<1, double>(a, cpl, groups, st);
  }
}

}  // namespace kpp
