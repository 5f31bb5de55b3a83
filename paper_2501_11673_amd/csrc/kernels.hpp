// Internal kernel launchers of the block-step library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace kpp {

// Solver scalars kept on the device so that no step needs the host
// (Section 5.4: window sums, checkpoint counter, running rate estimate).
struct DevState {
  double rho;        // momentum parameter for the next step
  double rhat;       // weighted average of window ratios (eq. (weighted))
  double E0, E1;     // window sums of ||r_t||^2 (Algorithms 2 and 5)
  double c;          // (1 - rho)/(1 + rho) used by the current step's update
  double thr;        // eps^2 ||b||^2
  double last_E1;    // E1 of the last checkpoint (estimated residual)
  double rho_before; // rho before the last checkpoint's revision
  int64_t t;         // steps completed
  int32_t ckpt;      // checkpoints that revised rho
  int32_t have_rhat;
  int32_t cand;      // the last checkpoint met E1 <= thr (host confirms)
  int32_t ckpts;     // checkpoints seen
  int32_t err;       // device-side error code (0 = none)
  int32_t pad;
};

constexpr int kMaxBlock = 512;      // largest supported block size s
constexpr int kLdsCholMax = 128;    // blocks up to this size are factored in LDS

// Host-visible copy of a launch's end state (pinned, coherent host memory).
struct HostMirror {
  DevState ds;
  int32_t err;
  int32_t fp64_count;
  uint32_t seq;   // raised last
  uint32_t pad;
};
static_assert(sizeof(DevState) % 8 == 0 && offsetof(HostMirror, err) % 8 == 0 &&
                  offsetof(HostMirror, fp64_count) == offsetof(HostMirror, err) + 4,
              "HostMirror: the error words are stored as one 8-byte word");

// Factor-time checks.  only: process just the blocks with only[k] != 0.
// flag (low-precision pass): instead of failing, set flag[k] = 1 when the
// factor breaks down or kappa(G) >= (max L_ii / min L_ii)^2 exceeds
// kappa_max, count it in *counter and leave that block to an FP64 redo.
struct FactorCheck {
  const int32_t* only = nullptr;
  int32_t* flag = nullptr;
  int32_t* counter = nullptr;
  double kappa_max = 1.0 / 0.0;
};

// r-partials of the block residual: rpart[i * P + p] = sum_{j in chunk p} A[rows[i], j] x[j]
void launch_block_gemv_partial(const double* A, int64_t lda, int64_t n, const int32_t* rows,
                               int32_t sb, const double* x, double* rpart, int32_t P,
                               int64_t chunk, hipStream_t st);

// r = sum_p rpart - b_S; E-sum and checkpoint bookkeeping; y = G^{-1} r
void launch_block_project(const double* rpart, int32_t P, const double* b, const int32_t* rows,
                          int32_t sb, const double* Ginv, int32_t ldl, double* y, DevState* ds,
                          int32_t zeta, int32_t adaptive, hipStream_t st);

// x, m update with w = A_S^T y (Kaczmarz++) or w = I_S^T y (CD++)
void launch_update(int32_t kind, const double* A, int64_t lda, int64_t n, const int32_t* rows,
                   int32_t sb, const double* y, const DevState* ds, double eta, double* x,
                   double* mom, hipStream_t st);

// Regularized Grams of nb blocks into column-major s x s slots (lower part);
// block k is staged at rows[k * s], lens[k] and goes to slot slot_of[k], whose
// first element is G[slot_of[k] * stride].  Kaczmarz++ Grams use the MFMA
// SYRK below and need gram_syrk_work(s, n, nb) doubles of workspace in ws.
void launch_gram(int32_t kind, const double* A, int64_t lda, int64_t n, const int32_t* rows,
                 const int32_t* lens, int32_t s, int32_t nb, double lambda, double* G, int64_t stride,
                 const int32_t* slot_of, double* ws, hipStream_t st, const int32_t* only = nullptr);

// The same Grams from an FP32 copy of A (FP32 products, FP32 accumulation),
// written to the FP64 slots.
void launch_gram_f32(int32_t kind, const float* A, int64_t lda, int64_t n, const int32_t* rows,
                     const int32_t* lens, int32_t s, int32_t nb, double lambda, double* G, int64_t stride,
                     const int32_t* slot_of, double* ws, hipStream_t st);

// Kaczmarz++ Grams A_S A_S^T + lambda I on the matrix cores: a workgroup
// forms every 16 x 16 tile of a block's lower triangle over one column chunk
// (16x16x4 MFMA, FP64, or FP32 in / FP32 accumulate), reading the block's
// rows once; FP64 partial tiles are summed in chunk order.  The rows are cut
// into gram_groups(s) groups of 16; gram_syrk_plan gives the split (ntiles =
// lower tiles per block, nchunks column chunks of `chunk` columns).
constexpr int kGramTile = 16;
constexpr int kGramTargetGroups = 512;
constexpr int kGramMinPanels = 8;       // a chunk spans at least this many LDS panels
inline int32_t gram_groups(int32_t s) {
  int32_t g = 2;
  while (16 * g < s) g *= 2;
  return g;
}
inline int32_t gram_panel(int32_t groups) { return groups <= 4 ? 32 : (groups <= 16 ? 16 : 8); }
void gram_syrk_plan(int32_t s, int64_t n, int32_t nb, int32_t* nchunks, int64_t* chunk, int32_t* ntiles);
size_t gram_syrk_work(int32_t s, int64_t n, int32_t nb);
void launch_gram_syrk(const double* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens, int32_t s,
                      int32_t nb, double lambda, double* G, int64_t stride, const int32_t* slot_of,
                      const int32_t* only, double* ws, hipStream_t st);
void launch_gram_syrk_f32(const float* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens, int32_t s,
                          int32_t nb, double lambda, double* G, int64_t stride, const int32_t* slot_of,
                          double* ws, hipStream_t st);

// In-place Cholesky of nb slots; breakdown sets *err = 1.  Blocks of
// kLdsCholMax+1 .. kFusedMaxBlock rows are factored in LDS panels.
void launch_cholesky(double* G, int32_t s, int64_t stride, const int32_t* lens, int32_t nb,
                     const int32_t* slot_of, int32_t* err, hipStream_t st, FactorCheck chk = FactorCheck());

// G^{-1} = L^{-T} L^{-1} of each slot's factor (at +s*s, full symmetric);
// blocks larger than kLdsCholMax use the slot's last s*s doubles as scratch
// (blocked in LDS up to kFusedMaxBlock rows).  With chk.flag set
// (low-precision pass), blocks whose Frobenius condition number exceeds
// chk.kappa_max are flagged; launch_cholesky with the same check must have run
// first (it leaves ||G||_F^2 in the slot).
void launch_factor_inverse(double* slots, int64_t stride, int32_t s, const int32_t* lens, int32_t nb,
                           const int32_t* slot_of, hipStream_t st, FactorCheck chk = FactorCheck(),
                           const int32_t* skip = nullptr);

// Blocks of at most kFactorSmallMax rows: Cholesky in place (breakdown sets
// *err = 1) and, if want_inverse, G^{-1} at +s*s, one register-resident
// workgroup per block.
constexpr int kFactorSmallMax = 128;
void launch_factor_small(double* slots, int64_t stride, int32_t s, const int32_t* lens, int32_t nb,
                         const int32_t* slot_of, int32_t want_inverse, int32_t* err, hipStream_t st,
                         FactorCheck chk = FactorCheck());

// rows[slot_of[k] * s + i] = stage_rows[k * s + i]; lens[slot_of[k]] = stage_lens[k]
void launch_scatter_rows(const int32_t* stage_rows, const int32_t* stage_lens, const int32_t* slot_of,
                         int32_t nb, int32_t s, int32_t* rows, int32_t* lens, hipStream_t st);

// Memo slot size (doubles): column-major L, G^{-1}, scratch.
inline int64_t slot_doubles(int32_t s) { return 3 * static_cast<int64_t>(s) * s; }

// ||A x - b||^2 partial sums per row group (deterministic), then a final sum.
void launch_residual_sq(const double* A, int64_t lda, int64_t m, int64_t n, const double* x,
                        const double* b, double* part, int32_t nparts, double* out,
                        hipStream_t st);

// finiteness check of an m x n strided matrix and a vector; sets *flag = 1 on NaN/Inf
void launch_check_finite(const double* A, int64_t lda, int64_t m, int64_t n, const double* b,
                         int32_t* flag, hipStream_t st);

// the run's starting state, *err = 0 and mom[0..n) = 0, in one launch
void launch_state_init(DevState* ds, double rho0, double thr, int32_t* err, double* mom, int64_t n, hipStream_t st);
// a[0..na), b[0..nb), c[0..nc) = 0 in one launch
void launch_zero3(double* a, int64_t na, double* b, int64_t nb, double* c, int64_t nc, hipStream_t st);

// out[i * n + j] = (float) A[i * lda + j]   (row-major FP32 copy, leading dimension n)
void launch_convert_f32(const double* A, int64_t lda, int64_t m, int64_t n, float* out, hipStream_t st);
// bfloat16 copy (leading dimension n): each entry rounded to FP32, then to
// the nearest bfloat16 (ties to even), kept as its 16 bits
void launch_convert_bf16(const double* A, int64_t lda, int64_t m, int64_t n, uint16_t* out, hipStream_t st);

// r = b - A x (FP64), rowsq[i] = r_i^2, *out = sum_i rowsq[i] in a fixed order
void launch_residual_vec(const double* A, int64_t lda, int64_t m, int64_t n, const double* x,
                         const double* b, double* r, double* rowsq, double* out, hipStream_t st);

// x += d  (FP64)
void launch_axpy1(double* x, const double* d, int64_t n, hipStream_t st);

// d = A^T z (m x n row-major A, FP64, fixed summation order over the rows);
// ws: gemv_t_splits(m, n) * n doubles of partial sums (unused for one split)
int32_t gemv_t_splits(int64_t m, int64_t n);
void launch_gemv_t(const double* A, int64_t lda, int64_t m, int64_t n, const double* z, double* d, double* ws,
                   hipStream_t st);

// Arguments of the fused persistent engine (fused.hip): W block steps of one
// system per launch, `groups` workgroups each owning 64 * cpl columns.
struct FusedArgs {
  const void* A;             // double, or float for the mixed-precision inner solver
  int64_t lda;
  int64_t n;
  const double* b;
  const int32_t* rows;       // slot table: rows of slot q at rows[q * s]
  const int32_t* lens;       // slot table: block length of slot q
  const double* L;           // slot table: factor data of slot q at L[q * slot_stride]
  int64_t slot_stride;
  int32_t s;
  int32_t W;                 // steps in this launch
  const int32_t* step_slot;  // slot used by step k of this launch
  double* x;
  double* mom;
  double* part;              // 2 x groups x s partial residuals (double-buffered by step parity)
  uint32_t* flags;           // one flag per workgroup, 128 bytes apart
  uint32_t epoch;            // flag value after step k of this launch: epoch + k + 1
  int32_t zeta;
  int32_t adaptive;
  double eta;
  DevState* ds;
  int32_t* err;              // bit 1: a wait exceeded spin_limit
  int64_t spin_limit;
  uint64_t* phase_ticks;     // optional (nullptr): wall-clock ticks per step phase, workgroup 0
  int32_t stop_on_cand;      // 1: end the launch after a checkpoint whose stop test passes
  int32_t vec_rows;          // 1: A and lda keep every row 16-byte aligned (vector tile loads)
  // Kaczmarz++ with m < n only (optional, nullptr = off): the dual of the
  // iterate and of the momentum, x = A^T zx and m = A^T zm in exact
  // arithmetic (m FP64 entries each, in and out like x and mom)
  double* zx;
  double* zm;
  int64_t mrows;
  // Kaczmarz++ only: 1 = y = G^{-1} r is split across the team (each
  // workgroup forms ceil(s/G) rows, then one all-gather of y through ypart,
  // 2 x s doubles, and a second set of flags); 0 = every workgroup forms all of y
  double* ypart;
  int32_t ysplit;
  // Kaczmarz++ with blocks of at most kTwoMaxBlock rows only: 1 = exchange
  // through row owners in two rounds.  Owner k (workgroup k) sums the G
  // partials of block rows R_k = [kOwnRows k, kOwnRows (k + 1)), forms its
  // part of y, c_k = G^{-1}[:, R_k] r_{R_k}, and ||r_{R_k}||^2, and publishes
  // them (kOwnStride doubles at ypart + kOwnOffset, double-buffered by step
  // parity) under the second set of flags; every workgroup sums the c_k in
  // owner order.  ysplit is then ignored.
  int32_t xchg2;
  // optional (nullptr = off; single teams only): at the end of the launch
  // workgroup 0 writes the DevState, *err and *fp64_count (when given) to this
  // host-visible mirror with system-scope stores and then raises mirror->seq
  // to seq, so that the host can read the state without a copy
  HostMirror* mirror;
  const int32_t* fp64_count;
  uint32_t seq;
  // 1: a launch enqueued before the previous one ended: it runs no step when
  // the previous launch ended at a checkpoint whose stop test passed
  // (DevState::cand), leaving the state as it is (the host then confirms the
  // stop, or launches the window again with skip_on_cand = 0)
  int32_t skip_on_cand;
};
constexpr int kTwoMaxBlock = 128;
constexpr int kOwnRows = 8;
constexpr int kOwnMax = kTwoMaxBlock / kOwnRows;
constexpr int kOwnStride = kTwoMaxBlock + 8;   // c_k, then ||r_{R_k}||^2 at kTwoMaxBlock

constexpr int kFusedPhases = 8;

constexpr int kFusedMaxBlock = 256;   // the fused engine gives one thread per block row
constexpr int kFusedMaxGroups = 256;
constexpr int kFlagWordsAlloc = 1024 * kFusedMaxGroups;   // up to 4 KB between flags
// the y all-gather's flags start this many words into the flag area
constexpr int kYFlagOffset = kFlagWordsAlloc / 2;
// exchange buffer per system: partial residuals, then the y all-gather
// (ypart), then the owners' contributions of the two-round exchange
constexpr size_t kOwnOffset = 2 * kFusedMaxBlock;   // from ypart
constexpr size_t kPartDoubles = 2 * static_cast<size_t>(kFusedMaxGroups) * kFusedMaxBlock + kOwnOffset +
                                2 * static_cast<size_t>(kOwnMax) * kOwnStride;

// prec: 0 FP64 A, 1 FP32 A, 2 bfloat16 A (widened to FP32 in the tile)
void launch_fused(int32_t kind, int32_t prec, const FusedArgs& a, int32_t cpl, int32_t groups, hipStream_t st);

// Workgroups of the step kernel for (kind, precision, cpl) that one compute
// unit can hold at once (the occupancy query; 0 if it fails).  A team must be
// resident as a whole: its workgroups wait for each other every step.
int32_t fused_blocks_per_cu(int32_t kind, int32_t prec, int32_t cpl);

// Several independent runs in one launch: team t has the workgroups
// [team_start[t], team_start[t + 1]) and the arguments args[t] (device
// memory); every team has the same kind, precision and cpl.  The caller keeps
// team_start[nteams] <= the number of compute units (one workgroup each) so
// that every team is resident at once.
void launch_fused_multi(int32_t kind, bool a_fp32, const FusedArgs* args, const int32_t* team_start,
                        int32_t nteams, int32_t total_groups, int32_t cpl, hipStream_t st);

// p[i] = base + step * i for i < n (step 0: a fill; step 1: consecutive ids)
void launch_fill_i32(int32_t* p, int64_t n, int32_t base, int32_t step, hipStream_t st);
// p[i] = 0 for i < n (a kernel rather than a memset node)
void launch_zero_f64(double* p, int64_t n, hipStream_t st);

// Split-Gram plan with at most max_work doubles of partial tiles: fewer
// column chunks than gram_syrk_plan when its split would not fit (nb blocks
// must fit with one chunk each: nb * ntiles * 64 * 64 <= max_work).  The
// launcher forms the same Grams as launch_gram (Kaczmarz++, FP64 A).
void gram_syrk_plan_capped(int32_t s, int64_t n, int32_t nb, size_t max_work, int32_t* nchunks, int64_t* chunk,
                           int32_t* ntiles);
void launch_gram_syrk_capped(const double* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens,
                             int32_t s, int32_t nb, double lambda, double* G, int64_t stride, const int32_t* slot_of,
                             double* ws, size_t max_work, hipStream_t st);

// Per-device scratch of the no-allocation entry point (noalloc.hip): a
// file-scope device array of kNoAllocScratchBytes.  noalloc_scratch returns
// its device address on `device`, which must be the current device; the
// address is resolved once per device and kept.
constexpr size_t kNoAllocScratchBytes = size_t{16} << 20;
hipError_t noalloc_scratch(int device, void** out);

// Randomized Hadamard transform (rht.hip): out = Do H_M Di X Dc along the row
// index of a row-major X, where Di, Dc, Do are optional diagonals of signs
// times a scale, X is zero-padded to M rows (rows >= rows_valid) and ncols
// columns (columns >= cols_valid), and output rows >= rows_out are dropped.
// transpose_out stores out[col * ld_out + row].  M is a power of two up to
// kFhtMaxRows; M > 4096 takes two passes, whose intermediate lives in out when
// the last pass can run in place there, otherwise in work (M x ncols).  in
// must not overlap out unless the transform is a single in-place pass without
// transpose.
constexpr int kFhtMaxDigitLog = 12;
constexpr int64_t kFhtMaxRows = int64_t{1} << (2 * kFhtMaxDigitLog);
struct FhtSpec {
  const double* in = nullptr;
  int64_t ld_in = 0;
  int64_t rows_valid = 0, cols_valid = 0;
  const int8_t* isign = nullptr;
  const int8_t* csign = nullptr;
  double iscale = 1.0, cscale = 1.0;
  double* out = nullptr;
  int64_t ld_out = 0;
  int64_t rows_out = 0;
  const int8_t* osign = nullptr;
  double oscale = 1.0;
  int32_t transpose_out = 0;
  int64_t M = 0, ncols = 0;
  double* work = nullptr;
};
inline int fht_passes(int64_t M) { return M > (int64_t{1} << kFhtMaxDigitLog) ? 2 : 1; }
void launch_fht(const FhtSpec& s, hipStream_t st);

}  // namespace kpp
