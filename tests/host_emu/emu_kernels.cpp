// CPU stand-ins for the library's kernel launchers (host-logic test): every
// device range a kernel would touch is checked against the live allocations
// of the stand-in runtime, and the solver state evolves with a modelled block
// residual so that checkpoints, stops and refinement rounds occur.  Nothing
// here computes the method; parity of the numbers is tested on the GPU.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>

#include "kernels.hpp"
#include "lsqr.hpp"
#include "multi.hpp"
#include "sparse.hpp"

namespace kpp {
namespace {
double model_rr(int64_t t) { return std::pow(0.985, static_cast<double>(t)); }
void emu_step(DevState* ds, int32_t zeta, bool* stop) {
  emu_check(ds, sizeof(DevState), "DevState");
  DevState& s = *ds;
  const double rr = model_rr(s.t);
  const int64_t period = 2 * static_cast<int64_t>(zeta);
  const int64_t ph = s.t % period;
  if (ph < zeta) s.E0 += rr; else s.E1 += rr;
  if (stop) *stop = false;
  if (ph == period - 1) {
    s.ckpts += 1;
    s.last_E1 = s.E1;
    s.cand = s.E1 <= s.thr;
    if (stop) *stop = s.cand;
    s.E0 = s.E1 = 0.0;
  }
  s.t += 1;
}
void check_rows(const int32_t* rows, int32_t sb, const char* what) {
  emu_check(rows, sizeof(int32_t) * sb, what);
}
void check_A(const void* A, size_t esz, int64_t lda, const int32_t* rows, int32_t sb, int64_t n, const char* what) {
  for (int32_t i = 0; i < sb; ++i) {
    const int64_t r = rows[i];
    if (r < 0) { std::fprintf(stderr, "EMU: negative row %lld in %s\n", (long long)r, what); std::abort(); }
    emu_check(static_cast<const char*>(A) + esz * (r * lda), esz * n, what);
  }
}
}  // namespace

void launch_block_gemv_partial(const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb,
                               const double* x, double* rpart, int32_t P, int64_t, hipStream_t) {
  check_rows(rows, sb, "gemv rows");
  check_A(A, 8, lda, rows, sb, n, "gemv A");
  emu_check(x, 8 * n, "gemv x");
  emu_check(rpart, 8 * sb * P, "gemv rpart");
}
void launch_block_project(const double* rpart, int32_t P, const double* b, const int32_t* rows, int32_t sb,
                          const double* Ginv, int32_t ldl, double* y, DevState* ds, int32_t zeta, int32_t,
                          hipStream_t) {
  emu_check(rpart, 8 * sb * P, "project rpart");
  check_rows(rows, sb, "project rows");
  for (int i = 0; i < sb; ++i) emu_check(b + rows[i], 8, "project b");
  emu_check(Ginv, 8 * (static_cast<size_t>(sb - 1) * ldl + sb), "project Ginv");
  emu_check(y, 8 * sb, "project y");
  emu_step(ds, zeta, nullptr);
}
void launch_update(int32_t kind, const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb,
                   const double* y, const DevState* ds, double, double* x, double* mom, hipStream_t) {
  check_rows(rows, sb, "update rows");
  if (kind == 0) check_A(A, 8, lda, rows, sb, n, "update A");
  emu_check(y, 8 * sb, "update y");
  emu_check(ds, sizeof(DevState), "update ds");
  emu_check(x, 8 * n, "update x");
  emu_check(mom, 8 * n, "update mom");
}
static void check_slots(const double* G, int64_t stride, int32_t s, const int32_t* lens, int32_t nb,
                        const int32_t* slot_of, int64_t span, const char* what) {
  emu_check(lens, 4 * nb, what);
  emu_check(slot_of, 4 * nb, what);
  for (int k = 0; k < nb; ++k) {
    if (lens[k] < 1 || lens[k] > s) { std::fprintf(stderr, "EMU: %s len %d\n", what, lens[k]); std::abort(); }
    emu_check(G + slot_of[k] * stride, 8 * span, what);
  }
}
void launch_gram(int32_t kind, const double* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens,
                 int32_t s, int32_t nb, double, double* G, int64_t stride, const int32_t* slot_of, double* ws,
                 hipStream_t, const int32_t* only) {
  if (nb <= 0) return;
  check_slots(G, stride, s, lens, nb, slot_of, static_cast<int64_t>(s) * s, "gram slots");
  for (int k = 0; k < nb; ++k) {
    if (only && !only[k]) continue;
    check_rows(rows + static_cast<int64_t>(k) * s, lens[k], "gram rows");
    check_A(A, 8, lda, rows + static_cast<int64_t>(k) * s, lens[k], n, "gram A");
  }
  if (kind == 0) emu_check(ws, 8 * gram_syrk_work(s, n, nb), "gram ws");
}
void launch_gram_f32(int32_t kind, const float* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens,
                     int32_t s, int32_t nb, double, double* G, int64_t stride, const int32_t* slot_of, double* ws,
                     hipStream_t) {
  if (nb <= 0) return;
  check_slots(G, stride, s, lens, nb, slot_of, static_cast<int64_t>(s) * s, "gram32 slots");
  for (int k = 0; k < nb; ++k) check_A(A, 4, lda, rows + static_cast<int64_t>(k) * s, lens[k], n, "gram32 A");
  if (kind == 0) emu_check(ws, 8 * gram_syrk_work(s, n, nb), "gram32 ws");
}
void launch_gram_syrk_capped(const double* A, int64_t lda, int64_t n, const int32_t* rows, const int32_t* lens,
                             int32_t s, int32_t nb, double, double* G, int64_t stride, const int32_t* slot_of,
                             double* ws, size_t max_work, hipStream_t) {
  if (nb <= 0) return;
  check_slots(G, stride, s, lens, nb, slot_of, static_cast<int64_t>(s) * s, "gram capped slots");
  for (int k = 0; k < nb; ++k) check_A(A, 8, lda, rows + static_cast<int64_t>(k) * s, lens[k], n, "gram capped A");
  int32_t nc, nt;
  int64_t chunk;
  gram_syrk_plan_capped(s, n, nb, max_work, &nc, &chunk, &nt);
  const size_t work = static_cast<size_t>(nb) * nt * nc * kGramTile * kGramTile;
  if (work > max_work) { std::fprintf(stderr, "EMU: capped gram plan exceeds its cap\n"); std::abort(); }
  emu_check(ws, 8 * work, "gram capped ws");
}
void launch_fill_i32(int32_t* p, int64_t n, int32_t base, int32_t step, hipStream_t) {
  emu_check(p, 4 * static_cast<size_t>(n), "fill i32");
  for (int64_t i = 0; i < n; ++i) p[i] = base + step * static_cast<int32_t>(i);
}
void launch_zero_f64(double* p, int64_t n, hipStream_t) {
  emu_check(p, 8 * static_cast<size_t>(n), "zero f64");
  for (int64_t i = 0; i < n; ++i) p[i] = 0.0;
}
hipError_t noalloc_scratch(int, void** out) {
  static void* p = nullptr;
  if (!p && hipMalloc(&p, kNoAllocScratchBytes) != hipSuccess) return hipErrorOutOfMemory;
  *out = p;
  return hipSuccess;
}
void launch_gram_syrk(const double*, int64_t, int64_t, const int32_t*, const int32_t*, int32_t, int32_t, double,
                      double*, int64_t, const int32_t*, const int32_t*, double*, hipStream_t) {}
void launch_gram_syrk_f32(const float*, int64_t, int64_t, const int32_t*, const int32_t*, int32_t, int32_t, double,
                          double*, int64_t, const int32_t*, double*, hipStream_t) {}
void launch_cholesky(double* G, int32_t s, int64_t stride, const int32_t* lens, int32_t nb, const int32_t* slot_of,
                     int32_t* err, hipStream_t, FactorCheck chk) {
  if (nb <= 0) return;
  const int64_t ss = static_cast<int64_t>(s) * s;
  check_slots(G, stride, s, lens, nb, slot_of, chk.flag ? 3 * ss : ss, "cholesky slots");
  emu_check(err, 4, "cholesky err");
  if (chk.flag) { emu_check(chk.flag, 4 * nb, "cholesky flag"); for (int k = 0; k < nb; ++k) chk.flag[k] = 0; }
}
void launch_factor_inverse(double* slots, int64_t stride, int32_t s, const int32_t* lens, int32_t nb,
                           const int32_t* slot_of, hipStream_t, FactorCheck, const int32_t*) {
  if (nb <= 0) return;
  check_slots(slots, stride, s, lens, nb, slot_of, 3 * static_cast<int64_t>(s) * s, "inverse slots");
}
void launch_factor_small(double* slots, int64_t stride, int32_t s, const int32_t* lens, int32_t nb,
                         const int32_t* slot_of, int32_t want_inverse, int32_t* err, hipStream_t, FactorCheck chk) {
  if (nb <= 0) return;
  check_slots(slots, stride, s, lens, nb, slot_of, (want_inverse ? 2 : 1) * static_cast<int64_t>(s) * s,
              "factor_small slots");
  emu_check(err, 4, "factor_small err");
  if (chk.flag) { emu_check(chk.flag, 4 * nb, "factor_small flag"); for (int k = 0; k < nb; ++k) chk.flag[k] = (k % 3 == 0); }
  if (chk.counter) emu_check(chk.counter, 4, "factor_small counter");
}
void launch_scatter_rows(const int32_t* stage_rows, const int32_t* stage_lens, const int32_t* slot_of, int32_t nb,
                         int32_t s, int32_t* rows, int32_t* lens, hipStream_t) {
  if (nb <= 0) return;
  emu_check(stage_rows, 4 * static_cast<size_t>(nb) * s, "scatter stage rows");
  emu_check(stage_lens, 4 * nb, "scatter stage lens");
  emu_check(slot_of, 4 * nb, "scatter slot_of");
  for (int k = 0; k < nb; ++k) {
    emu_check(rows + static_cast<int64_t>(slot_of[k]) * s, 4 * s, "scatter rows");
    emu_check(lens + slot_of[k], 4, "scatter lens");
    for (int i = 0; i < s; ++i) rows[slot_of[k] * s + i] = stage_rows[k * s + i];
    lens[slot_of[k]] = stage_lens[k];
  }
}
// scenario switches (set by the driver): the next g_emu_refuse_confirms true
// residuals come out huge, so that the host turns down that many stop
// candidates; counts of step-kernel launches enqueued ahead and of those that
// ran no step
int g_emu_refuse_confirms = 0;
int64_t g_emu_ahead_launches = 0, g_emu_skipped_launches = 0;
void launch_residual_sq(const double* A, int64_t lda, int64_t m, int64_t n, const double* x, const double* b,
                        double* part, int32_t, double* out, hipStream_t) {
  emu_check(A, 8 * (static_cast<size_t>(m - 1) * lda + n), "residual A");
  emu_check(x, 8 * n, "residual x");
  emu_check(b, 8 * m, "residual b");
  emu_check(part, 8 * m, "residual rowsq");
  emu_check(out, 8, "residual out");
  *out = 0.0;
  if (g_emu_refuse_confirms > 0) {
    --g_emu_refuse_confirms;
    *out = 1e300;
  }
}
void launch_check_finite(const double* A, int64_t lda, int64_t m, int64_t n, const double* b, int32_t* flag,
                         hipStream_t) {
  emu_check(A, 8 * (static_cast<size_t>(m - 1) * lda + n), "finite A");
  emu_check(b, 8 * m, "finite b");
  emu_check(flag, 4, "finite flag");
}
// The device routine's pass chain: the first pass reads in (rows < rows_valid,
// columns < min(cols_valid, ncols)), the last one writes out (rows < rows_out,
// transposed or not), and with two passes the intermediate lives in out when
// the last pass runs in place there, otherwise in work (M x ncols).
void launch_fht(const FhtSpec& s, hipStream_t) {
  if (s.M < 1 || (s.M & (s.M - 1)) || s.M > kFhtMaxRows || s.ncols < 1 || s.rows_valid < 1 ||
      s.rows_valid > s.M || s.cols_valid < 1 || s.rows_out < 1 || s.rows_out > s.M) {
    std::fprintf(stderr, "EMU: bad fht shape M=%lld ncols=%lld\n", (long long)s.M, (long long)s.ncols);
    std::abort();
  }
  const int64_t cin = std::min(s.cols_valid, s.ncols);
  emu_check(s.in, 8 * (static_cast<size_t>(s.rows_valid - 1) * s.ld_in + cin), "fht in");
  if (s.isign) emu_check(s.isign, static_cast<size_t>(s.rows_valid), "fht row signs");
  if (s.csign) emu_check(s.csign, static_cast<size_t>(cin), "fht column signs");
  if (s.osign) emu_check(s.osign, static_cast<size_t>(s.rows_out), "fht output signs");
  if (s.transpose_out)
    emu_check(s.out, 8 * (static_cast<size_t>(s.ncols - 1) * s.ld_out + s.rows_out), "fht out (transposed)");
  else
    emu_check(s.out, 8 * (static_cast<size_t>(s.rows_out - 1) * s.ld_out + s.ncols), "fht out");
  if (fht_passes(s.M) > 1) {
    const bool mid_is_out = !s.transpose_out && s.rows_out >= s.M && s.ld_out >= s.ncols;
    if (mid_is_out)
      emu_check(s.out, 8 * (static_cast<size_t>(s.M - 1) * s.ld_out + s.ncols), "fht intermediate in out");
    else
      emu_check(s.work, 8 * static_cast<size_t>(s.M) * s.ncols, "fht work");
  }
  // a single transposed pass cannot run in place (other workgroups still read what it writes)
  if (s.in == s.out && s.transpose_out && fht_passes(s.M) == 1) {
    std::fprintf(stderr, "EMU: transposed fht in place\n");
    std::abort();
  }
}

// LSQR projection: the ranges each launcher's kernels touch
void launch_factor_linv(double* slots, int64_t stride, int32_t s, const int32_t* lens, int32_t nb,
                        const int32_t* slot_of, hipStream_t) {
  emu_check(lens, 4 * static_cast<size_t>(nb), "linv lens");
  emu_check(slot_of, 4 * static_cast<size_t>(nb), "linv slots");
  for (int32_t k = 0; k < nb; ++k) {
    if (lens[k] < 1 || lens[k] > s) { std::fprintf(stderr, "EMU: linv block length %d\n", lens[k]); std::abort(); }
    emu_check(slots + static_cast<int64_t>(slot_of[k]) * stride, 8 * 3 * static_cast<size_t>(s) * s, "linv slot");
  }
}
void launch_sketch_gather(const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb, int32_t s,
                          double* Xt, hipStream_t) {
  check_rows(rows, sb, "sketch rows");
  check_A(A, 8, lda, rows, sb, n, "sketch A");
  emu_check(Xt, 8 * static_cast<size_t>(n) * s, "sketch Xt");
}
void launch_sketch_select(const double* Y, int32_t s, const int32_t* T, int32_t tau, int32_t sb, double,
                          double* Ahat, hipStream_t) {
  emu_check(T, 4 * static_cast<size_t>(tau), "sketch T");
  int32_t tmax = 0;
  for (int32_t k = 0; k < tau; ++k) tmax = std::max(tmax, T[k]);
  emu_check(Y, 8 * (static_cast<size_t>(tmax) * s + sb), "sketch Y");
  emu_check(Ahat, 8 * static_cast<size_t>(s) * tau, "sketch Ahat");
}
void launch_lsqr_start(const double* y, const double* Linv, int32_t s, int32_t sb, LsqrState* L, hipStream_t) {
  emu_check(y, 8 * static_cast<size_t>(sb), "lsqr y");
  emu_check(Linv, 8 * 2 * static_cast<size_t>(s) * s, "lsqr Linv and its transpose");
  emu_check(L, sizeof(LsqrState), "lsqr state");
  L->live = 0;   // the stand-in solves nothing: later LSQR kernels are no-ops
  for (int32_t i = 0; i < sb; ++i) L->zx[i] = 0.0;
}
int32_t lsqr_at_groups(int64_t n) { return static_cast<int32_t>((n + 255) / 256); }
int32_t lsqr_at_chunks(int32_t s) { return (s + 15) / 16; }
void launch_lsqr_at(const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb, const LsqrState* L,
                    double* ppart, double* p, double* partsq, hipStream_t) {
  check_rows(rows, sb, "lsqr rows");
  check_A(A, 8, lda, rows, sb, n, "lsqr A");
  emu_check(L, sizeof(LsqrState), "lsqr state");
  emu_check(ppart, 8 * static_cast<size_t>(lsqr_at_chunks(sb)) * n, "lsqr row-chunk parts");
  emu_check(p, 8 * static_cast<size_t>(n), "lsqr p");
  emu_check(partsq, 8 * static_cast<size_t>(lsqr_at_groups(n)), "lsqr partials");
}
void launch_lsqr_post(const double* partsq, int32_t ngroups, int32_t, double, int32_t, LsqrState* L, hipStream_t) {
  emu_check(partsq, 8 * static_cast<size_t>(ngroups), "lsqr partials");
  emu_check(L, sizeof(LsqrState), "lsqr state");
}
void launch_lsqr_mid(const double* rpart, int32_t P, const double* Linv, int32_t s, int32_t sb, double, LsqrState* L,
                     hipStream_t) {
  emu_check(rpart, 8 * static_cast<size_t>(sb) * P, "lsqr rpart");
  emu_check(Linv, 8 * 2 * static_cast<size_t>(s) * s, "lsqr Linv and its transpose");
  emu_check(L, sizeof(LsqrState), "lsqr state");
}

// several right-hand sides
void launch_block_gemm_partial(const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb,
                               const double* X, int64_t ldx, int32_t k, double* rpart, int32_t P, hipStream_t) {
  if (P != gemm_parts(n)) { std::fprintf(stderr, "EMU: gemm parts %d for n=%lld\n", P, (long long)n); std::abort(); }
  check_rows(rows, sb, "multi rows");
  check_A(A, 8, lda, rows, sb, n, "multi A");
  emu_check(X, 8 * (static_cast<size_t>(n - 1) * ldx + k), "multi X");
  emu_check(rpart, 8 * static_cast<size_t>(sb) * P * k, "multi rpart");
}
void launch_block_project_multi(const double* rpart, int32_t P, int32_t k, const double* B, int64_t ldb,
                                const int32_t* rows, int32_t sb, const double* Ginv, int32_t s, double* Y,
                                DevState* ds, const int32_t* frozen, int32_t zeta, int32_t, hipStream_t) {
  emu_check(rpart, 8 * static_cast<size_t>(sb) * P * k, "multi rpart");
  check_rows(rows, sb, "multi rows");
  for (int32_t i = 0; i < sb; ++i) emu_check(B + static_cast<int64_t>(rows[i]) * ldb, 8 * static_cast<size_t>(k), "multi B");
  emu_check(Ginv, 8 * static_cast<size_t>(s) * s, "multi Ginv");
  emu_check(Y, 8 * static_cast<size_t>(k) * s, "multi Y");
  emu_check(ds, sizeof(DevState) * k, "multi states");
  emu_check(frozen, 4 * static_cast<size_t>(k), "multi frozen");
  for (int32_t c = 0; c < k; ++c)
    if (!frozen[c]) emu_step(ds + c, zeta, nullptr);
}
void launch_update_multi(int32_t, const double* A, int64_t lda, int64_t n, const int32_t* rows, int32_t sb,
                         const double* Y, int32_t s, int32_t k, const DevState* ds, const int32_t* frozen, double,
                         double* X, int64_t ldx, double* M, hipStream_t) {
  check_rows(rows, sb, "multi rows");
  check_A(A, 8, lda, rows, sb, n, "multi A");
  emu_check(Y, 8 * static_cast<size_t>(k) * s, "multi Y");
  emu_check(ds, sizeof(DevState) * k, "multi states");
  emu_check(frozen, 4 * static_cast<size_t>(k), "multi frozen");
  emu_check(X, 8 * (static_cast<size_t>(n - 1) * ldx + k), "multi X");
  emu_check(M, 8 * static_cast<size_t>(n) * k, "multi momentum");
}
void launch_column(const double* X, int64_t ldx, int64_t n, int32_t c, double* out, hipStream_t) {
  emu_check(X, 8 * (static_cast<size_t>(n - 1) * ldx + c + 1), "column source");
  emu_check(out, 8 * static_cast<size_t>(n), "column out");
}

void launch_state_init(DevState* ds, double rho0, double thr, int32_t* err, double* mom, int64_t n, hipStream_t) {
  emu_check(ds, sizeof(DevState), "state init");
  emu_check(err, sizeof(int32_t), "state init err");
  emu_check(mom, 8 * static_cast<size_t>(n), "state init mom");
  DevState s{};
  s.rho = rho0; s.c = (1 - rho0) / (1 + rho0); s.thr = thr; s.rho_before = rho0;
  *ds = s;
  *err = 0;
  for (int64_t i = 0; i < n; ++i) mom[i] = 0.0;
}
void launch_zero3(double* a, int64_t na, double* b, int64_t nb, double* c, int64_t nc, hipStream_t) {
  emu_check(a, 8 * static_cast<size_t>(na), "zero3 a");
  for (int64_t i = 0; i < na; ++i) a[i] = 0.0;
  if (nb > 0) { emu_check(b, 8 * static_cast<size_t>(nb), "zero3 b"); for (int64_t i = 0; i < nb; ++i) b[i] = 0.0; }
  if (nc > 0) { emu_check(c, 8 * static_cast<size_t>(nc), "zero3 c"); for (int64_t i = 0; i < nc; ++i) c[i] = 0.0; }
}
void launch_convert_f32(const double* A, int64_t lda, int64_t m, int64_t n, float* out, hipStream_t) {
  emu_check(A, 8 * (static_cast<size_t>(m - 1) * lda + n), "convert A");
  emu_check(out, 4 * static_cast<size_t>(m) * n, "convert out");
}
void launch_convert_bf16(const double* A, int64_t lda, int64_t m, int64_t n, uint16_t* out, hipStream_t) {
  emu_check(A, 8 * (static_cast<size_t>(m - 1) * lda + n), "convert A");
  emu_check(out, 2 * static_cast<size_t>(m) * n, "convert out");
}
static std::map<const double*, int> g_rounds;
void launch_residual_vec(const double* A, int64_t lda, int64_t m, int64_t n, const double* x, const double* b,
                         double* r, double* rowsq, double* out, hipStream_t) {
  emu_check(A, 8 * (static_cast<size_t>(m - 1) * lda + n), "rvec A");
  emu_check(x, 8 * n, "rvec x");
  emu_check(b, 8 * m, "rvec b");
  emu_check(r, 8 * m, "rvec r");
  emu_check(rowsq, 8 * m, "rvec rowsq");
  emu_check(out, 8, "rvec out");
  const int k = g_rounds[x]++;
  double bb = 0.0;
  for (int64_t i = 0; i < m; ++i) bb += b[i] * b[i];
  *out = bb * std::pow(1e-4, 2.0 * k);
  if (*out < bb * 1e-30) g_rounds[x] = 0;
}
int32_t gemv_t_splits(int64_t m, int64_t n) {
  const int64_t cols = (n + 255) / 256;
  int64_t s = std::max<int64_t>(1, (2048 + cols - 1) / cols);
  s = std::min<int64_t>(s, std::max<int64_t>(1, m / 64));
  return static_cast<int32_t>(std::min<int64_t>(s, 64));
}
void launch_gemv_t(const double* A, int64_t lda, int64_t m, int64_t n, const double* z, double* d, double* ws,
                   hipStream_t) {
  if (gemv_t_splits(m, n) > 1) emu_check(ws, 8 * static_cast<size_t>(gemv_t_splits(m, n)) * n, "gemv_t ws");
  emu_check(A, 8 * (static_cast<size_t>(m - 1) * lda + n), "gemv_t A");
  emu_check(z, 8 * m, "gemv_t z");
  emu_check(d, 8 * n, "gemv_t d");
}
void launch_axpy1(double* x, const double* d, int64_t n, hipStream_t) {
  emu_check(x, 8 * n, "axpy x");
  emu_check(d, 8 * n, "axpy d");
}
// The step kernel's flags hold the step (epoch) each workgroup last
// published: a run continues exactly where the last one on the same flags
// stopped, or starts at 0 after the flags were cleared.
static std::map<const void*, uint32_t> g_next_epoch;
static std::mutex g_epoch_mu;
void emu_note_memset(const void* d) {
  std::lock_guard<std::mutex> lk(g_epoch_mu);
  g_next_epoch.erase(d);
}
static void check_epoch(const FusedArgs& a, int64_t steps_run) {
  std::lock_guard<std::mutex> lk(g_epoch_mu);
  auto it = g_next_epoch.find(a.flags);
  const uint32_t expect = it == g_next_epoch.end() ? 0u : it->second;
  if (a.epoch != expect) {
    std::fprintf(stderr, "EMU: step kernel epoch %u on flags that stopped at %u\n", a.epoch, expect);
    std::abort();
  }
  g_next_epoch[a.flags] = a.epoch + static_cast<uint32_t>(steps_run);
}

static void emu_fused(const FusedArgs& a, int32_t cpl, int32_t G, size_t esz) {
  const int64_t s = a.s;
  // the kernel reads the first step's slot (and its length) before its step
  // loop, whatever W is, unless it is a launch enqueued ahead that skips
  emu_check(a.ds, sizeof(DevState), "fused ds");
  if (a.W > 0 && !(a.skip_on_cand && a.ds->cand)) {
    emu_check(a.step_slot, 4 * static_cast<size_t>(a.W), "fused step_slot");
    emu_check(a.lens + a.step_slot[0], 4, "fused first lens");
  }
  emu_check(a.x, 8 * a.n, "fused x");
  emu_check(a.mom, 8 * a.n, "fused mom");
  emu_check(a.part, 8 * 2 * static_cast<size_t>(G) * s, "fused part");
  emu_check(a.flags, 4 * static_cast<size_t>(G) * 32, "fused flags");
  if (a.ysplit || a.xchg2) {
    emu_check(a.flags + kYFlagOffset, 4 * static_cast<size_t>(G) * 32, "fused y flags");
    emu_check(a.ypart, 8 * 2 * static_cast<size_t>(s), "fused ypart");
  }
  if (a.xchg2 && (s > kTwoMaxBlock || a.W < 0)) { std::fprintf(stderr, "EMU: two-level exchange with s > %d\n", kTwoMaxBlock); std::abort(); }
  if (a.xchg2) {
    // owners are workgroups 0 .. ceil(s / kOwnRows) - 1, each thread of one a partial
    if (G < kOwnMax || G > 256) { std::fprintf(stderr, "EMU: two-round exchange on %d workgroups\n", G); std::abort(); }
    emu_check(a.ypart + kOwnOffset, 8 * 2 * static_cast<size_t>(kOwnMax) * kOwnStride, "fused owner parts");
  }
  emu_check(a.err, 4, "fused err");
  if (G * 64 * cpl < a.n) { std::fprintf(stderr, "EMU: fused team too small\n"); std::abort(); }
  if (a.vec_rows && (reinterpret_cast<uintptr_t>(a.A) % 16 != 0 || (a.lda * esz) % 16 != 0)) {
    std::fprintf(stderr, "EMU: vector tile loads on unaligned rows\n");
    std::abort();
  }
  if (a.zx) {
    emu_check(a.zx, 8 * a.mrows, "fused zx");
    emu_check(a.zm, 8 * a.mrows, "fused zm");
    if ((a.mrows + G - 1) / G > 1024) { std::fprintf(stderr, "EMU: dual slice too long\n"); std::abort(); }
  }
  int64_t ran = 0;
  // a launch enqueued ahead runs no step after a checkpoint whose stop test passed
  emu_check(a.ds, sizeof(DevState), "fused ds");
  const int W = (a.skip_on_cand && a.ds->cand) ? 0 : a.W;
  if (a.skip_on_cand) ++g_emu_ahead_launches;
  if (a.skip_on_cand && W == 0) ++g_emu_skipped_launches;
  for (int k = 0; k < W; ++k) {
    const int q = a.step_slot[k];
    emu_check(a.lens + q, 4, "fused lens");
    const int sb = a.lens[q];
    if (sb < 1 || sb > s) { std::fprintf(stderr, "EMU: fused sb %d (slot %d, step %d)\n", sb, q, k); std::abort(); }
    emu_check(a.rows + q * s, 4 * sb, "fused rows");
    check_A(a.A, esz, a.lda, a.rows + q * s, sb, a.n, "fused A");
    for (int i = 0; i < sb; ++i) emu_check(a.b + a.rows[q * s + i], 8, "fused b");
    emu_check(a.L + q * a.slot_stride + s * s, 8 * static_cast<size_t>(s) * s, "fused Ginv");
    bool stop = false;
    emu_step(a.ds, a.zeta, &stop);
    ++ran;
    if (a.stop_on_cand && stop) break;
  }
  check_epoch(a, ran);
  if (a.mirror) {
    // the kernel's end-state mirror: state, error words, then the sequence number
    emu_check(a.mirror, sizeof(HostMirror), "fused host mirror");
    emu_check(a.err, 4, "fused err");
    a.mirror->ds = *a.ds;
    a.mirror->err = *a.err;
    if (a.fp64_count) emu_check(a.fp64_count, 4, "fused fp64 count");
    a.mirror->fp64_count = a.fp64_count ? *a.fp64_count : 0;
    a.mirror->seq = a.seq;
  }
}
void launch_fused(int32_t, int32_t prec, const FusedArgs& a, int32_t cpl, int32_t groups, hipStream_t) {
  emu_fused(a, cpl, groups, prec == 2 ? 2 : prec == 1 ? 4 : 8);
}
// the stand-in device holds one step-kernel workgroup per compute unit
int32_t fused_blocks_per_cu(int32_t, int32_t, int32_t) { return 1; }
void launch_fused_multi(int32_t, bool a_fp32, const FusedArgs* args, const int32_t* team_start, int32_t nteams,
                        int32_t total, int32_t cpl, hipStream_t) {
  emu_check(args, sizeof(FusedArgs) * nteams, "multi args");
  emu_check(team_start, 4 * (nteams + 1), "multi team_start");
  if (team_start[0] != 0 || team_start[nteams] != total || total > 256) { std::fprintf(stderr, "EMU: team table\n"); std::abort(); }
  for (int t = 0; t < nteams; ++t) emu_fused(args[t], cpl, team_start[t + 1] - team_start[t], a_fp32 ? 4 : 8);
}
// ---- sparse (CSR) systems: the stand-in device memory is host memory, so
// the launchers check the CSR structure they read and every entry they touch
void launch_csr_check(const int64_t* rp, const int32_t* ci, const double* cv, const double* b, int64_t m, int64_t n,
                      int64_t nnz, int32_t* flag, hipStream_t) {
  emu_check(rp, 8 * (m + 1), "csr row_ptr");
  emu_check(b, 8 * m, "csr b");
  emu_check(flag, 4, "csr flag");
  int bad = 0;
  for (int64_t i = 0; i < m; ++i) {
    const int64_t a = rp[i], e = rp[i + 1];
    if (!std::isfinite(b[i])) bad |= 4;
    if ((i == 0 && a != 0) || (i == m - 1 && e != nnz) || a < 0 || e < a || e > nnz) { bad |= 1; continue; }
    if (e > a) {
      emu_check(ci + a, 4 * (e - a), "csr col");
      emu_check(cv + a, 8 * (e - a), "csr val");
    }
    int64_t prev = -1;
    for (int64_t k = a; k < e; ++k) {
      if (ci[k] <= prev || ci[k] >= n) { bad |= 2; break; }
      prev = ci[k];
      if (!std::isfinite(cv[k])) bad |= 4;
    }
  }
  *flag |= bad;
}
namespace {
void check_csr_row(const int64_t* rp, const int32_t* ci, const double* cv, int64_t r, const char* what) {
  emu_check(rp + r, 16, what);
  const int64_t a = rp[r], e = rp[r + 1];
  if (e > a) {
    emu_check(ci + a, 4 * (e - a), what);
    if (cv) emu_check(cv + a, 8 * (e - a), what);
  }
}
}  // namespace
void launch_csr_rows_dot(const int64_t* rp, const int32_t* ci, const double* cv, const int32_t* rows, int32_t sb,
                         const double* u, const double* v, double t01, double* out, hipStream_t) {
  check_rows(rows, sb, "csr rows");
  for (int32_t i = 0; i < sb; ++i) {
    check_csr_row(rp, ci, cv, rows[i], "csr rows_dot");
    for (int64_t k = rp[rows[i]]; k < rp[rows[i] + 1]; ++k) {
      emu_check(u + ci[k], 8, "csr rows_dot u");
      if (t01 != 0.0) emu_check(v + ci[k], 8, "csr rows_dot v");
    }
  }
  emu_check(out, 8 * sb, "csr rows_dot out");
}
void launch_csc_apply(const CscArena& ar, int64_t off, int32_t z, const int32_t* nu, int32_t q, const double* y,
                      int32_t sb, double, double, double* u, double* v, hipStream_t) {
  emu_check(nu + q, 4, "csc nu");
  emu_check(ar.val + off, 8 * static_cast<size_t>(z + 1), "csc val");
  emu_check(ar.row + off, 4 * static_cast<size_t>(z + 1), "csc row");
  emu_check(ar.col + off, 4 * static_cast<size_t>(z + 1), "csc col");
  emu_check(ar.ptr + off, 4 * static_cast<size_t>(z + 1), "csc ptr");
  emu_check(y, 8 * sb, "csc y");
  if (nu[q] < 0 || nu[q] > z) { std::fprintf(stderr, "EMU: csc nu %d of %d\n", nu[q], z); std::abort(); }
  for (int32_t k = 0; k < nu[q]; ++k) {
    emu_check(u + ar.col[off + k], 8, "csc u");
    emu_check(v + ar.col[off + k], 8, "csc v");
  }
}
void launch_rows_apply(const int32_t* rows, int32_t sb, const double* y, double, double, double* u, double* v,
                       hipStream_t) {
  check_rows(rows, sb, "rows_apply rows");
  emu_check(y, 8 * sb, "rows_apply y");
  for (int32_t i = 0; i < sb; ++i) {
    emu_check(u + rows[i], 8, "rows_apply u");
    emu_check(v + rows[i], 8, "rows_apply v");
  }
}
void launch_lazy_fold(double* u, double* v, int64_t n, double, double, hipStream_t) {
  emu_check(u, 8 * n, "fold u");
  emu_check(v, 8 * n, "fold v");
}
// The stand-in build writes a valid copy with no columns (nu = 0): the
// step's back-projection then touches nothing.
void launch_csr_block_build(const int64_t* rp, const int32_t* ci, const double* cv, const int32_t* rows,
                            const int32_t* lens, const int32_t* slot_of, const int32_t* meta, int32_t nb, int32_t s,
                            double, double* G, int64_t stride, const CscArena& ar, int32_t* nu, double* ws, bool,
                            bool, int32_t* err, hipStream_t) {
  check_slots(G, stride, s, lens, nb, slot_of, static_cast<int64_t>(s) * s, "csr build G");
  emu_check(meta, 4 * static_cast<size_t>(kCsrMetaInts) * nb, "csr build meta");
  for (int32_t k = 0; k < nb; ++k) {
    const int32_t* mk = meta + kCsrMetaInts * k;
    auto get = [](const int32_t* w) {
      return static_cast<int64_t>((static_cast<uint64_t>(static_cast<uint32_t>(w[1])) << 32) |
                                  static_cast<uint32_t>(w[0]));
    };
    const int64_t off = get(mk);
    const int32_t z = mk[2];
    const int64_t wso = get(mk + 3);
    check_rows(rows + static_cast<int64_t>(k) * s, lens[k], "csr build rows");
    int64_t zz = 0;
    for (int32_t i = 0; i < lens[k]; ++i) {
      const int64_t r = rows[static_cast<int64_t>(k) * s + i];
      check_csr_row(rp, ci, cv, r, "csr build row");
      zz += rp[r + 1] - rp[r];
    }
    if (zz != z) { *err |= 4; continue; }
    emu_check(ar.val + off, 8 * static_cast<size_t>(z + 1), "csr build val");
    emu_check(ar.row + off, 4 * static_cast<size_t>(z + 1), "csr build row");
    emu_check(ar.col + off, 4 * static_cast<size_t>(z + 1), "csr build col");
    emu_check(ar.ptr + off, 4 * static_cast<size_t>(z + 1), "csr build ptr");
    if (wso >= 0) emu_check(ws + wso, 8 * csr_build_ws_doubles(z), "csr build ws");
    else if (z > kCsrLdsEntries) { std::fprintf(stderr, "EMU: LDS build of %d nonzeros\n", z); std::abort(); }
    emu_check(nu + slot_of[k], 4, "csr build nu");
    nu[slot_of[k]] = 0;
    ar.ptr[off] = z;
  }
}
void launch_csr_gram_cd(const int64_t* rp, const int32_t* ci, const double* cv, const int32_t* rows,
                        const int32_t* lens, const int32_t* slot_of, int32_t nb, int32_t s, double, double* G,
                        int64_t stride, hipStream_t) {
  check_slots(G, stride, s, lens, nb, slot_of, static_cast<int64_t>(s) * s, "csr gram_cd G");
  for (int32_t k = 0; k < nb; ++k)
    for (int32_t i = 0; i < lens[k]; ++i) {
      const int32_t r = rows[static_cast<int64_t>(k) * s + i];
      if (i > 0 && r <= rows[static_cast<int64_t>(k) * s + i - 1]) { std::fprintf(stderr, "EMU: CD rows not ascending\n"); std::abort(); }
      check_csr_row(rp, ci, cv, r, "csr gram_cd row");
    }
}
void launch_csr_residual_sq(const int64_t* rp, const int32_t* ci, const double* cv, const double* b, int64_t m,
                            const double* x, double* part, double* out, hipStream_t) {
  emu_check(rp, 8 * (m + 1), "csr resid rp");
  for (int64_t r = 0; r < m; ++r) {
    check_csr_row(rp, ci, cv, r, "csr resid row");
    for (int64_t k = rp[r]; k < rp[r + 1]; ++k) emu_check(x + ci[k], 8, "csr resid x");
  }
  emu_check(b, 8 * m, "csr resid b");
  emu_check(part, 8 * csr_residual_parts(m), "csr resid part");
  emu_check(out, 8, "csr resid out");
  *out = 0.0;
}
// team tables from the stand-in CSR arrays, exactly (binary searches)
void launch_csr_team_tables(int32_t kind, const int64_t* rp, const int32_t* ci, const int32_t* rows,
                            const int32_t* lens, const int32_t* slot_of, const int32_t* meta, const CscArena& ar,
                            const int32_t* nu, int32_t nb, int32_t s, int64_t n, int32_t G, int32_t* team,
                            hipStream_t) {
  emu_check(lens, 4 * nb, "team lens");
  emu_check(slot_of, 4 * nb, "team slot_of");
  const int64_t ts = csr_team_stride(s, G);
  for (int32_t k = 0; k < nb; ++k) {
    const int32_t* R = rows + static_cast<int64_t>(k) * s;
    check_rows(R, lens[k], "team rows");
    int32_t* TT = team + static_cast<int64_t>(slot_of[k]) * ts;
    emu_check(TT, 4 * static_cast<size_t>(ts), "team table");
    for (int32_t i = 0; i < lens[k]; ++i) {
      check_csr_row(rp, ci, nullptr, R[i], "team row");
      const int64_t a0 = rp[R[i]], a1 = rp[R[i] + 1];
      for (int32_t g = 0; g <= G; ++g) {
        int64_t e = a0;
        const int64_t c = g == G ? n : csr_slice_lo(n, G, g);
        while (e < a1 && ci[e] < c) ++e;
        TT[i * (G + 1) + g] = static_cast<int32_t>(e - a0);
      }
    }
    for (int32_t g = 0; g <= G; ++g) {
      const int64_t c = g == G ? n : csr_slice_lo(n, G, g);
      int32_t lo = 0;
      if (kind == 0) {
        emu_check(meta + kCsrMetaInts * k, 4 * kCsrMetaInts, "team meta");
        const int64_t off = static_cast<int64_t>((static_cast<uint64_t>(static_cast<uint32_t>(meta[kCsrMetaInts * k + 1])) << 32) |
                                                 static_cast<uint32_t>(meta[kCsrMetaInts * k]));
        emu_check(nu + slot_of[k], 4, "team nu");
        while (lo < nu[slot_of[k]] && ar.col[off + lo] < c) ++lo;
      } else {
        while (lo < lens[k] && R[lo] < c) ++lo;
      }
      TT[s * (G + 1) + g] = lo;
    }
  }
}
void launch_sparse_team(int32_t kind, const SparseTeamArgs& a, hipStream_t) {
  if (a.W <= 0) return;
  if (a.G < 1 || a.G > kSparseTeamMax) { std::fprintf(stderr, "EMU: team size %d\n", a.G); std::abort(); }
  emu_check(a.coef, 8 * 3 * static_cast<size_t>(a.W), "team coef");
  emu_check(a.step_info, 4 * kSparseStepInts * static_cast<size_t>(a.W), "team step_info");
  emu_check(a.xr, 8 * 2 * static_cast<size_t>(a.G) * a.s, "team xr");
  emu_check(a.xy, 8 * 2 * static_cast<size_t>(a.s), "team xy");
  emu_check(a.flags, 4 * (kYFlagOffset + a.G * kSparseFlagStride), "team flags");
  emu_check(a.err, 4, "team err");
  const int T1 = a.G + 1;
  for (int32_t k = 0; k < a.W; ++k) {
    const int32_t* in = a.step_info + kSparseStepInts * k;
    const int32_t q = in[0], sb = in[1], z = in[2];
    const int32_t* R = a.rows + static_cast<int64_t>(q) * a.s;
    check_rows(R, sb, "team rows");
    const int32_t* TT = a.team + static_cast<int64_t>(q) * a.team_stride;
    emu_check(TT, 4 * static_cast<size_t>(a.team_stride), "team table");
    int64_t zz = 0;
    for (int32_t i = 0; i < sb; ++i) {
      check_csr_row(a.rp, a.ci, a.cv, R[i], "team row");
      const int64_t base = a.rp[R[i]], len = a.rp[R[i] + 1] - base;
      zz += len;
      for (int g = 0; g < a.G; ++g) {
        const int32_t j0 = TT[i * T1 + g], j1 = TT[i * T1 + g + 1];
        if (j0 < 0 || j1 < j0 || j1 > len) { std::fprintf(stderr, "EMU: team row slice %d..%d of %lld\n", j0, j1, (long long)len); std::abort(); }
        for (int64_t e = base + j0; e < base + j1; ++e) {
          emu_check(a.u + a.ci[e], 8, "team gather u");
          if (a.coef[3 * k] != 0.0) emu_check(a.v + a.ci[e], 8, "team gather v");
        }
      }
      emu_check(a.b + R[i], 8, "team b");
    }
    if (zz != z) { std::fprintf(stderr, "EMU: team step %d nonzeros %lld vs %d\n", k, (long long)zz, z); std::abort(); }
    emu_check(a.L + q * a.slot_stride + static_cast<int64_t>(a.s) * a.s, 8 * static_cast<size_t>(a.s) * a.s,
              "team Ginv");
    const int32_t c0 = TT[a.s * T1], cG = TT[a.s * T1 + a.G];
    if (kind == 0) {
      const int64_t off = static_cast<int64_t>((static_cast<uint64_t>(static_cast<uint32_t>(in[4])) << 32) |
                                               static_cast<uint32_t>(in[3]));
      emu_check(a.ar.ptr + off, 4 * static_cast<size_t>(z + 1), "team ptr");
      if (c0 != 0 || cG < 0 || cG > z) { std::fprintf(stderr, "EMU: team column bounds %d %d\n", c0, cG); std::abort(); }
      for (int32_t c = 0; c < cG; ++c) {
        emu_check(a.u + a.ar.col[off + c], 8, "team u");
        emu_check(a.v + a.ar.col[off + c], 8, "team v");
      }
    } else {
      if (c0 != 0 || cG != sb) { std::fprintf(stderr, "EMU: team row bounds %d %d of %d\n", c0, cG, sb); std::abort(); }
      for (int32_t i = 0; i < sb; ++i) {
        emu_check(a.u + R[i], 8, "team u");
        emu_check(a.v + R[i], 8, "team v");
      }
    }
    emu_step(a.ds, a.zeta, nullptr);
  }
}
}  // namespace kpp
