// Solver and server scenarios through the C ABI on the CPU stand-ins: every
// kernel argument range is checked, and the sanitizers the test builds with
// check the host code (heap, undefined behaviour, data races).
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <thread>
#include <chrono>
#include "kpp.h"

static double* dev_vec(size_t n, double v) {
  void* p; hipMalloc(&p, n * 8); double* d = (double*)p; for (size_t i = 0; i < n; ++i) d[i] = v; return d;
}
#define CHECK(x) do { kpp_status s_ = (x); if (s_ < 0) { std::printf("FAIL %s -> %d: %s\n", #x, s_, kpp_last_error()); std::exit(1);} } while (0)

static void solve_case(const char* name, int kind, int64_t m, int64_t n, int s, int memo, int part, int nblocks,
                       int engine, int prec, int64_t T, double tol) {
  kpp_context* ctx; CHECK(kpp_context_create(0, nullptr, &ctx));
  double* A = dev_vec(m * n, 0.5); double* b = dev_vec(m, 1.0); double* x = dev_vec(n, 0.0);
  kpp_system* sys; CHECK(kpp_system_create(ctx, kind, m, n, A, n, b, &sys));
  for (int rep = 0; rep < 2; ++rep) {
    kpp_params p; CHECK(kpp_params_default(&p, kind));
    p.block_size = s; p.memo = memo; p.fixed_partition = part; p.num_blocks = nblocks; p.engine = engine;
    p.precision = prec; p.max_iters = T * (rep + 1) / 2; p.tol = tol; p.seed = 31; p.lambda = 1e-3;
    kpp_result r; kpp_status st = kpp_solve(sys, &p, x, &r);
    if (st < 0) { std::printf("FAIL %s: %d %s\n", name, st, kpp_last_error()); std::exit(1); }
    std::printf("%-22s T=%-6lld st=%d iters=%lld misses=%lld hits=%lld rounds=%d\n", name, (long long)p.max_iters, st,
                (long long)r.iters, (long long)r.memo_misses, (long long)r.memo_hits, r.refinements);
  }
  CHECK(kpp_system_destroy(sys)); CHECK(kpp_context_destroy(ctx));
  hipFree(A); hipFree(b); hipFree(x);
}

// A solve cut in two: the state of the first part moves to a fresh system
// through export/import and the second part resumes there.
static void resume_case(int kind, int64_t m, int64_t n, int s) {
  kpp_context* ctx; CHECK(kpp_context_create(0, nullptr, &ctx));
  double* A = dev_vec(m * n, 0.5); double* b = dev_vec(m, 1.0); double* x = dev_vec(n, 0.0);
  kpp_system* sys; CHECK(kpp_system_create(ctx, kind, m, n, A, n, b, &sys));
  size_t bytes = 0;
  if (kpp_state_export(sys, nullptr, &bytes) >= 0) { std::printf("FAIL: export without state\n"); std::exit(1); }
  kpp_params p; CHECK(kpp_params_default(&p, kind));
  p.block_size = s; p.max_iters = 70; p.tol = 0.0; p.seed = 5;
  kpp_result r; CHECK(kpp_solve(sys, &p, x, &r));
  CHECK(kpp_state_export(sys, nullptr, &bytes));
  std::vector<unsigned char> buf(bytes);
  CHECK(kpp_state_export(sys, buf.data(), &bytes));
  kpp_system* sys2; CHECK(kpp_system_create(ctx, kind, m, n, A, n, b, &sys2));
  CHECK(kpp_state_import(sys2, buf.data(), bytes));
  p.resume = 1; p.max_iters = 45;
  CHECK(kpp_solve(sys2, &p, x, &r));
  if (r.iters != 45) { std::printf("FAIL: resumed %lld steps\n", (long long)r.iters); std::exit(1); }
  // wrong shape and truncated buffers are refused
  kpp_system* sys3; CHECK(kpp_system_create(ctx, kind, m - 1, n - 1, A, n, b, &sys3));
  if (kpp_state_import(sys3, buf.data(), bytes) >= 0) { std::printf("FAIL: import into another shape\n"); std::exit(1); }
  if (kpp_state_import(sys2, buf.data(), bytes - 1) >= 0) { std::printf("FAIL: truncated import\n"); std::exit(1); }
  std::printf("resume kind=%d: 70 + %lld steps\n", kind, (long long)r.iters);
  CHECK(kpp_system_destroy(sys3)); CHECK(kpp_system_destroy(sys2)); CHECK(kpp_system_destroy(sys));
  CHECK(kpp_context_destroy(ctx));
  hipFree(A); hipFree(b); hipFree(x);
}

// Solves with randomized Hadamard preprocessing: a Kaczmarz++ system whose
// padded row count takes two transform passes, and a CD++ one; a second solve
// with the same seed reuses the transformed system, another seed rebuilds it.
static void rht_case(int kind, int64_t m, int64_t n, int s) {
  kpp_context* ctx; CHECK(kpp_context_create(0, nullptr, &ctx));
  double* A = dev_vec(m * n, 0.5); double* b = dev_vec(m, 1.0); double* x = dev_vec(n, 0.0);
  kpp_system* sys; CHECK(kpp_system_create(ctx, kind, m, n, A, n, b, &sys));
  for (uint64_t seed : {3ull, 3ull, 4ull}) {
    kpp_params p; CHECK(kpp_params_default(&p, kind));
    p.block_size = s; p.max_iters = 90; p.tol = 0.0; p.rht = 1; p.rht_seed = seed;
    kpp_result r; CHECK(kpp_solve(sys, &p, x, &r));
    std::printf("rht kind=%d m=%lld seed=%llu iters=%lld\n", kind, (long long)m, (unsigned long long)seed,
                (long long)r.iters);
  }
  kpp_params p; CHECK(kpp_params_default(&p, kind));
  p.block_size = s; p.rht = 1; p.resume = 1;
  kpp_result r;
  if (kpp_solve(sys, &p, x, &r) >= 0) { std::printf("FAIL: rht with resume\n"); std::exit(1); }
  CHECK(kpp_system_destroy(sys)); CHECK(kpp_context_destroy(ctx));
  hipFree(A); hipFree(b); hipFree(x);
}

// Kaczmarz++ with the LSQR projection (online, fixed partition, and a
// block size above the in-LDS factor limit, more new blocks in a window than
// one batched sketch factoring takes), and the combinations it rejects.
static void lsqr_case(int64_t m, int64_t n, int s, int memo, int64_t iters = 150) {
  kpp_context* ctx; CHECK(kpp_context_create(0, nullptr, &ctx));
  double* A = dev_vec(m * n, 0.5); double* b = dev_vec(m, 1.0); double* x = dev_vec(n, 0.0);
  kpp_system* sys; CHECK(kpp_system_create(ctx, KPP_KACZMARZ, m, n, A, n, b, &sys));
  kpp_params p; CHECK(kpp_params_default(&p, KPP_KACZMARZ));
  p.block_size = s; p.memo = memo; p.max_iters = iters; p.tol = 0.0; p.projection = 1; p.lsqr_iters = 3;
  kpp_result r; CHECK(kpp_solve(sys, &p, x, &r));
  std::printf("lsqr m=%lld n=%lld s=%d memo=%d iters=%lld misses=%lld\n", (long long)m, (long long)n, s, memo,
              (long long)r.iters, (long long)r.memo_misses);
  p.engine = 2;
  if (kpp_solve(sys, &p, x, &r) >= 0) { std::printf("FAIL: lsqr on the fused engine\n"); std::exit(1); }
  CHECK(kpp_system_destroy(sys)); CHECK(kpp_context_destroy(ctx));
  hipFree(A); hipFree(b); hipFree(x);
}

// Several right-hand sides (both kinds, memo modes, k not a power of two).
static void multi_case(int kind, int64_t m, int64_t n, int s, int memo, int k) {
  kpp_context* ctx; CHECK(kpp_context_create(0, nullptr, &ctx));
  double* A = dev_vec(m * n, 0.5); double* b = dev_vec(m, 1.0);
  double* B = dev_vec(m * (k + 1), 1.0); double* X = dev_vec(n * (k + 2), 0.0);
  kpp_system* sys; CHECK(kpp_system_create(ctx, kind, m, n, A, n, b, &sys));
  kpp_params p; CHECK(kpp_params_default(&p, kind));
  p.block_size = s; p.memo = memo; p.max_iters = 300; p.tol = 1e-10;
  std::vector<kpp_result> r(k);
  kpp_status st = kpp_solve_multi(sys, &p, k, B, k + 1, X, k + 2, r.data());
  if (st < 0) { std::printf("FAIL multi: %d %s\n", st, kpp_last_error()); std::exit(1); }
  std::printf("multi kind=%d k=%d st=%d iters[0]=%lld iters[k-1]=%lld misses=%lld\n", kind, k, st,
              (long long)r[0].iters, (long long)r[k - 1].iters, (long long)r[0].memo_misses);
  CHECK(kpp_system_destroy(sys)); CHECK(kpp_context_destroy(ctx));
  hipFree(A); hipFree(b); hipFree(B); hipFree(X);
}

static void serve_case() {
  kpp_context* ctx; CHECK(kpp_context_create(0, nullptr, &ctx));
  struct J { int kind; int64_t m, n; int s; int prec; double tol; };
  std::vector<J> jobs = {{1, 500, 500, 64, 0, 1e-10}, {1, 1100, 1100, 128, 1, 1e-6}, {1, 300, 300, 32, 1, 1e-10},
                         {0, 900, 350, 50, 0, 1e-10}, {1, 1500, 1500, 128, 0, 1e-10}, {0, 400, 1200, 64, 1, 1e-8}};
  std::vector<kpp_system*> syss; std::vector<double*> xs; std::vector<double*> bufs;
  kpp_server* srv; CHECK(kpp_server_create(ctx, 64ull << 30, 16, &srv));
  std::vector<uint64_t> ids;
  for (auto& j : jobs) {
    double* A = dev_vec(j.m * j.n, 0.5); double* b = dev_vec(j.m, 1.0); double* x = dev_vec(j.n, 0.0);
    bufs.push_back(A); bufs.push_back(b); xs.push_back(x);
    kpp_system* sys; CHECK(kpp_system_create(ctx, j.kind, j.m, j.n, A, j.n, b, &sys)); syss.push_back(sys);
    kpp_params p; CHECK(kpp_params_default(&p, j.kind));
    p.block_size = j.s; p.precision = j.prec; p.tol = j.tol; p.max_iters = 200000; p.seed = 7;
    p.memo = KPP_MEMO_ONLINE;
    uint64_t id; CHECK(kpp_server_submit(srv, sys, &p, x, &id)); ids.push_back(id);
  }
  // a second request on system 3
  { kpp_params p; CHECK(kpp_params_default(&p, 0)); p.block_size = 50; p.tol = 1e-10; p.seed = 7;
    uint64_t id; CHECK(kpp_server_submit(srv, syss[3], &p, xs[3], &id)); ids.push_back(id); }
  size_t got = 0;
  for (long it = 0; it < 200000000L && got < ids.size(); ++it) {
    uint64_t rid[16]; int32_t st[16]; kpp_result res[16]; int32_t n = 0;
    CHECK(kpp_server_poll(srv, 16, 0.0, rid, st, res, &n));
    for (int i = 0; i < n; ++i)
      std::printf("served id=%llu st=%d iters=%lld rounds=%d queued=%.4f total=%.4f\n", (unsigned long long)rid[i], st[i],
                  (long long)res[i].iters, res[i].refinements, res[i].seconds_queued, res[i].seconds_total);
    got += n;
  }
  kpp_server_info info; CHECK(kpp_server_stats(srv, &info));
  std::printf("server: completed=%lld rounds=%lld peak_active=%d peak_bytes=%llu\n", (long long)info.completed,
              (long long)info.rounds, info.peak_active, (unsigned long long)info.peak_bytes);
  CHECK(kpp_server_destroy(srv));
  for (auto* s : syss) CHECK(kpp_system_destroy(s));
  for (auto* p : bufs) hipFree(p);
  for (auto* p : xs) hipFree(p);
  CHECK(kpp_context_destroy(ctx));
  if (got != ids.size()) { std::printf("FAIL: %zu of %zu served\n", got, ids.size()); std::exit(1); }
}


// Sparse systems: random CSR structure in stand-in device memory (columns
// ascending in each row), solves in every memo mode, blocks past the LDS
// build size, resume, the block factor, and the refusals.
struct Csr {
  int64_t* rp; int32_t* ci; double* cv; int64_t nnz;
};
static Csr make_csr(int64_t m, int64_t n, int per_row, unsigned seed, bool symmetric_band) {
  std::vector<int64_t> rp(m + 1, 0);
  std::vector<int32_t> ci;
  std::vector<double> cv;
  unsigned st = seed;
  auto rnd = [&]() { st = st * 1664525u + 1013904223u; return st >> 8; };
  for (int64_t i = 0; i < m; ++i) {
    std::vector<int32_t> cols;
    if (symmetric_band) {
      for (int64_t j = std::max<int64_t>(0, i - per_row); j <= std::min<int64_t>(n - 1, i + per_row); ++j) cols.push_back((int32_t)j);
    } else {
      const int k = (i % 17 == 3) ? 0 : per_row;   // a few empty rows
      for (int t = 0; t < k; ++t) cols.push_back((int32_t)(rnd() % n));
      std::sort(cols.begin(), cols.end());
      cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    }
    for (int32_t c : cols) { ci.push_back(c); cv.push_back(c == i ? 4.0 : 0.25); }
    rp[i + 1] = (int64_t)ci.size();
  }
  Csr a;
  a.nnz = (int64_t)ci.size();
  void* p;
  hipMalloc(&p, (m + 1) * 8); a.rp = (int64_t*)p; std::memcpy(a.rp, rp.data(), (m + 1) * 8);
  hipMalloc(&p, std::max<int64_t>(1, a.nnz) * 4); a.ci = (int32_t*)p; std::memcpy(a.ci, ci.data(), a.nnz * 4);
  hipMalloc(&p, std::max<int64_t>(1, a.nnz) * 8); a.cv = (double*)p; std::memcpy(a.cv, cv.data(), a.nnz * 8);
  return a;
}
static void free_csr(Csr& a) { hipFree(a.rp); hipFree(a.ci); hipFree(a.cv); }

static void sparse_solve(const char* name, int kind, int64_t m, int64_t n, int per_row, int s, int memo, int part,
                         int engine, int64_t T, bool band) {
  kpp_context* ctx; CHECK(kpp_context_create(0, nullptr, &ctx));
  Csr a = make_csr(m, n, per_row, 7 + s, band);
  double* b = dev_vec(m, 1.0); double* x = dev_vec(n, 0.0);
  kpp_system* sys; CHECK(kpp_system_create_csr(ctx, kind, m, n, a.nnz, a.rp, a.ci, a.cv, b, &sys));
  for (int rep = 0; rep < 2; ++rep) {
    kpp_params p; CHECK(kpp_params_default(&p, kind));
    p.block_size = s; p.memo = memo; p.fixed_partition = part; p.engine = engine;
    p.max_iters = T * (rep + 1) / 2; p.tol = 0.0; p.seed = 3; p.lambda = 1e-3; p.keep_memo = 1;
    if (rep == 1) { p.adaptive_rho = 0; p.rho0 = 0.7; }   // folds every few steps
    kpp_result r; kpp_status st = kpp_solve(sys, &p, x, &r);
    if (st < 0) { std::printf("FAIL %s: %d %s\n", name, st, kpp_last_error()); std::exit(1); }
    std::printf("%-22s T=%-6lld st=%d iters=%lld misses=%lld hits=%lld\n", name, (long long)p.max_iters, st,
                (long long)r.iters, (long long)r.memo_misses, (long long)r.memo_hits);
  }
  double rn = 0.0; CHECK(kpp_residual_norm(sys, x, &rn));
  CHECK(kpp_system_destroy(sys)); CHECK(kpp_context_destroy(ctx));
  free_csr(a); hipFree(b); hipFree(x);
}

#define EXPECT_STATUS(x, want) do { kpp_status s_ = (x); if (s_ != (want)) { std::printf("FAIL %s -> %d (want %d): %s\n", #x, s_, (int)(want), kpp_last_error()); std::exit(1);} } while (0)

static void sparse_misc() {
  kpp_context* ctx; CHECK(kpp_context_create(0, nullptr, &ctx));
  const int64_t m = 400, n = 120;
  Csr a = make_csr(m, n, 5, 11, false);
  double* b = dev_vec(m, 1.0); double* x = dev_vec(n, 0.0);
  kpp_system* sys; CHECK(kpp_system_create_csr(ctx, 0, m, n, a.nnz, a.rp, a.ci, a.cv, b, &sys));
  // refused options
  kpp_params p; CHECK(kpp_params_default(&p, 0));
  p.block_size = 16; p.max_iters = 40; p.tol = 0.0; p.lambda = 1e-3;
  kpp_result r;
  { kpp_params q = p; q.precision = KPP_MIXED_FP32; EXPECT_STATUS(kpp_solve(sys, &q, x, &r), KPP_ERR_INVALID_ARG); }
  { kpp_params q = p; q.rht = 1; EXPECT_STATUS(kpp_solve(sys, &q, x, &r), KPP_ERR_INVALID_ARG); }
  { kpp_params q = p; q.projection = 1; EXPECT_STATUS(kpp_solve(sys, &q, x, &r), KPP_ERR_INVALID_ARG); }
  { kpp_params q = p; q.team_groups = 300; EXPECT_STATUS(kpp_solve(sys, &q, x, &r), KPP_ERR_INVALID_ARG); }
  double* B = dev_vec(m * 2, 1.0); double* X = dev_vec(n * 2, 0.0);
  EXPECT_STATUS(kpp_solve_multi(sys, &p, 2, B, 2, X, 2, nullptr), KPP_ERR_INVALID_ARG);
  uint64_t bytes = 0;
  EXPECT_STATUS(kpp_request_footprint(sys, &p, &bytes), KPP_ERR_INVALID_ARG);
  // block factor (Kaczmarz++ build kernel) and the no-allocation refusal
  std::vector<int32_t> rows = {0, 5, 9, 40, 77, 300, 1, 2, 3, -1, -1, -1}, lens = {6, 3};
  double* L = dev_vec(2 * 6 * 6, 0.0);
  CHECK(kpp_block_factor(sys, 6, 1e-3, 2, rows.data(), lens.data(), L));
  EXPECT_STATUS(kpp_block_factor_noalloc(sys, 6, 1e-3, 2, rows.data(), lens.data(), L), KPP_ERR_INVALID_ARG);
  // resume through export / import
  CHECK(kpp_solve(sys, &p, x, &r));
  size_t sz = 0; CHECK(kpp_state_export(sys, nullptr, &sz));
  std::vector<unsigned char> buf(sz); CHECK(kpp_state_export(sys, buf.data(), &sz));
  kpp_system* sys2; CHECK(kpp_system_create_csr(ctx, 0, m, n, a.nnz, a.rp, a.ci, a.cv, b, &sys2));
  CHECK(kpp_state_import(sys2, buf.data(), sz));
  kpp_params q = p; q.resume = 1; q.max_iters = 25;
  CHECK(kpp_solve(sys2, &q, x, &r));
  if (r.iters != 25) { std::printf("FAIL: sparse resume ran %lld\n", (long long)r.iters); std::exit(1); }
  CHECK(kpp_system_destroy(sys2));
  CHECK(kpp_system_destroy(sys));
  // malformed structures
  kpp_system* bad = nullptr;
  int32_t c0 = a.ci[0]; a.ci[0] = (int32_t)n;
  EXPECT_STATUS(kpp_system_create_csr(ctx, 0, m, n, a.nnz, a.rp, a.ci, a.cv, b, &bad), KPP_ERR_SHAPE);
  a.ci[0] = c0;
  EXPECT_STATUS(kpp_system_create_csr(ctx, 0, m, n, a.nnz + 1, a.rp, a.ci, a.cv, b, &bad), KPP_ERR_SHAPE);
  EXPECT_STATUS(kpp_system_create_csr(ctx, 1, m, n, a.nnz, a.rp, a.ci, a.cv, b, &bad), KPP_ERR_SHAPE);
  double v0 = a.cv[3]; a.cv[3] = 0.0 / 0.0;
  EXPECT_STATUS(kpp_system_create_csr(ctx, 0, m, n, a.nnz, a.rp, a.ci, a.cv, b, &bad), KPP_ERR_NONFINITE);
  a.cv[3] = v0;
  if (bad) { std::printf("FAIL: a refused system was returned\n"); std::exit(1); }
  // CD++ block factor needs ascending rows
  Csr c = make_csr(200, 200, 2, 5, true);
  double* bc = dev_vec(200, 1.0);
  kpp_system* cs; CHECK(kpp_system_create_csr(ctx, 1, 200, 200, c.nnz, c.rp, c.ci, c.cv, bc, &cs));
  std::vector<int32_t> crow = {3, 4, 9, 10}, crow_bad = {4, 3, 9, 10}, clen = {4};
  double* Lc = dev_vec(16, 0.0);
  CHECK(kpp_block_factor(cs, 4, 1e-8, 1, crow.data(), clen.data(), Lc));
  EXPECT_STATUS(kpp_block_factor(cs, 4, 1e-8, 1, crow_bad.data(), clen.data(), Lc), KPP_ERR_INVALID_ARG);
  CHECK(kpp_system_destroy(cs));
  std::printf("sparse misc ok\n");
  CHECK(kpp_context_destroy(ctx));
  free_csr(a); free_csr(c); hipFree(b); hipFree(bc); hipFree(x); hipFree(B); hipFree(X); hipFree(L); hipFree(Lc);
}

namespace kpp {
extern int g_emu_refuse_confirms;
extern int64_t g_emu_ahead_launches, g_emu_skipped_launches;
}

// Launches enqueued ahead of the current one: a FP64 solve to a tolerance
// enqueues the next window before the current one ends; when the host turns
// down a stop candidate (its true residual is too large) the launch enqueued
// ahead has run no step and the window is launched again, so the solve goes on
// to a later checkpoint and ends there.
static void ahead_case(int kind, int64_t m, int64_t n, int s) {
  kpp_context* ctx; CHECK(kpp_context_create(0, nullptr, &ctx));
  double* A = dev_vec(m * n, 0.5); double* b = dev_vec(m, 1.0); double* x = dev_vec(n, 0.0);
  kpp_system* sys; CHECK(kpp_system_create(ctx, kind, m, n, A, n, b, &sys));
  int64_t iters[2] = {0, 0}, skipped[2] = {0, 0}, ahead[2] = {0, 0};
  for (int refuse = 0; refuse < 2; ++refuse) {
    kpp_params p; CHECK(kpp_params_default(&p, kind));
    p.block_size = s; p.engine = 2; p.max_iters = 20000; p.tol = 1e-10; p.seed = 31; p.lambda = 1e-3;
    kpp::g_emu_refuse_confirms = refuse ? 2 : 0;
    kpp::g_emu_ahead_launches = kpp::g_emu_skipped_launches = 0;
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    kpp_result r; CHECK(kpp_solve(sys, &p, x, &r));
    if (!r.converged) { std::printf("FAIL ahead: not converged (refuse %d)\n", refuse); std::exit(1); }
    iters[refuse] = r.iters; skipped[refuse] = kpp::g_emu_skipped_launches; ahead[refuse] = kpp::g_emu_ahead_launches;
    std::printf("ahead kind=%d refuse=%d iters=%lld launches=%lld ahead=%lld skipped=%lld\n", kind, refuse,
                (long long)r.iters, (long long)r.kernel_launches, (long long)ahead[refuse], (long long)skipped[refuse]);
  }
  // every launch but the first is enqueued ahead; one skip at the stop, and
  // one more for each turned-down candidate
  if (ahead[0] < 2 || skipped[0] != 1 || skipped[1] != 3 || iters[1] <= iters[0]) {
    std::printf("FAIL ahead: iters %lld / %lld, skipped %lld / %lld\n", (long long)iters[0], (long long)iters[1],
                (long long)skipped[0], (long long)skipped[1]);
    std::exit(1);
  }
  CHECK(kpp_system_destroy(sys)); CHECK(kpp_context_destroy(ctx));
  hipFree(A); hipFree(b); hipFree(x);
}

int main(int argc, char** argv) {
  const char* only = argc > 1 ? argv[1] : "";
  if (!*only || !std::strcmp(only, "solve")) {
    for (int eng : {1, 2}) {
      solve_case("c1", 0, 1000, 200, 20, 1, 1, 0, eng, 0, 600, 0.0);
      solve_case("c2_small", 1, 1000, 1000, 128, 1, 1, 0, eng, 0, 320, 0.0);
      solve_case("c2_small_partition", 1, 1000, 1000, 128, 2, 1, 0, eng, 0, 160, 0.0);
      solve_case("c3_small", 0, 6000, 700, 256, 2, 1, 0, eng, 0, 200, 0.0);
      solve_case("c4_small", 0, 300, 5000, 64, 1, 1, 0, eng, 0, 200, 0.0);
      solve_case("tiny_under_off", 0, 30, 90, 7, 0, 1, 0, eng, 0, 150, 0.0);
      solve_case("tiny_fixed_subsets", 0, 80, 30, 9, 2, 0, 11, eng, 0, 200, 0.0);
    }
    solve_case("mixed_c3_small", 0, 6000, 700, 256, 2, 1, 0, 0, 1, 20000, 1e-10);
    solve_case("mixed_psd", 1, 1000, 1000, 128, 1, 1, 0, 0, 1, 20000, 1e-10);
    solve_case("bf16_c3_small", 0, 6000, 700, 256, 2, 1, 0, 0, 2, 20000, 1e-10);
    solve_case("bf16_c4_small", 0, 300, 5000, 64, 1, 1, 0, 0, 2, 20000, 1e-10);
    solve_case("bf16_psd", 1, 1000, 1000, 128, 1, 1, 0, 0, 2, 20000, 1e-10);
    // no step at all (max_iters = 0): nothing is launched
    solve_case("zero_steps", 0, 40, 10, 4, 1, 1, 0, 2, 0, 0, 0.0);
    ahead_case(0, 300, 5000, 64);
    ahead_case(1, 1000, 1000, 128);
    resume_case(1, 600, 600, 64);
    resume_case(0, 900, 300, 40);
    rht_case(0, 5000, 12, 16);
    rht_case(1, 100, 100, 16);
    lsqr_case(1000, 200, 20, 1);
    lsqr_case(700, 300, 160, 2);
    lsqr_case(400, 5000, 64, 0);
    lsqr_case(20000, 100, 16, 2, 600);   // 1250 blocks: about 480 new ones in the first window
    multi_case(0, 1000, 200, 20, 1, 5);
    multi_case(1, 600, 600, 64, 2, 32);
    multi_case(0, 300, 2500, 150, 0, 3);
  }
  if (!*only || !std::strcmp(only, "sparse")) {
    for (int eng : {0, 1, 2}) {
      sparse_solve("csr_kpp_online", 0, 2000, 500, 6, 32, 1, 1, eng, 400, false);
      sparse_solve("csr_kpp_fixed", 0, 2000, 500, 6, 32, 2, 1, eng, 300, false);
      sparse_solve("csr_kpp_off", 0, 600, 900, 8, 20, 0, 1, eng, 200, false);
    }
    sparse_solve("csr_kpp_big_blocks", 0, 600, 20000, 40, 150, 1, 1, 0, 60, false);
    sparse_solve("csr_kpp_big_off", 0, 600, 20000, 40, 150, 0, 1, 0, 30, false);
    sparse_solve("csr_cd_online", 1, 800, 800, 3, 40, 1, 1, 0, 300, true);
    sparse_solve("csr_cd_off", 1, 800, 800, 3, 40, 0, 1, 0, 100, true);
    sparse_solve("csr_cd_s300", 1, 900, 900, 2, 300, 2, 1, 0, 30, true);
    sparse_misc();
  }
  if (!*only || !std::strcmp(only, "serve")) serve_case();
  std::printf("EMU OK\n");
  return 0;
}
