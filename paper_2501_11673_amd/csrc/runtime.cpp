// Host runtime behind the C ABI (include/kpp.h): contexts, systems, the memo
// cache of block factors and the solver loop (Algorithms 2 and 5 of the paper,
// exact memoized Cholesky projection).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "kpp.h"
#include "schedule.hpp"

namespace {

thread_local std::string g_last_error = "no error";

kpp_status fail(kpp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(e_ == hipErrorOutOfMemory ? KPP_ERR_OOM : KPP_ERR_HIP, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                    \
  } while (0)

#define KPP_TRY(expr)                   \
  do {                                  \
    kpp_status s_ = (expr);             \
    if (s_ < 0) return s_;              \
  } while (0)

template <class T>
kpp_status dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return KPP_OK;
  HIP_TRY(hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)));
  return KPP_OK;
}

template <class T>
void dev_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

}  // namespace

struct kpp_context {
  int32_t device = 0;
  hipStream_t stream = nullptr;   // borrowed: all results are ordered on it
  hipStream_t side = nullptr;     // owned: memo-miss factorizations one window ahead
  int32_t cu_count = 0;
};

struct kpp_system {
  kpp_context* ctx = nullptr;
  int32_t kind = 0;
  int64_t m = 0, n = 0, lda = 0;
  const double* A = nullptr;
  const double* b = nullptr;
  double bnorm = 0.0;
  // device work buffers
  double* mom = nullptr;
  kpp::DevState* ds = nullptr;
  double* rpart = nullptr;
  int64_t rpart_cap = 0;
  double* y = nullptr;
  double* rowsq = nullptr;
  double* scal = nullptr;
  int32_t* err = nullptr;
  // memo cache: one slot per block (factor data, rows, length)
  double* L = nullptr;
  int32_t* rows = nullptr;
  int32_t* lens = nullptr;
  int32_t cap_slots = 0;
  int32_t slot_s = 0;
  int64_t slot_stride = 0;
  int32_t used_slots = 0;
  std::vector<int32_t> slot_of_block;
  // signature of the schedule the cache belongs to
  bool memo_valid = false;
  int32_t sig_s = 0, sig_memo = 0, sig_nb = 0, sig_part = 0, sig_prec = 0;
  uint64_t sig_seed = 0;
  double sig_lambda = 0.0;
  // per-window staging (pinned host mirror + device copy): block rows, lengths,
  // slot ids of the blocks to factor, and the slot of every step
  int32_t* h_stage[2] = {nullptr, nullptr};
  int32_t* d_stage[2] = {nullptr, nullptr};
  size_t stage_cap[2] = {0, 0};
  hipEvent_t ev_fact[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};  // start, end, ready
  kpp::DevState* h_ds = nullptr;
  int32_t* h_err = nullptr;
  // fused engine
  double* part = nullptr;
  uint32_t* flags = nullptr;
  uint32_t epoch = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  uint64_t* phase_ticks = nullptr;   // KPP_PHASE_PROFILE=1: fused-engine phase profile
  // mixed precision: FP32 copy of A (leading dimension n), outer residual, correction
  float* A32 = nullptr;
  double* gram_ws[2] = {nullptr, nullptr};   // split-Gram partial tiles, one per staging buffer
  size_t gram_ws_cap[2] = {0, 0};
  double* rvec = nullptr;
  double* dvec = nullptr;
  int32_t* fp64_count = nullptr;   // blocks refactored in FP64 (mixed precision)
};

namespace {

constexpr int kFlagWords = kpp::kFlagWordsAlloc;

void destroy_buffers(kpp_system* s) {
  dev_free(s->mom);
  dev_free(s->ds);
  dev_free(s->rpart);
  dev_free(s->y);
  dev_free(s->rowsq);
  dev_free(s->scal);
  dev_free(s->err);
  dev_free(s->L);
  dev_free(s->rows);
  dev_free(s->lens);
  for (int i = 0; i < 2; ++i) {
    dev_free(s->d_stage[i]);
    if (s->h_stage[i]) (void)hipHostFree(s->h_stage[i]);
    s->h_stage[i] = nullptr;
    s->stage_cap[i] = 0;
    for (auto& e : s->ev_fact[i])
      if (e) {
        (void)hipEventDestroy(e);
        e = nullptr;
      }
  }
  dev_free(s->part);
  dev_free(s->flags);
  dev_free(s->phase_ticks);
  dev_free(s->A32);
  for (int i = 0; i < 2; ++i) {
    dev_free(s->gram_ws[i]);
    s->gram_ws_cap[i] = 0;
  }
  dev_free(s->rvec);
  dev_free(s->dvec);
  dev_free(s->fp64_count);
  if (s->h_ds) (void)hipHostFree(s->h_ds);
  if (s->h_err) (void)hipHostFree(s->h_err);
  s->h_ds = nullptr;
  s->h_err = nullptr;
  for (auto& e : s->ev)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
  s->cap_slots = 0;
}

// Grow the slot table to hold `need` slots for block size s (keeps contents).
kpp_status ensure_slots(kpp_system* sys, int32_t need, int32_t s) {
  hipStream_t st = sys->ctx->stream;
  if (sys->slot_s != s) {
    // a different block size invalidates every cached factor
    dev_free(sys->L);
    dev_free(sys->rows);
    dev_free(sys->lens);
    sys->cap_slots = 0;
    sys->slot_s = s;
    sys->slot_stride = kpp::slot_doubles(s);
    sys->used_slots = 0;
    sys->slot_of_block.clear();
    sys->memo_valid = false;
  }
  if (need <= sys->cap_slots) return KPP_OK;
  // kernels in flight on either stream may read the old table
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipStreamSynchronize(sys->ctx->side));
  const int32_t cap = std::max<int32_t>(need, std::max<int32_t>(16, sys->cap_slots * 2));
  double* L = nullptr;
  int32_t *rows = nullptr, *lens = nullptr;
  const size_t sd = static_cast<size_t>(sys->slot_stride);
  KPP_TRY(dev_alloc(&L, sd * cap));
  KPP_TRY(dev_alloc(&rows, static_cast<size_t>(s) * cap));
  KPP_TRY(dev_alloc(&lens, cap));
  if (sys->cap_slots > 0) {
    HIP_TRY(hipMemcpyAsync(L, sys->L, sd * sys->cap_slots * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(rows, sys->rows, static_cast<size_t>(s) * sys->cap_slots * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(lens, sys->lens, sys->cap_slots * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  dev_free(sys->L);
  dev_free(sys->rows);
  dev_free(sys->lens);
  sys->L = L;
  sys->rows = rows;
  sys->lens = lens;
  sys->cap_slots = cap;
  return KPP_OK;
}

kpp_status ensure_stage(kpp_system* sys, int idx, size_t ints) {
  if (ints <= sys->stage_cap[idx]) return KPP_OK;
  const size_t cap = std::max<size_t>(ints, std::max<size_t>(4096, sys->stage_cap[idx] * 2));
  HIP_TRY(hipStreamSynchronize(sys->ctx->stream));
  HIP_TRY(hipStreamSynchronize(sys->ctx->side));
  dev_free(sys->d_stage[idx]);
  if (sys->h_stage[idx]) (void)hipHostFree(sys->h_stage[idx]);
  sys->h_stage[idx] = nullptr;
  sys->stage_cap[idx] = 0;
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&sys->h_stage[idx]), cap * sizeof(int32_t), hipHostMallocDefault));
  KPP_TRY(dev_alloc(&sys->d_stage[idx], cap));
  sys->stage_cap[idx] = cap;
  return KPP_OK;
}

// Workspace of the split Kaczmarz++ Gram for staging buffer idx.
kpp_status ensure_gram_ws(kpp_system* sys, int idx, size_t doubles) {
  if (doubles <= sys->gram_ws_cap[idx]) return KPP_OK;
  const size_t cap = std::max<size_t>(doubles, sys->gram_ws_cap[idx] * 2);
  HIP_TRY(hipStreamSynchronize(sys->ctx->stream));
  HIP_TRY(hipStreamSynchronize(sys->ctx->side));
  dev_free(sys->gram_ws[idx]);
  sys->gram_ws_cap[idx] = 0;
  KPP_TRY(dev_alloc(&sys->gram_ws[idx], cap));
  sys->gram_ws_cap[idx] = cap;
  return KPP_OK;
}

kpp_status check_params(const kpp_system* sys, const kpp_params* p) {
  if (!p) return fail(KPP_ERR_INVALID_ARG, "params is NULL");
  const int64_t rows = sys->kind == KPP_CD_PSD ? sys->n : sys->m;
  if (p->block_size < 1 || p->block_size > rows || p->block_size > kpp::kMaxBlock)
    return fail(KPP_ERR_INVALID_ARG, "block_size %d must be in [1, min(rows=%lld, %d)]",
                p->block_size, static_cast<long long>(rows), kpp::kMaxBlock);
  if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda))
    return fail(KPP_ERR_INVALID_ARG, "lambda must be finite and >= 0");
  if (!(p->tol >= 0.0)) return fail(KPP_ERR_INVALID_ARG, "tol must be >= 0");
  if (p->max_iters < 0) return fail(KPP_ERR_INVALID_ARG, "max_iters must be >= 0");
  if (p->memo < 0 || p->memo > 2) return fail(KPP_ERR_INVALID_ARG, "unknown memo mode %d", p->memo);
  if (p->memo == KPP_MEMO_FIXED && !p->fixed_partition && p->num_blocks < 1)
    return fail(KPP_ERR_INVALID_ARG, "fixed collection needs num_blocks >= 1");
  if (!(p->rho0 >= 0.0 && p->rho0 <= 1.0)) return fail(KPP_ERR_INVALID_ARG, "rho0 must be in [0, 1]");
  if (p->precision != KPP_FP64 && p->precision != KPP_MIXED_FP32)
    return fail(KPP_ERR_INVALID_ARG, "precision %d is not available in this build", p->precision);
  if (p->precision == KPP_MIXED_FP32) {
    if (p->engine == 1) return fail(KPP_ERR_INVALID_ARG, "mixed precision runs on the fused engine");
    if (p->block_size > kpp::kFusedMaxBlock)
      return fail(KPP_ERR_INVALID_ARG, "mixed precision takes block_size <= %d", kpp::kFusedMaxBlock);
    if (!(p->inner_tol > 0.0 && p->inner_tol < 1.0)) return fail(KPP_ERR_INVALID_ARG, "inner_tol must be in (0, 1)");
    if (p->refine_max_rounds < 1) return fail(KPP_ERR_INVALID_ARG, "refine_max_rounds must be >= 1");
  }
  if (p->engine < 0 || p->engine > 2) return fail(KPP_ERR_INVALID_ARG, "unknown engine %d", p->engine);
  if (p->engine == 2 && p->block_size > kpp::kFusedMaxBlock)
    return fail(KPP_ERR_INVALID_ARG, "the fused engine takes block_size <= %d", kpp::kFusedMaxBlock);
  if (p->team_groups < 0 || p->team_groups > kpp::kFusedMaxGroups)
    return fail(KPP_ERR_INVALID_ARG, "team_groups must be in [0, %d]", kpp::kFusedMaxGroups);
  return KPP_OK;
}

double default_eta(int32_t kind, int64_t m, int64_t n, int32_t s) {
  if (kind == KPP_CD_PSD) return s / (2.0 * static_cast<double>(n));
  return s / (2.0 * static_cast<double>(std::min(m, n)));
}

kpp_status residual_norm(kpp_system* sys, const double* x, double* out) {
  hipStream_t st = sys->ctx->stream;
  kpp::launch_residual_sq(sys->A, sys->lda, sys->m, sys->n, x, sys->b, sys->rowsq, 0, sys->scal, st);
  HIP_TRY(hipGetLastError());
  double v = 0.0;
  HIP_TRY(hipMemcpyAsync(&v, sys->scal, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *out = std::sqrt(v);
  return KPP_OK;
}

// Fused-engine geometry: columns per lane (cpl) and workgroups per step.  A
// wave holds ceil(s/4) block rows of cpl columns in registers (at most 64
// doubles per lane), so cpl <= 256/s; the smallest cpl that brings the team
// down to the target size is taken.
bool fused_geometry(int64_t n, int32_t s, int32_t target_groups, int32_t* cpl, int32_t* groups) {
  if (s > kpp::kFusedMaxBlock) return false;
  const int32_t gmax = target_groups > 0 ? target_groups : 32;
  const int32_t rows_per_wave = (s + 3) / 4;
  int32_t cmax = 1;
  while (cmax < 16 && 2 * cmax * rows_per_wave <= 64) cmax *= 2;
  int32_t c = 1;
  while (c < cmax && (n + 64 * c - 1) / (64 * c) > gmax) c *= 2;
  const int64_t g = (n + 64 * c - 1) / (64 * c);
  if (g > kpp::kFusedMaxGroups) return false;
  *cpl = c;
  *groups = static_cast<int32_t>(g);
  return true;
}

// The matrix and right-hand side one run of the block iteration works on: the
// caller's FP64 system, or (mixed precision) the FP32 copy of A with the
// current outer residual as right-hand side.
struct Source {
  const double* A64 = nullptr;
  const float* A32 = nullptr;
  int64_t lda = 0;
  const double* b = nullptr;
  double bnorm = 0.0;
};

struct CoreOpts {
  double tol = 0.0;
  int32_t confirm = 1;      // confirm a candidate stop with ||A x - b|| (FP64 system only)
  double rho0 = 0.0;
  int32_t keep_memo = 0;
  int64_t max_iters = 0;
};

struct CoreStats {
  int64_t iters = 0, hits = 0, misses = 0, launches = 0;
  bool converged = false;
  double true_rel = NAN, t_factor = 0.0, t_kernel = 0.0;
  kpp::DevState hs{};
  int32_t engine = 0;
};

kpp_status solve_core(kpp_system* sys, const kpp_params* p, const Source& src, const CoreOpts& o,
                      double* x, CoreStats* cs) {
  hipStream_t st = sys->ctx->stream;
  const bool fp32 = src.A32 != nullptr;
  const int32_t kind = sys->kind;
  const int64_t m = sys->m, n = sys->n;
  const int64_t N = kind == KPP_CD_PSD ? n : m;
  const int32_t s = p->block_size;
  const int32_t zeta = static_cast<int32_t>((N + s - 1) / s);
  double eta = p->eta < 0.0 ? default_eta(kind, m, n, s) : p->eta;
  if (!p->accel) eta = 0.0;
  const kpp::MemoMode mode = static_cast<kpp::MemoMode>(p->memo);
  const double B0 = kpp::online_rate(kind, m, n, s);
  std::unique_ptr<kpp::BlockSchedule> sch;
  try {
    sch.reset(new kpp::BlockSchedule(mode, N, s, p->seed, B0, p->num_blocks, p->fixed_partition != 0));
  } catch (const std::exception& e) {
    return fail(KPP_ERR_INVALID_ARG, "%s", e.what());
  }
  // engine
  int32_t cpl = 0, groups = 0;
  bool fused = false;
  if (p->engine != 1) fused = fused_geometry(n, s, p->team_groups, &cpl, &groups);
  if (p->engine == 2 && !fused) return fail(KPP_ERR_INVALID_ARG, "n=%lld is too wide for the fused engine", (long long)n);

  // memo cache: reuse only for an identical schedule definition; the slot
  // table is sized for this block size before any slot is handed out
  KPP_TRY(ensure_slots(sys, 16, s));
  const bool same_sig = sys->memo_valid && o.keep_memo && sys->sig_s == s && sys->sig_memo == p->memo &&
                        sys->sig_nb == p->num_blocks && sys->sig_part == p->fixed_partition &&
                        sys->sig_seed == p->seed && sys->sig_lambda == p->lambda &&
                        sys->sig_prec == (fp32 ? 1 : 0) && mode != kpp::MemoMode::Off;
  if (!same_sig) {
    sys->slot_of_block.clear();
    sys->used_slots = 0;
    sys->memo_valid = mode != kpp::MemoMode::Off;
    sys->sig_s = s;
    sys->sig_memo = p->memo;
    sys->sig_nb = p->num_blocks;
    sys->sig_part = p->fixed_partition;
    sys->sig_seed = p->seed;
    sys->sig_lambda = p->lambda;
    sys->sig_prec = fp32 ? 1 : 0;
  }
  if (mode == kpp::MemoMode::Fixed) KPP_TRY(ensure_slots(sys, sch->num_blocks(), s));
  // launch engine: column chunks of the block gemv
  const int64_t chunk = 2048;
  const int32_t P = static_cast<int32_t>((n + chunk - 1) / chunk);
  if (!fused && static_cast<int64_t>(s) * P > sys->rpart_cap) {
    dev_free(sys->rpart);
    KPP_TRY(dev_alloc(&sys->rpart, static_cast<size_t>(s) * P));
    sys->rpart_cap = static_cast<int64_t>(s) * P;
  }
  HIP_TRY(hipMemsetAsync(sys->mom, 0, n * sizeof(double), st));
  HIP_TRY(hipMemsetAsync(sys->err, 0, sizeof(int32_t), st));
  const double thr = o.tol * o.tol * src.bnorm * src.bnorm;
  kpp::launch_state_init(sys->ds, o.rho0, thr, st);
  HIP_TRY(hipGetLastError());

  const char* prof_env = std::getenv("KPP_PHASE_PROFILE");
  const bool phase_prof = fused && prof_env && prof_env[0] == '1';
  if (phase_prof) {
    if (!sys->phase_ticks) KPP_TRY(dev_alloc(&sys->phase_ticks, kpp::kFusedPhases));
    HIP_TRY(hipMemsetAsync(sys->phase_ticks, 0, kpp::kFusedPhases * sizeof(uint64_t), st));
  }
  int64_t hits = 0, misses = 0, t = 0;
  bool converged = false;
  double true_rel = NAN;
  double t_factor = 0.0, t_kernel = 0.0;
  int64_t launches = 0;
  kpp::DevState hs{};
  const int64_t max_iters = o.max_iters;
  const int64_t period = 2 * static_cast<int64_t>(zeta);
  const size_t sd = static_cast<size_t>(sys->slot_stride);

  // A window is the run of steps up to the next checkpoint.  Planning a window
  // draws its blocks, assigns memo slots and stages (pinned) the rows of its
  // new blocks plus the slot of every step; its memo misses are then factored
  // on the side stream while the previous window runs on the main stream.
  struct Window {
    int64_t t0 = 0, W = 0;
    int32_t nb = 0, idx = 0;
    size_t o_len = 0, o_slot = 0, o_step = 0;
    std::vector<int32_t> step_block, step_slot;
  };
  auto plan = [&](Window& w, int64_t t0, int idx) -> kpp_status {
    w.t0 = t0;
    w.idx = idx;
    w.W = std::min<int64_t>(period - (t0 % period), max_iters - t0);
    w.step_block.resize(w.W);
    w.step_slot.resize(w.W);
    std::vector<int32_t> pending, pending_slots;
    if (mode == kpp::MemoMode::Off) KPP_TRY(ensure_slots(sys, static_cast<int32_t>(2 * period), s));
    for (int64_t k = 0; k < w.W; ++k) {
      bool is_new = false;
      const int32_t b = sch->next(&is_new);
      w.step_block[k] = b;
      if (mode == kpp::MemoMode::Off) {
        // windows alternate between two halves of the slot table
        const int32_t q = static_cast<int32_t>(idx * period + k);
        w.step_slot[k] = q;
        pending.push_back(b);
        pending_slots.push_back(q);
        ++misses;
        continue;
      }
      if (static_cast<int32_t>(sys->slot_of_block.size()) <= b) sys->slot_of_block.resize(b + 1, -1);
      int32_t q = sys->slot_of_block[b];
      if (q < 0) {
        q = sys->used_slots++;
        sys->slot_of_block[b] = q;
        pending.push_back(b);
        pending_slots.push_back(q);
        ++misses;
      } else {
        ++hits;
      }
      w.step_slot[k] = q;
    }
    if (mode != kpp::MemoMode::Off) KPP_TRY(ensure_slots(sys, sys->used_slots, s));
    w.nb = static_cast<int32_t>(pending.size());
    w.o_len = static_cast<size_t>(w.nb) * s;
    w.o_slot = w.o_len + w.nb;
    w.o_step = w.o_slot + w.nb;
    const size_t need = w.o_step + static_cast<size_t>(w.W) + static_cast<size_t>(w.nb);  // + flags
    KPP_TRY(ensure_stage(sys, idx, need));
    int32_t* hs_ = sys->h_stage[idx];
    for (int32_t k = 0; k < w.nb; ++k) {
      const int32_t b = pending[k];
      const int32_t l = sch->len(b);
      std::copy(sch->rows(b), sch->rows(b) + l, hs_ + static_cast<size_t>(k) * s);
      std::fill(hs_ + static_cast<size_t>(k) * s + l, hs_ + static_cast<size_t>(k + 1) * s, 0);
      hs_[w.o_len + k] = l;
      hs_[w.o_slot + k] = pending_slots[k];
    }
    std::copy(w.step_slot.begin(), w.step_slot.end(), hs_ + w.o_step);
    return KPP_OK;
  };
  // upload the window's staging and factor its memo misses on `fs`
  auto enqueue_factor = [&](const Window& w, hipStream_t fs) -> kpp_status {
    const int idx = w.idx;
    const size_t need = w.o_step + static_cast<size_t>(w.W);
    HIP_TRY(hipMemcpyAsync(sys->d_stage[idx], sys->h_stage[idx], need * sizeof(int32_t), hipMemcpyHostToDevice, fs));
    HIP_TRY(hipEventRecord(sys->ev_fact[idx][0], fs));
    if (w.nb > 0) {
      const int32_t* d_srows = sys->d_stage[idx];
      const int32_t* d_slens = sys->d_stage[idx] + w.o_len;
      const int32_t* d_sslot = sys->d_stage[idx] + w.o_slot;
      kpp::launch_scatter_rows(d_srows, d_slens, d_sslot, w.nb, s, sys->rows, sys->lens, fs);
      if (kind == KPP_KACZMARZ) KPP_TRY(ensure_gram_ws(sys, idx, kpp::gram_syrk_work(s, n, w.nb)));
      double* gws = sys->gram_ws[idx];
      auto factor = [&](const kpp::FactorCheck& chk, const int32_t* skip) {
        if (s <= kpp::kFactorSmallMax) {
          kpp::launch_factor_small(sys->L, sys->slot_stride, s, d_slens, w.nb, d_sslot, 1, sys->err, fs, chk);
        } else {
          kpp::launch_cholesky(sys->L, s, sys->slot_stride, d_slens, w.nb, d_sslot, sys->err, fs, chk);
          kpp::launch_factor_inverse(sys->L, sys->slot_stride, s, d_slens, w.nb, d_sslot, fs, chk, skip);
        }
      };
      if (fp32) {
        // FP32 Grams; blocks whose factor breaks down or whose kappa(G) exceeds
        // 1e6 are formed again from the FP64 A and factored in FP64
        int32_t* flag = sys->d_stage[idx] + w.o_step + w.W;
        kpp::launch_gram_f32(kind, src.A32, src.lda, n, d_srows, d_slens, s, w.nb, p->lambda, sys->L,
                             sys->slot_stride, d_sslot, gws, fs);
        kpp::FactorCheck first;
        first.flag = flag;
        first.counter = sys->fp64_count;
        first.kappa_max = 1e6;
        factor(first, flag);
        kpp::launch_gram(kind, sys->A, sys->lda, n, d_srows, d_slens, s, w.nb, p->lambda, sys->L,
                         sys->slot_stride, d_sslot, gws, fs, flag);
        kpp::FactorCheck redo;
        redo.only = flag;
        factor(redo, nullptr);
      } else {
        kpp::launch_gram(kind, src.A64, src.lda, n, d_srows, d_slens, s, w.nb, p->lambda, sys->L,
                         sys->slot_stride, d_sslot, gws, fs);
        factor(kpp::FactorCheck(), nullptr);
      }
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipEventRecord(sys->ev_fact[idx][1], fs));
    return KPP_OK;
  };

  // the side stream's first work must follow this solve's initialisation
  HIP_TRY(hipEventRecord(sys->ev_fact[1][2], st));
  HIP_TRY(hipStreamWaitEvent(sys->ctx->side, sys->ev_fact[1][2], 0));
  Window win[2];
  bool have_next = false;
  if (max_iters > 0) {
    KPP_TRY(plan(win[0], 0, 0));
    KPP_TRY(enqueue_factor(win[0], st));  // nothing to overlap with yet
  }
  int cur = 0;
  while (t < max_iters && !converged) {
    Window& w = win[cur];
    if (have_next) HIP_TRY(hipStreamWaitEvent(st, sys->ev_fact[cur][1], 0));
    const int32_t* d_step = sys->d_stage[cur] + w.o_step;
    HIP_TRY(hipEventRecord(sys->ev[0], st));
    if (fused) {
      if (sys->epoch > 0x3fffffffu) {
        HIP_TRY(hipMemsetAsync(sys->flags, 0, kFlagWords * sizeof(uint32_t), st));
        sys->epoch = 0;
      }
      kpp::FusedArgs a{};
      a.A = fp32 ? static_cast<const void*>(src.A32) : static_cast<const void*>(src.A64);
      a.lda = src.lda;
      a.n = n;
      a.b = src.b;
      a.rows = sys->rows;
      a.lens = sys->lens;
      a.L = sys->L;
      a.slot_stride = sys->slot_stride;
      a.s = s;
      a.W = static_cast<int32_t>(w.W);
      a.step_slot = d_step;
      a.x = x;
      a.mom = sys->mom;
      a.part = sys->part;
      a.flags = sys->flags;
      a.epoch = sys->epoch;
      a.zeta = zeta;
      a.adaptive = p->adaptive_rho;
      a.eta = eta;
      a.ds = sys->ds;
      a.err = sys->err;
      a.spin_limit = int64_t{1} << 22;
      a.phase_ticks = phase_prof ? sys->phase_ticks : nullptr;
      kpp::launch_fused(kind, fp32, a, cpl, groups, st);
      sys->epoch += static_cast<uint32_t>(w.W);
      ++launches;
    } else {
      for (int64_t k = 0; k < w.W; ++k) {
        const int32_t q = w.step_slot[k];
        const int32_t sb = sch->len(w.step_block[k]);
        const int32_t* rows = sys->rows + static_cast<size_t>(q) * s;
        kpp::launch_block_gemv_partial(src.A64, src.lda, n, rows, sb, x, sys->rpart, P, chunk, st);
        kpp::launch_block_project(sys->rpart, P, src.b, rows, sb, sys->L + sd * q + static_cast<size_t>(s) * s,
                                  s, sys->y, sys->ds, zeta, p->adaptive_rho, st);
        kpp::launch_update(kind, src.A64, src.lda, n, rows, sb, sys->y, sys->ds, eta, x, sys->mom, st);
      }
      launches += 3 * w.W;
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(sys->ev[1], st));
    HIP_TRY(hipMemcpyAsync(sys->h_ds, sys->ds, sizeof(kpp::DevState), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(sys->h_err, sys->err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    // plan and factor the next window while this one runs
    const int64_t t_next = t + w.W;
    have_next = false;
    if (t_next < max_iters) {
      KPP_TRY(plan(win[cur ^ 1], t_next, cur ^ 1));
      KPP_TRY(enqueue_factor(win[cur ^ 1], sys->ctx->side));
      have_next = true;
    }
    HIP_TRY(hipStreamSynchronize(st));
    hs = *sys->h_ds;
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, sys->ev[0], sys->ev[1]));
    t_kernel += 1e-3 * ms;
    if (w.nb > 0) {
      HIP_TRY(hipEventElapsedTime(&ms, sys->ev_fact[cur][0], sys->ev_fact[cur][1]));
      t_factor += 1e-3 * ms;
    }
    const int32_t herr = *sys->h_err;
    if (herr & 2) {
      HIP_TRY(hipStreamSynchronize(sys->ctx->side));
      HIP_TRY(hipMemsetAsync(sys->flags, 0, kFlagWords * sizeof(uint32_t), st));
      HIP_TRY(hipStreamSynchronize(st));
      sys->epoch = 0;
      return fail(KPP_ERR_DEVICE, "a device-side wait exceeded its bound in the fused engine");
    }
    if (herr & 1) {
      HIP_TRY(hipStreamSynchronize(sys->ctx->side));
      return fail(KPP_ERR_NOT_SPD, "a regularized block Gram has no Cholesky factor (lambda=%g)", p->lambda);
    }
    t = t_next;
    if ((t % period) == 0 && hs.cand) {
      if (o.confirm) {
        double rn = 0.0;
        KPP_TRY(residual_norm(sys, x, &rn));
        true_rel = sys->bnorm > 0 ? rn / sys->bnorm : rn;
        if (rn <= o.tol * sys->bnorm) converged = true;
      } else {
        converged = true;
      }
    }
    cur ^= 1;
  }
  // factorizations planned past the stop are dropped from the counts; the
  // side stream is drained so that no work of this call is left in flight
  HIP_TRY(hipStreamSynchronize(sys->ctx->side));
  if (have_next && converged) {
    const Window& w = win[cur];
    misses -= w.nb;
    hits -= w.W - w.nb;
  }
  if (o.confirm && (!converged || std::isnan(true_rel))) {
    double rn = 0.0;
    KPP_TRY(residual_norm(sys, x, &rn));
    true_rel = sys->bnorm > 0 ? rn / sys->bnorm : rn;
  }
  if (phase_prof && t > 0) {
    uint64_t ticks[kpp::kFusedPhases];
    HIP_TRY(hipMemcpy(ticks, sys->phase_ticks, sizeof ticks, hipMemcpyDeviceToHost));
    int rate_khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, sys->ctx->device));
    static const char* names[kpp::kFusedPhases] = {"rows", "tile-dot", "publish", "wait", "reduce-r",
                                                   "solve+scalars", "update", "-"};
    std::fprintf(stderr, "[kpp phase profile] %lld steps, workgroup 0, us per step:", static_cast<long long>(t));
    for (int ph = 0; ph < kpp::kFusedPhases - 1; ++ph)
      std::fprintf(stderr, " %s=%.3f", names[ph], 1e3 * static_cast<double>(ticks[ph]) / rate_khz / static_cast<double>(t));
    std::fprintf(stderr, "\n");
  }
  cs->iters = t;
  cs->hits = hits;
  cs->misses = misses;
  cs->launches = launches;
  cs->converged = converged;
  cs->true_rel = true_rel;
  cs->t_factor = t_factor;
  cs->t_kernel = t_kernel;
  cs->hs = hs;
  cs->engine = fused ? 2 : 1;
  return converged ? KPP_OK : KPP_NOT_CONVERGED;
}


void fill_result(kpp_result* res, const kpp_system* sys, const kpp_params* p, int64_t iters, int64_t hits,
                 int64_t misses, bool converged, int32_t rounds, const CoreStats& last, double true_rel,
                 double est_rel, double rho_final, double seconds, double t_factor, double t_kernel,
                 int64_t launches, int64_t checkpoints, double bytes_per_elem) {
  if (!res) return;
  const int32_t kind = sys->kind;
  const int64_t n = sys->n;
  const int32_t s = p->block_size;
  res->iters = iters;
  res->memo_hits = hits;
  res->memo_misses = misses;
  res->factors_fp64 = misses;
  res->converged = converged ? 1 : 0;
  res->refinements = rounds;
  res->checkpoints = static_cast<int32_t>(checkpoints);
  res->engine_used = last.engine;
  res->est_rel_res = est_rel;
  res->true_rel_res = true_rel;
  res->rho_final = rho_final;
  res->seconds_total = seconds;
  res->seconds_factor = t_factor;
  const double sdb = s;
  const double nn = static_cast<double>(n);
  const double per_step = 2.0 * sdb * nn + 2.0 * sdb * sdb + (kind == KPP_CD_PSD ? 0.0 : 2.0 * sdb * nn) + 5.0 * nn;
  const double per_fact = sdb * sdb * sdb / 3.0 + (kind == KPP_CD_PSD ? 0.0 : sdb * sdb * nn);
  res->flops = per_step * static_cast<double>(iters) + per_fact * static_cast<double>(misses);
  res->bytes_algorithmic =
      static_cast<double>(iters) * (sdb * nn * bytes_per_elem + 0.5 * sdb * (sdb + 1) * 8.0 + 12.0 * sdb);
  res->kernel_seconds = t_kernel;
  res->kernel_launches = static_cast<double>(launches);
}

kpp_status solve_fp64(kpp_system* sys, const kpp_params* p, double* x, kpp_result* res) {
  using clock = std::chrono::steady_clock;
  const auto t0 = clock::now();
  Source src;
  src.A64 = sys->A;
  src.lda = sys->lda;
  src.b = sys->b;
  src.bnorm = sys->bnorm;
  CoreOpts o;
  o.tol = p->tol;
  o.confirm = p->confirm_true_residual;
  o.rho0 = p->rho0;
  o.keep_memo = p->keep_memo;
  o.max_iters = p->max_iters;
  CoreStats cs;
  KPP_TRY(solve_core(sys, p, src, o, x, &cs));
  double true_rel = cs.true_rel;
  if (std::isnan(true_rel)) {
    double rn = 0.0;
    KPP_TRY(residual_norm(sys, x, &rn));
    true_rel = sys->bnorm > 0 ? rn / sys->bnorm : rn;
  }
  const double est = sys->bnorm > 0 ? std::sqrt(cs.hs.last_E1) / sys->bnorm : std::sqrt(cs.hs.last_E1);
  fill_result(res, sys, p, cs.iters, cs.hits, cs.misses, cs.converged, 0, cs, true_rel, est,
              cs.converged ? cs.hs.rho_before : cs.hs.rho,
              std::chrono::duration<double>(clock::now() - t0).count(), cs.t_factor, cs.t_kernel, cs.launches,
              cs.hs.ckpts, 8.0);
  return cs.converged ? KPP_OK : KPP_NOT_CONVERGED;
}

// Mixed precision: classical iterative refinement.  The outer loop is FP64 --
// r = b - A x over the caller's FP64 A, x += d -- and each correction d comes
// from the block iteration on A32 d = r (FP32 A_S products and Grams, FP64
// factors, FP64 momentum and iterate) run to the relative tolerance inner_tol.
// The memo cache of block factors carries over from round to round.
kpp_status solve_mixed(kpp_system* sys, const kpp_params* p, double* x, kpp_result* res) {
  using clock = std::chrono::steady_clock;
  const auto t0 = clock::now();
  hipStream_t st = sys->ctx->stream;
  const int64_t m = sys->m, n = sys->n;
  if (!sys->A32) {
    KPP_TRY(dev_alloc(&sys->A32, static_cast<size_t>(m) * n));
    kpp::launch_convert_f32(sys->A, sys->lda, m, n, sys->A32, st);
    HIP_TRY(hipGetLastError());
  }
  if (!sys->rvec) KPP_TRY(dev_alloc(&sys->rvec, m));
  if (!sys->dvec) KPP_TRY(dev_alloc(&sys->dvec, n));
  if (!sys->fp64_count) KPP_TRY(dev_alloc(&sys->fp64_count, 1));
  HIP_TRY(hipMemsetAsync(sys->fp64_count, 0, sizeof(int32_t), st));
  int64_t iters = 0, hits = 0, misses = 0, launches = 0, ckpts = 0;
  double t_factor = 0.0, t_kernel = 0.0, rho = p->rho0, true_rel = NAN, est = NAN;
  bool converged = false;
  int32_t rounds = 0;
  CoreStats last;
  for (;;) {
    kpp::launch_residual_vec(sys->A, sys->lda, m, n, x, sys->b, sys->rvec, sys->rowsq, sys->scal, st);
    HIP_TRY(hipGetLastError());
    double rr = 0.0;
    HIP_TRY(hipMemcpyAsync(&rr, sys->scal, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double rn = std::sqrt(rr);
    true_rel = sys->bnorm > 0 ? rn / sys->bnorm : rn;
    if (rn <= p->tol * sys->bnorm) {
      converged = true;
      break;
    }
    if (rounds >= p->refine_max_rounds || iters >= p->max_iters) break;
    HIP_TRY(hipMemsetAsync(sys->dvec, 0, n * sizeof(double), st));
    Source src;
    src.A32 = sys->A32;
    src.lda = n;
    src.b = sys->rvec;
    src.bnorm = rn;
    CoreOpts o;
    o.tol = p->inner_tol;
    o.confirm = 0;
    o.rho0 = rho;
    o.keep_memo = rounds > 0 ? 1 : p->keep_memo;
    o.max_iters = p->max_iters - iters;
    CoreStats cs;
    KPP_TRY(solve_core(sys, p, src, o, sys->dvec, &cs));
    kpp::launch_axpy1(x, sys->dvec, n, st);
    HIP_TRY(hipGetLastError());
    ++rounds;
    iters += cs.iters;
    hits += cs.hits;
    misses += cs.misses;
    launches += cs.launches;
    ckpts += cs.hs.ckpts;
    t_factor += cs.t_factor;
    t_kernel += cs.t_kernel;
    rho = cs.converged ? cs.hs.rho_before : cs.hs.rho;
    est = rn > 0 ? std::sqrt(cs.hs.last_E1) / rn : 0.0;
    last = cs;
  }
  fill_result(res, sys, p, iters, hits, misses, converged, rounds, last, true_rel, est, rho,
              std::chrono::duration<double>(clock::now() - t0).count(), t_factor, t_kernel, launches, ckpts, 4.0);
  if (res) {
    int32_t nfp64 = 0;
    HIP_TRY(hipMemcpy(&nfp64, sys->fp64_count, sizeof(int32_t), hipMemcpyDeviceToHost));
    res->factors_fp64 = nfp64;
  }
  return converged ? KPP_OK : KPP_NOT_CONVERGED;
}

}  // namespace

extern "C" {

KPP_API int32_t kpp_abi_version(void) { return KPP_ABI_VERSION; }

KPP_API const char* kpp_last_error(void) { return g_last_error.c_str(); }

KPP_API kpp_status kpp_params_default(kpp_params* p, int32_t kind) {
  if (!p) return fail(KPP_ERR_INVALID_ARG, "params is NULL");
  if (kind != KPP_KACZMARZ && kind != KPP_CD_PSD) return fail(KPP_ERR_INVALID_ARG, "unknown kind %d", kind);
  std::memset(p, 0, sizeof(*p));
  p->block_size = 128;
  p->memo = KPP_MEMO_ONLINE;
  p->num_blocks = 0;
  p->fixed_partition = 1;
  p->accel = 1;
  p->adaptive_rho = 1;
  p->precision = KPP_FP64;
  p->confirm_true_residual = 1;
  p->lambda = 1e-8;
  p->tol = 1e-10;
  p->eta = -1.0;
  p->rho0 = 0.0;
  p->max_iters = 1000000;
  p->seed = 0x2501116730ull;
  p->keep_memo = 0;
  p->refine_max_rounds = 12;
  p->inner_tol = 1e-3;
  p->engine = 0;
  p->team_groups = 0;
  return KPP_OK;
}

KPP_API kpp_status kpp_context_create(int32_t device, void* hip_stream, kpp_context** out) {
  if (!out) return fail(KPP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(KPP_ERR_INVALID_ARG, "device %d of %d", device, count);
  HIP_TRY(hipSetDevice(device));
  auto* c = new (std::nothrow) kpp_context;
  if (!c) return fail(KPP_ERR_OOM, "host allocation failed");
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(KPP_ERR_HIP, "hipStreamCreateWithFlags failed");
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->cu_count = prop.multiProcessorCount;
  *out = c;
  return KPP_OK;
}

KPP_API kpp_status kpp_context_destroy(kpp_context* ctx) {
  if (ctx) {
    (void)hipSetDevice(ctx->device);
    if (ctx->side) {
      (void)hipStreamSynchronize(ctx->side);
      (void)hipStreamDestroy(ctx->side);
    }
  }
  delete ctx;
  return KPP_OK;
}

KPP_API kpp_status kpp_system_create(kpp_context* ctx, int32_t kind, int64_t m, int64_t n,
                                     const double* A_dev, int64_t lda, const double* b_dev,
                                     kpp_system** out) {
  if (!out) return fail(KPP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx || !A_dev || !b_dev) return fail(KPP_ERR_INVALID_ARG, "NULL context, A or b");
  if (kind != KPP_KACZMARZ && kind != KPP_CD_PSD) return fail(KPP_ERR_INVALID_ARG, "unknown kind %d", kind);
  if (m < 1 || n < 1) return fail(KPP_ERR_SHAPE, "empty system (m=%lld, n=%lld)", (long long)m, (long long)n);
  if (lda < n) return fail(KPP_ERR_SHAPE, "lda=%lld < n=%lld", (long long)lda, (long long)n);
  if (kind == KPP_CD_PSD && m != n) return fail(KPP_ERR_SHAPE, "CD++ needs a square matrix");
  if (m > (int64_t{1} << 31) - 1 || n > (int64_t{1} << 31) - 1) return fail(KPP_ERR_SHAPE, "dimension above 2^31-1");
  HIP_TRY(hipSetDevice(ctx->device));
  std::unique_ptr<kpp_system> sys(new (std::nothrow) kpp_system);
  if (!sys) return fail(KPP_ERR_OOM, "host allocation failed");
  sys->ctx = ctx;
  sys->kind = kind;
  sys->m = m;
  sys->n = n;
  sys->lda = lda;
  sys->A = A_dev;
  sys->b = b_dev;
  kpp_status stt;
  if ((stt = dev_alloc(&sys->mom, n)) < 0 || (stt = dev_alloc(&sys->ds, 1)) < 0 ||
      (stt = dev_alloc(&sys->y, kpp::kMaxBlock)) < 0 || (stt = dev_alloc(&sys->rowsq, m)) < 0 ||
      (stt = dev_alloc(&sys->scal, 4)) < 0 || (stt = dev_alloc(&sys->err, 4)) < 0 ||
      (stt = dev_alloc(&sys->part, 2 * static_cast<size_t>(kpp::kFusedMaxGroups) * kpp::kFusedMaxBlock)) < 0 ||
      (stt = dev_alloc(&sys->flags, kFlagWords)) < 0) {
    destroy_buffers(sys.get());
    return stt;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&sys->h_ds), sizeof(kpp::DevState), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&sys->h_err), sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
    destroy_buffers(sys.get());
    return fail(KPP_ERR_OOM, "pinned host allocation failed");
  }
  for (auto& e : sys->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      destroy_buffers(sys.get());
      return fail(KPP_ERR_HIP, "hipEventCreate failed");
    }
  }
  for (auto& pair : sys->ev_fact)
    for (auto& e : pair)
      if (hipEventCreate(&e) != hipSuccess) {
        destroy_buffers(sys.get());
        return fail(KPP_ERR_HIP, "hipEventCreate failed");
      }
  hipStream_t st = ctx->stream;
  HIP_TRY(hipMemsetAsync(sys->flags, 0, kFlagWords * sizeof(uint32_t), st));
  // finiteness of A and b, and ||b||
  HIP_TRY(hipMemsetAsync(sys->err, 0, sizeof(int32_t), st));
  kpp::launch_check_finite(A_dev, lda, m, n, b_dev, sys->err, st);
  HIP_TRY(hipGetLastError());
  int32_t bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, sys->err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (bad) {
    destroy_buffers(sys.get());
    return fail(KPP_ERR_NONFINITE, "A or b holds NaN or Inf");
  }
  std::vector<double> hb(m);
  HIP_TRY(hipMemcpyAsync(hb.data(), b_dev, m * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double bb = 0.0;
  for (double v : hb) bb += v * v;
  sys->bnorm = std::sqrt(bb);
  *out = sys.release();
  return KPP_OK;
}

KPP_API kpp_status kpp_system_destroy(kpp_system* sys) {
  if (!sys) return KPP_OK;
  if (sys->ctx) (void)hipSetDevice(sys->ctx->device);
  if (sys->ctx) (void)hipStreamSynchronize(sys->ctx->stream);
  destroy_buffers(sys);
  delete sys;
  return KPP_OK;
}

KPP_API kpp_status kpp_solve(kpp_system* sys, const kpp_params* p, double* x_dev, kpp_result* res) {
  if (!sys || !x_dev) return fail(KPP_ERR_INVALID_ARG, "NULL system or x");
  if (res) std::memset(res, 0, sizeof(*res));
  KPP_TRY(check_params(sys, p));
  HIP_TRY(hipSetDevice(sys->ctx->device));
  try {
    if (p->precision == KPP_MIXED_FP32) return solve_mixed(sys, p, x_dev, res);
    return solve_fp64(sys, p, x_dev, res);
  } catch (const std::bad_alloc&) {
    return fail(KPP_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(KPP_ERR_INVALID_ARG, "%s", e.what());
  }
}

KPP_API kpp_status kpp_schedule_generate(int32_t kind, int64_t m, int64_t n, const kpp_params* p,
                                         int64_t T, int32_t* step_block_host,
                                         int32_t* block_rows_host, int32_t* block_len_host,
                                         int32_t blocks_cap, int32_t* num_blocks_out) {
  if (!p || T < 0 || (T > 0 && !step_block_host) || !num_blocks_out)
    return fail(KPP_ERR_INVALID_ARG, "bad arguments");
  if (kind != KPP_KACZMARZ && kind != KPP_CD_PSD) return fail(KPP_ERR_INVALID_ARG, "unknown kind");
  const int64_t N = kind == KPP_CD_PSD ? n : m;
  const int32_t s = p->block_size;
  try {
    kpp::BlockSchedule sch(static_cast<kpp::MemoMode>(p->memo), N, s, p->seed,
                           kpp::online_rate(kind, m, n, s), p->num_blocks, p->fixed_partition != 0);
    for (int64_t t = 0; t < T; ++t) step_block_host[t] = sch.next(nullptr);
    const int32_t nb = sch.num_blocks();
    *num_blocks_out = nb;
    if (nb > blocks_cap) return fail(KPP_ERR_INVALID_ARG, "blocks_cap %d < %d blocks", blocks_cap, nb);
    for (int32_t b = 0; b < nb; ++b) {
      if (block_len_host) block_len_host[b] = sch.len(b);
      if (block_rows_host)
        for (int32_t i = 0; i < s; ++i) block_rows_host[static_cast<size_t>(b) * s + i] = i < sch.len(b) ? sch.rows(b)[i] : -1;
    }
  } catch (const std::exception& e) {
    return fail(KPP_ERR_INVALID_ARG, "%s", e.what());
  }
  return KPP_OK;
}

KPP_API kpp_status kpp_block_factor(kpp_system* sys, int32_t s, double lambda, int32_t nb,
                                    const int32_t* rows_host, const int32_t* len_host, double* L_dev) {
  if (!sys || !rows_host || !len_host || !L_dev || nb < 0) return fail(KPP_ERR_INVALID_ARG, "bad arguments");
  const int64_t N = sys->kind == KPP_CD_PSD ? sys->n : sys->m;
  if (s < 1 || s > kpp::kMaxBlock) return fail(KPP_ERR_INVALID_ARG, "block size %d out of range", s);
  if (!(lambda >= 0.0)) return fail(KPP_ERR_INVALID_ARG, "lambda must be >= 0");
  for (int32_t b = 0; b < nb; ++b) {
    if (len_host[b] < 1 || len_host[b] > s) return fail(KPP_ERR_INVALID_ARG, "block %d length %d", b, len_host[b]);
    for (int32_t i = 0; i < len_host[b]; ++i) {
      const int32_t r = rows_host[static_cast<size_t>(b) * s + i];
      if (r < 0 || r >= N) return fail(KPP_ERR_INVALID_ARG, "block %d row %d out of range", b, r);
    }
  }
  if (nb == 0) return KPP_OK;
  HIP_TRY(hipSetDevice(sys->ctx->device));
  hipStream_t st = sys->ctx->stream;
  int32_t *d_rows = nullptr, *d_lens = nullptr, *d_ids = nullptr;
  KPP_TRY(dev_alloc(&d_rows, static_cast<size_t>(nb) * s));
  KPP_TRY(dev_alloc(&d_lens, nb));
  KPP_TRY(dev_alloc(&d_ids, nb));
  std::vector<int32_t> ids(nb);
  for (int32_t b = 0; b < nb; ++b) ids[b] = b;
  HIP_TRY(hipMemcpyAsync(d_rows, rows_host, static_cast<size_t>(nb) * s * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_lens, len_host, nb * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_ids, ids.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(sys->err, 0, sizeof(int32_t), st));
  HIP_TRY(hipMemsetAsync(L_dev, 0, static_cast<size_t>(nb) * s * s * sizeof(double), st));
  if (sys->kind == KPP_KACZMARZ) KPP_TRY(ensure_gram_ws(sys, 0, kpp::gram_syrk_work(s, sys->n, nb)));
  kpp::launch_gram(sys->kind, sys->A, sys->lda, sys->n, d_rows, d_lens, s, nb, lambda, L_dev,
                   static_cast<int64_t>(s) * s, d_ids, sys->gram_ws[0], st);
  HIP_TRY(hipGetLastError());
  if (s <= kpp::kFactorSmallMax)
    kpp::launch_factor_small(L_dev, static_cast<int64_t>(s) * s, s, d_lens, nb, d_ids, 0, sys->err, st);
  else
    kpp::launch_cholesky(L_dev, s, static_cast<int64_t>(s) * s, d_lens, nb, d_ids, sys->err, st);
  HIP_TRY(hipGetLastError());
  int32_t herr = 0;
  HIP_TRY(hipMemcpyAsync(&herr, sys->err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  dev_free(d_rows);
  dev_free(d_lens);
  dev_free(d_ids);
  if (herr) return fail(KPP_ERR_NOT_SPD, "a regularized block Gram has no Cholesky factor");
  return KPP_OK;
}

KPP_API kpp_status kpp_residual_norm(kpp_system* sys, const double* x_dev, double* out_host) {
  if (!sys || !x_dev || !out_host) return fail(KPP_ERR_INVALID_ARG, "bad arguments");
  HIP_TRY(hipSetDevice(sys->ctx->device));
  return residual_norm(sys, x_dev, out_host);
}

}  // extern "C"
