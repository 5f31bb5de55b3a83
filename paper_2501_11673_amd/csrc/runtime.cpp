// Host runtime behind the C ABI (include/kpp.h): contexts, systems, the memo
// cache of block factors and the solver loop (Algorithms 2 and 5 of the paper,
// exact memoized Cholesky projection).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <stdexcept>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"
#include "lsqr.hpp"
#include "multi.hpp"
#include "kpp.h"
#include "schedule.hpp"
#include "sparse.hpp"

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

// The locals of these macros have names no caller uses (a caller's variable
// of the same name inside `expr` would otherwise be the macro's own local).
#define HIP_TRY(expr)                                                                             \
  do {                                                                                            \
    hipError_t hip_try_err_ = (expr);                                                             \
    if (hip_try_err_ != hipSuccess)                                                               \
      return fail(hip_try_err_ == hipErrorOutOfMemory ? KPP_ERR_OOM : KPP_ERR_HIP, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(hip_try_err_), __FILE__, __LINE__);                    \
  } while (0)

#define KPP_TRY(expr)                          \
  do {                                         \
    kpp_status kpp_try_status_ = (expr);       \
    if (kpp_try_status_ < 0) return kpp_try_status_; \
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
  // workgroups of k_fused<kind, cpl, precision> per compute unit
  // ([kind][fp32][log2 cpl]; -1 = not asked yet)
  // ([kind][precision of A: FP64, FP32, BF16][log2 cpl]; -1 = not asked yet)
  int32_t fused_per_cu[2][3][5] = {{{-1, -1, -1, -1, -1}, {-1, -1, -1, -1, -1}, {-1, -1, -1, -1, -1}},
                                   {{-1, -1, -1, -1, -1}, {-1, -1, -1, -1, -1}, {-1, -1, -1, -1, -1}}};
  // device address of this device's no-allocation scratch (noalloc.hip)
  unsigned char* scratch = nullptr;
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
  bool sig_explicit = false;
  // resumable state of the last FP64 kpp_solve, or of kpp_state_import: step
  // counter and checkpoint statistics, the schedule generator, and (on the
  // device, in mom) the momentum
  bool res_valid = false;
  int32_t res_s = 0;
  int64_t res_t = 0;
  kpp::DevState res_ds{};
  std::unique_ptr<kpp::BlockSchedule> res_sch;
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
  // end state of single-team step-kernel launches, written by the kernel
  // (pinned coherent host memory, two of them: launch number q writes
  // h_mirror[q % 2]; d_mirror is the device address)
  kpp::HostMirror* h_mirror = nullptr;
  kpp::HostMirror* d_mirror = nullptr;
  uint32_t mirror_seq = 0;
  // recorded after each step-kernel launch of the window held in staging
  // buffer i; that buffer's next window is uploaded after it
  hipEvent_t ev_win[2] = {nullptr, nullptr};
  // fused engine
  double* part = nullptr;
  uint32_t* flags = nullptr;
  uint32_t epoch = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  uint64_t* phase_ticks = nullptr;   // KPP_PHASE_PROFILE=1: fused-engine phase profile
  // mixed precision: FP32 copy of A (leading dimension n), outer residual, correction
  float* A32 = nullptr;
  uint16_t* A16 = nullptr;   // mixed precision with bfloat16 storage: the bfloat16 copy of A
  double* gram_ws[2] = {nullptr, nullptr};   // split-Gram partial tiles, one per staging buffer
  size_t gram_ws_cap[2] = {0, 0};
  double* rvec = nullptr;
  double* dvec = nullptr;
  double* xsave = nullptr;   // mixed precision: the iterate with the lowest true residual so far
  double* gemvt_ws = nullptr;      // partial sums of d = A^T z (wide mixed precision)
  double* zx = nullptr;    // mixed precision, wide Kaczmarz++: duals of the inner iterate and momentum
  double* zm = nullptr;
  int32_t* fp64_count = nullptr;   // blocks refactored in FP64 (mixed precision)
  // mixed precision: every FP32 Gram tried on this system failed the
  // conditioning test, so new blocks go straight to an FP64 Gram and factor
  bool fp32_gram_futile = false;
  int64_t fp64_direct = 0;         // blocks factored that way in the current solve
  int64_t fp32_tried = 0;          // blocks with an FP32 Gram attempt in the current solve
  // randomized Hadamard preprocessing (params.rht): the transformed padded
  // system (its own memo and resume state), the signs and the seed they came
  // from; formed on the first such solve
  kpp_system* rht_inner = nullptr;
  int8_t* rht_signs = nullptr;
  double* rht_A = nullptr;
  double* rht_b = nullptr;
  double* rht_x = nullptr;      // CD++: the transformed iterate
  double* rht_work = nullptr;   // two-pass transforms (R > 4096)
  int64_t rht_R = 0;
  uint64_t rht_seed = 0;
  // LSQR projection (params.projection = 1): per-step state, p = A_S^T z, the
  // partial norms, the sketch's staging and signs, and the sketch rows of the
  // new blocks of each staging buffer
  kpp::LsqrState* lsqr_state = nullptr;
  double* lsqr_p = nullptr;
  double* lsqr_ppart = nullptr;
  double* lsqr_part = nullptr;
  double* lsqr_Xt = nullptr;
  double* lsqr_Y = nullptr;
  double* lsqr_Ahat = nullptr;   // the sketches of up to lsqr_cap_chunk blocks, s x tau each
  int32_t* lsqr_iota = nullptr;   // their row indices in that stack: k s + i
  int8_t* lsqr_signs = nullptr;
  int32_t* lsqr_T[2] = {nullptr, nullptr};
  size_t lsqr_T_cap[2] = {0, 0};
  int64_t lsqr_cap_n = 0, lsqr_cap_N = 0;
  int32_t lsqr_cap_s = 0, lsqr_cap_tau = 0, lsqr_cap_chunk = 0;
  int32_t sig_proj = 0;
  // compressed sparse rows (kpp_system_create_csr): the caller's device
  // arrays (A is NULL), a host copy of the row pointers, the column-compressed
  // copies of the memoized Kaczmarz++ blocks (one arena, each block at a host-
  // assigned offset; nu per slot on the device) and the build workspace of
  // blocks too large for LDS, one per staging buffer
  bool csr = false;
  const int64_t* csr_rp = nullptr;
  const int32_t* csr_ci = nullptr;
  const double* csr_cv = nullptr;
  int64_t nnz = 0;
  std::vector<int64_t> h_rp;
  kpp::CscArena csc{};
  int64_t csc_cap = 0;    // entries of each arena array
  int64_t csc_top = 0;    // memoized blocks: next free entry
  int64_t csc_half = 0;   // no memo: each staging buffer owns half of the arena
  int32_t* csc_nu = nullptr;
  int32_t csc_nu_cap = 0;
  std::vector<int64_t> slot_csc_off;
  std::vector<int32_t> slot_csc_z;
  double* csr_ws[2] = {nullptr, nullptr};
  size_t csr_ws_cap[2] = {0, 0};
  int32_t csr_G = 1;                 // team size of the sparse step kernel (column slices of x)
  int32_t* csr_team = nullptr;       // per-slot team tables
  int32_t csr_team_cap = 0, csr_team_s = 0;
  double* csr_xr = nullptr;          // team exchange: r partials [2][G][s] and y [2][s]
  double* csr_xy = nullptr;
  // per-step coefficients of the deferred momentum form (pinned, device)
  double* h_coef = nullptr;
  double* d_coef = nullptr;
  size_t coef_cap = 0;
};

namespace {

constexpr int kFlagWords = kpp::kFlagWordsAlloc;

void drop_rht(kpp_system* s) {
  if (s->rht_inner) (void)kpp_system_destroy(s->rht_inner);
  s->rht_inner = nullptr;
  dev_free(s->rht_signs);
  dev_free(s->rht_A);
  dev_free(s->rht_b);
  dev_free(s->rht_x);
  dev_free(s->rht_work);
  s->rht_R = 0;
}

void drop_lsqr(kpp_system* s) {
  dev_free(s->lsqr_state);
  dev_free(s->lsqr_p);
  dev_free(s->lsqr_ppart);
  dev_free(s->lsqr_part);
  dev_free(s->lsqr_Xt);
  dev_free(s->lsqr_Y);
  dev_free(s->lsqr_Ahat);
  dev_free(s->lsqr_iota);
  dev_free(s->lsqr_signs);
  for (int i = 0; i < 2; ++i) {
    dev_free(s->lsqr_T[i]);
    s->lsqr_T_cap[i] = 0;
  }
  s->lsqr_cap_n = s->lsqr_cap_N = 0;
  s->lsqr_cap_s = s->lsqr_cap_tau = s->lsqr_cap_chunk = 0;
}

void destroy_buffers(kpp_system* s) {
  drop_rht(s);
  drop_lsqr(s);
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
  dev_free(s->A16);
  for (int i = 0; i < 2; ++i) {
    dev_free(s->gram_ws[i]);
    s->gram_ws_cap[i] = 0;
  }
  dev_free(s->rvec);
  dev_free(s->dvec);
  dev_free(s->xsave);
  dev_free(s->gemvt_ws);
  dev_free(s->zx);
  dev_free(s->zm);
  dev_free(s->fp64_count);
  dev_free(s->csc.val);
  dev_free(s->csc.row);
  dev_free(s->csc.col);
  dev_free(s->csc.ptr);
  dev_free(s->csc_nu);
  dev_free(s->csr_team);
  dev_free(s->csr_xr);
  dev_free(s->csr_xy);
  s->csr_team_cap = s->csr_team_s = 0;
  dev_free(s->d_coef);
  if (s->h_coef) (void)hipHostFree(s->h_coef);
  s->h_coef = nullptr;
  s->coef_cap = 0;
  s->csc_cap = s->csc_top = s->csc_half = 0;
  s->csc_nu_cap = 0;
  for (int i = 0; i < 2; ++i) {
    dev_free(s->csr_ws[i]);
    s->csr_ws_cap[i] = 0;
  }
  if (s->h_ds) (void)hipHostFree(s->h_ds);
  if (s->h_err) (void)hipHostFree(s->h_err);
  if (s->h_mirror) (void)hipHostFree(s->h_mirror);
  s->h_ds = nullptr;
  s->h_err = nullptr;
  s->h_mirror = nullptr;
  s->d_mirror = nullptr;
  for (auto& e : s->ev)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
  for (auto& e : s->ev_win)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
  s->cap_slots = 0;
}

// Wait for this system's work on the side stream (memo-miss factorizations):
// the stream runs in order, so the last event recorded for each staging
// buffer covers everything the system enqueued there.  Other systems' work on
// the shared side stream is not waited for.
kpp_status wait_side_work(kpp_system* sys) {
  HIP_TRY(hipEventSynchronize(sys->ev_fact[0][1]));
  HIP_TRY(hipEventSynchronize(sys->ev_fact[1][1]));
  return KPP_OK;
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
  if (sys->cap_slots > 0) {
    HIP_TRY(hipStreamSynchronize(st));
    KPP_TRY(wait_side_work(sys));
  }
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
  if (sys->stage_cap[idx] > 0) {
    HIP_TRY(hipStreamSynchronize(sys->ctx->stream));
    KPP_TRY(wait_side_work(sys));
  }
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
  if (sys->gram_ws_cap[idx] > 0) {
    HIP_TRY(hipStreamSynchronize(sys->ctx->stream));
    KPP_TRY(wait_side_work(sys));
  }
  dev_free(sys->gram_ws[idx]);
  sys->gram_ws_cap[idx] = 0;
  KPP_TRY(dev_alloc(&sys->gram_ws[idx], cap));
  sys->gram_ws_cap[idx] = cap;
  return KPP_OK;
}

// Sparse systems: the per-slot team tables for block size s (kept when the
// table grows; a new block size drops them with the slots they belong to).
kpp_status ensure_csr_team(kpp_system* sys, int32_t slots, int32_t s) {
  if (sys->csr_team_s != s) {
    dev_free(sys->csr_team);
    sys->csr_team_cap = 0;
    sys->csr_team_s = s;
  }
  if (slots <= sys->csr_team_cap) return KPP_OK;
  const int32_t cap = std::max<int32_t>(slots, std::max<int32_t>(16, 2 * sys->csr_team_cap));
  const size_t per = static_cast<size_t>(kpp::csr_team_stride(s, sys->csr_G));
  int32_t* t = nullptr;
  KPP_TRY(dev_alloc(&t, per * cap));
  if (sys->csr_team_cap > 0) {
    HIP_TRY(hipStreamSynchronize(sys->ctx->stream));
    KPP_TRY(wait_side_work(sys));
    HIP_TRY(hipMemcpy(t, sys->csr_team, per * sys->csr_team_cap * sizeof(int32_t), hipMemcpyDeviceToDevice));
  }
  dev_free(sys->csr_team);
  sys->csr_team = t;
  sys->csr_team_cap = cap;
  return KPP_OK;
}

// Sparse systems: the per-slot column counts of the Kaczmarz++ blocks (kept
// when the table grows).
kpp_status ensure_csc_nu(kpp_system* sys, int32_t slots) {
  if (slots <= sys->csc_nu_cap) return KPP_OK;
  const int32_t cap = std::max<int32_t>(slots, std::max<int32_t>(16, 2 * sys->csc_nu_cap));
  int32_t* nu = nullptr;
  KPP_TRY(dev_alloc(&nu, cap));
  if (sys->csc_nu_cap > 0) {
    HIP_TRY(hipStreamSynchronize(sys->ctx->stream));
    KPP_TRY(wait_side_work(sys));
    HIP_TRY(hipMemcpy(nu, sys->csc_nu, sys->csc_nu_cap * sizeof(int32_t), hipMemcpyDeviceToDevice));
  }
  dev_free(sys->csc_nu);
  sys->csc_nu = nu;
  sys->csc_nu_cap = cap;
  return KPP_OK;
}

// Sparse systems: grow the column-compressed arena to `need` entries per
// array, keeping the first `keep` (memoized blocks).  Kernels in flight on
// either stream may read the old arena, so both are drained first.
kpp_status ensure_csc(kpp_system* sys, int64_t need, int64_t keep) {
  if (need <= sys->csc_cap) return KPP_OK;
  const int64_t cap = std::max<int64_t>(need, std::max<int64_t>(int64_t{1} << 16, 2 * sys->csc_cap));
  HIP_TRY(hipStreamSynchronize(sys->ctx->stream));
  KPP_TRY(wait_side_work(sys));
  kpp::CscArena a;
  kpp_status stt;
  if ((stt = dev_alloc(&a.val, cap)) < 0 || (stt = dev_alloc(&a.row, cap)) < 0 || (stt = dev_alloc(&a.col, cap)) < 0 ||
      (stt = dev_alloc(&a.ptr, cap)) < 0) {
    dev_free(a.val);
    dev_free(a.row);
    dev_free(a.col);
    dev_free(a.ptr);
    return stt;
  }
  if (keep > 0) {
    HIP_TRY(hipMemcpy(a.val, sys->csc.val, keep * sizeof(double), hipMemcpyDeviceToDevice));
    HIP_TRY(hipMemcpy(a.row, sys->csc.row, keep * sizeof(int32_t), hipMemcpyDeviceToDevice));
    HIP_TRY(hipMemcpy(a.col, sys->csc.col, keep * sizeof(int32_t), hipMemcpyDeviceToDevice));
    HIP_TRY(hipMemcpy(a.ptr, sys->csc.ptr, keep * sizeof(int32_t), hipMemcpyDeviceToDevice));
  }
  dev_free(sys->csc.val);
  dev_free(sys->csc.row);
  dev_free(sys->csc.col);
  dev_free(sys->csc.ptr);
  sys->csc = a;
  sys->csc_cap = cap;
  return KPP_OK;
}

// Sparse systems: global workspace of the block build for staging buffer idx.
kpp_status ensure_csr_ws(kpp_system* sys, int idx, size_t doubles) {
  if (doubles <= sys->csr_ws_cap[idx]) return KPP_OK;
  const size_t cap = std::max<size_t>(doubles, sys->csr_ws_cap[idx] * 2);
  if (sys->csr_ws_cap[idx] > 0) {
    HIP_TRY(hipStreamSynchronize(sys->ctx->stream));
    KPP_TRY(wait_side_work(sys));
  }
  dev_free(sys->csr_ws[idx]);
  sys->csr_ws_cap[idx] = 0;
  KPP_TRY(dev_alloc(&sys->csr_ws[idx], cap));
  sys->csr_ws_cap[idx] = cap;
  return KPP_OK;
}

// Sparse systems: the per-step coefficient table (no launch reading the old
// one is in flight: every window is waited for before the next is launched).
kpp_status ensure_coef(kpp_system* sys, size_t doubles) {
  if (doubles <= sys->coef_cap) return KPP_OK;
  const size_t cap = std::max<size_t>(doubles, std::max<size_t>(3 * 1024, 2 * sys->coef_cap));
  HIP_TRY(hipStreamSynchronize(sys->ctx->stream));
  dev_free(sys->d_coef);
  if (sys->h_coef) (void)hipHostFree(sys->h_coef);
  sys->h_coef = nullptr;
  sys->coef_cap = 0;
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&sys->h_coef), cap * sizeof(double), hipHostMallocDefault));
  KPP_TRY(dev_alloc(&sys->d_coef, cap));
  sys->coef_cap = cap;
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
  if (p->precision != KPP_FP64 && p->precision != KPP_MIXED_FP32 && p->precision != KPP_MIXED_BF16)
    return fail(KPP_ERR_INVALID_ARG, "unknown precision %d", p->precision);
  if (p->precision != KPP_FP64) {
    if (p->engine == 1) return fail(KPP_ERR_INVALID_ARG, "mixed precision runs on the fused engine");
    if (p->block_size > kpp::kFusedMaxBlock)
      return fail(KPP_ERR_INVALID_ARG, "mixed precision takes block_size <= %d", kpp::kFusedMaxBlock);
    if (!(p->inner_tol > 0.0 && p->inner_tol < 1.0)) return fail(KPP_ERR_INVALID_ARG, "inner_tol must be in (0, 1)");
    if (p->refine_max_rounds < 1) return fail(KPP_ERR_INVALID_ARG, "refine_max_rounds must be >= 1");
  }
  if (p->engine < 0 || p->engine > 2) return fail(KPP_ERR_INVALID_ARG, "unknown engine %d", p->engine);
  if (p->engine == 2 && p->block_size > kpp::kFusedMaxBlock && !sys->csr)
    return fail(KPP_ERR_INVALID_ARG, "the fused engine takes block_size <= %d", kpp::kFusedMaxBlock);
  if (p->team_groups < 0 || p->team_groups > kpp::kFusedMaxGroups)
    return fail(KPP_ERR_INVALID_ARG, "team_groups must be in [0, %d]", kpp::kFusedMaxGroups);
  if (p->resume && p->precision != KPP_FP64) return fail(KPP_ERR_INVALID_ARG, "resume runs in FP64 only");
  if (p->rht != 0 && p->rht != 1) return fail(KPP_ERR_INVALID_ARG, "rht must be 0 or 1");
  if (p->projection != 0 && p->projection != 1) return fail(KPP_ERR_INVALID_ARG, "projection must be 0 or 1");
  if (p->projection == 1) {
    if (sys->kind != KPP_KACZMARZ) return fail(KPP_ERR_INVALID_ARG, "the LSQR projection is for Kaczmarz++");
    if (p->precision != KPP_FP64) return fail(KPP_ERR_INVALID_ARG, "the LSQR projection runs in FP64 only");
    if (p->engine == 2) return fail(KPP_ERR_INVALID_ARG, "the LSQR projection runs on the launch-per-phase engine");
    if (p->resume) return fail(KPP_ERR_INVALID_ARG, "resume does not combine with the LSQR projection");
    if (p->lsqr_iters < 1 || p->lsqr_iters > 256) return fail(KPP_ERR_INVALID_ARG, "lsqr_iters must be in [1, 256]");
    if (p->sketch_size < 0) return fail(KPP_ERR_INVALID_ARG, "sketch_size must be >= 0");
    int64_t N = 1;
    while (N < sys->n) N <<= 1;
    if (N > kpp::kFhtMaxRows) return fail(KPP_ERR_SHAPE, "n is too large for the sketch's Hadamard transform");
  }
  if (p->rht && p->resume) return fail(KPP_ERR_INVALID_ARG, "resume does not combine with rht");
  if (sys->csr) {
    // the sparse step runs in FP64 (engine 1: a launch per phase; otherwise
    // the team kernel), without the Hadamard preprocessing (it would
    // densify A) or the sketched projection
    if (p->precision != KPP_FP64) return fail(KPP_ERR_INVALID_ARG, "a sparse system solves in FP64 only");
    if (p->rht) return fail(KPP_ERR_INVALID_ARG, "the Hadamard preprocessing does not apply to a sparse system");
    if (p->projection != 0) return fail(KPP_ERR_INVALID_ARG, "a sparse system takes the exact projection only");
  }
  if (p->schedule) {
    if (p->schedule_len < 0) return fail(KPP_ERR_INVALID_ARG, "schedule_len must be >= 0");
    if (!p->block_rows || p->block_rows_count < 1)
      return fail(KPP_ERR_INVALID_ARG, "an explicit schedule needs block_rows and block_rows_count >= 1");
    if (p->precision != KPP_FP64) return fail(KPP_ERR_INVALID_ARG, "an explicit schedule runs in FP64 only");
  }
  return KPP_OK;
}

double default_eta(int32_t kind, int64_t m, int64_t n, int32_t s) {
  if (kind == KPP_CD_PSD) return s / (2.0 * static_cast<double>(n));
  return s / (2.0 * static_cast<double>(std::min(m, n)));
}

kpp_status residual_norm(kpp_system* sys, const double* x, double* out) {
  hipStream_t st = sys->ctx->stream;
  if (sys->csr)
    kpp::launch_csr_residual_sq(sys->csr_rp, sys->csr_ci, sys->csr_cv, sys->b, sys->m, x, sys->rowsq, sys->scal, st);
  else
    kpp::launch_residual_sq(sys->A, sys->lda, sys->m, sys->n, x, sys->b, sys->rowsq, 0, sys->scal, st);
  HIP_TRY(hipGetLastError());
  double v = 0.0;
  HIP_TRY(hipMemcpyAsync(&v, sys->scal, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *out = std::sqrt(v);
  return KPP_OK;
}

// Fused-engine geometry: columns per lane (cpl) and workgroups per step.  A
// lane holds 64 FP64 tile entries, or 128 FP32 ones when cpl >= 4; the four
// waves of a workgroup hold 4 * entries / cpl block rows, which must cover s.
int32_t fused_tile_elems(bool fp32, int32_t cpl) { return (fp32 && cpl >= 4) ? 128 : 64; }

bool fused_cpl_fits(int32_t s, bool fp32, int32_t cpl) {
  return s <= kpp::kFusedMaxBlock && 4 * fused_tile_elems(fp32, cpl) / cpl >= s;
}

int32_t fused_cpl_max(int32_t s, bool fp32) {
  int32_t c = 1;
  while (c < 16 && fused_cpl_fits(s, fp32, 2 * c)) c *= 2;
  return c;
}

// The smallest cpl that brings the team down to the target size (default 32
// workgroups: a step is bound by the load rate of each compute unit as much as
// by the exchange between workgroups, and 32 was the fastest at n = 4096).
bool fused_geometry(int64_t n, int32_t s, int32_t target_groups, bool fp32, int32_t* cpl, int32_t* groups) {
  if (s > kpp::kFusedMaxBlock) return false;
  const int32_t gmax = target_groups > 0 ? target_groups : 32;
  const int32_t cmax = fused_cpl_max(s, fp32);
  int32_t c = 1;
  while (c < cmax && (n + 64 * c - 1) / (64 * c) > gmax) c *= 2;
  const int64_t g = (n + 64 * c - 1) / (64 * c);
  if (g > kpp::kFusedMaxGroups) return false;
  *cpl = c;
  *groups = static_cast<int32_t>(g);
  return true;
}

// Workgroups of the step kernel that can be resident on the context's device
// at once.
int64_t fused_resident_groups(kpp_context* ctx, int32_t kind, int32_t prec, int32_t cpl) {
  int lc = 0;
  while ((1 << lc) < cpl && lc < 4) ++lc;
  int32_t& per = ctx->fused_per_cu[kind == KPP_CD_PSD ? 1 : 0][prec][lc];
  if (per < 0) {
    (void)hipSetDevice(ctx->device);
    per = kpp::fused_blocks_per_cu(kind == KPP_CD_PSD ? 1 : 0, prec, cpl);
  }
  return static_cast<int64_t>(per) * std::max(ctx->cu_count, 0);
}

// The matrix and right-hand side one run of the block iteration works on: the
// caller's FP64 system, or (mixed precision) the FP32 copy of A with the
// current outer residual as right-hand side.
struct Source {
  const double* A64 = nullptr;
  const float* A32 = nullptr;
  const uint16_t* A16 = nullptr;   // bfloat16 storage (then A32 is null)
  int64_t lda = 0;
  const double* b = nullptr;
  double bnorm = 0.0;
};

struct CoreOpts {
  double tol = 0.0;
  int32_t confirm = 1;      // confirm a candidate stop with ||A x - b|| (FP64 system only)
  double rho0 = 0.0;
  int32_t keep_memo = 0;
  int64_t max_iters = 0;       // steps in this run (after the resumed ones)
  bool resume = false;         // continue the system's saved state
  bool keep_state = false;     // save this run's state on the system at its end
  // end the run when the window residual estimate E1 has not fallen below
  // kStallRatio times its value kStallWindows window ends earlier (an inner
  // low-precision solve at its precision floor); 0 = never
  int32_t stop_on_stall = 0;
  // time each step-kernel launch with a pair of HIP events (kernel seconds)
  bool time_launches = true;
  // leave Grams and factors enqueued ahead on the side stream in flight when
  // the run ends (a run that follows on the same system orders its first
  // step after them through its own first window's factor event; the caller
  // waits for them before it returns)
  bool defer_side_wait = false;
  // duals of the iterate and momentum (m entries each, zero on entry), kept
  // by the fused engine for Kaczmarz++ when every workgroup's share of the m
  // rows fits its registers; CoreStats::dual says whether they were
  double* zx = nullptr;
  double* zm = nullptr;
};

// host seconds spent in window planning, split for the serving profile
// (KPP_SERVE_PROFILE): buffer growth, schedule and slots, factor enqueue
thread_local double t_prof_grow = 0.0, t_prof_sched = 0.0, t_prof_enqueue = 0.0, t_prof_slots = 0.0;
thread_local int64_t n_prof_slot_growth = 0;

double wall_now() {
  using clock = std::chrono::steady_clock;
  return std::chrono::duration<double>(clock::now().time_since_epoch()).count();
}

constexpr int kStallWindows = 12;
constexpr int64_t kDualRowsPerGroup = 1024;   // 4 rows per thread in the step kernel
constexpr double kStallRatio = 0.9;
// Kaczmarz++ blocks of at least this many rows split y = G^{-1} r across the
// team: forming all of y reads the whole s x s inverse in every workgroup
// (512 KB per workgroup per step at s = 256), one more exchange costs less
constexpr int32_t kYSplitMinBlock = 128;
// Kaczmarz++ teams of at least this many workgroups exchange r in two levels
// (row owners, then an all-gather of r): gathering every workgroup's partials
// in every workgroup reads G s doubles per workgroup per step (64 MB per step
// for 256 workgroups of 128-row blocks)
constexpr int32_t kTwoLevelMinGroups = 128;
// most sketches of the LSQR projection stacked for one batched factoring
constexpr int64_t kSketchBatch = 256;

struct CoreStats {
  int64_t iters = 0, hits = 0, misses = 0, launches = 0;
  bool converged = false;
  double true_rel = NAN, t_factor = 0.0, t_kernel = 0.0;
  kpp::DevState hs{};
  int32_t engine = 0;
  int32_t groups = 0, cpl = 0;   // fused geometry (0 for the launch-per-phase engine)
  bool dual = false;
  // sparse systems: nonzeros of the stepped blocks, gathered iterate entries
  // (one or two vectors a nonzero), folds of the deferred momentum form
  double csr_nnz = 0.0, csr_gathers = 0.0, csr_miss_nnz = 0.0;
  int64_t csr_folds = 0;
};

// One run of the block iteration (Algorithm 2 / Algorithm 5 with the exact
// memoized projection), advanced launch by launch: kpp_solve drives a run to
// its end on its own, the server advances many runs in shared launches.
//
// A window is the run of steps up to the `periods`-th next checkpoint.
// Planning a window draws its blocks, assigns memo slots and stages (pinned)
// the rows of its new blocks plus the slot of every step; its memo misses are
// then factored on the side stream while the previous window runs on the main
// stream.  With stop_on_cand a launch ends at a checkpoint whose stop test
// passes, and the rest of the window follows if the true residual does not
// confirm the stop; the iterates are the same as with one checkpoint per
// window.
class CoreRun {
 public:
  ~CoreRun() { drain(); }

  kpp_status begin(kpp_system* sys, const kpp_params* p, const Source& src, const CoreOpts& o, double* x,
                   int32_t periods, int32_t force_cpl) {
    sys_ = sys;
    prm_ = *p;
    src_ = src;
    o_ = o;
    x_ = x;
    st_ = sys->ctx->stream;
    side_ = sys->ctx->side;
    bf16_ = src.A16 != nullptr;
    fp32_ = src.A32 != nullptr || bf16_;
    kind_ = sys->kind;
    m_ = sys->m;
    n_ = sys->n;
    N_ = kind_ == KPP_CD_PSD ? n_ : m_;
    s_ = p->block_size;
    zeta_ = static_cast<int32_t>((N_ + s_ - 1) / s_);
    period_ = 2 * static_cast<int64_t>(zeta_);
    periods_ = std::max<int32_t>(1, periods);
    eta_ = p->eta < 0.0 ? default_eta(kind_, m_, n_, s_) : p->eta;
    if (!p->accel) eta_ = 0.0;
    csr_ = sys->csr;
    csr_window_ = csr_ && p->engine != 1;
    rho_now_ = o.rho0;
    mode_ = static_cast<kpp::MemoMode>(p->memo);
    max_iters_ = o.max_iters;
    const double B0 = kpp::online_rate(kind_, m_, n_, s_);
    try {
      if (p->schedule) {
        sch_.reset(new kpp::BlockSchedule(N_, s_, p->block_rows, p->block_rows_count, p->schedule, p->schedule_len));
        mode_ = kpp::MemoMode::Fixed;
        max_iters_ = std::min(max_iters_, p->schedule_len);
      } else {
        sch_.reset(new kpp::BlockSchedule(mode_, N_, s_, p->seed, B0, p->num_blocks, p->fixed_partition != 0));
      }
    } catch (const std::exception& e) {
      return fail(KPP_ERR_INVALID_ARG, "%s", e.what());
    }
    if (o.resume) {
      if (!sys->res_valid || !sys->res_sch || sys->res_s != s_)
        return fail(KPP_ERR_INVALID_ARG, "no saved state of a solve with block size %d to resume", s_);
      sch_ = std::move(sys->res_sch);
      sys->res_valid = false;
      mode_ = sch_->mode();
      t_ = t_start_ = sys->res_t;
      max_iters_ = t_ + o.max_iters;
      if (sch_->is_explicit()) max_iters_ = std::min(max_iters_, sch_->length());
      hs_ = sys->res_ds;
      rho_now_ = hs_.rho;
    }
    if (force_cpl > 0) {
      fused_ = fused_cpl_fits(s_, fp32_, force_cpl);
      cpl_ = force_cpl;
      groups_ = static_cast<int32_t>((n_ + 64 * cpl_ - 1) / (64 * cpl_));
      if (groups_ > kpp::kFusedMaxGroups) fused_ = false;
      if (!fused_) return fail(KPP_ERR_INVALID_ARG, "no fused geometry with %d columns per lane", force_cpl);
    } else {
      if (p->engine != 1 && !csr_) fused_ = fused_geometry(n_, s_, p->team_groups, fp32_, &cpl_, &groups_);
      if (p->engine == 2 && !fused_ && !csr_)
        return fail(KPP_ERR_INVALID_ARG, "n=%lld is too wide for the fused engine", (long long)n_);
    }
    // every workgroup of a team waits for the others each step, so the whole
    // team must be resident; otherwise the launch-per-phase engine runs (an
    // explicit request for the fused engine, a team size or the FP32 inner
    // solver, which needs the fused engine, is refused)
    if (fused_ && groups_ > fused_resident_groups(sys->ctx, kind_, prec(), cpl_)) {
      if (p->engine == 2 || p->team_groups > 0 || force_cpl > 0 || fp32_)
        return fail(KPP_ERR_INVALID_ARG, "a team of %d workgroups cannot be resident on this device (%lld)",
                    groups_, static_cast<long long>(fused_resident_groups(sys->ctx, kind_, prec(), cpl_)));
      fused_ = false;
    }
    lsqr_ = p->projection == 1;
    if (lsqr_) {
      fused_ = false;
      KPP_TRY(setup_lsqr(p));
    }
    dual_ = o.zx != nullptr && o.zm != nullptr && kind_ == KPP_KACZMARZ && fused_ && fp32_ && groups_ > 0 &&
            (m_ + groups_ - 1) / groups_ <= kDualRowsPerGroup;
    // memo cache: reuse only for an identical schedule definition.  The slot
    // table and the staging buffers are sized for the whole run before any
    // slot is handed out: growing them later waits for the device (a freed
    // buffer may still be read).  An online collection holds about
    // B0 (1 + ln(T / B0)) blocks after T steps (Section 5.2); 4 B0 covers
    // T up to ~20 B0, and the table still grows past that if needed.
    int64_t est_blocks = 16;
    if (mode_ == kpp::MemoMode::Fixed) est_blocks = sch_->num_blocks();
    if (mode_ == kpp::MemoMode::Online)
      est_blocks = std::min<int64_t>(static_cast<int64_t>(4.0 * B0) + 16, std::max<int64_t>(16, max_iters_ + 1));
    if (mode_ == kpp::MemoMode::Off) est_blocks = 2 * periods_ * period_;
    KPP_TRY(ensure_slots(sys, static_cast<int32_t>(std::min<int64_t>(est_blocks, 1 << 24)), s_));
    {
      const size_t stage = static_cast<size_t>(periods_ * period_) * (s_ + 4) + 16;
      KPP_TRY(ensure_stage(sys, 0, stage));
      KPP_TRY(ensure_stage(sys, 1, stage));
    }
    const bool same_sig = sys->memo_valid && (o.keep_memo || o.resume) && sys->sig_s == s_ && sys->sig_memo == p->memo &&
                          sys->sig_nb == p->num_blocks && sys->sig_part == p->fixed_partition &&
                          sys->sig_seed == p->seed && sys->sig_lambda == p->lambda &&
                          sys->sig_prec == prec() && mode_ != kpp::MemoMode::Off &&
                          !sch_->is_explicit() && !sys->sig_explicit && !lsqr_ && sys->sig_proj == 0;
    if (!same_sig) {
      sys->slot_of_block.clear();
      sys->used_slots = 0;
      sys->memo_valid = mode_ != kpp::MemoMode::Off;
      sys->sig_s = s_;
      sys->sig_memo = p->memo;
      sys->sig_nb = p->num_blocks;
      sys->sig_part = p->fixed_partition;
      sys->sig_seed = p->seed;
      sys->sig_lambda = p->lambda;
      sys->sig_prec = prec();
      sys->sig_explicit = sch_->is_explicit();
      sys->sig_proj = lsqr_ ? 1 : 0;
      sys->csc_top = 0;
    }
    if (csr_ && kind_ == KPP_KACZMARZ) KPP_TRY(ensure_csc_nu(sys, sys->cap_slots));
    if (csr_) KPP_TRY(ensure_csr_team(sys, sys->cap_slots, s_));
    // launch engine: column chunks of the block gemv
    P_ = csr_ ? 1 : static_cast<int32_t>((n_ + kChunk - 1) / kChunk);
    if (!fused_ && static_cast<int64_t>(s_) * P_ > sys->rpart_cap) {
      dev_free(sys->rpart);
      KPP_TRY(dev_alloc(&sys->rpart, static_cast<size_t>(s_) * P_));
      sys->rpart_cap = static_cast<int64_t>(s_) * P_;
    }
    const double thr = o.tol * o.tol * src.bnorm * src.bnorm;
    if (o.resume) {
      HIP_TRY(hipMemsetAsync(sys->err, 0, sizeof(int32_t), st_));
      // the momentum is still (or was imported) on the device
      kpp::DevState d = hs_;
      d.thr = thr;
      *sys->h_ds = d;
      HIP_TRY(hipMemcpyAsync(sys->ds, sys->h_ds, sizeof(kpp::DevState), hipMemcpyHostToDevice, st_));
      HIP_TRY(hipStreamSynchronize(st_));
    } else {
      kpp::launch_state_init(sys->ds, o.rho0, thr, sys->err, sys->mom, n_, st_);
    }
    HIP_TRY(hipGetLastError());
    const char* prof_env = std::getenv("KPP_PHASE_PROFILE");
    phase_prof_ = (fused_ || csr_window_) && prof_env && prof_env[0] == '1';
    if (phase_prof_) {
      if (!sys->phase_ticks) KPP_TRY(dev_alloc(&sys->phase_ticks, kpp::kFusedPhases));
      HIP_TRY(hipMemsetAsync(sys->phase_ticks, 0, kpp::kFusedPhases * sizeof(uint64_t), st_));
    }
    // the side stream's first work must follow this run's initialisation
    HIP_TRY(hipEventRecord(sys->ev_fact[1][2], st_));
    HIP_TRY(hipStreamWaitEvent(side_, sys->ev_fact[1][2], 0));
    begun_ = true;
    if (max_iters_ <= t_) {
      finished_ = true;
      return KPP_OK;
    }
    KPP_TRY(plan(win_[0], t_, 0));
    KPP_TRY(enqueue_factor(win_[0], side_));
    win_[0].on_side = true;
    return KPP_OK;
  }

  // Leave this run's state on the system for a later resume (after end()).
  void keep_state() {
    if (!sch_) return;
    sys_->res_valid = true;
    sys_->res_s = s_;
    sys_->res_t = t_;
    sys_->res_ds = hs_;
    sys_->res_sch = std::move(sch_);
  }

  bool finished() const { return finished_; }
  bool dual() const { return dual_; }
  bool fused() const { return fused_; }
  bool fp32() const { return fp32_; }
  int32_t prec() const { return bf16_ ? 2 : (fp32_ ? 1 : 0); }   // storage of A in the step kernel
  int32_t kind() const { return kind_; }
  int32_t cpl() const { return cpl_; }
  int32_t groups() const { return groups_; }
  int64_t steps() const { return t_; }
  bool converged() const { return converged_; }
  const kpp::DevState& state() const { return hs_; }
  void add_kernel_seconds(double sec) { t_kernel_ += sec; }
  void set_stop_on_cand(bool v) { stop_on_cand_ = v; }

  // Order the main stream after the current window's factors and, for the
  // fused engine, fill the step-kernel arguments for the rest of the window.
  kpp_status prepare(kpp::FusedArgs* a) {
    KPP_TRY(order_after_factors(cur_));
    if (!fused_) return KPP_OK;
    if (sys_->epoch > 0x3fffffffu) {
      HIP_TRY(hipMemsetAsync(sys_->flags, 0, kFlagWords * sizeof(uint32_t), st_));
      sys_->epoch = 0;
    }
    fill_args(a, cur_, sys_->epoch);
    return KPP_OK;
  }

  // The main stream waits for window i's factors (nothing to order after
  // factors that have completed already).
  kpp_status order_after_factors(int i) {
    Window& w = win_[i];
    if (w.on_side && !w.waited) {
      const hipError_t q = hipEventQuery(sys_->ev_fact[i][1]);
      if (q == hipErrorNotReady)
        HIP_TRY(hipStreamWaitEvent(st_, sys_->ev_fact[i][1], 0));
      else
        HIP_TRY(q);
      w.waited = true;
    }
    return KPP_OK;
  }

  // Launches enqueued ahead (solve_core): the next window's launch goes to the
  // stream before the current one ends, so that no host round trip separates
  // them.  It runs no step if the current launch ends at a checkpoint whose
  // stop test passes; the host then confirms the stop or launches the window
  // again.  Only single teams whose state comes back through the mirror, full
  // windows (no stop inside a launch), no stall test (it is decided on the
  // host after the launch) and one launch in flight.
  bool can_launch_ahead() const {
    if (!fused_ || csr_ || lsqr_ || !sys_->d_mirror || o_.stop_on_stall || stop_on_cand_) return false;
    if (!have_next_ || planned_ || finished_ || launches_in_flight_.size() != 1) return false;
    const Window& w = win_[cur_];
    const Window& nw = win_[cur_ ^ 1];
    return nw.t0 == w.t0 + w.W && sys_->epoch + static_cast<uint64_t>(w.W - w.done) + static_cast<uint64_t>(nw.W) <=
                                      0x3fffffffu;
  }
  kpp_status prepare_ahead(kpp::FusedArgs* a) {
    KPP_TRY(order_after_factors(cur_ ^ 1));
    const Window& w = win_[cur_];
    fill_args(a, cur_ ^ 1, sys_->epoch + static_cast<uint32_t>(w.W - w.done));
    a->skip_on_cand = 1;
    return KPP_OK;
  }
  int cur_window() const { return cur_; }

  void fill_args(kpp::FusedArgs* a, int wi, uint32_t epoch) {
    const Window& w = win_[wi];
    *a = kpp::FusedArgs{};
    a->A = bf16_ ? static_cast<const void*>(src_.A16)
                 : fp32_ ? static_cast<const void*>(src_.A32) : static_cast<const void*>(src_.A64);
    a->lda = src_.lda;
    a->n = n_;
    a->b = src_.b;
    a->rows = sys_->rows;
    a->lens = sys_->lens;
    a->L = sys_->L;
    a->slot_stride = sys_->slot_stride;
    a->s = s_;
    a->W = static_cast<int32_t>(w.W - w.done);
    a->step_slot = sys_->d_stage[wi] + w.o_step + w.done;
    a->x = x_;
    a->mom = sys_->mom;
    a->part = sys_->part;
    a->flags = sys_->flags;
    a->epoch = epoch;
    a->zeta = zeta_;
    a->adaptive = prm_.adaptive_rho;
    a->eta = eta_;
    a->ds = sys_->ds;
    a->err = sys_->err;
    a->spin_limit = int64_t{1} << 22;
    a->phase_ticks = phase_prof_ ? sys_->phase_ticks : nullptr;
    a->stop_on_cand = stop_on_cand_ ? 1 : 0;
    a->zx = dual_ ? o_.zx : nullptr;
    a->zm = dual_ ? o_.zm : nullptr;
    a->mrows = m_;
    a->ypart = sys_->part + 2 * static_cast<size_t>(kpp::kFusedMaxGroups) * kpp::kFusedMaxBlock;
    a->ysplit = (kind_ == KPP_KACZMARZ && s_ >= kYSplitMinBlock && groups_ >= 4) ? 1 : 0;
    a->xchg2 = (kind_ == KPP_KACZMARZ && s_ <= kpp::kTwoMaxBlock && groups_ >= kTwoLevelMinGroups) ? 1 : 0;
    {
      const size_t esz = bf16_ ? sizeof(uint16_t) : fp32_ ? sizeof(float) : sizeof(double);
      a->vec_rows = (reinterpret_cast<uintptr_t>(a->A) % 16 == 0 && (static_cast<size_t>(a->lda) * esz) % 16 == 0) ? 1 : 0;
    }
  }

  // One launch per phase for the rest of the window (engine 1).
  kpp_status launch_unfused() {
    Window& w = win_[cur_];
    const size_t sd = static_cast<size_t>(sys_->slot_stride);
    if (lsqr_) return launch_lsqr_steps();
    if (csr_) return launch_csr_steps();
    for (int64_t k = w.done; k < w.W; ++k) {
      const int32_t q = w.step_slot[k];
      const int32_t sb = sch_->len(w.step_block[k]);
      const int32_t* rows = sys_->rows + static_cast<size_t>(q) * s_;
      kpp::launch_block_gemv_partial(src_.A64, src_.lda, n_, rows, sb, x_, sys_->rpart, P_, kChunk, st_);
      kpp::launch_block_project(sys_->rpart, P_, src_.b, rows, sb, sys_->L + sd * q + static_cast<size_t>(s_) * s_,
                                s_, sys_->y, sys_->ds, zeta_, prm_.adaptive_rho, st_);
      kpp::launch_update(kind_, src_.A64, src_.lda, n_, rows, sb, sys_->y, sys_->ds, eta_, x_, sys_->mom, st_);
    }
    launches_ += 3 * (w.W - w.done);
    HIP_TRY(hipGetLastError());
    return KPP_OK;
  }

  // Steps with the LSQR projection: r and y = L^{-1} r (the projection kernel
  // with L^{-1} in place of G^{-1}: it also keeps the window sums), LSQR in the
  // block's coordinates, then the update with w = A_S^T z_x.
  kpp_status launch_lsqr_steps() {
    Window& w = win_[cur_];
    kpp_system* sys = sys_;
    const size_t sd = static_cast<size_t>(sys->slot_stride);
    const int32_t G = kpp::lsqr_at_groups(n_);
    kpp::LsqrState* L = sys->lsqr_state;
    const double* zx = reinterpret_cast<const double*>(reinterpret_cast<const char*>(L) + offsetof(kpp::LsqrState, zx));
    for (int64_t k = w.done; k < w.W; ++k) {
      const int32_t q = w.step_slot[k];
      const int32_t sb = sch_->len(w.step_block[k]);
      const int32_t* rows = sys->rows + static_cast<size_t>(q) * s_;
      const double* Li = sys->L + sd * q + static_cast<size_t>(s_) * s_;
      kpp::launch_block_gemv_partial(src_.A64, src_.lda, n_, rows, sb, x_, sys->rpart, P_, kChunk, st_);
      kpp::launch_block_project(sys->rpart, P_, src_.b, rows, sb, Li, s_, sys->y, sys->ds, zeta_, prm_.adaptive_rho,
                                st_);
      kpp::launch_lsqr_start(sys->y, Li, s_, sb, L, st_);
      kpp::launch_lsqr_at(src_.A64, src_.lda, n_, rows, sb, L, sys->lsqr_ppart, sys->lsqr_p, sys->lsqr_part, st_);
      kpp::launch_lsqr_post(sys->lsqr_part, G, sb, prm_.lambda, 1, L, st_);
      for (int32_t it = 0; it < lsqr_iters_; ++it) {
        kpp::launch_block_gemv_partial(src_.A64, src_.lda, n_, rows, sb, sys->lsqr_p, sys->rpart, P_, kChunk, st_);
        kpp::launch_lsqr_mid(sys->rpart, P_, Li, s_, sb, prm_.lambda, L, st_);
        kpp::launch_lsqr_at(src_.A64, src_.lda, n_, rows, sb, L, sys->lsqr_ppart, sys->lsqr_p, sys->lsqr_part, st_);
        kpp::launch_lsqr_post(sys->lsqr_part, G, sb, prm_.lambda, 0, L, st_);
      }
      kpp::launch_update(kind_, src_.A64, src_.lda, n_, rows, sb, zx, sys->ds, eta_, x_, sys->mom, st_);
    }
    launches_ += (7 + 5 * lsqr_iters_) * (w.W - w.done);
    HIP_TRY(hipGetLastError());
    return KPP_OK;
  }

  // Sparse steps: block rows, projection, back-projection on the deferred
  // iterate u + t01 v and momentum t11 v (x_ and the momentum buffer hold u
  // and v).  rho, hence c, is fixed inside a window (its checkpoint is the
  // window's last step and revises rho for the next one), so the host draws
  // up (t01, au, av) for every step.  u, v are folded back into x, m at the
  // window's end and before any step at which 1 / t11 or t01 / t11 would pass
  // kLazyBound: the deferred sums then stay within a factor kLazyBound of the
  // terms they hold.  The steps between folds run in one launch of the team
  // kernel, or (engine 1) three launches per step.
  kpp_status launch_csr_steps() {
    Window& w = win_[cur_];
    kpp_system* sys = sys_;
    const size_t sd = static_cast<size_t>(sys->slot_stride);
    const double c = (1.0 - rho_now_) / (1.0 + rho_now_);
    const int64_t W = w.W - w.done;
    if (W <= 0) return KPP_OK;
    KPP_TRY(ensure_coef(sys, static_cast<size_t>(3 * W)));
    double* cf = sys->h_coef;
    std::vector<int64_t> cut;              // sub-run boundaries (steps before which u, v are folded)
    std::vector<double> fold_at;           // (t01, t11) of each fold
    double t01 = 0.0, t11 = 1.0;
    for (int64_t k = 0; k < W; ++k) {
      if (t11 == 0.0 || 1.0 / t11 > kLazyBound || std::fabs(t01 / t11) > kLazyBound) {
        cut.push_back(k);
        fold_at.push_back(t01);
        fold_at.push_back(t11);
        t01 = 0.0;
        t11 = 1.0;
      }
      cf[3 * k] = t01;
      cf[3 * k + 1] = 1.0 - t01 / t11;
      cf[3 * k + 2] = 1.0 / t11;
      const int32_t z = sys->slot_csc_z[w.step_slot[w.done + k]];
      csr_nnz_ += z;
      csr_gathers_ += (t01 != 0.0 ? 2.0 : 1.0) * z;
      t01 += eta_ * c * t11;
      t11 *= c;
    }
    cut.push_back(W);
    fold_at.push_back(t01);
    fold_at.push_back(t11);
    auto fold = [&](size_t i) {
      const double f01 = fold_at[2 * i], f11 = fold_at[2 * i + 1];
      if (f01 == 0.0 && f11 == 1.0) return;
      kpp::launch_lazy_fold(x_, sys->mom, n_, f01, f11, st_);   // not counted as a step-kernel launch
      ++csr_folds_;
    };
    if (csr_window_) {
      HIP_TRY(hipMemcpyAsync(sys->d_coef, cf, static_cast<size_t>(3 * W) * sizeof(double), hipMemcpyHostToDevice, st_));
      if (sys->epoch > 0x3fffffffu) {
        HIP_TRY(hipMemsetAsync(sys->flags, 0, kFlagWords * sizeof(uint32_t), st_));
        sys->epoch = 0;
      }
      int64_t a0 = 0;
      for (size_t i = 0; i < cut.size(); ++i) {
        const int64_t a1 = cut[i];
        if (a1 > a0) {
          kpp::SparseTeamArgs a;
          a.rp = sys->csr_rp;
          a.ci = sys->csr_ci;
          a.cv = sys->csr_cv;
          a.b = src_.b;
          a.rows = sys->rows;
          a.L = sys->L;
          a.slot_stride = sys->slot_stride;
          a.team = sys->csr_team;
          a.team_stride = kpp::csr_team_stride(s_, sys->csr_G);
          a.step_info = sys->d_stage[cur_] + w.o_sinfo + static_cast<size_t>(kpp::kSparseStepInts) * (w.done + a0);
          a.coef = sys->d_coef + 3 * a0;
          a.ar = sys->csc;
          a.u = x_;
          a.v = sys->mom;
          a.ds = sys->ds;
          a.xr = sys->csr_xr;
          a.xy = sys->csr_xy;
          a.flags = sys->flags;
          a.epoch = sys->epoch;
          a.spin_limit = int64_t{1} << 22;
          a.err = sys->err;
          a.s = s_;
          a.W = static_cast<int32_t>(a1 - a0);
          a.zeta = zeta_;
          a.adaptive = prm_.adaptive_rho;
          a.G = sys->csr_G;
          a.phase_ticks = phase_prof_ ? sys->phase_ticks : nullptr;
          kpp::launch_sparse_team(kind_, a, st_);
          sys->epoch += static_cast<uint32_t>(a1 - a0);
          ++launches_;
        }
        fold(i);
        a0 = a1;
      }
    } else {
      size_t ci = 0;
      for (int64_t k = 0; k < W; ++k) {
        if (k == cut[ci]) fold(ci++);
        const int32_t q = w.step_slot[w.done + k];
        const int32_t sb = sch_->len(w.step_block[w.done + k]);
        const int32_t* rows = sys->rows + static_cast<size_t>(q) * s_;
        kpp::launch_csr_rows_dot(sys->csr_rp, sys->csr_ci, sys->csr_cv, rows, sb, x_, sys->mom, cf[3 * k], sys->rpart,
                                 st_);
        kpp::launch_block_project(sys->rpart, 1, src_.b, rows, sb, sys->L + sd * q + static_cast<size_t>(s_) * s_, s_,
                                  sys->y, sys->ds, zeta_, prm_.adaptive_rho, st_);
        if (kind_ == KPP_KACZMARZ)
          kpp::launch_csc_apply(sys->csc, sys->slot_csc_off[q], sys->slot_csc_z[q], sys->csc_nu, q, sys->y, sb,
                                cf[3 * k + 1], cf[3 * k + 2], x_, sys->mom, st_);
        else
          kpp::launch_rows_apply(rows, sb, sys->y, cf[3 * k + 1], cf[3 * k + 2], x_, sys->mom, st_);
      }
      fold(cut.size() - 1);
      launches_ += 3 * W;
    }
    HIP_TRY(hipGetLastError());
    return KPP_OK;
  }

  void count_fused_launch() { ++launches_; }

  // Single-team fused launches: the kernel writes its end state to the
  // system's host mirror (no copy-back; the host waits on the mirror).
  // Record a launch of window wi that solve_core enqueued: its end state
  // comes back through the host mirror (single fused teams) or by a copy, and
  // the window's staging buffer is free again once the stream passes the
  // event recorded here.
  void mirror_args(kpp::FusedArgs* a) {
    if (!fused_ || csr_ || !sys_->d_mirror) return;
    a->seq = ++sys_->mirror_seq;
    a->mirror = sys_->d_mirror + (a->seq & 1u);
    a->fp64_count = (fp32_ && sys_->fp64_count) ? sys_->fp64_count : nullptr;
  }
  kpp_status note_launch(const kpp::FusedArgs& a, int wi) {
    launches_in_flight_.push_back(Launch{a.mirror != nullptr, a.seq});
    HIP_TRY(hipEventRecord(sys_->ev_win[wi], st_));
    return KPP_OK;
  }

  // After the launch is enqueued: state copy-back, and the next window planned
  // and factored on the side stream while this one runs.
  kpp_status after_launch() {
    if (launches_in_flight_.empty() || !launches_in_flight_.back().mirrored) KPP_TRY(copy_back());
    KPP_TRY(plan_ahead());
    return enqueue_ahead();
  }

  // Wait for the oldest launch's end state: spin on its host mirror (the
  // stream may still be retiring the kernel), else drain the main stream.
  // A stream that went idle without the mirror raised falls back to a copy
  // (an error when a later launch has changed the state since).
  kpp_status wait_launch() {
    if (launches_in_flight_.empty()) {
      HIP_TRY(hipStreamSynchronize(st_));
      return KPP_OK;
    }
    const Launch l = launches_in_flight_.front();
    launches_in_flight_.pop_front();
    if (!l.mirrored) {
      HIP_TRY(hipStreamSynchronize(st_));
      return KPP_OK;
    }
    const kpp::HostMirror* hm = sys_->h_mirror + (l.seq & 1u);
    const volatile uint32_t* seq = &hm->seq;
    for (;;) {
      for (int i = 0; i < 4096; ++i)
        if (*seq == l.seq) {
          std::atomic_thread_fence(std::memory_order_acquire);
          std::memcpy(sys_->h_ds, const_cast<const kpp::DevState*>(&hm->ds), sizeof(kpp::DevState));
          sys_->h_err[0] = hm->err;
          if (fp32_ && sys_->fp64_count) sys_->h_err[1] = hm->fp64_count;
          return KPP_OK;
        }
      const hipError_t q = hipStreamQuery(st_);
      if (q == hipSuccess && *seq != l.seq) {
        if (!launches_in_flight_.empty()) {
          finished_ = true;
          return fail(KPP_ERR_DEVICE, "a step-kernel launch ended without reporting its state");
        }
        KPP_TRY(copy_back());
        HIP_TRY(hipStreamSynchronize(st_));
        return KPP_OK;
      }
      if (q != hipSuccess && q != hipErrorNotReady) return fail(KPP_ERR_HIP, "HIP error: %s", hipGetErrorString(q));
    }
  }
  // Steps the last finish() took (0: a launch enqueued ahead that ran none).
  int64_t last_ran() const { return last_ran_; }
  size_t launches_in_flight() const { return launches_in_flight_.size(); }

  // The three parts of after_launch, for callers that plan several runs at
  // once: the state copy-back (HIP calls on the main stream), the next
  // window's host planning (touches only this run and its system: runs of
  // different systems may plan concurrently), and its factorization on the
  // side stream (HIP calls).
  kpp_status copy_back() {
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(sys_->h_ds, sys_->ds, sizeof(kpp::DevState), hipMemcpyDeviceToHost, st_));
    HIP_TRY(hipMemcpyAsync(sys_->h_err, sys_->err, sizeof(int32_t), hipMemcpyDeviceToHost, st_));
    if (fp32_ && sys_->fp64_count)
      HIP_TRY(hipMemcpyAsync(sys_->h_err + 1, sys_->fp64_count, sizeof(int32_t), hipMemcpyDeviceToHost, st_));
    return KPP_OK;
  }
  kpp_status plan_ahead() {
    const Window& w = win_[cur_];
    const int64_t t_next = w.t0 + w.W;
    planned_ = false;
    if (!have_next_ && t_next < max_iters_) {
      KPP_TRY(plan(win_[cur_ ^ 1], t_next, cur_ ^ 1));
      planned_ = true;
    }
    return KPP_OK;
  }
  kpp_status enqueue_ahead() {
    if (!planned_) return KPP_OK;
    planned_ = false;
    KPP_TRY(enqueue_factor(win_[cur_ ^ 1], side_));
    win_[cur_ ^ 1].on_side = true;
    have_next_ = true;
    return KPP_OK;
  }

  // After the main stream has drained: progress, errors, checkpoint, stop.
  kpp_status finish() {
    hs_ = *sys_->h_ds;
    const int32_t herr = *sys_->h_err;
    if (herr & 2) {
      drain();
      HIP_TRY(hipMemsetAsync(sys_->flags, 0, kFlagWords * sizeof(uint32_t), st_));
      HIP_TRY(hipStreamSynchronize(st_));
      sys_->epoch = 0;
      finished_ = true;
      return fail(KPP_ERR_DEVICE, "a device-side wait exceeded its bound in the fused engine");
    }
    if (herr & 1) {
      drain();
      finished_ = true;
      return fail(KPP_ERR_NOT_SPD, "a regularized block Gram has no Cholesky factor (lambda=%g)", prm_.lambda);
    }
    if (herr & 4) {
      drain();
      finished_ = true;
      return fail(KPP_ERR_INVALID_ARG, "the sparse matrix's row pointers changed after the system was created");
    }
    rho_now_ = hs_.rho;
    Window& w = win_[cur_];
    // every FP32 Gram tried so far (at least 32 blocks) was redone in FP64:
    // later blocks of this system skip the FP32 attempt
    if (fp32_ && !sys_->fp32_gram_futile && w.fp32_tried >= 32 && sys_->h_err[1] >= w.fp32_tried)
      sys_->fp32_gram_futile = true;
    const int64_t ran = hs_.t - t_;
    last_ran_ = ran;
    if (ran < 0 || ran > w.W - w.done) {
      finished_ = true;
      return fail(KPP_ERR_DEVICE, "step count out of range after a launch");
    }
    for (int64_t k = w.done; k < w.done + ran; ++k) {
      if (w.step_new[k])
        ++misses_;
      else
        ++hits_;
    }
    if (fused_) sys_->epoch += static_cast<uint32_t>(ran);
    w.done += ran;
    t_ = hs_.t;
    if (w.done == w.W && w.nb > 0) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, sys_->ev_fact[cur_][0], sys_->ev_fact[cur_][1]));
      t_factor_ += 1e-3 * ms;
    }
    if (ran > 0 && (t_ % period_) == 0 && hs_.cand) {
      if (o_.confirm) {
        double rn = 0.0;
        KPP_TRY(residual_norm(sys_, x_, &rn));
        true_rel_ = sys_->bnorm > 0 ? rn / sys_->bnorm : rn;
        if (rn <= o_.tol * sys_->bnorm) converged_ = true;
      } else {
        converged_ = true;
      }
    }
    if (o_.stop_on_stall && ran > 0 && (t_ % period_) == 0 && !converged_) {
      e1_hist_.push_back(hs_.last_E1);
      const size_t k = e1_hist_.size();
      if (k > static_cast<size_t>(kStallWindows) &&
          !(e1_hist_[k - 1] < kStallRatio * e1_hist_[k - 1 - kStallWindows]))
        stalled_ = true;
    }
    if (converged_ || stalled_ || t_ >= max_iters_) {
      finished_ = true;
    } else if (w.done == w.W) {
      cur_ ^= 1;
      have_next_ = false;
    }
    return KPP_OK;
  }

  // Wait for the system's side-stream work (factorizations planned past the
  // stop included) and report the run.
  kpp_status end(CoreStats* cs) {
    if (o_.defer_side_wait)
      side_deferred_ = true;
    else
      KPP_TRY(wait_side_work(sys_));
    if (o_.confirm && (!converged_ || std::isnan(true_rel_))) {
      double rn = 0.0;
      KPP_TRY(residual_norm(sys_, x_, &rn));
      true_rel_ = sys_->bnorm > 0 ? rn / sys_->bnorm : rn;
    }
    if (phase_prof_ && t_ > 0) {
      uint64_t ticks[kpp::kFusedPhases];
      HIP_TRY(hipMemcpy(ticks, sys_->phase_ticks, sizeof ticks, hipMemcpyDeviceToHost));
      int rate_khz = 0;
      HIP_TRY(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, sys_->ctx->device));
      static const char* names[kpp::kFusedPhases] = {"rows", "tile-dot", "publish", "wait", "reduce-r",
                                                     "solve+scalars", "update", "-"};
      static const char* sparse_names[kpp::kFusedPhases] = {"slice-rows", "publish+r-wait", "reduce-r", "y-rows",
                                                            "publish+y-wait", "read-y", "back-projection", "-"};
      std::fprintf(stderr, "[kpp phase profile] %lld steps, workgroup 0, us per step:", static_cast<long long>(t_));
      for (int ph = 0; ph < kpp::kFusedPhases - 1; ++ph)
        std::fprintf(stderr, " %s=%.3f", csr_ ? sparse_names[ph] : names[ph],
                     1e3 * static_cast<double>(ticks[ph]) / rate_khz / static_cast<double>(t_));
      std::fprintf(stderr, "\n");
    }
    cs->iters = t_ - t_start_;
    cs->hits = hits_;
    cs->misses = misses_;
    cs->launches = launches_;
    cs->converged = converged_;
    cs->true_rel = true_rel_;
    cs->t_factor = t_factor_;
    cs->t_kernel = t_kernel_;
    cs->hs = hs_;
    cs->engine = (fused_ || csr_window_) ? 2 : 1;
    cs->groups = fused_ ? groups_ : 0;
    cs->cpl = fused_ ? cpl_ : 0;
    cs->dual = dual_;
    cs->csr_nnz = csr_nnz_;
    cs->csr_gathers = csr_gathers_;
    cs->csr_miss_nnz = csr_miss_nnz_;
    cs->csr_folds = csr_folds_;
    return converged_ ? KPP_OK : KPP_NOT_CONVERGED;
  }

  // Wait for this system's side-stream work (used on every exit path).
  void drain() {
    if (begun_ && !side_deferred_) (void)wait_side_work(sys_);
  }

 private:
  static constexpr int64_t kChunk = 2048;
  static constexpr double kLazyBound = 256.0;

  struct Window {
    int64_t t0 = 0, W = 0, done = 0;
    int32_t nb = 0, idx = 0;
    int64_t fp32_tried = 0;   // new blocks with an FP32 Gram attempt up to this window
    bool try32 = false;       // this window's new blocks try an FP32 Gram first
    bool on_side = false, waited = false;
    size_t o_len = 0, o_slot = 0, o_step = 0, o_csc = 0, o_sinfo = 0;
    bool csr_lds = false, csr_global = false;   // sparse Kaczmarz++: build variants this window needs
    std::vector<int32_t> step_block, step_slot;
    std::vector<char> step_new;
  };

  kpp_status plan(Window& w, int64_t t0, int idx) {
    const double tp0 = wall_now();
    const double grow0 = t_prof_grow;
    struct Done {
      double t0, g0;
      ~Done() { t_prof_sched += (wall_now() - t0) - (t_prof_grow - g0); }
    } done{tp0, grow0};
    kpp_system* sys = sys_;
    const int32_t s = s_;
    w.t0 = t0;
    w.idx = idx;
    w.done = 0;
    w.on_side = false;
    w.waited = false;
    const int64_t span = periods_ * period_;
    w.W = std::min<int64_t>(span - (t0 % period_), max_iters_ - t0);
    w.step_block.resize(w.W);
    w.step_slot.resize(w.W);
    w.step_new.assign(w.W, 0);
    std::vector<int32_t> pending, pending_slots;
    if (mode_ == kpp::MemoMode::Off) KPP_TRY(ensure_slots(sys, static_cast<int32_t>(2 * span), s));
    for (int64_t k = 0; k < w.W; ++k) {
      bool is_new = false;
      const int32_t b = sch_->next(&is_new);
      w.step_block[k] = b;
      if (mode_ == kpp::MemoMode::Off) {
        // windows alternate between two halves of the slot table
        const int32_t q = static_cast<int32_t>(idx * span + k);
        w.step_slot[k] = q;
        w.step_new[k] = 1;
        pending.push_back(b);
        pending_slots.push_back(q);
        continue;
      }
      if (static_cast<int32_t>(sys->slot_of_block.size()) <= b) sys->slot_of_block.resize(b + 1, -1);
      int32_t q = sys->slot_of_block[b];
      if (q < 0) {
        q = sys->used_slots++;
        sys->slot_of_block[b] = q;
        pending.push_back(b);
        pending_slots.push_back(q);
        w.step_new[k] = 1;
      }
      w.step_slot[k] = q;
    }
    if (mode_ != kpp::MemoMode::Off) {
      const double ts = wall_now();
      if (sys->used_slots > sys->cap_slots) ++n_prof_slot_growth;
      KPP_TRY(ensure_slots(sys, sys->used_slots, s));
      t_prof_slots += wall_now() - ts;
    }
    if (csr_ && kind_ == KPP_KACZMARZ) KPP_TRY(ensure_csc_nu(sys, sys->cap_slots));
    if (csr_) KPP_TRY(ensure_csr_team(sys, sys->cap_slots, s));
    w.nb = static_cast<int32_t>(pending.size());
    w.try32 = fp32_ && !bf16_ && !sys->fp32_gram_futile;   // bfloat16 storage: FP64 Grams
    if (w.try32) sys->fp32_tried += w.nb;
    w.fp32_tried = sys->fp32_tried;
    w.o_len = static_cast<size_t>(w.nb) * s;
    w.o_slot = w.o_len + w.nb;
    w.o_step = w.o_slot + w.nb;
    w.o_csc = w.o_step + static_cast<size_t>(w.W) + static_cast<size_t>(w.nb);   // after the flags
    w.o_sinfo = w.o_csc + (csr_ ? static_cast<size_t>(kpp::kCsrMetaInts) * w.nb : 0);
    const size_t need = w.o_sinfo + (csr_ ? static_cast<size_t>(kpp::kSparseStepInts) * w.W : 0);
    const double tg = wall_now();
    KPP_TRY(ensure_stage(sys, idx, need));
    t_prof_grow += wall_now() - tg;
    // the copy out of this host buffer that an earlier run left in flight on
    // the side stream has been read before the buffer is written again
    HIP_TRY(hipEventSynchronize(sys->ev_fact[idx][0]));
    int32_t* stage = sys->h_stage[idx];
    for (int32_t k = 0; k < w.nb; ++k) {
      const int32_t b = pending[k];
      const int32_t l = sch_->len(b);
      std::copy(sch_->rows(b), sch_->rows(b) + l, stage + static_cast<size_t>(k) * s);
      std::fill(stage + static_cast<size_t>(k) * s + l, stage + static_cast<size_t>(k + 1) * s, 0);
      stage[w.o_len + k] = l;
      stage[w.o_slot + k] = pending_slots[k];
    }
    std::copy(w.step_slot.begin(), w.step_slot.end(), stage + w.o_step);
    if (csr_) {
      KPP_TRY(plan_csr(w, pending, pending_slots));
      // each step's slot, block length, nonzeros and place in the arena
      for (int64_t k = 0; k < w.W; ++k) {
        int32_t* in = stage + w.o_sinfo + static_cast<size_t>(kpp::kSparseStepInts) * k;
        const int32_t q = w.step_slot[k];
        in[0] = q;
        in[1] = sch_->len(w.step_block[k]);
        in[2] = sys->slot_csc_z[q];
        kpp::csr_meta_put(in + 3, kind_ == KPP_KACZMARZ ? sys->slot_csc_off[q] : 0);
      }
    }
    if (lsqr_) {
      // the sketch rows of the new blocks, in step order
      auto& T = lsqr_T_host_[idx];
      T.resize(static_cast<size_t>(w.nb) * tau_);
      for (int32_t k = 0; k < w.nb; ++k) draw_sketch_rows(T.data() + static_cast<size_t>(k) * tau_);
    }
    return KPP_OK;
  }

  // Sparse systems: nonzeros of each new block (from the host copy of the row
  // pointers) and, for Kaczmarz++, its place in the column-compressed arena
  // (appended for memoized blocks; for runs without memo each staging buffer
  // fills its own half) and in the build workspace when it exceeds LDS.
  kpp_status plan_csr(Window& w, const std::vector<int32_t>& pending, const std::vector<int32_t>& slots) {
    kpp_system* sys = sys_;
    w.csr_lds = w.csr_global = false;
    if (w.nb == 0) return KPP_OK;
    const int32_t maxq = *std::max_element(slots.begin(), slots.end());
    if (static_cast<int32_t>(sys->slot_csc_z.size()) <= maxq) {
      sys->slot_csc_z.resize(static_cast<size_t>(maxq) + 1, 0);
      sys->slot_csc_off.resize(static_cast<size_t>(maxq) + 1, 0);
    }
    std::vector<int64_t> zs(w.nb);
    int64_t total = 0;
    for (int32_t k = 0; k < w.nb; ++k) {
      const int32_t b = pending[k];
      const int32_t* r = sch_->rows(b);
      const int32_t l = sch_->len(b);
      int64_t z = 0;
      for (int32_t i = 0; i < l; ++i) z += sys->h_rp[r[i] + 1] - sys->h_rp[r[i]];
      if (z > kpp::kCsrMaxBlockNnz)
        return fail(KPP_ERR_SHAPE, "a block of %d rows holds %lld nonzeros (at most %lld)", l,
                    static_cast<long long>(z), static_cast<long long>(kpp::kCsrMaxBlockNnz));
      zs[k] = z;
      total += z + 1;
      sys->slot_csc_z[slots[k]] = static_cast<int32_t>(z);
      csr_miss_nnz_ += static_cast<double>(z);
    }
    if (kind_ != KPP_KACZMARZ) return KPP_OK;
    int64_t base = 0;
    if (mode_ == kpp::MemoMode::Off) {
      if (total > sys->csc_half) {
        KPP_TRY(ensure_csc(sys, 2 * std::max(total, 2 * sys->csc_half), 0));
        sys->csc_half = sys->csc_cap / 2;
      }
      base = w.idx * sys->csc_half;
    } else {
      KPP_TRY(ensure_csc(sys, sys->csc_top + total, sys->csc_top));
      base = sys->csc_top;
      sys->csc_top += total;
    }
    int32_t* meta = sys->h_stage[w.idx] + w.o_csc;
    size_t wsd = 0;
    int64_t o = base;
    for (int32_t k = 0; k < w.nb; ++k) {
      const int64_t z = zs[k];
      sys->slot_csc_off[slots[k]] = o;
      int64_t wso = -1;
      if (z > kpp::kCsrLdsEntries) {
        wso = static_cast<int64_t>(wsd);
        wsd += kpp::csr_build_ws_doubles(z);
        w.csr_global = true;
      } else {
        w.csr_lds = true;
      }
      int32_t* mk = meta + static_cast<size_t>(kpp::kCsrMetaInts) * k;
      kpp::csr_meta_put(mk, o);
      mk[2] = static_cast<int32_t>(z);
      kpp::csr_meta_put(mk + 3, wso);
      o += z + 1;
    }
    if (wsd > 0) KPP_TRY(ensure_csr_ws(sys, w.idx, wsd));
    return KPP_OK;
  }

  // tau of the Nsk padded columns: the sorted first tau entries of a partial
  // Fisher-Yates shuffle of 0..Nsk-1 (the schedule's subset draw)
  void draw_sketch_rows(int32_t* out) {
    std::unordered_map<int64_t, int64_t> moved;
    auto at = [&](int64_t i) {
      auto it = moved.find(i);
      return it == moved.end() ? i : it->second;
    };
    for (int32_t j = 0; j < tau_; ++j) {
      const int64_t k = j + static_cast<int64_t>(sk_gen_.bounded(static_cast<uint64_t>(Nsk_ - j)));
      const int64_t vj = at(j), vk = at(k);
      moved[j] = vk;
      moved[k] = vj;
      out[j] = static_cast<int32_t>(vk);
    }
    std::sort(out, out + tau_);
  }

  kpp_status setup_lsqr(const kpp_params* p) {
    kpp_system* sys = sys_;
    Nsk_ = 1;
    while (Nsk_ < n_) Nsk_ <<= 1;
    tau_ = static_cast<int32_t>(std::min<int64_t>(p->sketch_size > 0 ? p->sketch_size : 2 * static_cast<int64_t>(s_), Nsk_));
    lsqr_iters_ = p->lsqr_iters;
    sk_gen_ = kpp::SplitMix64(p->sketch_seed);
    // a window's new blocks are factored in batches of up to this many
    // sketches (at most 2^25 doubles, 256 MB, of stacked sketches)
    const int64_t per = static_cast<int64_t>(s_) * tau_;
    chunk_ = static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(kSketchBatch, (int64_t{1} << 25) / per)));
    if (sys->lsqr_cap_n < n_ || sys->lsqr_cap_N < Nsk_ || sys->lsqr_cap_s < s_ || sys->lsqr_cap_tau < tau_ ||
        static_cast<int64_t>(sys->lsqr_cap_chunk) * sys->lsqr_cap_s * sys->lsqr_cap_tau < chunk_ * per ||
        static_cast<int64_t>(sys->lsqr_cap_chunk) * sys->lsqr_cap_s < static_cast<int64_t>(chunk_) * s_) {
      HIP_TRY(hipStreamSynchronize(st_));
      HIP_TRY(hipStreamSynchronize(side_));
      drop_lsqr(sys);
      kpp_status stt;
      const int32_t groups = kpp::lsqr_at_groups(n_);
      if ((stt = dev_alloc(&sys->lsqr_state, 1)) < 0 || (stt = dev_alloc(&sys->lsqr_p, n_)) < 0 ||
          (stt = dev_alloc(&sys->lsqr_ppart, static_cast<int64_t>(kpp::lsqr_at_chunks(s_)) * n_)) < 0 ||
          (stt = dev_alloc(&sys->lsqr_part, groups)) < 0 || (stt = dev_alloc(&sys->lsqr_Xt, n_ * s_)) < 0 ||
          (stt = dev_alloc(&sys->lsqr_Y, Nsk_ * s_)) < 0 ||
          (stt = dev_alloc(&sys->lsqr_Ahat, chunk_ * per)) < 0 ||
          (stt = dev_alloc(&sys->lsqr_iota, static_cast<int64_t>(chunk_) * s_)) < 0 ||
          (stt = dev_alloc(&sys->lsqr_signs, Nsk_)) < 0) {
        drop_lsqr(sys);
        return stt;
      }
      sys->lsqr_cap_n = n_;
      sys->lsqr_cap_N = Nsk_;
      sys->lsqr_cap_s = s_;
      sys->lsqr_cap_tau = tau_;
      sys->lsqr_cap_chunk = chunk_;
    }
    std::vector<int32_t> iota(static_cast<size_t>(chunk_) * s_);
    std::iota(iota.begin(), iota.end(), 0);
    std::vector<int8_t> sg(static_cast<size_t>(Nsk_));
    for (auto& v : sg) v = (sk_gen_.next() >> 63) ? int8_t{-1} : int8_t{1};
    HIP_TRY(hipMemcpy(sys->lsqr_iota, iota.data(), iota.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(sys->lsqr_signs, sg.data(), sg.size(), hipMemcpyHostToDevice));
    return KPP_OK;
  }

  // upload the window's staging and factor its memo misses on `fs`
  kpp_status enqueue_factor(const Window& w, hipStream_t fs) {
    struct Done {
      double t0;
      ~Done() { t_prof_enqueue += wall_now() - t0; }
    } done{wall_now()};
    kpp_system* sys = sys_;
    const int32_t s = s_;
    const int idx = w.idx;
    const size_t need = csr_ ? w.o_sinfo + static_cast<size_t>(kpp::kSparseStepInts) * w.W
                             : w.o_step + static_cast<size_t>(w.W);
    // the window that last used this staging buffer (and, without memo, this
    // half of the slot table) has left the main stream: the host may move on
    // once a launch's state is mirrored, before the kernel has retired
    HIP_TRY(hipStreamWaitEvent(fs, sys->ev_win[idx], 0));
    HIP_TRY(hipMemcpyAsync(sys->d_stage[idx], sys->h_stage[idx], need * sizeof(int32_t), hipMemcpyHostToDevice, fs));
    HIP_TRY(hipEventRecord(sys->ev_fact[idx][0], fs));
    if (w.nb > 0) {
      const int32_t* d_srows = sys->d_stage[idx];
      const int32_t* d_slens = sys->d_stage[idx] + w.o_len;
      const int32_t* d_sslot = sys->d_stage[idx] + w.o_slot;
      kpp::launch_scatter_rows(d_srows, d_slens, d_sslot, w.nb, s, sys->rows, sys->lens, fs);
      if (lsqr_) {
        KPP_TRY(enqueue_sketch_factor(w, fs));
        HIP_TRY(hipEventRecord(sys->ev_fact[idx][1], fs));
        return KPP_OK;
      }
      if (csr_) {
        if (kind_ == KPP_KACZMARZ)
          kpp::launch_csr_block_build(sys->csr_rp, sys->csr_ci, sys->csr_cv, d_srows, d_slens, d_sslot,
                                      sys->d_stage[idx] + w.o_csc, w.nb, s, prm_.lambda, sys->L, sys->slot_stride,
                                      sys->csc, sys->csc_nu, sys->csr_ws[idx], w.csr_lds, w.csr_global, sys->err, fs);
        else
          kpp::launch_csr_gram_cd(sys->csr_rp, sys->csr_ci, sys->csr_cv, d_srows, d_slens, d_sslot, w.nb, s,
                                  prm_.lambda, sys->L, sys->slot_stride, fs);
        kpp::launch_csr_team_tables(kind_, sys->csr_rp, sys->csr_ci, d_srows, d_slens, d_sslot,
                                    sys->d_stage[idx] + w.o_csc, sys->csc, sys->csc_nu, w.nb, s, n_, sys->csr_G,
                                    sys->csr_team, fs);
        if (s <= kpp::kFactorSmallMax) {
          kpp::launch_factor_small(sys->L, sys->slot_stride, s, d_slens, w.nb, d_sslot, 1, sys->err, fs);
        } else {
          kpp::launch_cholesky(sys->L, s, sys->slot_stride, d_slens, w.nb, d_sslot, sys->err, fs);
          kpp::launch_factor_inverse(sys->L, sys->slot_stride, s, d_slens, w.nb, d_sslot, fs);
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(sys->ev_fact[idx][1], fs));
        return KPP_OK;
      }
      if (kind_ == KPP_KACZMARZ) KPP_TRY(ensure_gram_ws(sys, idx, kpp::gram_syrk_work(s, n_, w.nb)));
      double* gws = sys->gram_ws[idx];
      auto factor = [&](const kpp::FactorCheck& chk, const int32_t* skip) {
        if (s <= kpp::kFactorSmallMax) {
          kpp::launch_factor_small(sys->L, sys->slot_stride, s, d_slens, w.nb, d_sslot, 1, sys->err, fs, chk);
        } else {
          kpp::launch_cholesky(sys->L, s, sys->slot_stride, d_slens, w.nb, d_sslot, sys->err, fs, chk);
          kpp::launch_factor_inverse(sys->L, sys->slot_stride, s, d_slens, w.nb, d_sslot, fs, chk, skip);
        }
      };
      if (fp32_ && !w.try32) {
        kpp::launch_gram(kind_, sys->A, sys->lda, n_, d_srows, d_slens, s, w.nb, prm_.lambda, sys->L,
                         sys->slot_stride, d_sslot, gws, fs);
        factor(kpp::FactorCheck(), nullptr);
        sys->fp64_direct += w.nb;
      } else if (fp32_) {
        // FP32 Grams; blocks whose factor breaks down or whose kappa(G) exceeds
        // 1e6 are formed again from the FP64 A and factored in FP64
        int32_t* flag = sys->d_stage[idx] + w.o_step + w.W;
        kpp::launch_gram_f32(kind_, src_.A32, src_.lda, n_, d_srows, d_slens, s, w.nb, prm_.lambda, sys->L,
                             sys->slot_stride, d_sslot, gws, fs);
        kpp::FactorCheck first;
        first.flag = flag;
        first.counter = sys->fp64_count;
        first.kappa_max = 1e6;
        factor(first, flag);
        kpp::launch_gram(kind_, sys->A, sys->lda, n_, d_srows, d_slens, s, w.nb, prm_.lambda, sys->L,
                         sys->slot_stride, d_sslot, gws, fs, flag);
        kpp::FactorCheck redo;
        redo.only = flag;
        factor(redo, nullptr);
      } else {
        kpp::launch_gram(kind_, src_.A64, src_.lda, n_, d_srows, d_slens, s, w.nb, prm_.lambda, sys->L,
                         sys->slot_stride, d_sslot, gws, fs);
        factor(kpp::FactorCheck(), nullptr);
      }
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipEventRecord(sys->ev_fact[idx][1], fs));
    return KPP_OK;
  }

  // New blocks of the LSQR projection: the sketch A_hat = A_S Pi^T of each,
  // then the Gram of A_hat, its Cholesky factor and L^{-1} in the block's slot.
  kpp_status enqueue_sketch_factor(const Window& w, hipStream_t fs) {
    kpp_system* sys = sys_;
    const int idx = w.idx;
    const auto& Th = lsqr_T_host_[idx];
    const size_t nT = Th.size();
    if (sys->lsqr_T_cap[idx] < nT) {
      HIP_TRY(hipStreamSynchronize(fs));
      dev_free(sys->lsqr_T[idx]);
      sys->lsqr_T_cap[idx] = 0;
      KPP_TRY(dev_alloc(&sys->lsqr_T[idx], nT));
      sys->lsqr_T_cap[idx] = nT;
    }
    HIP_TRY(hipMemcpyAsync(sys->lsqr_T[idx], Th.data(), nT * sizeof(int32_t), hipMemcpyHostToDevice, fs));
    // split-Gram workspace for a full batch and for the last, shorter one
    const int32_t tail = w.nb % chunk_;
    KPP_TRY(ensure_gram_ws(sys, idx, std::max(kpp::gram_syrk_work(s_, tau_, std::min(chunk_, w.nb)),
                                              tail ? kpp::gram_syrk_work(s_, tau_, tail) : size_t{0})));
    const int32_t* d_slens = sys->d_stage[idx] + w.o_len;
    const int32_t* d_sslot = sys->d_stage[idx] + w.o_slot;
    const double iscale = 1.0 / std::sqrt(static_cast<double>(Nsk_));
    const double scale = std::sqrt(static_cast<double>(Nsk_) / static_cast<double>(tau_));
    const size_t per = static_cast<size_t>(s_) * tau_;
    for (int32_t k0 = 0; k0 < w.nb; k0 += chunk_) {
      // the sketches of up to chunk_ new blocks, stacked s x tau each ...
      const int32_t nk = std::min(chunk_, w.nb - k0);
      for (int32_t j = 0; j < nk; ++j) {
        const int32_t k = k0 + j;
        const int32_t q = sys->h_stage[idx][w.o_slot + k];
        const int32_t sb = sys->h_stage[idx][w.o_len + k];
        const int32_t* rows = sys->rows + static_cast<size_t>(q) * s_;
        kpp::launch_sketch_gather(src_.A64, src_.lda, n_, rows, sb, s_, sys->lsqr_Xt, fs);
        kpp::FhtSpec f;
        f.in = sys->lsqr_Xt;
        f.ld_in = s_;
        f.rows_valid = n_;
        f.cols_valid = s_;
        f.isign = sys->lsqr_signs;
        f.iscale = iscale;
        f.out = sys->lsqr_Y;
        f.ld_out = s_;
        f.rows_out = Nsk_;
        f.M = Nsk_;
        f.ncols = s_;
        kpp::launch_fht(f, fs);
        kpp::launch_sketch_select(sys->lsqr_Y, s_, sys->lsqr_T[idx] + static_cast<size_t>(k) * tau_, tau_, sb, scale,
                                  sys->lsqr_Ahat + j * per, fs);
      }
      // ... then their Grams A_hat A_hat^T + lambda I, Cholesky factors and
      // inverses in one launch each (rows k s + i of the stack)
      kpp::launch_gram(KPP_KACZMARZ, sys->lsqr_Ahat, tau_, tau_, sys->lsqr_iota, d_slens + k0, s_, nk, prm_.lambda,
                       sys->L, sys->slot_stride, d_sslot + k0, sys->gram_ws[idx], fs);
      kpp::launch_cholesky(sys->L, s_, sys->slot_stride, d_slens + k0, nk, d_sslot + k0, sys->err, fs);
      kpp::launch_factor_linv(sys->L, sys->slot_stride, s_, d_slens + k0, nk, d_sslot + k0, fs);
    }
    HIP_TRY(hipGetLastError());
    return KPP_OK;
  }

  kpp_system* sys_ = nullptr;
  kpp_params prm_{};
  Source src_{};
  CoreOpts o_{};
  double* x_ = nullptr;
  hipStream_t st_ = nullptr, side_ = nullptr;
  bool fp32_ = false, bf16_ = false, fused_ = false, phase_prof_ = false, stop_on_cand_ = false, begun_ = false;
  bool side_deferred_ = false;   // end() left the side stream's work in flight (CoreOpts::defer_side_wait)
  int32_t chunk_ = 1;   // sketches per batched factoring (LSQR projection)
  int32_t kind_ = 0, s_ = 0, zeta_ = 0, periods_ = 1, cpl_ = 0, groups_ = 0, P_ = 0;
  int64_t m_ = 0, n_ = 0, N_ = 0, period_ = 0, max_iters_ = 0;
  double eta_ = 0.0;
  kpp::MemoMode mode_ = kpp::MemoMode::Online;
  std::unique_ptr<kpp::BlockSchedule> sch_;
  Window win_[2];
  int cur_ = 0;
  bool have_next_ = false;
  int64_t t_ = 0, t_start_ = 0, hits_ = 0, misses_ = 0, launches_ = 0;
  bool converged_ = false, finished_ = false, stalled_ = false, planned_ = false, dual_ = false;
  struct Launch {
    bool mirrored;
    uint32_t seq;
  };
  std::deque<Launch> launches_in_flight_;
  int64_t last_ran_ = 0;
  double true_rel_ = NAN, t_factor_ = 0.0, t_kernel_ = 0.0;
  kpp::DevState hs_{};
  std::vector<double> e1_hist_;
  // sparse systems
  bool csr_ = false;
  bool csr_window_ = false;   // one launch of the team kernel per run of steps between folds
  double rho_now_ = 0.0;   // rho of the current window's steps
  double csr_nnz_ = 0.0, csr_gathers_ = 0.0, csr_miss_nnz_ = 0.0;
  int64_t csr_folds_ = 0;
  // LSQR projection
  bool lsqr_ = false;
  int64_t Nsk_ = 0;
  int32_t tau_ = 0, lsqr_iters_ = 0;
  kpp::SplitMix64 sk_gen_{0};
  std::vector<int32_t> lsqr_T_host_[2];
};

// A run driven on its own: one launch per window.
kpp_status solve_core(kpp_system* sys, const kpp_params* p, const Source& src, const CoreOpts& o,
                      double* x, CoreStats* cs) {
  hipStream_t st = sys->ctx->stream;
  CoreRun run;
  KPP_TRY(run.begin(sys, p, src, o, x, 1, 0));
  // Each launch is timed by an event pair (ev[0..1] or ev[2..3], in turn),
  // read when the host retires the launch, unless the caller turned launch
  // timing off; a launch enqueued ahead that ran no step is neither timed
  // nor counted.
  std::deque<int> pairs;   // event pair of each launch in flight, oldest first
  int next_pair = 0;
  auto launch = [&](bool ahead) -> kpp_status {
    kpp::FusedArgs a{};
    const int wi = ahead ? (run.cur_window() ^ 1) : run.cur_window();
    if (ahead)
      KPP_TRY(run.prepare_ahead(&a));
    else
      KPP_TRY(run.prepare(&a));
    const int pr = next_pair;
    next_pair ^= 1;
    if (o.time_launches) HIP_TRY(hipEventRecord(sys->ev[2 * pr], st));
    if (run.fused()) {
      run.mirror_args(&a);
      kpp::launch_fused(run.kind(), run.prec(), a, run.cpl(), run.groups(), st);
    } else {
      KPP_TRY(run.launch_unfused());
    }
    HIP_TRY(hipGetLastError());
    if (o.time_launches) HIP_TRY(hipEventRecord(sys->ev[2 * pr + 1], st));
    KPP_TRY(run.note_launch(a, wi));
    pairs.push_back(pr);
    return KPP_OK;
  };
  // the oldest launch: its end state, the checkpoint, its time
  auto retire = [&]() -> kpp_status {
    KPP_TRY(run.wait_launch());
    const int pr = pairs.front();
    pairs.pop_front();
    KPP_TRY(run.finish());
    if (run.last_ran() > 0) {
      if (o.time_launches) {
        float ms = 0.0f;
        HIP_TRY(hipEventSynchronize(sys->ev[2 * pr + 1]));
        HIP_TRY(hipEventElapsedTime(&ms, sys->ev[2 * pr], sys->ev[2 * pr + 1]));
        run.add_kernel_seconds(1e-3 * ms);
      }
      if (run.fused()) run.count_fused_launch();
    }
    return KPP_OK;
  };
  // (a run can be over before its first window: max_iters reached already)
  if (!run.finished()) {
    KPP_TRY(launch(false));
    KPP_TRY(run.after_launch());
  }
  while (!run.finished()) {
    // the next window goes to the stream before this one ends
    const bool ahead = run.can_launch_ahead();
    if (ahead) KPP_TRY(launch(true));
    KPP_TRY(retire());
    if (run.finished()) break;
    if (ahead) {
      if (run.state().cand) {
        // the stop test passed but the true residual did not confirm it:
        // the launch enqueued ahead ran no step; launch the window again
        KPP_TRY(retire());
        if (run.finished()) break;
        KPP_TRY(launch(false));
      }
      KPP_TRY(run.after_launch());
      continue;
    }
    KPP_TRY(launch(false));
    KPP_TRY(run.after_launch());
  }
  // a launch enqueued ahead of the stop ran no step: let it leave the stream
  while (run.launches_in_flight() > 0) {
    KPP_TRY(run.wait_launch());
    pairs.pop_front();
  }
  KPP_TRY(run.end(cs));
  if (o.keep_state) run.keep_state();
  return KPP_OK;
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
  res->team_groups = last.groups;
  res->cols_per_lane = last.cpl;
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
  if (p->projection == 1) {
    double Nsk = 1.0;
    while (Nsk < nn) Nsk *= 2.0;
    const double tau = std::min(p->sketch_size > 0 ? static_cast<double>(p->sketch_size) : 2.0 * sdb, Nsk);
    const double t = p->lsqr_iters;
    const double step = 4.0 * sdb * nn + 5.0 * nn + sdb * sdb + t * (4.0 * sdb * nn + 2.0 * nn + 4.0 * sdb * sdb);
    const double fact = sdb * Nsk * std::log2(Nsk) + sdb * sdb * tau + 2.0 * sdb * sdb * sdb / 3.0;
    res->flops = step * static_cast<double>(iters) + fact * static_cast<double>(misses);
  }
  res->bytes_algorithmic =
      static_cast<double>(iters) * (sdb * nn * bytes_per_elem + 0.5 * sdb * (sdb + 1) * 8.0 + 12.0 * sdb);
  if (sys->csr) {
    // sparse steps: block rows (index and value of each nonzero, its iterate
    // entries, row pointers), the projection (s^2 inverse entries), the
    // back-projection (Kaczmarz++: the column-compressed copy, counting every
    // nonzero's column as distinct, and u, v read and written there; CD++: s
    // entries of u and v), and 32 n bytes per fold.  Factors: s^3 / 3 plus
    // the Gram's s z (Kaczmarz++) per miss.
    const double it = static_cast<double>(iters);
    const double z = last.csr_nnz, g = last.csr_gathers, folds = static_cast<double>(last.csr_folds);
    const bool kz = kind == KPP_KACZMARZ;
    res->flops = 2.0 * z + it * 2.0 * sdb * sdb + (kz ? 2.0 * z + 4.0 * z : 4.0 * sdb * it) + 3.0 * nn * folds +
                 static_cast<double>(misses) * sdb * sdb * sdb / 3.0 + (kz ? sdb * last.csr_miss_nnz : 0.0);
    res->bytes_algorithmic = 12.0 * z + 8.0 * g + it * (16.0 * sdb + 8.0 * sdb * sdb + 28.0 * sdb) +
                             (kz ? 12.0 * z + 40.0 * z : it * 36.0 * sdb) + 32.0 * nn * folds;
  }
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
  o.resume = p->resume != 0;
  o.keep_state = true;
  o.time_launches = p->no_launch_timing == 0;
  if (!o.resume) sys->res_valid = false;
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
// factors, FP64 momentum and iterate) run to the relative tolerance inner_tol;
// with bfloat16 storage the inner products read the bfloat16 copy of A and
// the Grams are formed in FP64.  The memo cache of block factors carries over
// from round to round.  A diverging refinement ends early; an unconverged
// solve returns the iterate with the lowest true residual it saw.
kpp_status solve_mixed(kpp_system* sys, const kpp_params* p, double* x, kpp_result* res) {
  sys->res_valid = false;   // the inner runs reuse the momentum buffer
  // the inner runs leave their factors enqueued ahead in flight; every exit
  // waits for them
  struct SideWait {
    kpp_system* s;
    ~SideWait() { (void)wait_side_work(s); }
  } side_wait{sys};
  using clock = std::chrono::steady_clock;
  const auto t0 = clock::now();
  hipStream_t st = sys->ctx->stream;
  const int64_t m = sys->m, n = sys->n;
  const bool bf16 = p->precision == KPP_MIXED_BF16;
  if (bf16 && !sys->A16) {
    KPP_TRY(dev_alloc(&sys->A16, static_cast<size_t>(m) * n));
    kpp::launch_convert_bf16(sys->A, sys->lda, m, n, sys->A16, st);
    HIP_TRY(hipGetLastError());
  }
  if (!bf16 && !sys->A32) {
    KPP_TRY(dev_alloc(&sys->A32, static_cast<size_t>(m) * n));
    kpp::launch_convert_f32(sys->A, sys->lda, m, n, sys->A32, st);
    HIP_TRY(hipGetLastError());
  }
  if (!sys->rvec) KPP_TRY(dev_alloc(&sys->rvec, m));
  if (!sys->dvec) KPP_TRY(dev_alloc(&sys->dvec, n));
  if (!sys->xsave) KPP_TRY(dev_alloc(&sys->xsave, n));
  const bool wide = sys->kind == KPP_KACZMARZ && m < n;
  if (wide && !sys->gemvt_ws) KPP_TRY(dev_alloc(&sys->gemvt_ws, static_cast<size_t>(kpp::gemv_t_splits(m, n)) * n));
  if (wide && !sys->zx) KPP_TRY(dev_alloc(&sys->zx, m));
  if (wide && !sys->zm) KPP_TRY(dev_alloc(&sys->zm, m));
  if (!sys->fp64_count) KPP_TRY(dev_alloc(&sys->fp64_count, 1));
  HIP_TRY(hipMemsetAsync(sys->fp64_count, 0, sizeof(int32_t), st));
  sys->fp64_direct = 0;
  sys->fp32_tried = 0;
  int64_t iters = 0, hits = 0, misses = 0, launches = 0, ckpts = 0;
  double t_factor = 0.0, t_kernel = 0.0, rho = p->rho0, true_rel = NAN, est = NAN;
  bool converged = false;
  int32_t rounds = 0;
  CoreStats last;
  // the iterate with the lowest true residual is kept (xsave); a residual that
  // is not finite or has grown past kRefineDiverge times that lowest one ends
  // the refinement (the inner precision cannot resolve the system:
  // kappa(A) u_inner >= 1), and an unconverged solve returns that iterate
  constexpr double kRefineDiverge = 10.0;
  double best_rn = INFINITY;
  for (;;) {
    kpp::launch_residual_vec(sys->A, sys->lda, m, n, x, sys->b, sys->rvec, sys->rowsq, sys->scal, st);
    HIP_TRY(hipGetLastError());
    double rr = 0.0;
    HIP_TRY(hipMemcpyAsync(&rr, sys->scal, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double rn = std::sqrt(rr);
    if (rn < best_rn) {
      best_rn = rn;
      HIP_TRY(hipMemcpyAsync(sys->xsave, x, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    true_rel = sys->bnorm > 0 ? rn / sys->bnorm : rn;
    const bool diverged = !(rn <= kRefineDiverge * best_rn);
    if (rn <= p->tol * sys->bnorm) {
      converged = true;
      break;
    }
    if (diverged || rounds >= p->refine_max_rounds || iters >= p->max_iters) {
      if (!(rn <= best_rn)) {   // return the best iterate seen
        HIP_TRY(hipMemcpyAsync(x, sys->xsave, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        true_rel = sys->bnorm > 0 ? best_rn / sys->bnorm : best_rn;
      }
      break;
    }
    kpp::launch_zero3(sys->dvec, n, sys->zx, wide ? m : 0, sys->zm, wide ? m : 0, st);
    Source src;
    if (bf16)
      src.A16 = sys->A16;
    else
      src.A32 = sys->A32;
    src.lda = n;
    src.b = sys->rvec;
    src.bnorm = rn;
    CoreOpts o;
    o.zx = wide ? sys->zx : nullptr;
    o.zm = wide ? sys->zm : nullptr;
    o.tol = p->inner_tol;
    o.confirm = 0;
    o.stop_on_stall = 1;
    o.time_launches = p->no_launch_timing == 0;
    o.defer_side_wait = true;
    o.rho0 = rho;
    o.keep_memo = rounds > 0 ? 1 : p->keep_memo;
    o.max_iters = p->max_iters - iters;
    CoreStats cs;
    KPP_TRY(solve_core(sys, p, src, o, sys->dvec, &cs));
    // a wide system's correction is A^T zx with the FP64 A: in the row space
    // of A, so the refined x converges to the minimum-norm solution
    if (cs.dual) kpp::launch_gemv_t(sys->A, sys->lda, m, n, sys->zx, sys->dvec, sys->gemvt_ws, st);
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
  // the last inner run's Grams and factors enqueued ahead (they fill slots
  // that later solves may use, and the FP64-redo counter)
  KPP_TRY(wait_side_work(sys));
  fill_result(res, sys, p, iters, hits, misses, converged, rounds, last, true_rel, est, rho,
              std::chrono::duration<double>(clock::now() - t0).count(), t_factor, t_kernel, launches, ckpts,
              bf16 ? 2.0 : 4.0);
  if (res) {
    int32_t nfp64 = 0;
    HIP_TRY(hipMemcpy(&nfp64, sys->fp64_count, sizeof(int32_t), hipMemcpyDeviceToHost));
    res->factors_fp64 = nfp64 + sys->fp64_direct;
  }
  return converged ? KPP_OK : KPP_NOT_CONVERGED;
}


// --------------------------------------------------------------------------
// Serving: continuous batching of solves.  A worker thread owns the context's
// streams.  Every round it admits queued requests that fit (device-memory
// budget, compute units, active-request cap, one active request per system),
// then advances every active run by one window of its own length in a single
// persistent launch per (kind, precision, columns-per-lane) group: team t of
// the launch is run t's workgroups, so requests of different sizes and step
// counts share the device.  A window spans k_r checkpoint periods, k_r chosen
// per request so that windows are about kServeRoundSteps steps; a team stops
// early at a checkpoint whose stop test passes.  Each run's iterates are those
// of the same request served alone.
// --------------------------------------------------------------------------

constexpr int64_t kServeRoundSteps = 128;

double now_seconds() {
  using clock = std::chrono::steady_clock;
  return std::chrono::duration<double>(clock::now().time_since_epoch()).count();
}

struct ServeReq {
  uint64_t id = 0;
  kpp_system* sys = nullptr;
  kpp_params p{};
  double* x = nullptr;
  bool mixed = false;
  size_t footprint = 0;
  int32_t groups = 0, cpl = 0, periods = 1;
  double t_submit = 0.0, t_admit = 0.0, t_start = 0.0;
  kpp_status status = KPP_OK;
  kpp_result res{};
  std::unique_ptr<CoreRun> run;
  // refinement bookkeeping (mixed precision) and totals over runs
  int32_t rounds = 0;
  int64_t iters = 0, hits = 0, misses = 0, launches = 0, ckpts = 0;
  double t_factor = 0.0, t_kernel = 0.0, rho = 0.0, true_rel = NAN, est = NAN, last_rn = 0.0;
  CoreStats last;
  bool complete = false;
};

// Checkpoint periods per window of a served request: about kServeRoundSteps
// steps, so that requests of different sizes take similar time per round.
int32_t serve_periods(const kpp_system* sys, const kpp_params* p) {
  const int64_t N = sys->kind == KPP_CD_PSD ? sys->n : sys->m;
  const int64_t period = 2 * ((N + p->block_size - 1) / p->block_size);
  return static_cast<int32_t>(std::max<int64_t>(1, kServeRoundSteps / period));
}

// Device memory a request needs while it runs, beyond the caller's A, b and x:
// memo slots, the FP32 copy of A (mixed precision), state vectors, staging.
size_t serve_footprint(const kpp_system* sys, const kpp_params* p, int32_t periods) {
  const int64_t N = sys->kind == KPP_CD_PSD ? sys->n : sys->m;
  const int32_t s = p->block_size;
  const int64_t zeta = (N + s - 1) / s;
  int64_t blocks = 0;
  if (p->memo == KPP_MEMO_FIXED)
    blocks = p->fixed_partition ? zeta : p->num_blocks;
  else if (p->memo == KPP_MEMO_OFF)
    blocks = 4 * periods * zeta;
  else
    blocks = static_cast<int64_t>(4.0 * kpp::online_rate(sys->kind, sys->m, sys->n, s)) + 16;
  size_t bytes = static_cast<size_t>(blocks) * (static_cast<size_t>(kpp::slot_doubles(s)) * 8 + 4 * (s + 1));
  if (p->precision == KPP_MIXED_FP32) {
    bytes += static_cast<size_t>(sys->m) * sys->n * 4 + 8 * (sys->m + sys->n);
    if (sys->kind == KPP_KACZMARZ && sys->m < sys->n)   // duals and the partial sums of A^T z
      bytes += 8 * (2 * static_cast<size_t>(sys->m) + static_cast<size_t>(kpp::gemv_t_splits(sys->m, sys->n)) * sys->n);
  }
  bytes += 8 * static_cast<size_t>(sys->n) * 2 + 2 * 4 * static_cast<size_t>(s) * (4 * periods * zeta + 2 * s);
  return bytes;
}

}  // namespace

// A small pool of host threads that run one indexed job at a time (the
// calling thread takes part); used to plan the next windows of many runs.
// Indices are handed out under the mutex and tagged with the job's
// generation, so an index runs exactly once and a thread that is late for one
// job cannot take indices of the next.
class HostPool {
 public:
  explicit HostPool(int nthreads) {
    for (int i = 0; i < nthreads; ++i) threads_.emplace_back([this] { work(); });
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      quit_ = true;
    }
    cv_.notify_all();
    for (auto& t : threads_) t.join();
  }
  // fn(i) for i in [0, n), returns when all are done
  void run(int n, const std::function<void(int)>& fn) {
    if (n <= 0) return;
    uint64_t gen;
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn;
      n_ = n;
      next_ = 0;
      done_ = 0;
      gen = ++gen_;
    }
    cv_.notify_all();
    drain(gen);
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [&] { return done_ == n_; });
    fn_ = nullptr;
  }

 private:
  bool grab(uint64_t gen, int* i, const std::function<void(int)>** fn) {
    std::lock_guard<std::mutex> lk(mu_);
    if (gen != gen_ || next_ >= n_) return false;
    *i = next_++;
    *fn = fn_;
    return true;
  }
  void drain(uint64_t gen) {
    int i;
    const std::function<void(int)>* fn;
    while (grab(gen, &i, &fn)) {
      (*fn)(i);
      std::lock_guard<std::mutex> lk(mu_);
      if (++done_ == n_) cv_done_.notify_all();
    }
  }
  void work() {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return quit_ || gen_ != seen; });
        if (quit_) return;
        seen = gen_;
      }
      drain(seen);
    }
  }
  std::vector<std::thread> threads_;
  std::mutex mu_;
  std::condition_variable cv_, cv_done_;
  const std::function<void(int)>* fn_ = nullptr;
  int n_ = 0, next_ = 0, done_ = 0;
  uint64_t gen_ = 0;
  bool quit_ = false;
};

struct kpp_server {
  kpp_context* ctx = nullptr;
  std::unique_ptr<HostPool> pool;
  uint64_t budget = 0;
  int32_t max_active = 0;
  int32_t cu_budget = 0;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stopping = false;
  uint64_t next_id = 1;
  std::deque<ServeReq*> queue;           // guarded by mu
  std::vector<ServeReq*> active;         // worker thread only
  std::deque<ServeReq*> done;            // guarded by mu
  std::vector<kpp_system*> busy;         // systems with an active request (worker thread only)
  // device and pinned host copies of one launch's team table
  kpp::FusedArgs* d_args = nullptr;
  int32_t* d_team = nullptr;
  kpp::FusedArgs* h_args = nullptr;
  int32_t* h_team = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // statistics (guarded by mu)
  int64_t submitted = 0, completed = 0, rejected = 0, rounds = 0;
  int32_t n_active = 0, peak_active = 0;
  uint64_t bytes_active = 0, peak_bytes = 0;
  double busy_seconds = 0.0;
  int32_t groups_active = 0;
  // KPP_SERVE_PROFILE=1: host seconds per worker-loop section, printed at destroy
  bool prof = false;
  double prof_s[6] = {0, 0, 0, 0, 0, 0};
  double prof_grow = 0.0, prof_sched = 0.0, prof_enqueue = 0.0, prof_slots = 0.0;   // from the worker thread
  int64_t prof_slot_growth = 0;
};

namespace {

// Final numbers of a finished request (worker thread).  The request is handed
// to the caller later, by serve_handoff, after the worker's last use of it.
void serve_complete(kpp_server* srv, ServeReq* r) {
  (void)srv;
  if (r->run) {
    r->run->drain();
    r->run.reset();
  }
  kpp_result* res = &r->res;
  std::memset(res, 0, sizeof(*res));
  if (r->status >= 0) {
    fill_result(res, r->sys, &r->p, r->iters, r->hits, r->misses, r->status == KPP_OK, r->rounds, r->last,
                r->true_rel, r->est, r->rho, now_seconds() - r->t_submit, r->t_factor, r->t_kernel, r->launches,
                r->ckpts, r->mixed ? 4.0 : 8.0);
    if (r->mixed && r->sys->fp64_count) {
      int32_t nfp64 = 0;
      if (hipMemcpy(&nfp64, r->sys->fp64_count, sizeof(int32_t), hipMemcpyDeviceToHost) == hipSuccess)
        res->factors_fp64 = nfp64 + r->sys->fp64_direct;
    }
  }
  res->seconds_total = now_seconds() - r->t_submit;
  res->seconds_queued = r->t_admit - r->t_submit;
  r->complete = true;
}

// Move the worker's completed requests to the done queue; once there, a
// request belongs to kpp_server_poll (which deletes it) and the worker does
// not touch it again.
void serve_handoff(kpp_server* srv) {
  std::vector<ServeReq*> finished, keep;
  for (ServeReq* r : srv->active) {
    if (r->complete) {
      srv->busy.erase(std::find(srv->busy.begin(), srv->busy.end(), r->sys));
      finished.push_back(r);
    } else {
      keep.push_back(r);
    }
  }
  srv->active.swap(keep);
  if (finished.empty()) return;
  std::lock_guard<std::mutex> lk(srv->mu);
  for (ServeReq* r : finished) {
    srv->bytes_active -= r->footprint;
    srv->groups_active -= r->groups;
    srv->n_active -= 1;
    srv->completed += 1;
    srv->done.push_back(r);
  }
  srv->cv_done.notify_all();
}

// Start the next run of request r: the FP64 solve, or the next refinement
// round (mixed precision).  Sets r->status and returns false when r is over.
bool serve_next_run(kpp_server* srv, ServeReq* r) {
  kpp_system* sys = r->sys;
  hipStream_t st = sys->ctx->stream;
  auto failed = [&](kpp_status s) {
    r->status = s;
    return false;
  };
  if (!r->mixed) {
    Source src;
    src.A64 = sys->A;
    src.lda = sys->lda;
    src.b = sys->b;
    src.bnorm = sys->bnorm;
    CoreOpts o;
    o.tol = r->p.tol;
    o.confirm = r->p.confirm_true_residual;
    o.rho0 = r->p.rho0;
    o.keep_memo = r->p.keep_memo;
    o.max_iters = r->p.max_iters;
    r->run.reset(new CoreRun);
    r->run->set_stop_on_cand(true);
    const kpp_status s = r->run->begin(sys, &r->p, src, o, r->x, r->periods, r->cpl);
    if (s < 0) return failed(s);
    return true;
  }
  // mixed precision: r = b - A x in FP64; stop, or solve A32 d = r approximately
  kpp::launch_residual_vec(sys->A, sys->lda, sys->m, sys->n, r->x, sys->b, sys->rvec, sys->rowsq, sys->scal, st);
  if (hipGetLastError() != hipSuccess) return failed(fail(KPP_ERR_HIP, "residual launch failed"));
  double rr = 0.0;
  if (hipMemcpyAsync(&rr, sys->scal, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return failed(fail(KPP_ERR_HIP, "residual copy failed"));
  const double rn = std::sqrt(rr);
  r->true_rel = sys->bnorm > 0 ? rn / sys->bnorm : rn;
  if (rn <= r->p.tol * sys->bnorm) {
    r->status = KPP_OK;
    return false;
  }
  if (r->rounds >= r->p.refine_max_rounds || r->iters >= r->p.max_iters) {
    r->status = KPP_NOT_CONVERGED;
    return false;
  }
  if (hipMemsetAsync(sys->dvec, 0, sys->n * sizeof(double), st) != hipSuccess)
    return failed(fail(KPP_ERR_HIP, "memset failed"));
  const bool wide = sys->kind == KPP_KACZMARZ && sys->m < sys->n;
  if (wide && (hipMemsetAsync(sys->zx, 0, sys->m * sizeof(double), st) != hipSuccess ||
               hipMemsetAsync(sys->zm, 0, sys->m * sizeof(double), st) != hipSuccess))
    return failed(fail(KPP_ERR_HIP, "memset failed"));
  Source src;
  src.A32 = sys->A32;
  src.lda = sys->n;
  src.b = sys->rvec;
  src.bnorm = rn;
  CoreOpts o;
  o.zx = wide ? sys->zx : nullptr;
  o.zm = wide ? sys->zm : nullptr;
  o.tol = r->p.inner_tol;
  o.confirm = 0;
  o.stop_on_stall = 1;
  o.rho0 = r->rho;
  o.keep_memo = r->rounds > 0 ? 1 : r->p.keep_memo;
  o.max_iters = r->p.max_iters - r->iters;
  r->run.reset(new CoreRun);
  r->run->set_stop_on_cand(true);
  const kpp_status s = r->run->begin(sys, &r->p, src, o, sys->dvec, r->periods, r->cpl);
  if (s < 0) return failed(s);
  r->est = NAN;
  r->last_rn = rn;
  return true;
}

// A run of request r has ended: fold its numbers in, apply the correction
// (mixed precision) and start the next run if there is one.
bool serve_run_ended(kpp_server* srv, ServeReq* r) {
  CoreStats cs;
  const kpp_status s = r->run->end(&cs);
  if (s < 0) {
    r->status = s;
    return false;
  }
  r->iters += cs.iters;
  r->hits += cs.hits;
  r->misses += cs.misses;
  r->launches += cs.launches;
  r->ckpts += cs.hs.ckpts;
  r->t_factor += cs.t_factor;
  r->t_kernel += cs.t_kernel;
  r->last = cs;
  if (!r->mixed) {
    r->true_rel = cs.true_rel;
    r->rho = cs.converged ? cs.hs.rho_before : cs.hs.rho;
    r->est = r->sys->bnorm > 0 ? std::sqrt(cs.hs.last_E1) / r->sys->bnorm : std::sqrt(cs.hs.last_E1);
    r->status = cs.converged ? KPP_OK : KPP_NOT_CONVERGED;
    r->run.reset();
    return false;
  }
  if (cs.dual)
    kpp::launch_gemv_t(r->sys->A, r->sys->lda, r->sys->m, r->sys->n, r->sys->zx, r->sys->dvec, r->sys->gemvt_ws,
                       r->sys->ctx->stream);
  kpp::launch_axpy1(r->x, r->sys->dvec, r->sys->n, r->sys->ctx->stream);
  if (hipGetLastError() != hipSuccess) {
    r->status = fail(KPP_ERR_HIP, "axpy launch failed");
    return false;
  }
  r->rounds += 1;
  r->rho = cs.converged ? cs.hs.rho_before : cs.hs.rho;
  r->est = r->last_rn > 0 ? std::sqrt(cs.hs.last_E1) / r->last_rn : 0.0;
  r->run.reset();
  return serve_next_run(srv, r);
}

// First work of an admitted request (worker thread).
bool serve_start(kpp_server* srv, ServeReq* r) {
  kpp_system* sys = r->sys;
  hipStream_t st = sys->ctx->stream;
  r->t_start = now_seconds();
  if (r->mixed) {
    auto failed = [&](kpp_status s) {
      r->status = s;
      return false;
    };
    if (!sys->A32) {
      if (dev_alloc(&sys->A32, static_cast<size_t>(sys->m) * sys->n) < 0) return failed(KPP_ERR_OOM);
      kpp::launch_convert_f32(sys->A, sys->lda, sys->m, sys->n, sys->A32, st);
    }
    if (!sys->rvec && dev_alloc(&sys->rvec, sys->m) < 0) return failed(KPP_ERR_OOM);
    if (!sys->dvec && dev_alloc(&sys->dvec, sys->n) < 0) return failed(KPP_ERR_OOM);
    if (sys->kind == KPP_KACZMARZ && sys->m < sys->n) {
      if (!sys->zx && dev_alloc(&sys->zx, sys->m) < 0) return failed(KPP_ERR_OOM);
      if (!sys->zm && dev_alloc(&sys->zm, sys->m) < 0) return failed(KPP_ERR_OOM);
      if (!sys->gemvt_ws &&
          dev_alloc(&sys->gemvt_ws, static_cast<size_t>(kpp::gemv_t_splits(sys->m, sys->n)) * sys->n) < 0)
        return failed(KPP_ERR_OOM);
    }
    if (!sys->fp64_count && dev_alloc(&sys->fp64_count, 1) < 0) return failed(KPP_ERR_OOM);
    if (hipMemsetAsync(sys->fp64_count, 0, sizeof(int32_t), st) != hipSuccess) return failed(KPP_ERR_HIP);
    sys->fp64_direct = 0;
    sys->fp32_tried = 0;
    r->rho = r->p.rho0;
  }
  return serve_next_run(srv, r);
}

// One round: a window of every active run, one launch per group.
void serve_round(kpp_server* srv) {
  hipStream_t st = srv->ctx->stream;
  std::vector<ServeReq*> live;
  for (ServeReq* r : srv->active)
    if (!r->complete && r->run && !r->run->finished()) live.push_back(r);
  if (live.empty()) return;
  // groups of runs that can share one launch
  std::vector<std::vector<ServeReq*>> groups;
  for (ServeReq* r : live) {
    bool placed = false;
    for (auto& g : groups) {
      ServeReq* h = g.front();
      if (h->run->kind() == r->run->kind() && h->run->fp32() == r->run->fp32() && h->run->cpl() == r->run->cpl()) {
        g.push_back(r);
        placed = true;
        break;
      }
    }
    if (!placed) groups.push_back({r});
  }
  std::vector<ServeReq*> launched;
  double tp = now_seconds();
  (void)hipEventRecord(srv->ev[0], st);
  int32_t off_args = 0, off_team = 0;
  for (auto& g : groups) {
    std::vector<ServeReq*> team;
    for (ServeReq* r : g) {
      const kpp_status s = r->run->prepare(&srv->h_args[off_args + static_cast<int32_t>(team.size())]);
      if (s < 0) {
        r->status = s;
        continue;
      }
      team.push_back(r);
    }
    if (team.empty()) continue;
    const int32_t n_t = static_cast<int32_t>(team.size());
    int32_t* ht = srv->h_team + off_team;
    int32_t total = 0;
    ht[0] = 0;
    for (int32_t i = 0; i < n_t; ++i) {
      total += team[i]->run->groups();
      ht[i + 1] = total;
    }
    if (hipMemcpyAsync(srv->d_args + off_args, srv->h_args + off_args, n_t * sizeof(kpp::FusedArgs),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(srv->d_team + off_team, ht, (n_t + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st) !=
            hipSuccess) {
      for (ServeReq* r : team) r->status = fail(KPP_ERR_HIP, "team table upload failed");
      continue;
    }
    ServeReq* h = team.front();
    kpp::launch_fused_multi(h->run->kind(), h->run->fp32(), srv->d_args + off_args, srv->d_team + off_team, n_t,
                            total, h->run->cpl(), st);
    if (hipGetLastError() != hipSuccess) {
      for (ServeReq* r : team) r->status = fail(KPP_ERR_HIP, "step launch failed");
      continue;
    }
    for (ServeReq* r : team) {
      r->run->count_fused_launch();
      launched.push_back(r);
    }
    off_args += n_t;
    off_team += n_t + 1;
  }
  (void)hipEventRecord(srv->ev[1], st);
  if (srv->prof) {
    const double t = now_seconds();
    srv->prof_s[1] += t - tp;
    tp = t;
  }
  // next windows: copy-back and factor enqueue in order, host planning in parallel
  for (ServeReq* r : launched) {
    const kpp_status s = r->run->copy_back();
    if (s < 0) r->status = s;
  }
  srv->pool->run(static_cast<int>(launched.size()), [&](int i) {
    ServeReq* r = launched[i];
    if (r->status < 0) return;
    const kpp_status s = r->run->plan_ahead();
    if (s < 0) r->status = s;
  });
  for (ServeReq* r : launched) {
    if (r->status < 0) continue;
    const kpp_status s = r->run->enqueue_ahead();
    if (s < 0) r->status = s;
  }
  if (srv->prof) {
    const double t = now_seconds();
    srv->prof_s[2] += t - tp;
    tp = t;
  }
  (void)hipStreamSynchronize(st);
  if (srv->prof) {
    const double t = now_seconds();
    srv->prof_s[3] += t - tp;
    tp = t;
  }
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, srv->ev[0], srv->ev[1]);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->rounds += 1;
    srv->busy_seconds += 1e-3 * ms;
  }
  for (ServeReq* r : launched) {
    if (r->status < 0) continue;
    r->run->add_kernel_seconds(1e-3 * ms);
    const kpp_status s = r->run->finish();
    if (s < 0) r->status = s;
  }
  if (srv->prof) srv->prof_s[4] += now_seconds() - tp;
}

void serve_loop(kpp_server* srv) {
  (void)hipSetDevice(srv->ctx->device);
  for (;;) {
    std::vector<ServeReq*> admitted;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      // admission in arrival order; a request whose system is busy waits
      // without holding back later ones, one that does not fit stops the scan
      for (auto it = srv->queue.begin(); it != srv->queue.end();) {
        ServeReq* r = *it;
        if (std::find(srv->busy.begin(), srv->busy.end(), r->sys) != srv->busy.end()) {
          ++it;
          continue;
        }
        if (srv->n_active >= srv->max_active || srv->bytes_active + r->footprint > srv->budget ||
            srv->groups_active + r->groups > srv->cu_budget)
          break;
        srv->bytes_active += r->footprint;
        srv->groups_active += r->groups;
        srv->n_active += 1;
        srv->peak_active = std::max(srv->peak_active, srv->n_active);
        srv->peak_bytes = std::max<uint64_t>(srv->peak_bytes, srv->bytes_active);
        r->t_admit = now_seconds();
        srv->busy.push_back(r->sys);
        admitted.push_back(r);
        it = srv->queue.erase(it);
      }
      if (admitted.empty() && srv->active.empty()) {
        if (srv->stopping && srv->queue.empty()) return;
        srv->cv_work.wait_for(lk, std::chrono::milliseconds(2));
        continue;
      }
    }
    double t0 = now_seconds();
    for (ServeReq* r : admitted) {
      srv->active.push_back(r);
      if (!serve_start(srv, r)) {
        serve_complete(srv, r);
      }
    }
    if (srv->prof) srv->prof_s[0] += now_seconds() - t0;
    serve_round(srv);
    t0 = now_seconds();
    // runs that ended start their next refinement round or complete
    for (ServeReq* r : srv->active) {
      if (r->complete) continue;
      if (r->status < 0) {
        serve_complete(srv, r);
        continue;
      }
      if (r->run && r->run->finished()) {
        if (!serve_run_ended(srv, r)) serve_complete(srv, r);
      } else if (!r->run) {
        serve_complete(srv, r);
      }
    }
    serve_handoff(srv);
    if (srv->prof) {
      srv->prof_s[5] += now_seconds() - t0;
      srv->prof_grow = t_prof_grow;
      srv->prof_sched = t_prof_sched;
      srv->prof_enqueue = t_prof_enqueue;
      srv->prof_slots = t_prof_slots;
      srv->prof_slot_growth = n_prof_slot_growth;
    }
  }
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// randomized Hadamard preprocessing (Definition d:rht; Algorithms 2 to 5)
// ---------------------------------------------------------------------------
namespace {

bool is_pow2(int64_t v) { return v >= 1 && (v & (v - 1)) == 0; }
int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

kpp_status check_rht_size(int64_t rows, int64_t R) {
  if (!is_pow2(R) || R < rows || R > kpp::kFhtMaxRows)
    return fail(KPP_ERR_SHAPE, "R=%lld must be a power of two in [%lld, %lld]", static_cast<long long>(R),
                static_cast<long long>(rows), static_cast<long long>(kpp::kFhtMaxRows));
  return KPP_OK;
}

// H D [x; 0] (forward) or the first nx entries of D H x (back), D = diag(d)/sqrt(R)
kpp_status rht_vector(hipStream_t st, int64_t R, const int8_t* signs, const double* x, int64_t nx, double* y,
                      bool back, double* work) {
  kpp::FhtSpec f;
  f.in = x;
  f.ld_in = 1;
  f.rows_valid = back ? R : nx;
  f.cols_valid = 1;
  f.out = y;
  f.ld_out = 1;
  f.rows_out = back ? nx : R;
  f.M = R;
  f.ncols = 1;
  f.work = work;
  const double scale = 1.0 / std::sqrt(static_cast<double>(R));
  if (back) {
    f.osign = signs;
    f.oscale = scale;
  } else {
    f.isign = signs;
    f.iscale = scale;
  }
  kpp::launch_fht(f, st);
  HIP_TRY(hipGetLastError());
  return KPP_OK;
}

kpp_status rht_general(hipStream_t st, int64_t m, int64_t n, const double* A, int64_t lda, const double* b,
                       const int8_t* signs, int64_t R, double* At, int64_t ldt, double* bt) {
  kpp::FhtSpec f;
  f.in = A;
  f.ld_in = lda;
  f.rows_valid = m;
  f.cols_valid = n;
  f.isign = signs;
  f.iscale = 1.0 / std::sqrt(static_cast<double>(R));
  f.out = At;
  f.ld_out = ldt;
  f.rows_out = R;
  f.M = R;
  f.ncols = n;
  kpp::launch_fht(f, st);   // two passes run in place on At
  HIP_TRY(hipGetLastError());
  return rht_vector(st, R, signs, b, m, bt, false, nullptr);
}

kpp_status rht_psd(hipStream_t st, int64_t n, const double* A, int64_t lda, const double* b, const int8_t* signs,
                   int64_t R, double* At, int64_t ldt, double* bt, double* work) {
  const double scale = 1.0 / std::sqrt(static_cast<double>(R));
  // (H D A D)^T into At, then H applied to it in place: H (H D A D)^T = H D A D H
  kpp::FhtSpec f;
  f.in = A;
  f.ld_in = lda;
  f.rows_valid = n;
  f.cols_valid = n;
  f.isign = signs;
  f.iscale = scale;
  f.csign = signs;
  f.cscale = scale;
  f.out = At;
  f.ld_out = ldt;
  f.rows_out = R;
  f.transpose_out = 1;
  f.M = R;
  f.ncols = R;
  f.work = work;
  kpp::launch_fht(f, st);
  HIP_TRY(hipGetLastError());
  kpp::FhtSpec g;
  g.in = At;
  g.ld_in = ldt;
  g.rows_valid = R;
  g.cols_valid = R;
  g.out = At;
  g.ld_out = ldt;
  g.rows_out = R;
  g.M = R;
  g.ncols = R;
  kpp::launch_fht(g, st);
  HIP_TRY(hipGetLastError());
  return rht_vector(st, R, signs, b, n, bt, false, nullptr);
}

// Additions of the transforms as the paper counts them (Appendix on SymFHT):
// FHT of an n x d matrix n d log2 n, SymFHT by its recursion (two half-size
// SymFHTs, two FHTs of the off-diagonal block, 7 (n/2)^2 block sums).
double fht_adds(double n, double d) { return n > 1.0 ? n * d * std::log2(n) : 0.0; }
double symfht_adds(int64_t n) {
  if (n <= 1) return 0.0;
  const int64_t h = n / 2;
  const double hd = static_cast<double>(h);
  return 2.0 * symfht_adds(h) + 2.0 * fht_adds(hd, hd) + 7.0 * hd * hd;
}

void draw_signs(uint64_t seed, int64_t N, int8_t* out) {
  kpp::SplitMix64 g(seed);
  for (int64_t i = 0; i < N; ++i) out[i] = (g.next() >> 63) ? int8_t{-1} : int8_t{1};
}

// Form (or reuse) the transformed system of sys for this seed; *built tells
// whether this call formed it.
kpp_status prepare_rht(kpp_system* sys, uint64_t seed, bool* built) {
  *built = false;
  const bool psd = sys->kind == KPP_CD_PSD;
  const int64_t rows = psd ? sys->n : sys->m;
  const int64_t R = next_pow2(rows);
  KPP_TRY(check_rht_size(rows, R));
  if (sys->rht_inner && sys->rht_seed == seed) return KPP_OK;
  hipStream_t st = sys->ctx->stream;
  HIP_TRY(hipStreamSynchronize(st));
  drop_rht(sys);
  const int64_t cols = psd ? R : sys->n;
  kpp_status stt;
  if ((stt = dev_alloc(&sys->rht_signs, R)) < 0 || (stt = dev_alloc(&sys->rht_A, R * cols)) < 0 ||
      (stt = dev_alloc(&sys->rht_b, R)) < 0 || (psd && (stt = dev_alloc(&sys->rht_x, R)) < 0) ||
      (kpp::fht_passes(R) > 1 && (stt = dev_alloc(&sys->rht_work, psd ? R * R : R)) < 0)) {
    drop_rht(sys);
    return stt;
  }
  std::vector<int8_t> h(static_cast<size_t>(R));
  draw_signs(seed, R, h.data());
  HIP_TRY(hipMemcpyAsync(sys->rht_signs, h.data(), static_cast<size_t>(R), hipMemcpyHostToDevice, st));
  kpp_status r = psd ? rht_psd(st, sys->n, sys->A, sys->lda, sys->b, sys->rht_signs, R, sys->rht_A, R, sys->rht_b,
                               sys->rht_work)
                     : rht_general(st, sys->m, sys->n, sys->A, sys->lda, sys->b, sys->rht_signs, R, sys->rht_A,
                                   sys->n, sys->rht_b);
  if (r < 0) {
    drop_rht(sys);
    return r;
  }
  HIP_TRY(hipStreamSynchronize(st));   // the signs' host copy goes out of scope
  r = kpp_system_create(sys->ctx, sys->kind, R, cols, sys->rht_A, cols, sys->rht_b, &sys->rht_inner);
  if (r < 0) {
    drop_rht(sys);
    return r;
  }
  sys->rht_R = R;
  sys->rht_seed = seed;
  *built = true;
  return KPP_OK;
}

kpp_status solve_rht(kpp_system* sys, const kpp_params* p, double* x, kpp_result* res) {
  bool built = false;
  KPP_TRY(prepare_rht(sys, p->rht_seed, &built));
  sys->res_valid = false;
  hipStream_t st = sys->ctx->stream;
  kpp_params q = *p;
  q.rht = 0;
  kpp_result r{};
  kpp_status out;
  if (sys->kind == KPP_CD_PSD) {
    const int64_t R = sys->rht_R;
    KPP_TRY(rht_vector(st, R, sys->rht_signs, x, sys->n, sys->rht_x, false, nullptr));
    out = kpp_solve(sys->rht_inner, &q, sys->rht_x, &r);
    if (out < 0) return out;
    KPP_TRY(rht_vector(st, R, sys->rht_signs, sys->rht_x, sys->n, x, true, sys->rht_work));
  } else {
    out = kpp_solve(sys->rht_inner, &q, x, &r);
    if (out < 0) return out;
  }
  double rn = 0.0;
  KPP_TRY(residual_norm(sys, x, &rn));
  r.true_rel_res = rn / (sys->bnorm > 0.0 ? sys->bnorm : 1.0);
  // the inner solve confirmed its stop on the transformed system; the result
  // counts as converged only if the original system agrees
  if (out == KPP_OK && p->tol > 0.0 && !(r.true_rel_res <= p->tol)) {
    out = KPP_NOT_CONVERGED;
    r.converged = 0;
  }
  // the transforms' additions: A and b when this solve formed them, and for
  // CD++ the iterate in and out
  const double Rd = static_cast<double>(sys->rht_R);
  if (sys->kind == KPP_CD_PSD) {
    if (built) r.flops += symfht_adds(sys->rht_R) + fht_adds(Rd, 1.0);
    r.flops += 2.0 * fht_adds(Rd, 1.0);
  } else if (built) {
    r.flops += fht_adds(Rd, static_cast<double>(sys->n)) + fht_adds(Rd, 1.0);
  }
  if (res) *res = r;
  return out;
}

}  // namespace

KPP_API kpp_status kpp_rht_signs(uint64_t seed, int64_t N, int8_t* signs_host) {
  if (N < 0 || (N > 0 && !signs_host)) return fail(KPP_ERR_INVALID_ARG, "N < 0 or NULL output");
  draw_signs(seed, N, signs_host);
  return KPP_OK;
}

KPP_API kpp_status kpp_rht_general(kpp_context* ctx, int64_t m, int64_t n, const double* A, int64_t lda,
                                   const double* b, const int8_t* signs, int64_t R, double* At, int64_t ldt,
                                   double* bt) {
  if (!ctx || !A || !b || !signs || !At || !bt) return fail(KPP_ERR_INVALID_ARG, "NULL argument");
  if (m < 1 || n < 1) return fail(KPP_ERR_SHAPE, "empty matrix");
  if (lda < n || ldt < n) return fail(KPP_ERR_INVALID_ARG, "leading dimension below n");
  KPP_TRY(check_rht_size(m, R));
  HIP_TRY(hipSetDevice(ctx->device));
  return rht_general(ctx->stream, m, n, A, lda, b, signs, R, At, ldt, bt);
}

KPP_API kpp_status kpp_rht_psd(kpp_context* ctx, int64_t n, const double* A, int64_t lda, const double* b,
                               const int8_t* signs, int64_t R, double* At, int64_t ldt, double* bt,
                               double* work) {
  if (!ctx || !A || !b || !signs || !At || !bt) return fail(KPP_ERR_INVALID_ARG, "NULL argument");
  if (n < 1) return fail(KPP_ERR_SHAPE, "empty matrix");
  if (lda < n || ldt < R) return fail(KPP_ERR_INVALID_ARG, "leading dimension too small");
  KPP_TRY(check_rht_size(n, R));
  if (kpp::fht_passes(R) > 1 && !work) return fail(KPP_ERR_INVALID_ARG, "R > 4096 needs R x R doubles of work");
  HIP_TRY(hipSetDevice(ctx->device));
  return rht_psd(ctx->stream, n, A, lda, b, signs, R, At, ldt, bt, work);
}

KPP_API kpp_status kpp_rht_vector(kpp_context* ctx, int64_t R, const int8_t* signs, const double* x, int64_t nx,
                                  double* y, int32_t direction, double* work) {
  if (!ctx || !signs || !x || !y) return fail(KPP_ERR_INVALID_ARG, "NULL argument");
  if (direction != 0 && direction != 1) return fail(KPP_ERR_INVALID_ARG, "direction must be 0 or 1");
  if (nx < 1) return fail(KPP_ERR_SHAPE, "empty vector");
  KPP_TRY(check_rht_size(nx, R));
  if (direction == 1 && nx < R && kpp::fht_passes(R) > 1 && !work)
    return fail(KPP_ERR_INVALID_ARG, "R > 4096 with nx < R needs R doubles of work");
  HIP_TRY(hipSetDevice(ctx->device));
  return rht_vector(ctx->stream, R, signs, x, nx, y, direction == 1, work);
}

// ---------------------------------------------------------------------------
// several right-hand sides on one system (the multi-RHS form): one schedule,
// one memo, one pass over A_S per step for all of them
// ---------------------------------------------------------------------------
namespace {

extern "C++" {
// a device array freed when it goes out of scope
template <class T>
struct DevVec {
  T* p = nullptr;
  ~DevVec() { dev_free(p); }
  kpp_status alloc(size_t count) {
    dev_free(p);
    return dev_alloc(&p, count);
  }
};
}

kpp_status solve_multi(kpp_system* sys, const kpp_params* p, int32_t k, const double* B, int64_t ldb, double* X,
                       int64_t ldx, kpp_result* res) {
  using clock = std::chrono::steady_clock;
  const auto t_begin = clock::now();
  hipStream_t st = sys->ctx->stream;
  const int32_t kind = sys->kind;
  const int64_t m = sys->m, n = sys->n, N = kind == KPP_CD_PSD ? n : m;
  const int32_t s = p->block_size;
  const int32_t zeta = static_cast<int32_t>((N + s - 1) / s);
  const int64_t period = 2 * static_cast<int64_t>(zeta);
  double eta = p->eta < 0.0 ? default_eta(kind, m, n, s) : p->eta;
  if (!p->accel) eta = 0.0;
  const auto mode = static_cast<kpp::MemoMode>(p->memo);
  kpp::BlockSchedule sch(mode, N, s, p->seed, kpp::online_rate(kind, m, n, s), p->num_blocks,
                         p->fixed_partition != 0);
  const int32_t P = kpp::gemm_parts(n);
  const int64_t stride = kpp::slot_doubles(s);
  // ||b_c|| on the host
  std::vector<double> hb(static_cast<size_t>(m) * ldb);
  HIP_TRY(hipMemcpy(hb.data(), B, hb.size() * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<double> bn(k, 0.0);
  for (int64_t i = 0; i < m; ++i)
    for (int32_t c = 0; c < k; ++c) bn[c] += hb[static_cast<size_t>(i) * ldb + c] * hb[static_cast<size_t>(i) * ldb + c];
  for (auto& v : bn) v = std::sqrt(v);
  DevVec<double> mom, rpart, Y, xcol, bcol, rowsq, scal, ws, L;
  DevVec<kpp::DevState> ds;
  DevVec<int32_t> frozen, err, rows, lens, ids;
  KPP_TRY(mom.alloc(static_cast<size_t>(n) * k));
  KPP_TRY(rpart.alloc(static_cast<size_t>(s) * P * k));
  KPP_TRY(Y.alloc(static_cast<size_t>(k) * s));
  KPP_TRY(xcol.alloc(n));
  KPP_TRY(bcol.alloc(m));
  KPP_TRY(rowsq.alloc(m));
  KPP_TRY(scal.alloc(4));
  KPP_TRY(ds.alloc(k));
  KPP_TRY(frozen.alloc(k));
  KPP_TRY(err.alloc(1));
  if (kind == KPP_KACZMARZ) KPP_TRY(ws.alloc(kpp::gram_syrk_work(s, n, static_cast<int32_t>(period))));
  HIP_TRY(hipMemsetAsync(mom.p, 0, static_cast<size_t>(n) * k * sizeof(double), st));
  HIP_TRY(hipMemsetAsync(frozen.p, 0, k * sizeof(int32_t), st));
  HIP_TRY(hipMemsetAsync(err.p, 0, sizeof(int32_t), st));
  std::vector<kpp::DevState> hds(k);
  for (int32_t c = 0; c < k; ++c) {
    kpp::DevState d{};
    d.rho = p->rho0;
    d.c = (1.0 - p->rho0) / (1.0 + p->rho0);
    d.rho_before = p->rho0;
    d.thr = p->tol * p->tol * bn[c] * bn[c];
    hds[c] = d;
  }
  HIP_TRY(hipMemcpy(ds.p, hds.data(), k * sizeof(kpp::DevState), hipMemcpyHostToDevice));
  // memo slots (one for every block in OFF mode: factored at every step)
  int64_t cap = period;   // OFF: the blocks of one window
  if (mode == kpp::MemoMode::Fixed) cap = sch.num_blocks();
  if (mode == kpp::MemoMode::Online) cap = std::min<int64_t>(static_cast<int64_t>(4.0 * kpp::online_rate(kind, m, n, s)) + 16,
                                                            std::max<int64_t>(16, p->max_iters + 1));
  cap = std::max<int64_t>(cap, 1);
  auto grow = [&](int64_t want) -> kpp_status {
    if (want <= cap && L.p) return KPP_OK;
    const int64_t nc = std::max(want, L.p ? 2 * cap : cap);
    HIP_TRY(hipStreamSynchronize(st));
    DevVec<double> L2;
    DevVec<int32_t> r2, l2, i2;
    KPP_TRY(L2.alloc(static_cast<size_t>(nc) * stride));
    KPP_TRY(r2.alloc(static_cast<size_t>(nc) * s));
    KPP_TRY(l2.alloc(nc));
    KPP_TRY(i2.alloc(nc));
    if (L.p) {
      HIP_TRY(hipMemcpy(L2.p, L.p, static_cast<size_t>(cap) * stride * sizeof(double), hipMemcpyDeviceToDevice));
      HIP_TRY(hipMemcpy(r2.p, rows.p, static_cast<size_t>(cap) * s * sizeof(int32_t), hipMemcpyDeviceToDevice));
      HIP_TRY(hipMemcpy(l2.p, lens.p, static_cast<size_t>(cap) * sizeof(int32_t), hipMemcpyDeviceToDevice));
    }
    std::vector<int32_t> iota(static_cast<size_t>(nc));
    std::iota(iota.begin(), iota.end(), 0);
    HIP_TRY(hipMemcpy(i2.p, iota.data(), iota.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    std::swap(L.p, L2.p);
    std::swap(rows.p, r2.p);
    std::swap(lens.p, l2.p);
    std::swap(ids.p, i2.p);
    cap = nc;
    return KPP_OK;
  };
  KPP_TRY(grow(cap));
  std::vector<int32_t> slot_of;
  std::vector<int32_t> stage_rows, stage_lens;
  std::vector<int32_t> hfrozen(k, 0);
  std::vector<int64_t> iters(k, -1);
  std::vector<double> true_rel(k, NAN);
  int64_t t = 0, hits = 0, misses = 0;
  int32_t used = 0;
  auto confirm = [&](int32_t c, double* out) -> kpp_status {
    kpp::launch_column(X, ldx, n, c, xcol.p, st);
    kpp::launch_column(B, ldb, m, c, bcol.p, st);
    kpp::launch_residual_sq(sys->A, sys->lda, m, n, xcol.p, bcol.p, rowsq.p, 0, scal.p, st);
    HIP_TRY(hipGetLastError());
    double v = 0.0;
    HIP_TRY(hipMemcpyAsync(&v, scal.p, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *out = std::sqrt(v);
    return KPP_OK;
  };
  int32_t active = k;
  std::vector<int32_t> wblock, wslot;
  while (t < p->max_iters && active > 0) {
    // one checkpoint window: its steps drawn first (the schedule never looks
    // at x), its new blocks factored in one batch, then its steps
    const int64_t W = std::min<int64_t>(period - t % period, p->max_iters - t);
    wblock.assign(W, 0);
    wslot.assign(W, 0);
    stage_rows.clear();
    stage_lens.clear();
    int32_t q0 = -1, nb = 0;
    for (int64_t j = 0; j < W; ++j) {
      bool is_new = false;
      const int32_t b = sch.next(&is_new);
      wblock[j] = b;
      int32_t q;
      bool fresh = true;
      if (mode == kpp::MemoMode::Off) {
        q = static_cast<int32_t>(j);
      } else {
        if (static_cast<int32_t>(slot_of.size()) <= b) slot_of.resize(b + 1, -1);
        if (slot_of[b] < 0) {
          KPP_TRY(grow(used + 1));
          slot_of[b] = used++;
        } else {
          fresh = false;
        }
        q = slot_of[b];
      }
      wslot[j] = q;
      if (fresh) {
        if (q0 < 0) q0 = q;   // new slots of a window are consecutive
        const int32_t sb = sch.len(b);
        stage_rows.insert(stage_rows.end(), sch.rows(b), sch.rows(b) + sb);
        stage_rows.insert(stage_rows.end(), static_cast<size_t>(s - sb), 0);
        stage_lens.push_back(sb);
        ++nb;
        ++misses;
      } else {
        ++hits;
      }
    }
    if (nb > 0) {
      HIP_TRY(hipMemcpy(rows.p + static_cast<size_t>(q0) * s, stage_rows.data(), stage_rows.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(lens.p + q0, stage_lens.data(), stage_lens.size() * sizeof(int32_t), hipMemcpyHostToDevice));
      kpp::launch_gram(kind, sys->A, sys->lda, n, rows.p + static_cast<size_t>(q0) * s, lens.p + q0, s, nb, p->lambda,
                       L.p, stride, ids.p + q0, ws.p, st);
      if (s <= kpp::kFactorSmallMax) {
        kpp::launch_factor_small(L.p, stride, s, lens.p + q0, nb, ids.p + q0, 1, err.p, st);
      } else {
        kpp::launch_cholesky(L.p, s, stride, lens.p + q0, nb, ids.p + q0, err.p, st);
        kpp::launch_factor_inverse(L.p, stride, s, lens.p + q0, nb, ids.p + q0, st);
      }
    }
    for (int64_t j = 0; j < W; ++j) {
      const int32_t q = wslot[j];
      const int32_t sb = sch.len(wblock[j]);
      const int32_t* r = rows.p + static_cast<size_t>(q) * s;
      const double* Gi = L.p + static_cast<size_t>(q) * stride + static_cast<size_t>(s) * s;
      kpp::launch_block_gemm_partial(sys->A, sys->lda, n, r, sb, X, ldx, k, rpart.p, P, st);
      kpp::launch_block_project_multi(rpart.p, P, k, B, ldb, r, sb, Gi, s, Y.p, ds.p, frozen.p, zeta,
                                      p->adaptive_rho, st);
      kpp::launch_update_multi(kind, sys->A, sys->lda, n, r, sb, Y.p, s, k, ds.p, frozen.p, eta, X, ldx, mom.p, st);
    }
    HIP_TRY(hipGetLastError());
    t += W;
    {
      int32_t herr = 0;
      HIP_TRY(hipMemcpyAsync(hds.data(), ds.p, k * sizeof(kpp::DevState), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(&herr, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (herr) return fail(KPP_ERR_NOT_SPD, "a regularized block Gram has no Cholesky factor (lambda=%g)", p->lambda);
      bool changed = false;
      for (int32_t c = 0; c < k; ++c) {
        if (hfrozen[c] || !(t % period == 0 && hds[c].cand)) continue;
        double rn = 0.0;
        if (p->confirm_true_residual) KPP_TRY(confirm(c, &rn));
        if (!p->confirm_true_residual || rn <= p->tol * bn[c]) {
          hfrozen[c] = 1;
          iters[c] = t;
          true_rel[c] = p->confirm_true_residual ? rn / (bn[c] > 0.0 ? bn[c] : 1.0) : NAN;
          --active;
          changed = true;
        }
      }
      if (changed && active > 0)
        HIP_TRY(hipMemcpy(frozen.p, hfrozen.data(), k * sizeof(int32_t), hipMemcpyHostToDevice));
    }
  }
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipMemcpy(hds.data(), ds.p, k * sizeof(kpp::DevState), hipMemcpyDeviceToHost));
  bool all = true;
  for (int32_t c = 0; c < k; ++c) {
    if (!hfrozen[c]) {
      iters[c] = t;
      all = false;
    }
    if (std::isnan(true_rel[c])) {
      double rn = 0.0;
      KPP_TRY(confirm(c, &rn));
      true_rel[c] = rn / (bn[c] > 0.0 ? bn[c] : 1.0);
    }
  }
  const double seconds = std::chrono::duration<double>(clock::now() - t_begin).count();
  if (res) {
    for (int32_t c = 0; c < k; ++c) {
      kpp_result& r = res[c];
      std::memset(&r, 0, sizeof(r));
      CoreStats cs{};
      cs.engine = 1;
      fill_result(&r, sys, p, iters[c], hits, misses, hfrozen[c] != 0, 0, cs, true_rel[c],
                  std::sqrt(hds[c].last_E1) / (bn[c] > 0.0 ? bn[c] : 1.0), hds[c].rho, seconds, 0.0, 0.0,
                  3 * t, hds[c].ckpts, 8.0);
    }
  }
  return all ? KPP_OK : KPP_NOT_CONVERGED;
}

}  // namespace

KPP_API kpp_status kpp_solve_multi(kpp_system* sys, const kpp_params* p, int32_t k, const double* B_dev, int64_t ldb,
                                   double* X_dev, int64_t ldx, kpp_result* res) {
  if (!sys || !B_dev || !X_dev) return fail(KPP_ERR_INVALID_ARG, "NULL system, B or X");
  if (sys->csr) return fail(KPP_ERR_INVALID_ARG, "several right-hand sides take a dense system");
  if (k < 1 || k > kpp::kMaxRhs) return fail(KPP_ERR_INVALID_ARG, "k must be in [1, %d]", kpp::kMaxRhs);
  if (ldb < k || ldx < k) return fail(KPP_ERR_INVALID_ARG, "leading dimensions must be >= k");
  KPP_TRY(check_params(sys, p));
  if (p->precision != KPP_FP64 || p->rht || p->projection || p->resume || p->schedule)
    return fail(KPP_ERR_INVALID_ARG, "several right-hand sides: FP64 with the seeded schedule only");
  HIP_TRY(hipSetDevice(sys->ctx->device));
  sys->res_valid = false;
  try {
    return solve_multi(sys, p, k, B_dev, ldb, X_dev, ldx, res);
  } catch (const std::bad_alloc&) {
    return fail(KPP_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(KPP_ERR_INVALID_ARG, "%s", e.what());
  }
}

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
  p->refine_max_rounds = 40;
  // Kaczmarz++ 1e-3 (the 2048 x 32768 workload: 17.2-18.1 ms to 1e-10 over three schedule
  // seeds, 18.4-29.2 ms at 1e-2), CD++ 1e-2 (the fastest on the n = 4096 workload)
  p->inner_tol = kind == KPP_KACZMARZ ? 1e-3 : 1e-2;
  p->engine = 0;
  p->team_groups = 0;
  p->lsqr_iters = 8;
  p->sketch_seed = 0x5ca7c4ull;
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
  void* scr = nullptr;
  const hipError_t se = kpp::noalloc_scratch(device, &scr);
  if (se != hipSuccess || !scr) {
    (void)hipStreamDestroy(c->side);
    delete c;
    return fail(KPP_ERR_HIP, "no device address for the scratch array on device %d: %s", device,
                hipGetErrorString(se));
  }
  c->scratch = static_cast<unsigned char*>(scr);
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

namespace {

// The buffers every system holds (momentum, state, staging events, flags).
kpp_status alloc_system(kpp_context* ctx, int32_t kind, int64_t m, int64_t n, const double* b_dev,
                        std::unique_ptr<kpp_system>* out) {
  HIP_TRY(hipSetDevice(ctx->device));
  std::unique_ptr<kpp_system> sys(new (std::nothrow) kpp_system);
  if (!sys) return fail(KPP_ERR_OOM, "host allocation failed");
  sys->ctx = ctx;
  sys->kind = kind;
  sys->m = m;
  sys->n = n;
  sys->b = b_dev;
  kpp_status stt;
  if ((stt = dev_alloc(&sys->mom, n)) < 0 || (stt = dev_alloc(&sys->ds, 1)) < 0 ||
      (stt = dev_alloc(&sys->y, kpp::kMaxBlock)) < 0 || (stt = dev_alloc(&sys->rowsq, m)) < 0 ||
      (stt = dev_alloc(&sys->scal, 4)) < 0 || (stt = dev_alloc(&sys->err, 4)) < 0 ||
      (stt = dev_alloc(&sys->part, kpp::kPartDoubles)) < 0 ||
      (stt = dev_alloc(&sys->flags, kFlagWords)) < 0) {
    destroy_buffers(sys.get());
    return stt;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&sys->h_ds), sizeof(kpp::DevState), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&sys->h_err), 2 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&sys->h_mirror), 2 * sizeof(kpp::HostMirror),
                    hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
    destroy_buffers(sys.get());
    return fail(KPP_ERR_OOM, "pinned host allocation failed");
  }
  std::memset(sys->h_mirror, 0, 2 * sizeof(kpp::HostMirror));
  if (hipHostGetDevicePointer(reinterpret_cast<void**>(&sys->d_mirror), sys->h_mirror, 0) != hipSuccess) {
    destroy_buffers(sys.get());
    return fail(KPP_ERR_HIP, "hipHostGetDevicePointer failed");
  }
  for (auto& e : sys->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      destroy_buffers(sys.get());
      return fail(KPP_ERR_HIP, "hipEventCreate failed");
    }
  }
  for (auto& e : sys->ev_win) {
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
  if (hipMemsetAsync(sys->flags, 0, kFlagWords * sizeof(uint32_t), ctx->stream) != hipSuccess ||
      hipMemsetAsync(sys->err, 0, sizeof(int32_t), ctx->stream) != hipSuccess) {
    destroy_buffers(sys.get());
    return fail(KPP_ERR_HIP, "hipMemsetAsync failed");
  }
  *out = std::move(sys);
  return KPP_OK;
}

// Frees a system's buffers on every early return of its creation.
struct SystemGuard {
  std::unique_ptr<kpp_system>& sys;
  ~SystemGuard() {
    if (sys) destroy_buffers(sys.get());
  }
};

// ||b|| on the host (b is m doubles on the device).
kpp_status host_bnorm(kpp_system* sys) {
  hipStream_t st = sys->ctx->stream;
  std::vector<double> hb(sys->m);
  HIP_TRY(hipMemcpyAsync(hb.data(), sys->b, sys->m * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double bb = 0.0;
  for (double v : hb) bb += v * v;
  sys->bnorm = std::sqrt(bb);
  return KPP_OK;
}

}  // namespace

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
  std::unique_ptr<kpp_system> sys;
  KPP_TRY(alloc_system(ctx, kind, m, n, b_dev, &sys));
  SystemGuard guard{sys};
  sys->lda = lda;
  sys->A = A_dev;
  hipStream_t st = ctx->stream;
  // finiteness of A and b, and ||b||
  kpp::launch_check_finite(A_dev, lda, m, n, b_dev, sys->err, st);
  HIP_TRY(hipGetLastError());
  int32_t bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, sys->err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (bad) return fail(KPP_ERR_NONFINITE, "A or b holds NaN or Inf");
  KPP_TRY(host_bnorm(sys.get()));
  *out = sys.release();
  return KPP_OK;
}

KPP_API kpp_status kpp_system_create_csr(kpp_context* ctx, int32_t kind, int64_t m, int64_t n, int64_t nnz,
                                         const int64_t* row_ptr_dev, const int32_t* col_dev, const double* val_dev,
                                         const double* b_dev, kpp_system** out) {
  if (!out) return fail(KPP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx || !row_ptr_dev || !b_dev) return fail(KPP_ERR_INVALID_ARG, "NULL context, row pointers or b");
  if (nnz < 0) return fail(KPP_ERR_SHAPE, "nnz=%lld < 0", (long long)nnz);
  if (nnz > 0 && (!col_dev || !val_dev)) return fail(KPP_ERR_INVALID_ARG, "NULL column indices or values");
  if (kind != KPP_KACZMARZ && kind != KPP_CD_PSD) return fail(KPP_ERR_INVALID_ARG, "unknown kind %d", kind);
  if (m < 1 || n < 1) return fail(KPP_ERR_SHAPE, "empty system (m=%lld, n=%lld)", (long long)m, (long long)n);
  if (kind == KPP_CD_PSD && m != n) return fail(KPP_ERR_SHAPE, "CD++ needs a square matrix");
  if (m > (int64_t{1} << 31) - 1 || n > (int64_t{1} << 31) - 1) return fail(KPP_ERR_SHAPE, "dimension above 2^31-1");
  std::unique_ptr<kpp_system> sys;
  KPP_TRY(alloc_system(ctx, kind, m, n, b_dev, &sys));
  SystemGuard guard{sys};
  sys->csr = true;
  sys->csr_rp = row_ptr_dev;
  sys->csr_ci = col_dev;
  sys->csr_cv = val_dev;
  sys->nnz = nnz;
  // team of one workgroup per 256 columns, at most kSparseTeamMax
  sys->csr_G = static_cast<int32_t>(std::min<int64_t>(kpp::kSparseTeamMax, std::max<int64_t>(1, (n + 255) / 256)));
  KPP_TRY(dev_alloc(&sys->csr_xr, 2 * static_cast<size_t>(sys->csr_G) * kpp::kMaxBlock));
  KPP_TRY(dev_alloc(&sys->csr_xy, 2 * static_cast<size_t>(kpp::kMaxBlock)));
  hipStream_t st = ctx->stream;
  kpp::launch_csr_check(row_ptr_dev, col_dev, val_dev, b_dev, m, n, nnz, sys->err, st);
  HIP_TRY(hipGetLastError());
  int32_t bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, sys->err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (bad & 3)
    return fail(KPP_ERR_SHAPE, (bad & 1) ? "row pointers are not a CSR layout of nnz entries"
                                         : "a column index is out of range or not increasing within its row");
  if (bad) return fail(KPP_ERR_NONFINITE, "the values or b hold NaN or Inf");
  HIP_TRY(hipMemsetAsync(sys->err, 0, sizeof(int32_t), st));
  try {
    sys->h_rp.resize(static_cast<size_t>(m) + 1);
  } catch (const std::bad_alloc&) {
    return fail(KPP_ERR_OOM, "host allocation failed");
  }
  HIP_TRY(hipMemcpyAsync(sys->h_rp.data(), row_ptr_dev, (m + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  KPP_TRY(host_bnorm(sys.get()));
  *out = sys.release();
  return KPP_OK;
}

KPP_API kpp_status kpp_system_destroy(kpp_system* sys) {
  if (!sys) return KPP_OK;
  if (sys->ctx) (void)hipSetDevice(sys->ctx->device);
  if (sys->ctx) (void)hipStreamSynchronize(sys->ctx->stream);
  if (sys->ctx && sys->ctx->side) (void)hipStreamSynchronize(sys->ctx->side);
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
    if (p->rht) return solve_rht(sys, p, x_dev, res);
    if (p->precision != KPP_FP64) return solve_mixed(sys, p, x_dev, res);
    return solve_fp64(sys, p, x_dev, res);
  } catch (const std::bad_alloc&) {
    return fail(KPP_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(KPP_ERR_INVALID_ARG, "%s", e.what());
  }
}

namespace {
constexpr uint32_t kStateMagic = 0x4b505358u;   // "KPSX"
constexpr uint32_t kStateVersion = 1;
struct StateHeader {
  uint32_t magic, version;
  int32_t kind, s;
  int64_t m, n, t;
  uint64_t sched_bytes;
};
}  // namespace

KPP_API kpp_status kpp_state_export(const kpp_system* sys, void* host_buf, size_t* bytes) {
  if (!sys || !bytes) return fail(KPP_ERR_INVALID_ARG, "NULL argument");
  if (!sys->res_valid || !sys->res_sch) return fail(KPP_ERR_INVALID_ARG, "the system holds no solver state");
  std::vector<uint8_t> sched;
  try {
    sys->res_sch->save(&sched);
  } catch (const std::bad_alloc&) {
    return fail(KPP_ERR_OOM, "host allocation failed");
  }
  const size_t need = sizeof(StateHeader) + sizeof(kpp::DevState) + static_cast<size_t>(sys->n) * sizeof(double) +
                      sched.size();
  if (!host_buf) {
    *bytes = need;
    return KPP_OK;
  }
  if (*bytes < need) return fail(KPP_ERR_INVALID_ARG, "buffer of %zu bytes, %zu needed", *bytes, need);
  HIP_TRY(hipSetDevice(sys->ctx->device));
  StateHeader h{kStateMagic, kStateVersion, sys->kind, sys->res_s, sys->m, sys->n, sys->res_t, sched.size()};
  uint8_t* out = static_cast<uint8_t*>(host_buf);
  std::memcpy(out, &h, sizeof h);
  std::memcpy(out + sizeof h, &sys->res_ds, sizeof(kpp::DevState));
  double* mom = reinterpret_cast<double*>(out + sizeof h + sizeof(kpp::DevState));
  HIP_TRY(hipStreamSynchronize(sys->ctx->stream));
  HIP_TRY(hipMemcpy(mom, sys->mom, static_cast<size_t>(sys->n) * sizeof(double), hipMemcpyDeviceToHost));
  std::memcpy(out + sizeof h + sizeof(kpp::DevState) + static_cast<size_t>(sys->n) * sizeof(double), sched.data(),
              sched.size());
  *bytes = need;
  return KPP_OK;
}

KPP_API kpp_status kpp_state_import(kpp_system* sys, const void* host_buf, size_t bytes) {
  if (!sys || !host_buf) return fail(KPP_ERR_INVALID_ARG, "NULL argument");
  StateHeader h;
  if (bytes < sizeof h) return fail(KPP_ERR_INVALID_ARG, "state buffer too short");
  const uint8_t* in = static_cast<const uint8_t*>(host_buf);
  std::memcpy(&h, in, sizeof h);
  if (h.magic != kStateMagic || h.version != kStateVersion) return fail(KPP_ERR_INVALID_ARG, "not a solver state");
  if (h.kind != sys->kind || h.m != sys->m || h.n != sys->n)
    return fail(KPP_ERR_SHAPE, "the state belongs to a %lld x %lld system of kind %d", static_cast<long long>(h.m),
                static_cast<long long>(h.n), h.kind);
  const size_t need = sizeof h + sizeof(kpp::DevState) + static_cast<size_t>(sys->n) * sizeof(double) + h.sched_bytes;
  if (bytes != need) return fail(KPP_ERR_INVALID_ARG, "state buffer of %zu bytes, %zu expected", bytes, need);
  kpp::DevState ds;
  std::memcpy(&ds, in + sizeof h, sizeof ds);
  std::unique_ptr<kpp::BlockSchedule> sch;
  try {
    sch.reset(new kpp::BlockSchedule(kpp::BlockSchedule::load(
        in + sizeof h + sizeof(kpp::DevState) + static_cast<size_t>(sys->n) * sizeof(double), h.sched_bytes)));
  } catch (const std::exception& e) {
    return fail(KPP_ERR_INVALID_ARG, "%s", e.what());
  }
  const int64_t rows = sys->kind == KPP_CD_PSD ? sys->n : sys->m;
  if (sch->block_size() != h.s || h.t < 0 || ds.t != h.t)
    return fail(KPP_ERR_INVALID_ARG, "inconsistent solver state");
  for (int32_t b = 0; b < sch->num_blocks(); ++b)
    if (sch->rows(b)[sch->len(b) - 1] >= rows) return fail(KPP_ERR_INVALID_ARG, "inconsistent solver state");
  HIP_TRY(hipSetDevice(sys->ctx->device));
  HIP_TRY(hipStreamSynchronize(sys->ctx->stream));
  HIP_TRY(hipMemcpy(sys->mom, in + sizeof h + sizeof(kpp::DevState), static_cast<size_t>(sys->n) * sizeof(double),
                    hipMemcpyHostToDevice));
  sys->res_ds = ds;
  sys->res_t = h.t;
  sys->res_s = h.s;
  sys->res_sch = std::move(sch);
  sys->res_valid = true;
  sys->memo_valid = false;   // factors are formed again on first use
  return KPP_OK;
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
    if (p->schedule && T > p->schedule_len)
      return fail(KPP_ERR_INVALID_ARG, "T = %lld exceeds schedule_len", static_cast<long long>(T));
    kpp::BlockSchedule sch = p->schedule
        ? kpp::BlockSchedule(N, s, p->block_rows, p->block_rows_count, p->schedule, p->schedule_len)
        : kpp::BlockSchedule(static_cast<kpp::MemoMode>(p->memo), N, s, p->seed, kpp::online_rate(kind, m, n, s),
                             p->num_blocks, p->fixed_partition != 0);
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
  if (sys->csr && sys->kind == KPP_CD_PSD)
    for (int32_t b = 0; b < nb; ++b)
      for (int32_t i = 1; i < len_host[b]; ++i)
        if (rows_host[static_cast<size_t>(b) * s + i] <= rows_host[static_cast<size_t>(b) * s + i - 1])
          return fail(KPP_ERR_INVALID_ARG, "block %d: rows of a sparse CD++ block must ascend", b);
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
  kpp::CscArena ar;
  int32_t *d_meta = nullptr, *d_nu = nullptr;
  double* d_ws = nullptr;
  if (sys->csr && sys->kind == KPP_KACZMARZ) {
    // the memo-miss kernel of sparse Kaczmarz++ blocks, with an arena and
    // build workspace of this call's own
    std::vector<int32_t> meta(static_cast<size_t>(kpp::kCsrMetaInts) * nb);
    int64_t total = 0;
    size_t wsd = 0;
    bool any_lds = false, any_global = false;
    for (int32_t b = 0; b < nb; ++b) {
      int64_t z = 0;
      for (int32_t i = 0; i < len_host[b]; ++i) {
        const int32_t r = rows_host[static_cast<size_t>(b) * s + i];
        z += sys->h_rp[r + 1] - sys->h_rp[r];
      }
      if (z > kpp::kCsrMaxBlockNnz) return fail(KPP_ERR_SHAPE, "block %d holds %lld nonzeros", b, (long long)z);
      int64_t wso = -1;
      if (z > kpp::kCsrLdsEntries) {
        wso = static_cast<int64_t>(wsd);
        wsd += kpp::csr_build_ws_doubles(z);
        any_global = true;
      } else {
        any_lds = true;
      }
      int32_t* mk = meta.data() + static_cast<size_t>(kpp::kCsrMetaInts) * b;
      kpp::csr_meta_put(mk, total);
      mk[2] = static_cast<int32_t>(z);
      kpp::csr_meta_put(mk + 3, wso);
      total += z + 1;
    }
    KPP_TRY(dev_alloc(&ar.val, total));
    KPP_TRY(dev_alloc(&ar.row, total));
    KPP_TRY(dev_alloc(&ar.col, total));
    KPP_TRY(dev_alloc(&ar.ptr, total));
    KPP_TRY(dev_alloc(&d_nu, nb));
    KPP_TRY(dev_alloc(&d_meta, meta.size()));
    if (wsd > 0) KPP_TRY(dev_alloc(&d_ws, wsd));
    HIP_TRY(hipMemcpyAsync(d_meta, meta.data(), meta.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    kpp::launch_csr_block_build(sys->csr_rp, sys->csr_ci, sys->csr_cv, d_rows, d_lens, d_ids, d_meta, nb, s, lambda,
                                L_dev, static_cast<int64_t>(s) * s, ar, d_nu, d_ws, any_lds, any_global, sys->err, st);
  } else if (sys->csr) {
    kpp::launch_csr_gram_cd(sys->csr_rp, sys->csr_ci, sys->csr_cv, d_rows, d_lens, d_ids, nb, s, lambda, L_dev,
                            static_cast<int64_t>(s) * s, st);
  } else {
    if (sys->kind == KPP_KACZMARZ) KPP_TRY(ensure_gram_ws(sys, 0, kpp::gram_syrk_work(s, sys->n, nb)));
    kpp::launch_gram(sys->kind, sys->A, sys->lda, sys->n, d_rows, d_lens, s, nb, lambda, L_dev,
                     static_cast<int64_t>(s) * s, d_ids, sys->gram_ws[0], st);
  }
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
  dev_free(ar.val);
  dev_free(ar.row);
  dev_free(ar.col);
  dev_free(ar.ptr);
  dev_free(d_nu);
  dev_free(d_meta);
  dev_free(d_ws);
  if (herr & 4) return fail(KPP_ERR_INVALID_ARG, "the sparse matrix's row pointers changed after the system was created");
  if (herr) return fail(KPP_ERR_NOT_SPD, "a regularized block Gram has no Cholesky factor");
  return KPP_OK;
}

// Scratch layout of kpp_block_factor_noalloc: the breakdown flag, then the
// staged rows, lengths and slot ids, then the split-Gram workspace.
constexpr size_t kNaStageOffset = 256;
constexpr size_t kNaGramOffset = size_t{1} << 20;
constexpr int64_t kNaStageInts = static_cast<int64_t>((kNaGramOffset - kNaStageOffset) / sizeof(int32_t));
constexpr size_t kNaGramDoubles = (kpp::kNoAllocScratchBytes - kNaGramOffset) / sizeof(double);

KPP_API kpp_status kpp_block_factor_noalloc(kpp_system* sys, int32_t s, double lambda, int32_t nb,
                                            const int32_t* rows_host, const int32_t* len_host, double* L_dev) {
  if (!sys || !rows_host || !len_host || !L_dev || nb < 0) return fail(KPP_ERR_INVALID_ARG, "bad arguments");
  if (sys->csr) return fail(KPP_ERR_INVALID_ARG, "the no-allocation factor takes a dense system");
  const int64_t N = sys->kind == KPP_CD_PSD ? sys->n : sys->m;
  if (s < 1 || s > kpp::kMaxBlock) return fail(KPP_ERR_INVALID_ARG, "block size %d out of range", s);
  if (!(lambda >= 0.0)) return fail(KPP_ERR_INVALID_ARG, "lambda must be >= 0");
  if (static_cast<int64_t>(nb) * (s + 2) > kNaStageInts)
    return fail(KPP_ERR_INVALID_ARG,
                "nb * (s + 2) = %lld exceeds the %lld entries the no-allocation scratch stages",
                static_cast<long long>(nb) * (s + 2), static_cast<long long>(kNaStageInts));
  for (int32_t b = 0; b < nb; ++b) {
    if (len_host[b] < 1 || len_host[b] > s) return fail(KPP_ERR_INVALID_ARG, "block %d length %d", b, len_host[b]);
    for (int32_t i = 0; i < len_host[b]; ++i) {
      const int32_t r = rows_host[static_cast<size_t>(b) * s + i];
      if (r < 0 || r >= N) return fail(KPP_ERR_INVALID_ARG, "block %d row %d out of range", b, r);
    }
  }
  if (nb == 0) return KPP_OK;
  const int32_t ng = kpp::gram_groups(s);
  const size_t per_block = static_cast<size_t>(ng) * (ng + 1) / 2 * kpp::kGramTile * kpp::kGramTile;
  const int32_t batch = static_cast<int32_t>(std::min<size_t>(static_cast<size_t>(nb), kNaGramDoubles / per_block));
  if (batch < 1) return fail(KPP_ERR_INVALID_ARG, "block size %d exceeds the no-allocation Gram workspace", s);
  HIP_TRY(hipSetDevice(sys->ctx->device));
  unsigned char* base = sys->ctx->scratch;
  if (!base) return fail(KPP_ERR_HIP, "the context has no scratch address");
  hipStream_t st = sys->ctx->stream;
  int32_t* d_err = reinterpret_cast<int32_t*>(base);
  int32_t* d_rows = reinterpret_cast<int32_t*>(base + kNaStageOffset);
  int32_t* d_lens = d_rows + static_cast<size_t>(nb) * s;
  int32_t* d_ids = d_lens + nb;
  double* ws = reinterpret_cast<double*>(base + kNaGramOffset);
  HIP_TRY(hipMemcpyAsync(d_rows, rows_host, static_cast<size_t>(nb) * s * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_lens, len_host, nb * sizeof(int32_t), hipMemcpyHostToDevice, st));
  kpp::launch_fill_i32(d_ids, nb, 0, 1, st);
  kpp::launch_fill_i32(d_err, 1, 0, 0, st);
  kpp::launch_zero_f64(L_dev, static_cast<int64_t>(nb) * s * s, st);
  const int64_t ss = static_cast<int64_t>(s) * s;
  if (sys->kind == KPP_KACZMARZ) {
    for (int32_t b0 = 0; b0 < nb; b0 += batch) {
      const int32_t k = std::min(batch, nb - b0);
      kpp::launch_gram_syrk_capped(sys->A, sys->lda, sys->n, d_rows + static_cast<size_t>(b0) * s, d_lens + b0, s, k,
                                   lambda, L_dev, ss, d_ids + b0, ws, kNaGramDoubles, st);
    }
  } else {
    kpp::launch_gram(sys->kind, sys->A, sys->lda, sys->n, d_rows, d_lens, s, nb, lambda, L_dev, ss, d_ids, nullptr,
                     st);
  }
  HIP_TRY(hipGetLastError());
  if (s <= kpp::kFactorSmallMax)
    kpp::launch_factor_small(L_dev, ss, s, d_lens, nb, d_ids, 0, d_err, st);
  else
    kpp::launch_cholesky(L_dev, s, ss, d_lens, nb, d_ids, d_err, st);
  HIP_TRY(hipGetLastError());
  int32_t herr = 0;
  HIP_TRY(hipMemcpyAsync(&herr, d_err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (herr) return fail(KPP_ERR_NOT_SPD, "a regularized block Gram has no Cholesky factor");
  return KPP_OK;
}

KPP_API kpp_status kpp_residual_norm(kpp_system* sys, const double* x_dev, double* out_host) {
  if (!sys || !x_dev || !out_host) return fail(KPP_ERR_INVALID_ARG, "bad arguments");
  HIP_TRY(hipSetDevice(sys->ctx->device));
  return residual_norm(sys, x_dev, out_host);
}


KPP_API kpp_status kpp_server_create(kpp_context* ctx, uint64_t hbm_budget_bytes, int32_t max_active,
                                     kpp_server** out) {
  if (!out) return fail(KPP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(KPP_ERR_INVALID_ARG, "context is NULL");
  if (max_active < 1 || max_active > kpp::kFusedMaxGroups)
    return fail(KPP_ERR_INVALID_ARG, "max_active must be in [1, %d]", kpp::kFusedMaxGroups);
  if (hbm_budget_bytes == 0) return fail(KPP_ERR_INVALID_ARG, "hbm_budget_bytes must be > 0");
  HIP_TRY(hipSetDevice(ctx->device));
  auto* srv = new (std::nothrow) kpp_server;
  if (!srv) return fail(KPP_ERR_OOM, "host allocation failed");
  srv->ctx = ctx;
  srv->budget = hbm_budget_bytes;
  srv->max_active = max_active;
  srv->cu_budget = ctx->cu_count > 0 ? std::min<int32_t>(ctx->cu_count, kpp::kFusedMaxGroups) : 64;
  const char* prof_env = std::getenv("KPP_SERVE_PROFILE");
  srv->prof = prof_env && prof_env[0] == '1';
  const size_t n_args = static_cast<size_t>(max_active);
  const size_t n_team = 2 * static_cast<size_t>(max_active) + 2;
  kpp_status st = KPP_OK;
  if ((st = dev_alloc(&srv->d_args, n_args)) < 0 || (st = dev_alloc(&srv->d_team, n_team)) < 0 ||
      hipHostMalloc(reinterpret_cast<void**>(&srv->h_args), n_args * sizeof(kpp::FusedArgs), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&srv->h_team), n_team * sizeof(int32_t), hipHostMallocDefault) !=
          hipSuccess ||
      hipEventCreate(&srv->ev[0]) != hipSuccess || hipEventCreate(&srv->ev[1]) != hipSuccess) {
    dev_free(srv->d_args);
    dev_free(srv->d_team);
    if (srv->h_args) (void)hipHostFree(srv->h_args);
    if (srv->h_team) (void)hipHostFree(srv->h_team);
    for (auto& e : srv->ev)
      if (e) (void)hipEventDestroy(e);
    delete srv;
    return fail(st < 0 ? st : KPP_ERR_HIP, "server buffers could not be allocated");
  }
  try {
    srv->pool.reset(new HostPool(7));
    srv->worker = std::thread(serve_loop, srv);
  } catch (const std::exception&) {
    dev_free(srv->d_args);
    dev_free(srv->d_team);
    (void)hipHostFree(srv->h_args);
    (void)hipHostFree(srv->h_team);
    for (auto& e : srv->ev) (void)hipEventDestroy(e);
    delete srv;
    return fail(KPP_ERR_HIP, "the worker thread could not be started");
  }
  *out = srv;
  return KPP_OK;
}

KPP_API kpp_status kpp_request_footprint(kpp_system* sys, const kpp_params* p, uint64_t* bytes_out) {
  if (!sys || !bytes_out) return fail(KPP_ERR_INVALID_ARG, "NULL argument");
  if (sys->csr) return fail(KPP_ERR_INVALID_ARG, "the server takes dense systems");
  KPP_TRY(check_params(sys, p));
  if (p->precision == KPP_MIXED_BF16) return fail(KPP_ERR_INVALID_ARG, "bfloat16 storage is for kpp_solve");
  *bytes_out = serve_footprint(sys, p, serve_periods(sys, p));
  return KPP_OK;
}

KPP_API kpp_status kpp_server_submit(kpp_server* srv, kpp_system* sys, const kpp_params* p, double* x_dev,
                                     uint64_t* id_out) {
  if (!srv || !sys || !x_dev || !id_out) return fail(KPP_ERR_INVALID_ARG, "NULL argument");
  *id_out = 0;
  if (sys->ctx != srv->ctx) return fail(KPP_ERR_INVALID_ARG, "the system belongs to another context");
  if (sys->csr) return fail(KPP_ERR_INVALID_ARG, "the server takes dense systems");
  KPP_TRY(check_params(sys, p));
  if (p->engine == 1) return fail(KPP_ERR_INVALID_ARG, "the server runs the fused engine only");
  if (p->schedule) return fail(KPP_ERR_INVALID_ARG, "explicit schedules are for kpp_solve");
  if (p->resume) return fail(KPP_ERR_INVALID_ARG, "resume is for kpp_solve");
  if (p->rht) return fail(KPP_ERR_INVALID_ARG, "rht is for kpp_solve (submit a system transformed by kpp_rht_psd)");
  if (p->projection) return fail(KPP_ERR_INVALID_ARG, "the LSQR projection is for kpp_solve");
  if (p->precision == KPP_MIXED_BF16) return fail(KPP_ERR_INVALID_ARG, "bfloat16 storage is for kpp_solve");
  sys->res_valid = false;
  auto* r = new (std::nothrow) ServeReq;
  if (!r) return fail(KPP_ERR_OOM, "host allocation failed");
  r->sys = sys;
  r->p = *p;
  r->x = x_dev;
  r->mixed = p->precision == KPP_MIXED_FP32;
  r->periods = serve_periods(sys, p);
  // the most columns per lane: the fewest compute units per request
  r->cpl = fused_cpl_max(p->block_size, r->mixed);
  r->groups = static_cast<int32_t>((sys->n + 64 * r->cpl - 1) / (64 * r->cpl));
  r->footprint = serve_footprint(sys, p, r->periods);
  std::lock_guard<std::mutex> lk(srv->mu);
  if (p->block_size > kpp::kFusedMaxBlock || r->groups > srv->cu_budget || r->footprint > srv->budget) {
    srv->rejected += 1;
    const size_t need = r->footprint;
    const int32_t g = r->groups;
    delete r;
    return fail(KPP_ERR_REJECTED, "request needs %zu bytes and %d compute units (budget %llu bytes, %d units)", need,
                g, static_cast<unsigned long long>(srv->budget), srv->cu_budget);
  }
  if (srv->stopping) {
    delete r;
    return fail(KPP_ERR_INVALID_ARG, "the server is shutting down");
  }
  r->id = srv->next_id++;
  r->t_submit = now_seconds();
  srv->queue.push_back(r);
  srv->submitted += 1;
  *id_out = r->id;
  srv->cv_work.notify_one();
  return KPP_OK;
}

KPP_API kpp_status kpp_server_poll(kpp_server* srv, int32_t cap, double wait_seconds, uint64_t* ids,
                                   int32_t* status, kpp_result* res, int32_t* n_out) {
  if (!srv || !n_out || cap < 0 || (cap > 0 && (!ids || !status))) return fail(KPP_ERR_INVALID_ARG, "bad arguments");
  *n_out = 0;
  std::unique_lock<std::mutex> lk(srv->mu);
  if (srv->done.empty() && wait_seconds > 0.0)
    srv->cv_done.wait_for(lk, std::chrono::duration<double>(wait_seconds), [&] { return !srv->done.empty(); });
  int32_t n = 0;
  while (n < cap && !srv->done.empty()) {
    ServeReq* r = srv->done.front();
    srv->done.pop_front();
    ids[n] = r->id;
    status[n] = r->status;
    if (res) res[n] = r->res;
    delete r;
    ++n;
  }
  *n_out = n;
  return KPP_OK;
}

KPP_API kpp_status kpp_server_stats(kpp_server* srv, kpp_server_info* out) {
  if (!srv || !out) return fail(KPP_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = srv->submitted;
  out->completed = srv->completed;
  out->rejected = srv->rejected;
  out->rounds = srv->rounds;
  out->queued = static_cast<int32_t>(srv->queue.size());
  out->active = srv->n_active;
  out->peak_active = srv->peak_active;
  out->cu_budget = srv->cu_budget;
  out->bytes_active = srv->bytes_active;
  out->peak_bytes = srv->peak_bytes;
  out->busy_seconds = srv->busy_seconds;
  return KPP_OK;
}

KPP_API kpp_status kpp_server_destroy(kpp_server* srv) {
  if (!srv) return KPP_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  if (srv->prof)
    std::fprintf(stderr,
                 "[kpp serve profile] %lld rounds, host s: start %.3f, prepare+launch %.3f, plan+factor %.3f, "
                 "wait %.3f, finish %.3f, transitions %.3f (all planning: buffer growth %.3f, schedule %.3f "
                 "of which slot table %.3f in %lld growths, factor enqueue %.3f); device busy %.3f\n",
                 static_cast<long long>(srv->rounds), srv->prof_s[0], srv->prof_s[1], srv->prof_s[2], srv->prof_s[3],
                 srv->prof_s[4], srv->prof_s[5], srv->prof_grow, srv->prof_sched, srv->prof_slots,
                 static_cast<long long>(srv->prof_slot_growth), srv->prof_enqueue, srv->busy_seconds);
  for (ServeReq* r : srv->done) delete r;
  srv->done.clear();
  (void)hipSetDevice(srv->ctx->device);
  dev_free(srv->d_args);
  dev_free(srv->d_team);
  if (srv->h_args) (void)hipHostFree(srv->h_args);
  if (srv->h_team) (void)hipHostFree(srv->h_team);
  for (auto& e : srv->ev)
    if (e) (void)hipEventDestroy(e);
  delete srv;
  return KPP_OK;
}

}  // extern "C"
