/*
 * kpp.h -- C ABI of the MI355X Kaczmarz++ / CD++ block-step library.
 *
 * The library solves a consistent linear system A x = b by the accelerated,
 * Tikhonov-regularized, memoized randomized block step of
 *   M. Derezinski, D. Needell, E. Rebrova, J. Yang,
 *   "Randomized Kaczmarz Methods with Beyond-Krylov Convergence" (arXiv 2501.11673):
 *   - Kaczmarz++ (general m x n, over- or under-determined; Algorithm 5 with the
 *     exact Cholesky projection, "K++(Cholesky)" of Appendix F.1), and
 *   - CD++ (square positive semidefinite A; Algorithm 2 without the randomized
 *     Hadamard preprocessing, "CD++ w/o RHT" of Section 6.3).
 * One step, for a row block S of size s (Section 1.1, eq. (bk), eq. (momentum)):
 *   r = A_S x - b_S
 *   y = (A_S A_S^T + lambda I)^{-1} r      (CD++: (A_SS + lambda I)^{-1} r)
 *         through the memoized Cholesky factor of that block (Section 4.2, 5.2)
 *   w = A_S^T y                            (CD++: w = I_S^T y, eq. (cd-update))
 *   m <- (1 - rho)/(1 + rho) (m - w);  x <- x - w + eta m
 * with rho revised every 2*zeta steps from block-residual window sums
 * (Section 5.4, eq. (residual), eq. (weighted)).
 *
 * Conventions
 *   - Every pointer named *_dev is device memory of the context's device
 *     (for example a torch tensor's data_ptr()).  Host pointers are named *_host.
 *   - Matrices are row-major FP64 with a leading dimension (lda >= n).
 *   - The caller owns A, b and x; the library never frees them and they must
 *     outlive the kpp_system (or the served request) that refers to them.
 *     A and b must not change while a kpp_system refers to them: the library
 *     keeps values derived from them (||b||, the FP32 copy of A, memoized
 *     factors, the randomized Hadamard transforms); to solve with other
 *     values, create a new system.
 *     The library owns memo caches, low-precision copies, state and workspaces.
 *   - All work is enqueued on the context's stream (borrowed, never destroyed;
 *     NULL means the device's null stream).  Calls return after that stream's
 *     work for the call has completed.
 *   - Every call returns a kpp_status; negative values are errors, after which
 *     outputs are unspecified and kpp_last_error() describes the failure.
 *     No C++ exception crosses this boundary.
 *   - A context, and the systems created on it, must be used by one host
 *     thread at a time.
 */
#ifndef KPP_H_
#define KPP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KPP_API __attribute__((visibility("default")))
#define KPP_ABI_VERSION 6

typedef enum kpp_status {
  KPP_OK = 0,
  KPP_NOT_CONVERGED = 1,      /* max_iters reached; x holds the last iterate            */
  KPP_ERR_INVALID_ARG = -1,   /* a parameter is out of range or a pointer is NULL       */
  KPP_ERR_SHAPE = -2,         /* inconsistent sizes (lda < n, CD++ with m != n, ...)    */
  KPP_ERR_NOT_SPD = -3,       /* a regularized block Gram has no Cholesky factor        */
  KPP_ERR_NONFINITE = -4,     /* A or b holds NaN or Inf                                 */
  KPP_ERR_OOM = -5,           /* device allocation failed                                */
  KPP_ERR_HIP = -6,           /* a HIP runtime call failed                               */
  KPP_ERR_REJECTED = -7,      /* serving: the request does not fit the HBM budget        */
  KPP_ERR_DEVICE = -8         /* a device-side wait exceeded its bound (never expected)  */
} kpp_status;

typedef enum kpp_kind {
  KPP_KACZMARZ = 0,           /* general m x n system: Kaczmarz++                        */
  KPP_CD_PSD = 1              /* square PSD system: CD++                                 */
} kpp_kind;

typedef enum kpp_memo {
  KPP_MEMO_OFF = 0,           /* a new random block at every step, factor not kept
                                 ("w/o Memo", Section 6.2)                                */
  KPP_MEMO_ONLINE = 1,        /* Bernoulli(min(1, B0/t)) new blocks (Section 5.2)        */
  KPP_MEMO_FIXED = 2          /* collection drawn up front (Algorithm 1): a random
                                 partition, or num_blocks random s-subsets               */
} kpp_memo;

typedef enum kpp_precision {
  KPP_FP64 = 0,               /* every product in FP64                                   */
  KPP_MIXED_FP32 = 1,         /* FP32 block products and Grams, FP64 residual, factor
                                 of ill-conditioned blocks and x accumulation, with
                                 iterative refinement (outer loop FP64)                  */
  KPP_MIXED_BF16 = 2          /* as MIXED_FP32 with a bfloat16 copy of A for the block
                                 products (widened to FP32, FP32 accumulation) and FP64
                                 Grams; converges only when kappa(A) is well below
                                 2^8; kpp_solve only.  Both mixed modes end a
                                 diverging refinement early (a true residual not
                                 finite or 10x its lowest) and return, when they do
                                 not converge, the iterate with the lowest true
                                 residual (KPP_NOT_CONVERGED)                            */
} kpp_precision;

/* Solver parameters.  kpp_params_default() fills every field. */
typedef struct kpp_params {
  int32_t block_size;         /* s, 1 <= s <= rows (m for Kaczmarz++, n for CD++)       */
  int32_t memo;               /* kpp_memo                                                */
  int32_t num_blocks;         /* FIXED without partition: B >= 1                         */
  int32_t fixed_partition;    /* FIXED: 1 = random partition into ceil(rows/s) blocks    */
  int32_t accel;              /* 0: eta = 0 ("w/o Accel", Table 1)                       */
  int32_t adaptive_rho;       /* 1: revise rho at checkpoints (Section 5.4)              */
  int32_t precision;          /* kpp_precision                                           */
  int32_t confirm_true_residual; /* 1: a candidate stop is confirmed by ||Ax-b|| (FP64) */
  double lambda;              /* lambda >= 0 (default 1e-8, Section 6.2)                */
  double tol;                 /* eps: stop when ||Ax - b|| <= eps ||b|| (eq. (residual-error)) */
  double eta;                 /* < 0: default s / (2 min(m, n)) (CD++: s / (2n))         */
  double rho0;                /* initial rho (default 0, Algorithm 2)                    */
  int64_t max_iters;          /* upper bound on block steps                              */
  uint64_t seed;              /* schedule seed (SplitMix64 draws; see kpp_schedule_generate) */
  int32_t keep_memo;          /* 1: keep factors from an earlier solve with the same
                                 schedule settings; 0: start with an empty cache          */
  int32_t refine_max_rounds;  /* mixed precision: outer refinement rounds (default 40)   */
  double inner_tol;           /* mixed precision: relative tolerance of each inner solve
                                 (default 1e-3 for Kaczmarz++, 1e-2 for CD++); an inner
                                 solve also ends when its residual estimate stalls
                                 (FP32 precision floor)                               */
  int32_t engine;             /* 0: auto, 1: one launch per phase, 2: fused persistent  */
  int32_t team_groups;        /* fused engine: workgroups sharing one step (0: auto)    */
  /* Optional caller-given block schedule (host memory, read during kpp_solve;
   * the caller keeps ownership).  When schedule is not NULL it replaces the
   * memo/seed/num_blocks/fixed_partition settings: step t uses block
   * schedule[t] of the table block_rows (block_rows_count x block_size row
   * indices, ascending, a shorter block padded with -1), each block is
   * factored on first use and kept for the rest of the solve (Algorithm 1's
   * fixed collection with the paper's "if no factor is cached for S" rule),
   * and a solve runs at most min(max_iters, schedule_len) steps.  FP64 and
   * kpp_solve only: mixed precision and kpp_server_submit reject it with
   * KPP_ERR_INVALID_ARG, as does a malformed table or an id out of range. */
  const int32_t* schedule;
  int64_t schedule_len;
  const int32_t* block_rows;
  int32_t block_rows_count;
  /* 1: continue the saved state of this system (the last FP64 kpp_solve on
   * it, or kpp_state_import) instead of starting with zero momentum, rho0 and
   * a fresh schedule: x_dev must hold the iterate that solve returned, and
   * max_iters counts the further steps.  FP64 and kpp_solve only. */
  int32_t resume;
  /* 1: randomized Hadamard preprocessing (Definition d:rht; the RHT lines of
   * Algorithms 2 and 5).  Signs d_i from SplitMix64(rht_seed) (kpp_rht_signs),
   * rows padded with zeros to R = the next power of two of the row count.
   * Kaczmarz++ runs on (H D A) x = H D b, CD++ on (H D A D H) xbar = H D b with
   * xbar0 = H D x0 and x = D H xbar.  The transformed system is formed on the
   * device on the first such solve and kept with the system (an R x n or
   * R x R FP64 copy) until a solve asks for another rht_seed; memo, resume
   * state and an explicit schedule (rows 0..R-1) then belong to it.
   * true_rel_res is recomputed on the original system.  R <= 2^24.  resume
   * and kpp_server_submit reject rht = 1 (KPP_ERR_INVALID_ARG). */
  int32_t rht;
  /* 1: kpp_solve does not time its step-kernel launches: no HIP event pair
   * goes to the stream around each launch (each pair adds a few microseconds
   * between consecutive launches) and kernel_seconds reports 0.  Default 0:
   * every launch is timed (kernel_seconds). */
  int32_t no_launch_timing;
  uint64_t rht_seed;
  /* Kaczmarz++ projection (Section 4.1).  0: exact, w = A_S^T (A_S A_S^T +
   * lambda I)^{-1} r through the memoized Cholesky factor.  1: the inexact
   * Proj of Algorithm 5: on a new block the SRHT sketch A_hat = A_S Pi^T with
   * tau rows (Lemma l:inner; n padded to a power of two N) and
   * L = chol(A_hat A_hat^T + lambda I) are formed and L^{-1} memoized; each
   * step runs lsqr_iters LSQR iterations from zero on
   * min || L^{-1} [A_S, sqrt(lambda) I] z - L^{-1} r || and takes w = z[0:n].
   * The sketch draws come from SplitMix64(sketch_seed): N signs, then tau
   * sketch rows per new block in step order.  Kaczmarz++, FP64, kpp_solve,
   * launch-per-phase engine (engine 0 or 1) only; resume and an explicit
   * engine 2 are rejected (KPP_ERR_INVALID_ARG), and the factors are not kept
   * for a later solve. */
  int32_t projection;
  int32_t lsqr_iters;         /* t_max, 1..256 (default 8, Appendix F.1)              */
  int32_t sketch_size;        /* tau; 0: 2 s (Section 6.2), capped at N               */
  int32_t reserved3;
  uint64_t sketch_seed;
} kpp_params;

/* Per-solve report. */
typedef struct kpp_result {
  int64_t iters;              /* block steps executed (all refinement rounds)            */
  int64_t memo_hits;
  int64_t memo_misses;        /* factorizations performed                               */
  int64_t factors_fp64;       /* mixed precision: blocks factored in FP64                */
  int32_t converged;
  int32_t refinements;        /* outer refinement rounds (mixed precision)               */
  int32_t checkpoints;
  int32_t engine_used;
  double est_rel_res;         /* sqrt(E1) / ||b|| at the last checkpoint                 */
  double true_rel_res;        /* ||A x - b|| / ||b|| in FP64 at return                   */
  double rho_final;
  double seconds_total;
  double seconds_factor;      /* time in Gram + Cholesky                                 */
  double flops;               /* 2sn (+2sn K++) + 2s^2 + 5n per step; s^3/3 (+s^2 n) per factor;
                                 with rht: the transform's additions as the paper counts
                                 them (SymFHT or FHT of A and FHT of b when the solve
                                 formed them; CD++ also FHTs of the iterate in and out);
                                 projection 1: per step 4sn + 5n + s^2 + t_max (4sn + 2n
                                 + 4s^2), per factor s N log2 N + s^2 tau + 2 s^3 / 3 */
  double bytes_algorithmic;   /* per step: s n b_A (A_S) + s(s+1)/2 * 8 (factor) + 12 s (b_S, rows) */
  double kernel_seconds;      /* device time of the step kernels (HIP events), all launches;
                                 0 with params.no_launch_timing */
  double kernel_launches;     /* number of step-kernel launches (fused: one per window)  */
  double seconds_queued;      /* serving: time from submission to admission             */
  int32_t team_groups;        /* fused engine: workgroups sharing one step (0: launch-per-phase) */
  int32_t cols_per_lane;      /* fused engine: columns of x each lane holds (0: launch-per-phase) */
} kpp_result;

/* Serving statistics (kpp_server_stats). */
typedef struct kpp_server_info {
  int64_t submitted;          /* accepted by kpp_server_submit                           */
  int64_t completed;          /* finished (any status), including not yet polled         */
  int64_t rejected;           /* refused by kpp_server_submit with KPP_ERR_REJECTED      */
  int64_t rounds;             /* shared step launches issued                             */
  int32_t queued;             /* waiting for admission now                               */
  int32_t active;             /* admitted and not finished now                           */
  int32_t peak_active;        /* largest number of requests on the device at once        */
  int32_t cu_budget;          /* workgroups (one per compute unit) shared by active runs */
  uint64_t bytes_active;      /* admitted device-memory footprint now                    */
  uint64_t peak_bytes;        /* largest admitted footprint                              */
  double busy_seconds;        /* device time of the shared step launches                 */
} kpp_server_info;

typedef struct kpp_context kpp_context;
typedef struct kpp_system kpp_system;
typedef struct kpp_server kpp_server;

/* ABI version (KPP_ABI_VERSION). */
KPP_API int32_t kpp_abi_version(void);

/* Message for the last failed call on this host thread (never NULL). */
KPP_API const char* kpp_last_error(void);

/* Defaults of Algorithms 2 and 5: lambda 1e-8, rho0 0, eta from s and the
 * shape, zeta = ceil(rows / s), online memoization, acceleration on. */
KPP_API kpp_status kpp_params_default(kpp_params* p, int32_t kind);

/* Context on HIP device `device`, enqueueing on `hip_stream` (a hipStream_t,
 * borrowed; may be NULL). */
KPP_API kpp_status kpp_context_create(int32_t device, void* hip_stream, kpp_context** out);
KPP_API kpp_status kpp_context_destroy(kpp_context* ctx);

/* A system A x = b (Section 1.1).  A_dev: m x n row-major FP64 with leading
 * dimension lda >= n; b_dev: m values.  kind = KPP_CD_PSD requires m == n and
 * A symmetric positive semidefinite (only the entries the blocks touch are
 * read).  Checks that A and b are finite (KPP_ERR_NONFINITE). */
KPP_API kpp_status kpp_system_create(kpp_context* ctx, int32_t kind, int64_t m, int64_t n,
                                     const double* A_dev, int64_t lda, const double* b_dev,
                                     kpp_system** out);

/* A sparse system A x = b in compressed sparse rows (the sparse inputs of
 * Section 1's limitations and of the Conclusions, for which Section 3 lets
 * the Hadamard preprocessing be dropped).  row_ptr_dev: m + 1 int64 offsets
 * (row_ptr[0] = 0, row_ptr[m] = nnz, non-decreasing); col_dev, val_dev: nnz
 * column indices (strictly increasing within each row, in [0, n)) and FP64
 * values; b_dev: m values.  All device memory owned by the caller and read,
 * never written, for the system's lifetime; col_dev and val_dev may be NULL
 * when nnz = 0.  kind = KPP_CD_PSD requires m == n and A symmetric PSD (the
 * lower triangle of each block's A_SS is read).  The structure is checked on
 * the device (KPP_ERR_SHAPE) as is finiteness of values and b
 * (KPP_ERR_NONFINITE); the row pointers are copied to the host, and must not
 * change afterwards (a solve that finds different block nonzero counts
 * returns KPP_ERR_INVALID_ARG).
 *
 * kpp_solve, kpp_state_export/import, kpp_residual_norm and kpp_block_factor
 * take such a system; a solve runs in FP64 on the launch-per-phase engine
 * with the exact projection and without rht (KPP_ERR_INVALID_ARG for other
 * precision, engine, projection or rht values), and the iterates are those of
 * the same solve on the dense matrix up to rounding.  A block holds at most
 * 2^20 nonzeros (KPP_ERR_SHAPE).  kpp_solve_multi, kpp_block_factor_noalloc
 * and the server take dense systems only.  In kpp_result, bytes_algorithmic
 * counts every nonzero's column of a Kaczmarz++ block as distinct (an upper
 * bound on the back-projection's traffic). */
KPP_API kpp_status kpp_system_create_csr(kpp_context* ctx, int32_t kind, int64_t m, int64_t n, int64_t nnz,
                                         const int64_t* row_ptr_dev, const int32_t* col_dev,
                                         const double* val_dev, const double* b_dev, kpp_system** out);
KPP_API kpp_status kpp_system_destroy(kpp_system* sys);

/* Run the solver from x_dev (in: x0, out: final iterate; n FP64 values).
 * Returns KPP_OK when ||A x - b|| <= tol ||b|| was confirmed, KPP_NOT_CONVERGED
 * when max_iters steps ran first.  `res` may be NULL. */
KPP_API kpp_status kpp_solve(kpp_system* sys, const kpp_params* p, double* x_dev,
                             kpp_result* res);

/* Resume support.  After an FP64 kpp_solve a system holds what is needed to
 * continue that solve: the momentum vector, the step counter and checkpoint
 * statistics (rho, r_hat, E0, E1: Section 5.4) and the block schedule's
 * generator (Section 5.2).  kpp_state_export writes it to host memory owned by
 * the caller (host_buf NULL: only *bytes is set to the size needed; otherwise
 * *bytes is the buffer's size on entry and the size written on return;
 * KPP_ERR_INVALID_ARG when it is too small or the system holds no state).
 * kpp_state_import loads such a buffer into a system of the same kind and
 * shape (KPP_ERR_SHAPE otherwise); a kpp_solve with params.resume = 1 then
 * continues from it.  The memo cache is not part of the state: factors are
 * formed again on first use.  Continuing a CD++ solve this way gives the same
 * iterates, bit for bit, as one uninterrupted solve; Kaczmarz++ agrees up to
 * the rounding of Grams formed in a different batch.  The state holds no x:
 * the caller keeps the iterate it passed to kpp_solve. */
KPP_API kpp_status kpp_state_export(const kpp_system* sys, void* host_buf, size_t* bytes);
KPP_API kpp_status kpp_state_import(kpp_system* sys, const void* host_buf, size_t bytes);

/* Several right-hand sides on one system (A x_c = b_c, c < k <= 32): the k
 * solves share the block schedule, the memoized factors and every pass over
 * A_S (each A_S element is read once per step for all of them); each keeps
 * its own momentum, window sums and adaptive rho (Algorithms 2 and 5), is
 * confirmed against its own true residual and stops at its own step, exactly
 * where a kpp_solve of that right-hand side with the same parameters would.
 * B_dev: m x k row-major (leading dimension ldb >= k); X_dev: n x k row-major
 * (ldx >= k), in: the k starting iterates, out: the results; both device
 * memory owned by the caller; the system's own b is not used.  res: k results
 * (host) or NULL; the memo counts are the shared ones.  FP64, the seeded
 * schedule and the launch-per-phase kernels only: rht, projection, resume, an
 * explicit schedule or another precision give KPP_ERR_INVALID_ARG.  Returns
 * KPP_OK when every right-hand side converged, else KPP_NOT_CONVERGED. */
KPP_API kpp_status kpp_solve_multi(kpp_system* sys, const kpp_params* p, int32_t k, const double* B_dev,
                                   int64_t ldb, double* X_dev, int64_t ldx, kpp_result* res);

/* Randomized Hadamard preprocessing (Definition d:rht; Algorithm 4, FHT;
 * Algorithm 3 and Section 5.3, the symmetric transform).  H is the Sylvester
 * Hadamard matrix (H_1 = 1, H_2k = [[H_k, H_k], [H_k, -H_k]]); R is a power of
 * two; D = diag(signs) / sqrt(R).  Inputs are zero-padded to R.  All matrix and
 * vector pointers are device memory owned by the caller, row-major FP64;
 * signs is a device array of R int8 values +1 / -1.  The calls enqueue on the
 * context's stream and return without waiting.  Outputs must not overlap
 * inputs.  KPP_ERR_SHAPE: R not a power of two, R below the row count, or
 * R > 2^24; KPP_ERR_INVALID_ARG: a NULL pointer or a leading dimension too
 * small. */

/* N signs: signs_host[i] = +1 when the top bit of the i-th SplitMix64(seed)
 * output is 0, else -1 (host memory, caller-owned).  These are the signs
 * kpp_solve uses with params.rht = 1 and params.rht_seed = seed. */
KPP_API kpp_status kpp_rht_signs(uint64_t seed, int64_t N, int8_t* signs_host);

/* Kaczmarz++ (Algorithm 5): At (R x n, leading dimension ldt >= n) = H D A
 * and bt (R) = H D b, with A (m x n, lda >= n) and b (m) padded to R >= m rows. */
KPP_API kpp_status kpp_rht_general(kpp_context* ctx, int64_t m, int64_t n, const double* A, int64_t lda,
                                   const double* b, const int8_t* signs, int64_t R, double* At,
                                   int64_t ldt, double* bt);

/* CD++ (Algorithm 2): At (R x R, ldt >= R) = H D A D H and bt (R) = H D b, with
 * A (n x n symmetric, lda >= n) padded to R x R and b to R entries.  The
 * transform runs as H (H D A D)^T, two passes over At.  work: R x R doubles of
 * scratch when R > 4096 (may be NULL otherwise). */
KPP_API kpp_status kpp_rht_psd(kpp_context* ctx, int64_t n, const double* A, int64_t lda, const double* b,
                               const int8_t* signs, int64_t R, double* At, int64_t ldt, double* bt,
                               double* work);

/* Vector transforms of Algorithm 2.  direction 0: y (R entries) = H D [x; 0]
 * for x of nx <= R entries (the transformed start xbar0).  direction 1:
 * y (nx entries) = the first nx entries of D H x for x of R entries (the
 * returned x = D FHT(xbar)).  work: R doubles of scratch when R > 4096 and
 * direction 1 with nx < R (may be NULL otherwise). */
KPP_API kpp_status kpp_rht_vector(kpp_context* ctx, int64_t R, const int8_t* signs, const double* x,
                                  int64_t nx, double* y, int32_t direction, double* work);

/* The block schedule kpp_solve uses for these settings, on the host (Section
 * 5.2; Algorithms 1, 2, 5).  rows = m (Kaczmarz++) or n (CD++).  Writes the
 * block id of each of the T steps to step_block_host[T] and each block's rows
 * (sorted ascending) to block_rows_host[b * s + i], its size to
 * block_len_host[b], for b < *num_blocks_out (at most blocks_cap blocks).
 * SplitMix64 draws as documented in the library's schedule source. */
KPP_API kpp_status kpp_schedule_generate(int32_t kind, int64_t m, int64_t n, const kpp_params* p,
                                         int64_t T, int32_t* step_block_host,
                                         int32_t* block_rows_host, int32_t* block_len_host,
                                         int32_t blocks_cap, int32_t* num_blocks_out);

/* Regularized block Grams and their Cholesky factors on the device (the memo
 * miss path, Algorithm 1 and Algorithm 2).  rows_host[b * s + i], i <
 * len_host[b]: the rows of block b.  L_dev receives nb column-major s x s
 * lower factors (entry (i, j) of block b at L_dev[b*s*s + j*s + i]; the strict
 * upper triangle is zeroed).  Returns KPP_ERR_NOT_SPD if a Gram has no factor. */
KPP_API kpp_status kpp_block_factor(kpp_system* sys, int32_t s, double lambda, int32_t nb,
                                    const int32_t* rows_host, const int32_t* len_host,
                                    double* L_dev);

/* kpp_block_factor for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, layout, results and errors as
 * kpp_block_factor, but it calls no hipMalloc, hipFree or allocating library
 * routine.  Its scratch (the staged rows, lengths and slot ids, the
 * breakdown flag and the split-Gram partial tiles) is one 16 MiB array per
 * device (KPP_NOALLOC_SCRATCH_BYTES) that the library holds from its first
 * context on that device until the process ends.  Limits: nb * (s + 2) <=
 * KPP_NOALLOC_STAGE_ENTRIES (KPP_ERR_INVALID_ARG beyond it); Kaczmarz++
 * Grams are formed in batches of blocks with fewer column chunks when the
 * default split would not fit, so factors may differ from kpp_block_factor's
 * by rounding (they are identical when the default split fits).  Every call
 * on a device shares that device's array: calls that overlap on one device
 * (another thread, another context's stream) race and must be serialized by
 * the caller.  The call returns after its work on the context's stream. */
#define KPP_NOALLOC_SCRATCH_BYTES (16u << 20)
#define KPP_NOALLOC_STAGE_ENTRIES 262080
KPP_API kpp_status kpp_block_factor_noalloc(kpp_system* sys, int32_t s, double lambda, int32_t nb,
                                            const int32_t* rows_host, const int32_t* len_host,
                                            double* L_dev);

/* ||A x - b||_2 in FP64 (eq. (residual-error)); x_dev device, result on host. */
KPP_API kpp_status kpp_residual_norm(kpp_system* sys, const double* x_dev, double* out_host);

/*
 * Serving: continuous batching of solves (each one the solve kpp_solve runs).
 * A worker thread owned by the server runs every admitted request on the
 * context's streams; from kpp_server_create until kpp_server_destroy returns,
 * the context and the systems with submitted requests are used by that thread,
 * and the caller uses them only through kpp_server_* calls (creating further
 * systems on the context is allowed).  Requests wait in arrival order and are
 * admitted while (a) the sum of their device-memory footprints (memo cache,
 * FP32 copy of A, state and staging; the caller's A, b, x not counted) stays
 * within hbm_budget_bytes, (b) their workgroups (one per compute unit:
 * ceil(n / (64 c)), c = columns per lane, the most the block size s allows --
 * FP64: 2 for s <= 128, else 1; mixed precision: 4 for s <= 128, else 1) fit on
 * the device, (c) at most
 * max_active are active, and (d) no other request on the same system is active;
 * a request held back only by (d) does not hold back later ones.  Every round
 * advances each active request by a window of its own length, all of them in
 * one persistent launch, so that requests of different sizes overlap on the
 * device; a request's iterates do not depend on what else is being served.
 */

/* Device-memory footprint admission charges for a request (bytes). */
KPP_API kpp_status kpp_request_footprint(kpp_system* sys, const kpp_params* p, uint64_t* bytes_out);

/* Start a server on ctx (the worker thread starts at once). */
KPP_API kpp_status kpp_server_create(kpp_context* ctx, uint64_t hbm_budget_bytes, int32_t max_active,
                                     kpp_server** out);

/* Queue a solve of sys from x_dev (in: x0, out: final iterate), with the
 * parameters of kpp_solve (engine 1 is not available here).  Returns at once
 * with the request id; KPP_ERR_REJECTED if the request alone exceeds the
 * memory budget or the device.  sys, x_dev and *p's values are captured; x_dev
 * must stay valid until the request has been polled. */
KPP_API kpp_status kpp_server_submit(kpp_server* srv, kpp_system* sys, const kpp_params* p, double* x_dev,
                                     uint64_t* id_out);

/* Collect up to cap finished requests (waiting up to wait_seconds for the
 * first one): ids[i], status[i] (what kpp_solve would return) and, if res is
 * not NULL, res[i] with seconds_total = submission to completion and
 * seconds_queued = submission to admission. */
KPP_API kpp_status kpp_server_poll(kpp_server* srv, int32_t cap, double wait_seconds, uint64_t* ids,
                                   int32_t* status, kpp_result* res, int32_t* n_out);

KPP_API kpp_status kpp_server_stats(kpp_server* srv, kpp_server_info* out);

/* Finish every submitted request, stop the worker and free the server;
 * results not polled are dropped. */
KPP_API kpp_status kpp_server_destroy(kpp_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* KPP_H_ */
