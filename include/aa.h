/*
 * aa.h -- C ABI of the MI355X (gfx950) Anderson-acceleration library.
 *
 * Anderson acceleration (AA) of a fixed-point map G with a window of m past
 * differences, following Lockhart, Gardner, Woodward, Thomas and Olson,
 * "Performance of Low Synchronization Orthogonalization Methods in Anderson
 * Accelerated Fixed Point Solvers" (arXiv 2110.09667):
 *   Alg. 1  -- the AA iteration,
 *   Alg. 2  -- the least-squares solve through a windowed QR of F_i
 *              (QRDelete by Givens rotations when the window is full, then
 *              QRAdd, then R gamma = Q^T f_i),
 *   Algs. 3-6 -- QRAdd by MGS, ICWY-MGS, CGS-2 and DCGS-2.
 * Everything is FP64.  Every step runs in the library's HIP kernels.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 * - Pointers named d_* are device pointers (HBM of the current HIP device),
 *   h_* are host pointers.  Vectors of length n are contiguous FP64, 8-byte
 *   aligned; 16-byte alignment is not required.
 * - Ownership: the library never allocates device memory.  The caller passes
 *   a workspace (d_workspace, size from aa_workspace_size, 256-byte aligned)
 *   that holds Q, the history of G differences, R, T and all scratch; the
 *   caller keeps it alive until aa_destroy.  The context itself is a small
 *   host allocation freed by aa_destroy.
 * - Streams: all device work of a context is enqueued on the stream given to
 *   aa_init (or aa_set_stream); calls return without waiting unless stated.
 *   One context must not be used from two host threads at once.
 * - Errors: every entry point returns an aa_status.  Argument and state errors
 *   are detected on the host before anything is enqueued and leave the context
 *   unchanged.  Device-side breakdown (the new column numerically in the span
 *   of the window: R_kk <= 64 eps ||R_{0:k,k}||, or non-finite) is latched in
 *   the workspace and reported by the next aa_get_info.  In aa_step a
 *   breakdown ends the iteration: that step returns x_{i+1} = G(x_i) (no
 *   extrapolation from the broken factorization) and later steps change
 *   nothing until aa_reset, which restarts AA from the current iterate.  The
 *   library never aborts and never prints.
 */
#ifndef AA_H
#define AA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aa_ctx aa_ctx;
typedef struct aa_batch aa_batch;
typedef struct aa_mlp aa_mlp;

/* QRAdd variants (Sec. 3): Alg. 3, Alg. 5, Alg. 6, Alg. 4, and the delayed
 * CGS-2 whose normalization is lagged as well (the stable form Sec. 3.4
 * describes after Swirydowicz et al. and Bielich et al., which the paper does
 * not run in AA).  AA_DCGS2_LAG adds a column with ONE reduction: the block
 * dot products [Q^T v | Q^T q_{k-1} | v^T v] reorthogonalize and normalize the
 * previous column q_{k-1} (its correction s = Q_{:,0:k-2}^T q_{k-1}, its norm
 * sqrt(q_{k-1}^T q_{k-1} - s^T s)), project v once on the updated basis and
 * give the new column's norm by Pythagoras, R_kk = sqrt(v^T v - ||R_{0:k-1,k}||^2),
 * with no reduction over the new column; one more pass writes both columns.
 * Q R = F_i holds after every add and the LSP solve uses the newest column
 * as it stands (orthogonalized once); its reorthogonalization happens in the
 * next add.  A non-positive squared norm (the new column numerically in the
 * span of Q) latches AA_EBREAKDOWN.  Grid-wide passes only (no one-workgroup
 * step, no batched path, no AA_FUSE_DELETE). */
typedef enum { AA_MGS = 0, AA_CGS2 = 1, AA_DCGS2 = 2, AA_ICWY = 3,
               AA_DCGS2_LAG = 4 } aa_variant;

typedef enum {
  AA_OK = 0,
  AA_EINVAL = -1,      /* bad argument (size, pointer, alignment, enum)     */
  AA_EHIP = -2,        /* a HIP runtime call failed                          */
  AA_EBREAKDOWN = -3,  /* F_i lost full column rank: the new column's R_kk
                          is at most 64 eps times its column norm (or zero,
                          negative, non-finite)                              */
  AA_ESTATE = -4,      /* QRAdd on a full window, QRDelete on an empty one   */
  AA_ENOSPACE = -5     /* workspace smaller than aa_workspace_size           */
} aa_status;

/* Flags of aa_init. */
enum {
  /* Alg. 6 read literally: R_{0:k-2,k-1} += s.  Default adds R_{k-1,k-1} s,
   * which keeps Q R = F_i (the factorization Alg. 2 relies on). */
  AA_DCGS2_LITERAL = 1u << 1,
  /* ICWY: after QRDelete, update T without a reduction (the alternative
   * reading of Sec. 3.2's T update): the Givens kernel rotates the old Gram
   * matrix I + L + L^T of the columns 0..k-2 like the columns of Q and keeps
   * its strict lower rows 0..k-3 as the new T; the rotation pass then streams
   * Q without the Gram.  The last row of T (the column that old column k-1
   * entered) is recomputed by the next QRAdd's first reduction before any
   * read (Alg. 4), so aa_get_qr reports rows 0..k-2 only as current.  One
   * reduction fewer per recycled iteration.  Grid-wide passes only; with
   * AA_FUSE_DELETE the fused Gram refreshes T instead.  Not for the batched
   * entry points (AA_EINVAL). */
  AA_ICWY_T_TRANSFORM = 1u << 2,
  /* Alg. 6: reorthogonalize the previous column when m_i >= 3 instead of the
   * printed m_i > 3. */
  AA_DCGS2_GUARD_GE3 = 1u << 4,
  /* aa_step with CGS-2, DCGS-2 or ICWY: form c = Q^T f_i inside the QRAdd
   * passes (Q^T f with the first pass's block dot products, c_k = w^T f /
   * R_kk with the norm of the new column) and solve R gamma = c in the last
   * pass's tail, instead of a separate pass over Q after QRAdd (Alg. 2, last
   * line).  Same c, different rounding order; saves one pass over Q and one
   * reduction per iteration.  MGS and the first QRAdd keep the separate
   * pass. */
  AA_FUSE_RHS = 1u << 3,
  /* aa_step (and the batched entry points) with CGS-2, DCGS-2 or ICWY once
   * the window is full: QRDelete's rotation pass also stages Delta f (and
   * f_i with AA_FUSE_RHS) beside the rotated columns, and one matrix-core
   * Gram of [Q Delta f f] yields ICWY's T refresh (Sec. 3.2) together with
   * every block dot product of the QRAdd's first pass (Algs. 4-6: Q^T Delta
   * f, the Gram row of the last column, Q^T f_i).  Same quantities, different
   * rounding order; one pass over Q fewer per iteration, and for ICWY one
   * reduction fewer (2 per iteration including the delete instead of 3).
   * MGS is unaffected.  Windows of up to 62 columns (63 without
   * AA_FUSE_RHS); wider ones keep the separate passes. */
  AA_FUSE_DELETE = 1u << 5,
  /* Workspace for the QR update only (aa_qr_add / aa_qr_delete /
   * aa_qr_solve); aa_step is then unavailable.  Saves (m + 3) n doubles. */
  AA_QR_ONLY = 1u << 8
};

/* Largest window (columns of Q).  65 lets a full 64-column basis receive one
 * more column in the QRAdd microbenchmark. */
#define AA_MAX_COLS 65

/* Why an iteration has ended (aa_info.stopped). */
enum {
  AA_RUNNING = 0,
  AA_STOPPED_TEST = 1,      /* the stopping test of aa_set_stop held        */
  AA_STOPPED_BREAKDOWN = 2, /* a breakdown (status AA_EBREAKDOWN)           */
  AA_STOPPED_CAP = 3        /* the iteration cap of aa_set_stop was reached */
};

/* Stopping tests of aa_set_stop (Alg. 1 stops on the step length; the
 * workloads stop on the relative residual, reading A2). */
enum {
  AA_STOP_RESIDUAL = 0,     /* ||f_i||_2 <= tol ||f_0||_2 at the start of i  */
  AA_STOP_STEP = 1          /* ||x_i - x_{i-1}||_2 < tol at the start of i   */
};

typedef struct {
  int64_t iter;      /* index i of the next aa_step call                    */
  int m_i;           /* columns used by the last step (min(m, i))           */
  int k;             /* columns currently in Q                              */
  double res_norm;   /* ||f_i||_2 of the last step, f_i = G(x_i) - x_i      */
  double res0_norm;  /* ||f_0||_2                                           */
  double step_norm;  /* ||x_{i+1} - x_i||_2 of the last step                */
  int status;        /* AA_OK or a latched device-side error                */
  int stopped;       /* AA_RUNNING or why the iteration ended               */
  int64_t stop_iter; /* the iteration i at which it ended (x_i is the
                        answer of a stopping test or cap; G(x_i) was
                        returned by the step that broke down)               */
} aa_info;

/* Bytes of device workspace for a window of m columns over vectors of
 * length n (n >= 1; 1 <= m <= 64, or m = AA_MAX_COLS = 65 with AA_QR_ONLY
 * and a variant other than ICWY).  AA_EINVAL otherwise. */
aa_status aa_workspace_size(int64_t n, int m, int variant, unsigned flags,
                            size_t *bytes);

/* Create a context on the current HIP device.  d_workspace must be 256-byte
 * aligned and at least aa_workspace_size bytes; it is initialized on
 * `stream` (a hipStream_t, or NULL for the default stream). */
aa_status aa_init(aa_ctx **ctx, int64_t n, int m, int variant, unsigned flags,
                  void *d_workspace, size_t bytes, void *stream);

aa_status aa_set_stream(aa_ctx *ctx, void *stream);

/* One AA iteration (Alg. 1), asynchronous on the context's stream.
 * Call i = 0 (the first call): d_g = G(x_0); returns x_1 = G(x_0).
 * Call i >= 1: d_x = x_i, d_g = G(x_i); forms f_i, Delta f_{i-1} and
 * Delta g_{i-1}, updates the QR of F_i (QRDelete when i > m, then QRAdd),
 * solves R gamma = Q^T f_i and writes x_{i+1} = G(x_i) - sum gamma_j
 * Delta g_{i-m_i+j} to d_x_next.  d_x_next may alias d_x but not d_g. */
aa_status aa_step(aa_ctx *ctx, const double *d_x, const double *d_g,
                  double *d_x_next);

/* Replay steady-state iterations from HIP graphs (enable 1) or enqueue every
 * pass (0, the default).  Alg. 1 repeats the same passes once the window is
 * full; with graphs on, aa_step captures that iteration the first time each
 * ring-slot phase (i - 1) mod m comes round with the given x, G(x), x_next
 * pointers and replays it afterwards (one launch instead of about a dozen,
 * which at n below a few million is what an iteration costs).  Needs a
 * non-NULL stream; not used while profiling, for the one-workgroup step, or
 * after aa_qr_add / aa_qr_delete left k != m.  New pointers recapture that
 * phase; aa_reset, aa_set_stream, aa_set_grid, aa_set_fused_threshold and
 * aa_qr_load drop the graphs. */
aa_status aa_set_graph(aa_ctx *ctx, int enable);

/* Waits for the context's stream and reports the state of the last step. */
aa_status aa_get_info(aa_ctx *ctx, aa_info *h_info);

/* Stopping rule of aa_step (Alg. 1's tol and maxIters), evaluated on the
 * device so that a driver loop needs no per-step synchronization: with mode
 * AA_STOP_RESIDUAL the iteration ends at the start of iteration i >= 1 when
 * ||f_i||_2 <= tol ||f_0||_2; with AA_STOP_STEP when ||x_i - x_{i-1}||_2 < tol
 * (the paper's test on the step, in the 2-norm).  tol <= 0 disables the
 * test.  max_iter >= 1 caps the iterations i (0: no cap).  Once the iteration
 * has ended (test, cap or breakdown) every further aa_step leaves the state
 * unchanged and writes x_next = x (the host enqueues the same launches; they
 * return at once), and aa_get_info reports why and at which i; aa_reset
 * starts over.  Defaults: no test, no cap. */
aa_status aa_set_stop(aa_ctx *ctx, double tol, int64_t max_iter, int mode);

/* QRAdd (Alg. 2 with Alg. 3, 4, 5 or 6): append d_v (length n, not modified)
 * as column k; k -> k + 1.  AA_ESTATE if k == m. */
aa_status aa_qr_add(aa_ctx *ctx, const double *d_v);

/* QRDelete (Alg. 2): drop column 0 by Givens rotations; k -> k - 1.
 * ICWY also refreshes every row of T (T_ab = q_a^T q_b, b < a) with one
 * reduction.  (Inside aa_step, where a QRAdd always follows, the refresh
 * leaves the newest row to that QRAdd, whose first reduction recomputes it,
 * Alg. 4; the state after the step is the same.)  AA_ESTATE if k == 0. */
aa_status aa_qr_delete(aa_ctx *ctx);

/* Solve R gamma = Q^T d_f (Alg. 2, last line); d_gamma receives k doubles
 * (device).  AA_ESTATE if k == 0; AA_EINVAL if k > 64 (the solve is for
 * windows of at most 64 columns). */
aa_status aa_qr_solve(aa_ctx *ctx, const double *d_f, double *d_gamma);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc) and hold no
 * context: the same solve as aa_qr_solve (R gamma = Q^T f, the same kernels)
 * on a caller's factorization.  d_Q: k columns of length n, leading dimension
 * ldq >= n (device); d_R: k x k upper triangular, column-major, leading
 * dimension ldr >= k, nonsingular (device); d_f: n doubles (device); d_gamma:
 * k doubles out (device).  1 <= k <= 64, else AA_EINVAL.  Asynchronous on
 * `stream`.  Allocates nothing: the reduction partials live in a fixed
 * 257 KiB device array that every GPU the library runs on keeps until the
 * process ends, shared by all calls on that GPU -- calls that overlap on one
 * GPU (other streams, other host threads) race and must be serialized by the
 * caller. */
aa_status aa_qr_solve_noalloc(const double *d_Q, int64_t ldq, int64_t n, int k,
                              const double *d_R, int ldr, const double *d_f,
                              double *d_gamma, void *stream);

/* Copy R and T (k x k, column-major, leading dimension k) to host buffers
 * (either may be NULL) and report k.  Waits for the stream. */
aa_status aa_get_qr(aa_ctx *ctx, double *h_R, double *h_T, int *k);

/* Device pointer to Q (column j at *d_Q + j * *ldq) and its leading
 * dimension; Q lives in the caller's workspace. */
aa_status aa_qr_basis(aa_ctx *ctx, double **d_Q, int64_t *ldq);

/* Load an existing factorization (k columns of Q with leading dimension ldq,
 * k x k R, optional k x k T) -- used to start the QRAdd microbenchmark from a
 * given orthonormal basis.  Waits for the stream. */
aa_status aa_qr_load(aa_ctx *ctx, int k, const double *d_Q, int64_t ldq,
                     const double *h_R, const double *h_T);

/* Forget the history (k = 0, iteration index 0); keeps the workspace. */
aa_status aa_reset(aa_ctx *ctx);

aa_status aa_destroy(aa_ctx *ctx);

/* Number of reduction finalizations ("Syncs", Sec. 3) enqueued so far by
 * QRAdd, QRDelete and the right-hand side Q^T f, for comparison with the
 * paper's counts (Sec. 4.1).  Host-side counter, no wait. */
aa_status aa_sync_counts(aa_ctx *ctx, int64_t *add, int64_t *del, int64_t *rhs);

/* ---------------- measurement and tuning ---------------------------------- */

/* Kernel kinds, for per-kernel timing. */
typedef enum {
  AA_K_DOTS = 0,    /* block dot products Q^T [x, y] (+ x^T x)            */
  AA_K_UPDATE = 1,  /* v - Q c with fused dot / norm (+ DCGS-2 reorth)    */
  AA_K_CGS2B = 2,   /* CGS-2 second pass                                  */
  AA_K_GIVENS = 3,  /* Givens rotations from R (one wavefront)            */
  AA_K_ROTATE = 4,  /* rotation sweep over Q (+ ICWY Gram)                */
  AA_K_SCALE = 5,   /* q_k = w / R_kk                                     */
  AA_K_HISTORY = 6, /* f_i, Delta f, Delta g                              */
  AA_K_XUPDATE = 7, /* x_{i+1} = G(x_i) - sum gamma_j Delta g_j           */
  AA_K_FUSED = 8,   /* whole iteration in one workgroup (small n)         */
  AA_K_FINALIZE = 9, /* one-workgroup reduction + dense tail after a pass  */
  AA_K_COUNT = 10
} aa_kernel_kind;

/* Enable (1) or disable (0) per-launch timing: every pass the context
 * enqueues is bracketed by hipEvents on the context's stream, with one more
 * event between a streaming pass and its finalize kernel, so the pass and the
 * finalize are timed apart (events are created on the first enable; no device
 * memory is allocated).  Event records order the stream more strictly than
 * plain launches, so profiled steps run slightly slower than unprofiled
 * ones.  Disabling or aa_profile_reset discards what was recorded. */
aa_status aa_profile_enable(aa_ctx *ctx, int enable);

/* Totals for one kernel kind since the last reset: elapsed milliseconds
 * (sum of the event pairs), number of launches, and algorithmic HBM bytes
 * (each vector a launch must read or write counted once, 8 n bytes per
 * vector).  Waits for the context's stream. */
aa_status aa_profile_read(aa_ctx *ctx, int kind, double *ms, int64_t *launches,
                          double *bytes);
aa_status aa_profile_reset(aa_ctx *ctx);

/* Upper bounds on the workgroups of the streaming passes and of the ICWY
 * Gram pass (defaults 512 and 1024; each in [1, 4096]; the Gram pass also
 * keeps (workgroups) x (k-1)(k-2)/2 within its partials buffer).  A pass is
 * further limited to the workgroups of its kernel that the device holds at
 * once (one round), as the occupancy query reports. */
aa_status aa_set_grid(aa_ctx *ctx, int stream_max, int gram_max);

/* Largest n for which aa_step runs the whole iteration in one workgroup (one
 * launch instead of one per pass; default 20480 / m -- beyond that the
 * grid-wide passes are faster; 0 disables; m <= 64). */
aa_status aa_set_fused_threshold(aa_ctx *ctx, int64_t n_max);

/* ---------------- batched AA: many independent instances ------------------ */

/* Thousands of independent AA instances of uneven length n and window m
 * advance one iteration each per persistent launch: every workgroup pulls
 * instances from a work counter (largest n*m first) and runs the whole
 * iteration of Alg. 1 for that instance -- the model map G, history, QRDelete,
 * QRAdd by the chosen variant, R gamma = Q^T f_i, the x update -- so every
 * Sync of Sec. 3 becomes a workgroup barrier.  An instance stops (and is
 * skipped from then on) when ||f_i|| <= tol ||f_0|| at the start of iteration
 * i, when i reaches max_iter, or on breakdown. */
typedef struct {
  int64_t n;          /* vector length; n = s^dim                             */
  int m;              /* window, 1 <= m <= 64                                 */
  int dim;            /* model map G(u) = u - omega (A u + c u^3 - f) on an
                         s^dim Dirichlet grid (dim 1, 2 or 3)                 */
  int64_t s;          /* grid points per side                                 */
  double h, omega, c; /* spacing, relaxation weight, cubic coefficient        */
  const double *d_f;  /* right-hand side f, n doubles (device, caller-owned)  */
  double *d_x;        /* iterate: x_0 on entry; the current x_i afterwards
                         (device, caller-owned, 16-byte aligned)              */
} aa_batch_instance;

typedef struct {
  int64_t iter;       /* index i of the next iteration                        */
  int64_t stop_iter;  /* iteration i at which the instance stopped, -1 if not */
  int k, m_i, active, status;
  double res_norm;    /* ||f_i||_2 at the last history formation              */
  double res0_norm;   /* ||f_0||_2                                            */
  int64_t g_evals;    /* evaluations of G so far                              */
  int64_t accepted;   /* learned candidates accepted by the guard             */
  double loss;        /* last training loss sample of this instance           */
  int pending;        /* internal: iteration split across the network call    */
  int g_valid;        /* internal: G(x_i) already known (accepted candidate)  */
} aa_batch_state;

/* aa_batch_init flag: also allocate the learned step's candidate vectors and
 * feature / output buffers (required by aa_batch_run_learned and
 * aa_batch_train). */
enum { AA_BATCH_LEARNED = 1u << 9 };

aa_status aa_batch_workspace_size(int count, const aa_batch_instance *h_inst,
                                  int variant, unsigned flags, size_t *bytes);

/* h_inst: count descriptors (host; copied).  The workspace (device,
 * 256-byte aligned, caller-owned) holds every instance's Q, history, R, T and
 * the schedule.  flags: the QRAdd readings of aa_init (AA_DCGS2_LITERAL,
 * AA_DCGS2_GUARD_GE3), the pass fusions AA_FUSE_RHS and AA_FUSE_DELETE, and
 * AA_BATCH_LEARNED.  Each instance stops (on the device) at the start of the
 * first iteration with ||f_i|| <= tol ||f_0||, at max_iter, or on a
 * breakdown.  stream: a hipStream_t; a non-NULL stream lets aa_batch_run
 * replay a captured HIP graph. */
aa_status aa_batch_init(aa_batch **b, int count, const aa_batch_instance *h_inst,
                        int variant, unsigned flags, double tol, int64_t max_iter,
                        void *d_workspace, size_t bytes, void *stream);

/* Enqueue `iters` batched iterations (asynchronous). */
aa_status aa_batch_run(aa_batch *b, int iters);

/* Copy the per-instance states (h_states: count entries, may be NULL) and the
 * number of active instances (may be NULL).  Waits for the stream. */
aa_status aa_batch_read(aa_batch *b, aa_batch_state *h_states, int *h_active);

/* Schedule knobs (the autotuner's search space): persistent workgroups
 * (0 = 2 per compute unit), instance order (0 = largest n*m first,
 * 1 = as given), graph replay on/off. */
aa_status aa_batch_set_schedule(aa_batch *b, int grid, int order, int use_graph);

typedef struct {
  int grid;          /* persistent workgroups chosen                         */
  int order;         /* instance order chosen (as aa_batch_set_schedule)     */
  double ms_per_iter;/* its measured time per batched iteration              */
  int trials;        /* candidate schedules timed (0: taken from the cache)  */
  int pairs;         /* tiles chosen: row pairs per lane (aa_batch_set_tiles)*/
} aa_batch_schedule;

/* Tiles of the persistent kernel's passes: each lane streams `pairs` pairs
 * of consecutive rows per tile (2 or 4: tiles of 1024 or 2048 rows for the
 * 256-thread workgroup; two builds of the kernel).  Default 4. */
aa_status aa_batch_set_tiles(aa_batch *b, int pairs);

/* Large instances on many workgroups.  The persistent kernel gives every
 * instance one workgroup, which streams some 20 GB/s; while thousands are
 * active that fills the chip, but once at most `active_max` instances are
 * active (0: a quarter of the compute units) the active instances with
 * n >= min_n leave the persistent kernel and run their iterations on the
 * single-instance grid-wide passes (up to 1024 workgroups each), one
 * instance after another, the remaining ones staying in the persistent
 * kernel.  A split instance keeps its memory, its state and the batch's
 * stopping test (relative residual, iteration cap); its partial sums are
 * taken in another order (results agree to rounding), and a breakdown ends
 * it in the iteration that detects it with x_{i+1} = G(x_i), as aa_step
 * does.  The policy is evaluated when aa_batch_run starts (a wait for the
 * stream); split iterations are enqueued by the host, not replayed as
 * graphs; the learned entry points and the autotuner return every instance
 * to the persistent kernel first.  min_n = 0 disables the split (and
 * returns split instances).  Default: min_n = 65536, active_max = 0. */
aa_status aa_batch_set_split(aa_batch *b, int64_t min_n, int active_max);

/* Instances currently on the split path (as of the last aa_batch_run). */
aa_status aa_batch_split_count(const aa_batch *b, int *count);

/* Schedule autotuner (the batched path's tuning step; not in the paper).
 * Times `iters` real iterations of the batch under each candidate schedule
 * -- tiles {4, 2} row pairs per lane x persistent workgroups in {1, 2, 3, 4}
 * per compute unit (capped at the instance count) x instance order {largest
 * n*m first, as given} -- with events on the batch's stream, and keeps the
 * fastest (graph replay stays as set).  The iterations it runs are ordinary
 * progress of the batch, so call it once the windows are full (after max m
 * iterations) for a fair comparison.  With cache_path non-NULL the result is
 * looked up first in, and afterwards appended to, a text file of lines
 * "<gcn arch> <workload signature> <grid> <order> <pairs> <ms per
 * iteration>"; the signature hashes the format, the variant, the flags and
 * every instance's (n, m, dim).  A cache hit applies the stored schedule and
 * runs nothing.  best may be NULL.  Waits for the stream. */
aa_status aa_batch_autotune(aa_batch *b, int iters, const char *cache_path,
                            aa_batch_schedule *best);

/* Learned-guarded iterations (not part of the paper): after R gamma = Q^T f_i
 * the network proposes delta gamma and beta from R and Q^T f_i; the candidate
 * x_c = G(x_i) - G_i gamma' - (1 - beta)(f_i - Q R gamma'), gamma' = gamma +
 * delta gamma, is accepted iff ||G(x_c) - x_c|| < ||f_i|| (then G(x_c) serves
 * as G(x_{i+1})); otherwise the plain AA step x_{i+1} = G(x_i) - G_i gamma is
 * taken.  net must have max_batch >= count; the batch needs AA_BATCH_LEARNED. */
aa_status aa_batch_run_learned(aa_batch *b, aa_mlp *net, int iters);

/* Training iterations: plain AA steps (the trajectory the network learns
 * from); at each one the candidate's one-step loss log(||G(x_c)-x_c||^2 /
 * ||f_i||^2) is back-propagated through G (the adjoint of the symmetric
 * stencil map) into delta gamma and beta, then through the network, and one
 * Adam step (learning rate lr) is taken per iteration. */
aa_status aa_batch_train(aa_batch *b, aa_mlp *net, int iters, float lr);

/* Copy the learned step's buffers of the last iteration (count x 230
 * features, count x 21 network outputs, count x 21 loss gradients w.r.t. the
 * outputs, each may be NULL).  Waits. */
aa_status aa_batch_read_learning(aa_batch *b, float *h_feat, float *h_out, float *h_dout);

aa_status aa_batch_destroy(aa_batch *b);

/* ---------------- the learned mixing-weight network ---------------------- */

/* A small network that reads the n-independent state of the windowed QR --
 * the upper triangle of R and c = Q^T f_i, zero-padded to a 20-column window
 * and divided by ||f_i|| (230 features) -- and proposes a correction to the
 * mixing weights gamma (20 outputs) and a damping logit (1 output):
 * 230 -> 256 -> 256 -> 256 -> 21, GELU (erf form), BF16 operands on the
 * matrix cores with FP32 accumulation, FP32 master weights, Adam.  Not part
 * of the paper: an addition that never replaces the FP64 method (see the
 * guarded batched step). */
#define AA_MLP_FEATURES 230
#define AA_MLP_OUTPUTS 21

/* Parameters in the packed order W0 [256 x 256], b0 [256], W1, b1, W2, b2,
 * W3 [256 x 64], b3 [64] (row-major; inputs 230..255 and outputs 21..63 are
 * padding and stay zero). */
int64_t aa_mlp_param_count(void);
aa_status aa_mlp_workspace_size(int max_batch, size_t *bytes);
/* Seeded initialization: hidden layers N(0, 2/fan_in), last layer zero with
 * the damping-logit bias at +4 (no correction, beta = sigmoid(4)). */
aa_status aa_mlp_init(aa_mlp **net, int max_batch, uint64_t seed, void *d_workspace,
                      size_t bytes, void *stream);
aa_status aa_mlp_reseed(aa_mlp *net, uint64_t seed);
aa_status aa_mlp_set_params(aa_mlp *net, const float *h_params);  /* waits */
aa_status aa_mlp_get_params(aa_mlp *net, float *h_params);        /* waits */
aa_status aa_mlp_get_grads(aa_mlp *net, float *h_grads);          /* waits */
/* d_x: batch x 230 FP32 features; d_out: batch x 21 FP32 outputs (may be
 * NULL).  Keeps the activations for aa_mlp_backward. */
aa_status aa_mlp_forward(aa_mlp *net, int batch, const float *d_x, float *d_out);
/* d_dout: batch x 21 gradient of the loss w.r.t. the outputs of the last
 * forward (same batch); accumulates the parameter gradients. */
aa_status aa_mlp_backward(aa_mlp *net, int batch, const float *d_dout);
/* One Adam step with the accumulated gradients, which are then cleared. */
aa_status aa_mlp_adam(aa_mlp *net, float lr, float beta1, float beta2, float eps);
aa_status aa_mlp_destroy(aa_mlp *net);

/* ---------------- model fixed-point maps and seeded inputs --------------- */

/* d_out = d_u - omega (A d_u + c d_u^3 - d_f), A the (2 dim + 1)-point
 * Dirichlet Laplacian on an s^dim grid (x fastest) scaled by 1/h^2.
 * dim in {1, 2, 3}; d_out must not alias d_u. */
aa_status aa_problem_apply(int dim, int64_t s, double h, double omega, double c,
                           const double *d_f, const double *d_u, double *d_out,
                           void *stream);

/* Seeded inputs: element i of stream (seed, stream) is SplitMix64's output
 * function of a per-stream counter origin plus i; uniforms in [0, 1) scaled
 * to [lo, hi); normals by the Box-Muller cosine branch. */
aa_status aa_fill_uniform(double *d_out, int64_t n, uint64_t seed,
                          uint64_t stream_id, uint64_t offset, double lo,
                          double hi, void *stream);
aa_status aa_fill_normal(double *d_out, int64_t n, uint64_t seed,
                         uint64_t stream_id, uint64_t offset, void *stream);

/* The EM map of Sec. 5.3 (the paper's third test problem): the means of a
 * three-component univariate normal mixture with known proportions alpha and
 * standard deviations sigma, estimated from unlabeled samples.  With the
 * current means mu = d_u[0..2],
 *   w_ik = alpha_i N(x_k; mu_i, sigma_i^2) / sum_j alpha_j N(x_k; mu_j, sigma_j^2),
 *   G(mu)_i = sum_k x_k w_ik / sum_k w_ik,
 * written to every replica: d_out[3 r + i] = G(mu)_i for r < n / 3 (the
 * paper estimates one set of means redundantly in every entry of the AA
 * vector, so the map costs O(nsamples + n)).  d_x: nsamples doubles
 * (device); d_u, d_out: n doubles, n a positive multiple of 3 (d_out may
 * alias d_u); d_work: at least AA_EM_WORK_DOUBLES doubles of device scratch
 * owned by the caller.  alpha_i > 0, sigma_i > 0.  Sums in a fixed order
 * (deterministic).  Asynchronous on `stream`. */
#define AA_EM_WORK_DOUBLES 6144
typedef struct {
  double alpha[3];
  double sigma[3];
} aa_em_mixture;
aa_status aa_em_apply(const aa_em_mixture *h_mix, const double *d_x, int64_t nsamples,
                      const double *d_u, double *d_out, int64_t n, double *d_work,
                      void *stream);

/* The fixed-point maps of the paper's 2D test problems on the unit square,
 * N x N interior points (x fastest, h = 1 / (N + 1)), zero Dirichlet values:
 *   AA_PDE_HEAT_NL1, AA_PDE_HEAT_NL2 -- the steady heat equation with a
 *     nonlinear term of Sec. 5.1, u_xx + u_yy + c(u) = f with
 *     c(u) = u + u e^u + u e^-u + (u - e^u)^2 (term 1) or 100 (u - u^2)
 *     (term 2); G(u) = A^{-1}(c(u) - b), b = f at the grid points;
 *   AA_PDE_BRATU -- the Bratu problem of Sec. 5.2, u_xx + u_yy + lambda e^u
 *     = 0; G(u) = A^{-1}(lambda e^u);
 * A = -L_h, L_h the 5-point Laplacian (second-order centred differences).
 * Each evaluation solves A x = rhs by the conjugate gradient preconditioned
 * with one geometric-multigrid V(1,1) cycle (the paper uses a structured
 * multigrid preconditioner of an external library; this one is the
 * library's own): red-black Gauss-Seidel, red then black before the coarse
 * correction and black then red after it, full weighting, bilinear
 * interpolation, coarse point I at fine point 2 I + 1, coarse levels the
 * 5-point operator at spacing 2^l h whose last row and column keep the
 * boundary at its true distance (diagonal (1 + 2^l) / H^2 from that side:
 * the 1D Galerkin products).  The grid halves while N is even; the sizes must
 * reach one of at most 32 (N = a 2^j with odd a <= 32, N <= 65536), else
 * AA_EINVAL.  The solve starts from x = 0 and stops before iteration k when
 * ||r_k||_2 <= tol ||rhs||_2, or at max_iter (not converged: see
 * aa_pde2d_last).  The stopping test runs on the device; the host reads the
 * solve's state after a batch of iterations sized by the previous solve, so
 * aa_pde2d_apply and aa_pde2d_solve return after the stream has reached
 * the end of the solve (they synchronize `stream`).
 *
 * Workspace: caller-owned device memory of aa_pde2d_workspace_size bytes,
 * 256-byte aligned (about 7 N^2 doubles), kept alive until
 * aa_pde2d_destroy; the context is a small host allocation.  One context
 * per stream; calls on one context must not overlap. */
typedef struct aa_pde2d aa_pde2d;
enum { AA_PDE_HEAT_NL1 = 1, AA_PDE_HEAT_NL2 = 2, AA_PDE_BRATU = 3 };
aa_status aa_pde2d_workspace_size(int64_t N, int max_iter, size_t *bytes);
aa_status aa_pde2d_init(aa_pde2d **ctx, int64_t N, int problem, double lambda, double tol,
                        int max_iter, void *d_workspace, size_t bytes, void *stream);
/* d_out = G(d_u); d_b: the heat problems' source f at the grid points (N^2
 * doubles; ignored and may be null for Bratu).  d_out may alias d_u. */
aa_status aa_pde2d_apply(aa_pde2d *ctx, const double *d_b, const double *d_u, double *d_out);
/* d_x = A^{-1} d_rhs by the same PCG (d_x must not alias d_rhs). */
aa_status aa_pde2d_solve(aa_pde2d *ctx, const double *d_rhs, double *d_x);
/* d_z = B d_r, one V-cycle (the preconditioner) on the fine grid; async. */
aa_status aa_pde2d_vcycle(aa_pde2d *ctx, const double *d_r, double *d_z);
/* iters >= 0: every later solve runs exactly that many PCG iterations
 * (<= max_iter) regardless of the tolerance; -1 restores the test. */
aa_status aa_pde2d_set_iters(aa_pde2d *ctx, int iters);
/* PCG iterations of the last solve and whether it met the tolerance. */
aa_status aa_pde2d_last(const aa_pde2d *ctx, int *h_iters, int *h_converged);
aa_status aa_pde2d_set_stream(aa_pde2d *ctx, void *stream);
aa_status aa_pde2d_destroy(aa_pde2d *ctx);

/* Measurement: the sustained HBM bandwidth of an access pattern, with the
 * streaming passes' tiles, loads, stores and launch shape (at most 1024
 * workgroups, one resident round).  Reads `reads` vectors of length n from
 * d_src (vector j at d_src + j * ld) and writes `writes` vectors to d_dst
 * (each the sum of the read ones); with writes == 0 every workgroup writes
 * one partial sum to d_sink (at least 1024 doubles).  (reads, writes) in
 * {(1,0), (4,0), (8,0), (1,1), (2,1), (3,1), (8,1), (1,2)}, else AA_EINVAL.
 * Asynchronous on `stream`. */
aa_status aa_bandwidth_probe(int reads, int writes, const double *d_src, int64_t ld,
                             double *d_dst, int64_t n, double *d_sink, void *stream);

/* Library version string. */
const char *aa_version(void);

#ifdef __cplusplus
}
#endif
#endif /* AA_H */
