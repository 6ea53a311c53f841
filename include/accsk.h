/*
 * accsk.h -- C ABI of the MI355X (gfx950) Acc-Sinkhorn library.
 *
 * Entropy-regularized optimal transport (paper Sec. 1, eq:EOT):
 *     min_{P in Pi(a,b)}  <C,P> + eps * sum_ij P_ij (log P_ij - 1)
 * solved in the dual (Sec. 2, eq:dual-obj / eq:dual-min) by log-domain
 * Sinkhorn (eq:u-update, eq:v-update, normalized as eq:normalized-sinkhorn) or
 * by Acc-Sinkhorn (Algorithm A2MD inside the homotopy of Algorithm
 * A2MD-homotopy, Sec. 4), stopped by the L1 marginal rule eq:l1tol.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named as device pointers must point to device memory of the
 *   current HIP device; all work is enqueued on `stream` (a hipStream_t passed
 *   as void*, NULL = the legacy default stream).  The caller owns every input
 *   and output buffer.  The library owns only scratch memory it allocates
 *   stream-ordered inside the call and frees before returning.
 * - Matrices are row-major with a leading dimension (in elements) >= the row
 *   length.  Potentials are FP64.
 * - Marginals a (length n) and b (length m) must be finite and > 0; they are
 *   rescaled to unit mass inside the call (eq:Fc needs 1'a = 1'b = 1).
 * - Potentials returned are f = eps*u and g = eps*v in cost units, so that
 *   P_ij = exp((f_i + g_j - C_ij)/eps) (eq:P-from-dual); g is centred
 *   (sum_j g_j = 0, the gauge of eq:Fc).
 * - Calls that fill an accsk_result (host pointer) block until their work on
 *   `stream` has finished.  Other calls only enqueue work.
 * - Stream-ordered forms (names ending in _async) take the result records in
 *   device memory (or host-mapped pinned memory) instead and only enqueue
 *   work: the records are written by the device when the stream reaches the
 *   end of the solve, so several solves can be queued back to back, overlap
 *   host work, and be waited for with one event or stream synchronization.
 *   Their return value reports what the host can check before enqueueing
 *   (INVALID_ARG, SHAPE, OOM, HIP_ERROR); a problem's own outcome (OK,
 *   NOT_CONVERGED, NONFINITE, INVALID_ARG for a non-positive marginal entry,
 *   DIVERGED) is in its record's `status`, and its kernel_ms is measured on the
 *   device clock.  Input buffers must stay valid until the stream has passed
 *   the call's work.
 * - Errors are reported by the return value; no exception crosses the ABI.
 *   On any status other than ACCSK_OK / ACCSK_NOT_CONVERGED the output
 *   buffers are unspecified.
 */
#ifndef ACCSK_H
#define ACCSK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ACCSK_OK = 0,
    ACCSK_INVALID_ARG = 1,   /* bad scalar argument or non-positive marginal entry */
    ACCSK_SHAPE = 2,         /* sizes / leading dimensions / alignment not supported */
    ACCSK_NONFINITE = 3,     /* NaN or Inf met in the cost or the marginals */
    ACCSK_NOT_CONVERGED = 4, /* max_iter reached; outputs hold the last iterate */
    ACCSK_DIVERGED = 5,      /* the marginal error became non-finite during the solve */
    ACCSK_OOM = 6,           /* device allocation failed or HBM budget exceeded */
    ACCSK_HIP_ERROR = 7,     /* a HIP runtime call failed */
    ACCSK_BUSY = 8           /* serving queue full; retry later */
} accsk_status;

typedef enum { ACCSK_SINKHORN = 0, ACCSK_ACC = 1 } accsk_method;

/* Hand-off of w = alpha*y between homotopy stages (alpha changes with mu):
 * Y_CONTINUOUS keeps y (w scaled by alpha_new/alpha_old, the state the
 * homotopy analysis of Theorem thm:homotopy carries); LITERAL passes w
 * unchanged as Algorithm A2MD-homotopy prints it. */
typedef enum { ACCSK_W_LITERAL = 0, ACCSK_W_Y_CONTINUOUS = 1 } accsk_w_rule;

/* On-the-fly costs from point clouds X (n x d) and Y (m x d):
 * SQEUCLID: C_ij = ||x_i - y_j||^2 / scale   (Sec. 5, colour transfer)
 * COSINE:   C_ij = (1 - <x_i, y_j>) / scale  (Sec. 5, word alignment; unit rows) */
typedef enum { ACCSK_SQEUCLID = 0, ACCSK_COSINE = 1 } accsk_cost;

typedef struct {
    int32_t method;     /* accsk_method */
    int32_t w_rule;     /* accsk_w_rule */
    double eps;         /* regularization, > 0 */
    double tol;         /* stop when ||P1-a||_1 + ||P'1-b||_1 < tol (eq:l1tol), > 0 */
    int64_t max_iter;   /* cap on iterations (It), >= 0 */
    double mu0;         /* homotopy start, 0 < mu0 < 1 (Algorithm A2MD-homotopy) */
    int64_t m0;         /* inner iterations of the first stage, >= 1 */
    int32_t split;      /* point-cloud cross terms X Y^T: 0 = FP64 dot products (default),
                           2 or 3 = BF16 matrix cores on a 2- or 3-piece split of X and Y */
    int32_t flags;      /* ACCSK_FLAG_* bits */
    double *err_trace;  /* optional device FP64 buffer, NULL for none: err_trace[k] receives the L1
                           marginal error (eq:l1tol, as the stop test computes it) of the iterate
                           evaluated by the k-th Sinkhorn step, for k < trace_len.  Calls on one
                           problem only (accsk_solve_dense, accsk_solve_points, batches of one);
                           with several problems, or on a server, it is INVALID_ARG */
    int64_t trace_len;  /* entries of err_trace, >= 0 */
} accsk_params;

#define ACCSK_FLAG_NO_COST 1       /* skip the final <C,P> pass */
#define ACCSK_FLAG_NO_SERPENTINE 2 /* traverse C in the same row order every step */
#define ACCSK_FLAG_ON_THE_FLY 4    /* point-cloud solves: form C_ij on the fly in every step (never stored);
                                      implied when m > 8192.  FP64 dot products for d <= 16; the BF16
                                      matrix-core cross term of p->split (2 or 3) pieces for 16 < d <= 128
                                      (split 0 with d > 16 is SHAPE) */
#define ACCSK_FLAG_RESTART 8       /* Acc-Sinkhorn: when the reduced dual objective f(x) = 1 - <u,a> - <x,b>
                                      rises (stability monitor), reset the extrapolation w <- alpha x.  A
                                      safeguard of this library (function-value restart), not the paper's
                                      algorithm; off by default */
#define ACCSK_FLAG_CONDITIONS 16   /* Acc-Sinkhorn: evaluate, in FP64 at every iterate, the two boundedness
                                      conditions of Theorem thm:condition-boundedness (App. B) with the metric
                                      D(p(x)) of eq:D (the logarithmic mean of the column sums c and b) and the
                                      shifted Lyapunov function of its proof, and count violations and rises
                                      (accsk_result.cond1_violations, cond2_violations, lyap_increases).  A
                                      monitor: the iterates are unchanged.  Costs O(m) FP64 work per step,
                                      done by one workgroup; batches of several problems and servers refuse it */

typedef struct {
    int64_t iters;          /* It: accepted iterates after x_0 (Sinkhorn: v-updates) */
    int64_t sinkhorn_steps; /* Sinkhorn steps evaluated (= iters + 1) */
    int64_t fallback_steps; /* steps that needed the exact column-max pass */
    int64_t fval_increases; /* stability monitor: steps at which f(x) = 1 - <u,a> - <x,b> (Lemma coercivity)
                               rose by more than 1e-8 + 1e-12 |f| over the previous iterate */
    int64_t restarts;       /* extrapolation resets done under ACCSK_FLAG_RESTART */
    int64_t cond1_violations; /* ACCSK_FLAG_CONDITIONS: iterates at which the first condition of Theorem
                                 thm:condition-boundedness, ||grad f(x_k)||^2 in the metric D_k^-1 D_k+1 D_k^-1
                                 < (4 - alpha^2 - 2 alpha^(1/2)) / (2 alpha (1+alpha)^2) D_phi*(0, grad f(x_k)),
                                 failed (pairs of consecutive iterates of one homotopy stage); -1 if not evaluated */
    int64_t cond2_violations; /* the same for the second condition, ||v_k||^2 in the metric D_k+1 - D_k
                                 < alpha^(3/2) ||v_k+1||^2 in D_k+1 (v = w/alpha - x) */
    int64_t lyap_increases;   /* rises of the proof's shifted Lyapunov function f(x) + (mu/2)||v||_D^2
                                 - theta/(1+alpha) D_phi*(0, grad f(x)) within a stage; -1 if not evaluated */
    double marginal_err;    /* eq:l1tol at the returned iterate, column part (row part is 0 by the exact row solve) */
    double eot_value;       /* dual value <f,a> + <g,b> - eps*sum P (equals the EOT optimum at
                               convergence), FP64-evaluated unless ACCSK_FLAG_NO_COST; problems that
                               accsk_solve_batch gives one workgroup sum FP32 exponentials in FP64
                               instead (sum P to ~1e-8 relative) */
    double transport_cost;  /* <C,P> at the returned potentials (NaN if skipped), evaluated as eot_value */
    double dual_fval;       /* reduced dual objective f(x) = 1 - <u,a> - <x,b> at eps = 1 (Lemma coercivity) */
    double kernel_ms;       /* duration of the solve kernel (HIP events on `stream`); for a batch, the
                               launch that solved this problem (shared by the problems of that launch) */
    int32_t converged;      /* 1 if marginal_err < tol */
    int32_t status;         /* accsk_status of the call */
} accsk_result;

/* Fills the defaults: ACC, Y_CONTINUOUS, eps 1e-2, tol 1e-6, max_iter 100000,
 * mu0 and m0 as calibrated on the FP64 oracle, split 0, flags 0. */
void accsk_default_params(accsk_params *p);

/* Human-readable name of a status code (static storage). */
const char *accsk_status_string(int status);

/*
 * Upper bound of the device workspace (bytes) that accsk_solve_dense,
 * accsk_solve_batch or accsk_solve_batch_strided allocates for `count`
 * problems of at most n x m.  The library allocates it stream-ordered from the
 * device's default memory pool (hipMallocAsync / hipFreeAsync on the caller's
 * stream), so a caller can pre-size that pool with this figure.  Needs the
 * current device (its CU count).  Errors: INVALID_ARG (bytes NULL, count < 1),
 * SHAPE (n or m < 1), HIP_ERROR (no device).
 */
accsk_status accsk_workspace_bytes(int64_t n, int64_t m, int64_t count, size_t *bytes);

/*
 * Measured HBM read bandwidth (GB/s), the reference beside the published peak
 * for kernels bound by reading HBM: a read-only stream kernel (grid-stride
 * float4 loads, 4 to 16 in flight per thread) over the first `bytes` (rounded
 * down to 16) of the device buffer buf (16-byte aligned), timed with HIP
 * events over `reps` launches after one warm-up, in three launch shapes; the
 * best rate is returned.  A buffer larger than the 256 MB last-level cache
 * measures HBM; a smaller one re-read measures what the cache adds.  Not part
 * of the solve.  Errors: INVALID_ARG, OOM, HIP_ERROR.
 */
accsk_status accsk_read_bandwidth(const void *buf, int64_t bytes, int32_t reps, double *gbps, void *stream);

/*
 * Measured ceiling of the FP32 exponential (v_exp_f32), the reference for the
 * exponential-bound solvers: 8 independent chains a <- 2^(-a) per thread, 8
 * waves per SIMD on every CU, timed with HIP events over `reps` launches after
 * one warm-up; *per_s receives the best rate in exponentials per second.  Not
 * part of the solve.  Errors: INVALID_ARG, OOM, HIP_ERROR.
 */
accsk_status accsk_exp_rate(int32_t reps, double *per_s, void *stream);

/* Library version string (static storage). */
const char *accsk_version(void);

/*
 * Dense solve on an explicit FP32 cost (Sec. 2 dual, Sec. 4 algorithms).
 * C: device, n x m row-major, leading dimension ldc >= m.  a: device FP64[n],
 * b: device FP64[m].  f_out: device FP64[n], g_out: device FP64[m].
 * res: host.  Sizes: 1 <= n, 1 <= m.  For m <= 8192 this is accsk_solve_batch
 * with one problem: n*m <= 65536 is solved by one workgroup; larger problems by
 * cooperating workgroups that each own a block of about 16 rows, and every
 * Sinkhorn step reads C once (row and column sums fused).
 * Larger m, or a row block too large for on-chip memory, uses the tiled
 * solver (a row sweep and a column sweep, two reads of C per step).
 * Returns ACCSK_OK, ACCSK_NOT_CONVERGED (outputs valid), or an error.
 */
accsk_status accsk_solve_dense(const float *C, int64_t n, int64_t m, int64_t ldc,
                               const double *a, const double *b, const accsk_params *p,
                               double *f_out, double *g_out, accsk_result *res, void *stream);

/*
 * Stream-ordered form of accsk_solve_dense (same arguments, routing, kernels
 * and results): res is a device pointer (or host-mapped pinned memory) to one
 * accsk_result, written by the device; the call returns once the work is
 * enqueued (Sec. 2 problem statement: (C; a, b; eps; tol) -> (f, g, cost, It)).
 */
accsk_status accsk_solve_dense_async(const float *C, int64_t n, int64_t m, int64_t ldc,
                                     const double *a, const double *b, const accsk_params *p,
                                     double *f_out, double *g_out, accsk_result *res, void *stream);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * serving loops or harnesses that forbid hipMalloc): accsk_solve_dense with
 * the same arguments, routing, kernels and results, but no device allocation
 * by the library (no hipMalloc, hipMallocAsync or HIP events).  Its workspace
 * is one fixed device array of ACCSK_NOALLOC_SCRATCH_BYTES per GPU, held from
 * the library's load until the process ends; kernel_ms is then measured on the
 * device clock.  Every call on one GPU uses that GPU's array, so calls whose
 * work overlaps on one GPU (other streams, other host threads) race and must
 * be serialized by the caller; work enqueued on one stream is ordered.
 * Limits: m <= 8192, and a workspace (one workgroup or one cooperative launch
 * of up to one workgroup per compute unit, plus the FP64 evaluation) within
 * ACCSK_NOALLOC_SCRATCH_BYTES, e.g. n = m = 8192 or n up to about 100000 at
 * m = 8192; larger problems, and problems whose row blocks do not fit on chip
 * (which accsk_solve_dense hands to the tiled solver), return ACCSK_SHAPE
 * before any work is enqueued.  The call blocks like accsk_solve_dense.
 */
#define ACCSK_NOALLOC_SCRATCH_BYTES ((size_t)48 << 20)
accsk_status accsk_solve_dense_noalloc(const float *C, int64_t n, int64_t m, int64_t ldc,
                                       const double *a, const double *b, const accsk_params *p,
                                       double *f_out, double *g_out, accsk_result *res, void *stream);

/*
 * Transport plan rows [row0, row0+rows) from potentials (eq:P-from-dual):
 * P_ij = exp((f_i + g_j - C_ij)/eps), written as FP32 to P (device,
 * rows x m, leading dimension ldp >= m).  f, g: device FP64 (full length).
 */
accsk_status accsk_plan_dense(const float *C, int64_t n, int64_t m, int64_t ldc, double eps,
                              const double *f, const double *g, int64_t row0, int64_t rows,
                              float *P, int64_t ldp, void *stream);

/*
 * FP64-accumulated evaluation of potentials (f, g) on an explicit cost
 * (eq:P-from-dual, eq:l1tol, eq:dual-obj): out (host FP64[5]) receives
 * ||P1 - a||_1, ||P'1 - b||_1, <f,a> + <g,b> - eps*sum P, <C,P>, sum P,
 * with a, b used as given (the caller normalizes).
 */
accsk_status accsk_eval_dense(const float *C, int64_t n, int64_t m, int64_t ldc, double eps,
                              const double *a, const double *b, const double *f, const double *g,
                              double *out, void *stream);

/* One problem of a batch (explicit FP32 cost).  All pointers are device
 * pointers; C is n x m row-major with leading dimension ldc >= m. */
typedef struct {
    const float *C;
    int64_t n, m, ldc;
    const double *a, *b; /* marginals, > 0, normalized inside */
    double *f, *g;       /* outputs: potentials in cost units */
    double eps;          /* regularization of this problem, > 0 */
} accsk_problem;

/*
 * Batched solve of independent dense problems (Sec. 2 dual, Sec. 4
 * algorithms, stopping rule eq:l1tol per problem).  A problem that fits one
 * workgroup (m <= 1024, n <= 4096 and (8m + 4n) * 8 bytes <= 150 KiB) is
 * owned by one workgroup when n*m <= 65536 or the batch has more than 64
 * problems: iterate, extrapolation state and homotopy counters stay in
 * on-chip memory and no grid-wide barrier is used.  Other problems
 * (m <= 8192) share persistent launches, a group of workgroups per problem
 * with its own barrier (a problem whose row blocks do not fit on chip goes to
 * the tiled solver).  Every problem stops on its own test.  probs: host array of `count` descriptors (the library copies it);
 * res: host array of `count` results.  p supplies method, tol, max_iter,
 * mu0, m0, w_rule and flags (p->eps is ignored; each problem has its own).
 * Limits per problem: 1 <= m <= 8192, 1 <= n.
 * Returns ACCSK_OK if every problem converged, ACCSK_NOT_CONVERGED if some hit
 * max_iter, otherwise the first error (per-problem status in res[k].status).
 */
accsk_status accsk_solve_batch(const accsk_problem *probs, int64_t count, const accsk_params *p,
                               accsk_result *res, void *stream);

/*
 * accsk_solve_batch for `batch` problems of one shape stored as strided arrays
 * (Sec. 2 dual, Sec. 4 algorithms, eq:l1tol per problem; same routing and
 * kernels).  Problem k: cost C + k*stride_c (device FP32, n x m row-major,
 * leading dimension ldc >= m, stride_c >= (n-1)*ldc + m), marginals a + k*n and
 * b + k*m (device FP64, > 0, normalized inside), outputs f_out + k*n and
 * g_out + k*m (device FP64).  eps: host FP64[batch] of per-problem
 * regularizations, or NULL for p->eps in every problem.  res: host array of
 * `batch` results.  The descriptors are built on the host, so a large batch
 * costs one call.  Returns as accsk_solve_batch.
 */
accsk_status accsk_solve_batch_strided(const float *C, int64_t batch, int64_t n, int64_t m, int64_t ldc,
                                       int64_t stride_c, const double *a, const double *b, const double *eps,
                                       const accsk_params *p, double *f_out, double *g_out, accsk_result *res,
                                       void *stream);

/* Stream-ordered form of accsk_solve_batch_strided: res is a device array of
 * `batch` records written by the device (eps, when given, is still a host
 * array); returns once the work is enqueued. */
accsk_status accsk_solve_batch_strided_async(const float *C, int64_t batch, int64_t n, int64_t m, int64_t ldc,
                                             int64_t stride_c, const double *a, const double *b, const double *eps,
                                             const accsk_params *p, double *f_out, double *g_out,
                                             accsk_result *res, void *stream);

/*
 * Cost matrix from point clouds (Sec. 5: squared Euclidean for colour
 * transfer, cosine for word alignment).  X: device FP32 n x d, Y: device FP32
 * m x d (row-major, rows contiguous).  C: device FP32 n x m, leading
 * dimension ldc >= m.  cost_scale s > 0 divides the raw cost.
 * split: 0 = FP64 dot products (C exact up to its FP32 rounding); 2 or 3 =
 * BF16 matrix cores on a 2- or 3-piece BF16 split of X and Y (cross-term
 * pieces down to 2^-16 or 2^-24 relative, FP32 accumulation per 32-wide K
 * chunk, chunks summed in FP64).  Limits: d <= 512.
 */
accsk_status accsk_cost_points(const float *X, const float *Y, int64_t n, int64_t m, int64_t d, int kind,
                               double cost_scale, int split, float *C, int64_t ldc, void *stream);

/*
 * accsk_cost_points for a batch of equal-shape problems in one launch: X is
 * batch x n x d, Y batch x m x d (problems consecutive), and problem k's cost
 * goes to C + k n ldc (leading dimension ldc >= m).  Same arguments, costs and
 * limits otherwise; batch >= 1.
 */
accsk_status accsk_cost_points_batched(const float *X, const float *Y, int64_t batch, int64_t n, int64_t m,
                                       int64_t d, int kind, double cost_scale, int split, float *C, int64_t ldc,
                                       void *stream);

/*
 * Point-cloud solve: builds the cost as accsk_cost_points does (with
 * p->split) into library scratch memory and solves EOT on it.  a, b, f_out,
 * g_out as for accsk_solve_dense.  With ACCSK_FLAG_ON_THE_FLY, or when
 * m > 8192, the cost is instead formed on the fly in every step from X and Y
 * by the tiled solver (a row sweep and a column sweep per step; nothing of
 * size n x m is stored): FP64 dot products for d <= 16, and for
 * 16 < d <= 128 with p->split 2 or 3 the cross term x_i . y_j on BF16 matrix
 * cores (Sec. 5 costs: |x|^2 + |y|^2 - 2 x.y or 1 - x.y, norms in FP64) with
 * all products of a 16 x 16 tile accumulated in FP32.  For m > 8192 with
 * d > 128, or with split 0 and d > 16, the cost is built explicitly and
 * solved by the tiled solver.  Limits: d <= 512.
 */
accsk_status accsk_solve_points(const float *X, const float *Y, int64_t n, int64_t m, int64_t d, int kind,
                                double cost_scale, const double *a, const double *b, const accsk_params *p,
                                double *f_out, double *g_out, accsk_result *res, void *stream);

/*
 * Transport plan rows [row0, row0+rows) for point clouds (eq:P-from-dual):
 * P_ij = exp((f_i + g_j - C_ij)/eps) with C_ij formed in FP64 from X and Y
 * (as accsk_cost_points with split 0; cost_scale s divides the raw cost),
 * written as FP32 to P (device, rows x m, leading dimension ldp >= m).
 * f: device FP64[n], g: device FP64[m].  Limits: d <= 512.
 */
accsk_status accsk_plan_points(const float *X, const float *Y, int64_t n, int64_t m, int64_t d, int kind,
                               double cost_scale, double eps, const double *f, const double *g, int64_t row0,
                               int64_t rows, float *P, int64_t ldp, void *stream);

/*
 * Barycentric projection of X through the plan (the colour-transfer map of
 * Sec. 5): T_i = sum_j P_ij y_j / sum_j P_ij with P_ij = exp((f_i + g_j -
 * C_ij)/eps) recomputed tile by tile (C in FP64, FP32 exponentials of FP64
 * arguments, FP64 sums), never stored.  T: device FP32 n x d.  Limits: d <= 448.
 */
accsk_status accsk_barycentric_points(const float *X, const float *Y, int64_t n, int64_t m, int64_t d, int kind,
                                      double cost_scale, double eps, const double *f, const double *g, float *T,
                                      void *stream);

/*
 * Row top-k of the plan (the retrieval of Sec. 5 word alignment): for each row
 * i the k columns with the largest P_ij, in decreasing order, decided on
 * g_j - C_ij in FP64 (ties: lower column first).  idx: device int64 n x k;
 * val: device FP64 n x k plan values (may be NULL).  k in {1, 5, 8}.
 */
accsk_status accsk_topk_points(const float *X, const float *Y, int64_t n, int64_t m, int64_t d, int kind,
                               double cost_scale, double eps, const double *f, const double *g, int k,
                               int64_t *idx, double *val, void *stream);

/*
 * Exact maximum of the raw point-cloud cost (before division by a scale):
 * max_ij ||x_i - y_j||^2 (SQEUCLID) or max_ij (1 - <x_i, y_j>) (COSINE), each
 * entry summed in FP64 as accsk_cost_points does with split 0 (Sec. 5 divides
 * the colour-transfer cost by its maximum).  out: host double.  Limits: d <= 512.
 */
accsk_status accsk_cost_max_points(const float *X, const float *Y, int64_t n, int64_t m, int64_t d, int kind,
                                   double *out, void *stream);

/*
 * Batch of `batch` independent point-cloud problems of equal shape: X is
 * batch x n x d, Y batch x m x d, a batch x n, b batch x m, f_out batch x n,
 * g_out batch x m (all contiguous device arrays); res: host array of `batch`
 * results.  Every problem stops on its own test (accsk_solve_batch).
 */
accsk_status accsk_solve_points_batched(const float *X, const float *Y, int64_t batch, int64_t n, int64_t m,
                                        int64_t d, int kind, double cost_scale, const double *a,
                                        const double *b, const accsk_params *p, double *f_out, double *g_out,
                                        accsk_result *res, void *stream);

/* Stream-ordered form of accsk_solve_points_batched (and, with batch = 1, of
 * accsk_solve_points): res is a device array of `batch` records written by the
 * device; returns once the work is enqueued. */
accsk_status accsk_solve_points_batched_async(const float *X, const float *Y, int64_t batch, int64_t n,
                                              int64_t m, int64_t d, int kind, double cost_scale, const double *a,
                                              const double *b, const accsk_params *p, double *f_out,
                                              double *g_out, accsk_result *res, void *stream);

/*
 * Gradients of the EOT value at the potentials (f, g) by the envelope theorem
 * (dEOT/dC = P with P_ij = exp((f_i + g_j - C_ij)/eps), eq:P-from-dual), for a
 * batch of equal-shape point-cloud problems laid out as in
 * accsk_solve_points_batched.  P is recomputed tile by tile (never stored),
 * with the cost formed in FP64 from X and Y.  grad_scale: device FP64[batch]
 * upstream gradient per problem, or NULL for 1.  Outputs (device, scaled by
 * grad_scale): dX (batch x n x d FP32), dY (batch x m x d FP32) and, if not
 * NULL, da (batch x n FP64) = (f - <f, a/sum a>)/sum a and db likewise, the
 * gradients with respect to un-normalized marginals.  a, b may be NULL when
 * da, db are.  Limits: d <= 448.
 */
accsk_status accsk_backward_points(const float *X, const float *Y, int64_t batch, int64_t n, int64_t m,
                                   int64_t d, int kind, double cost_scale, double eps, const double *a,
                                   const double *b, const double *f, const double *g, const double *grad_scale,
                                   float *dX, float *dY, double *da, double *db, void *stream);

/*
 * Gradients of the EOT value of an explicit-cost problem at the potentials
 * (f, g) by the envelope theorem (eq:P-from-dual): dC = grad_scale * P with
 * P_ij = exp((f_i + g_j - C_ij)/eps) (FP64 argument and exponential, written as
 * FP32, device n x m with leading dimension lddc >= m), and, if not NULL,
 * da = grad_scale * (f - <f, a/sum a>)/sum a and db likewise (device FP64), the
 * gradients with respect to un-normalized marginals.  C (leading dimension
 * ldc >= m) may be NULL when dC is; a, b may be NULL when da, db are.
 * grad_scale: device FP64[1] upstream gradient, or NULL for 1.  f, g are the
 * potentials a solve returned (device FP64).  Nothing is allocated; the call
 * only enqueues work on stream.
 */
accsk_status accsk_backward_dense(const float *C, int64_t n, int64_t m, int64_t ldc, double eps,
                                  const double *a, const double *b, const double *f, const double *g,
                                  const double *grad_scale, float *dC, int64_t lddc, double *da, double *db,
                                  void *stream);

/*
 * ---------------------------------------------------------------------------
 * Serving loop (continuous batching of point-cloud requests).
 *
 * A server owns one persistent kernel on its own stream: requests of uneven
 * (n, m, eps) are admitted while others run, each is solved by one workgroup
 * (cost built on the device, then the Sec. 4 Algorithms A2MD / A2MD-homotopy
 * with the Sec. 2 row solve, stop on eq:l1tol per request), and each retires
 * on its own test.  Admission is by HBM footprint: every request needs an
 * n x ceil4(m) FP32 cost block from the server's arena of hbm_budget bytes; a
 * request waits until a block fits (later requests that fit may go first).
 * Results do not depend on which other requests are in flight.
 * ---------------------------------------------------------------------------
 */
typedef struct accsk_request {
    const float *X;      /* device FP32 n x d, rows contiguous */
    const float *Y;      /* device FP32 m x d */
    int64_t n, m, d;     /* 1 <= n, m <= 512, 1 <= d <= 512 */
    int32_t kind;        /* ACCSK_SQEUCLID or ACCSK_COSINE */
    int32_t reserved;    /* 0 */
    double cost_scale;   /* s > 0: C = raw cost / s */
    const double *a;     /* device FP64 [n], positive (normalized inside) */
    const double *b;     /* device FP64 [m] */
    double eps;          /* > 0 */
    double *f_out;       /* device FP64 [n] */
    double *g_out;       /* device FP64 [m] */
} accsk_request;

typedef struct accsk_server accsk_server;

/*
 * Creates a server on the current device.  hbm_budget: bytes of the cost
 * arena (allocated here).  max_slots: worker workgroups (requests solved at
 * once), 0 = as many as stay resident (up to three per compute unit, minus
 * one for the dispatcher).  p: method, tol, max_iter, mu0, m0, w_rule, flags and the
 * cost split (0, 2, 3) used for every request (p->eps is ignored).
 * Returns ACCSK_OOM if the arena cannot be allocated.
 */
accsk_status accsk_server_create(size_t hbm_budget, int max_slots, const accsk_params *p, accsk_server **out);

/*
 * Queues one request and returns its ticket.  The request's buffers must stay
 * valid (and unchanged) until accsk_server_poll reports it done; they must be
 * ready when submitted (synchronize their producers first).  Errors:
 * INVALID_ARG, SHAPE (limits above), OOM (cost block larger than the whole
 * budget), HIP_ERROR (an earlier launch failed).
 */
accsk_status accsk_server_submit(accsk_server *srv, const accsk_request *req, uint64_t *ticket);

/*
 * Non-blocking: *done = 1 and *res filled once the request has finished
 * (res->kernel_ms = its time on the device); the ticket is then released.
 * times (optional, 3 doubles): submit, admission and completion instants on
 * the accsk_clock_seconds() clock.  INVALID_ARG for an unknown ticket.
 */
accsk_status accsk_server_poll(accsk_server *srv, uint64_t ticket, accsk_result *res, int *done, double *times);

/* info[5]: worker workgroups, waiting requests, requests in flight, kernel launches, free arena bytes. */
accsk_status accsk_server_info(accsk_server *srv, int64_t *info);

/*
 * Admission by HBM footprint, counted since the server was created.
 * stats[6]: requests that waited for arena space (a first-fit search over the
 * free blocks found none large enough for their n x ceil4(m) FP32 cost), failed
 * first-fit searches in total, requests admitted ahead of an earlier waiting
 * request that did not fit, peak arena bytes in use, peak requests in flight,
 * arena size (hbm_budget).  INVALID_ARG for NULL arguments.
 */
accsk_status accsk_server_admission(accsk_server *srv, int64_t *stats);

/* Stops the persistent kernel once the requests in flight have finished, and frees the server. */
accsk_status accsk_server_destroy(accsk_server *srv);

/* Monotonic host clock (seconds) used for the serving timestamps. */
double accsk_clock_seconds(void);

#ifdef __cplusplus
}
#endif

#endif /* ACCSK_H */
