/*
 * cqk.h -- C ABI of libcqk, an MI355X (gfx950) library for the continuous
 * quadratic knapsack problem and its simplex / l1-ball special cases.
 *
 * Problem (Secchin & Silva, "Parallel Newton methods for the continuous
 * quadratic knapsack problem", Section 1, eq. (CQK)):
 *
 *     min_x 1/2 x^T D x - a^T x   s.t.  b^T x = r,  l <= x <= u,
 *
 * with D = diag(d), d_i > 0, b_i > 0 (the paper assumes b > 0 throughout),
 * l_i <= u_i; bounds may be -inf / +inf.  The solver is the semismooth Newton
 * method on the dual equation phi(lam) = b^T x(lam) = r (Section 2.1,
 * eq. (xopt), eq. (opt), eq. (phideriv), Algorithm 1), with variable fixing
 * (Section 2.2) done as compaction of the indices the Newton bracket has
 * resolved, and the stopping criteria of Section 5.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array argument is a DEVICE pointer owned by the caller, contiguous,
 *   with element i at ptr[i].  Any alignment of the element type is accepted
 *   (the kernels move 16 bytes per lane per access either way).  Outputs must
 *   not alias inputs: some calls write parts of x before they have finished
 *   reading y.
 * - Work is enqueued on the context's HIP stream (cqk_create / cqk_set_stream)
 *   and is ordered with the caller's other work on that stream.
 * - Errors are returned as cqk_status; nothing aborts or throws across the
 *   ABI.  Host-side argument errors return before anything is enqueued.
 *   A call given a cqk_info also stores a non-OK return value in
 *   info->status, whatever step it stopped at (its other fields are then
 *   filled only if the call reached the solver).
 * - With opts->sync != 0 (the default) the call waits for the result and
 *   fills *info.  Outputs are then final.
 * - With opts->sync = 0, or while the context's stream is capturing a HIP
 *   graph, a dense-output call only enqueues its work and returns CQK_OK
 *   (info->status = CQK_OK, nothing else filled); its outcome stays in device
 *   memory and cqk_ctx_last_info() waits for the stream and reads it.  The
 *   single-instance calls (cqk_solve_*, cqk_project_*) then queue every pass
 *   their iteration cap allows (2 max_iter + 4 general, max_iter + 2
 *   simplex / l1; each returns at once after the loop has stopped, a few
 *   microseconds), so keep opts->max_iter near what the problem needs.
 *   Per-pass timing (opts->timing) is skipped then.  The sparse-output calls,
 *   the SPG driver and the tuners always wait: under capture they return
 *   CQK_INVALID_ARG without enqueuing anything, and the sparse calls also with
 *   sync = 0.
 * - No call allocates device memory while its stream is capturing: if the
 *   workspace reserved before the capture (cqk_reserve) is too small, the call
 *   returns CQK_NO_MEMORY without enqueuing anything.
 * - On any status other than CQK_OK and CQK_NOT_CONVERGED the contents of the
 *   output array are unspecified.  CQK_NOT_CONVERGED writes x(lam_last).
 * - The context owns a device workspace that grows on demand (hipMalloc) and
 *   is reused between calls; cqk_reserve() grows it ahead of time (before a
 *   graph capture: cqk_reserve(ctx, n, 0) for a single call of n indices,
 *   cqk_reserve(ctx, 0, nseg) for a batched call of nseg rows).
 * - A context is not thread safe; use one context per host thread.
 */
#ifndef CQK_H
#define CQK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cqk_status {
  CQK_OK = 0,
  CQK_INFEASIBLE = 1,     /* r outside [b^T l, b^T u] (Algorithm 1 exits) */
  CQK_INVALID_ARG = 2,    /* bad argument or input data (see each call) */
  CQK_NOT_CONVERGED = 3,  /* max_iter reached; x = x(lam_last) written */
  CQK_DEVICE_ERROR = 4,   /* a HIP runtime call failed */
  CQK_NO_MEMORY = 5,      /* workspace allocation failed */
  CQK_BUFFER_TOO_SMALL = 6  /* sparse output: the support exceeds the
                               capacity; nothing written, count returned.
                               No-allocation call: more rows than its fixed
                               buffers hold; nothing enqueued */
} cqk_status;

/* Initial multiplier (Section 2.1 eq. (CQKlambda0); Section 3.1 Alg. 2). */
typedef enum cqk_lambda0_mode {
  CQK_LAMBDA0_ZERO = 0,     /* lam_0 = 0 */
  CQK_LAMBDA0_FORMULA = 1,  /* lam_0 = (r - s)/q over all indices, eq. (CQKlambda0) */
  CQK_LAMBDA0_CONDAT = 2,   /* simplex / l1 only: Algorithm 2 run per thread
                               chunk on a sample of y, merged by eq. (lambdaJ)
                               (Section 4), then one pass over y that keeps
                               the values above the merged bound */
  CQK_LAMBDA0_USER = 3      /* lam_0 = opts->lambda0_user */
} cqk_lambda0_mode;

typedef enum cqk_compaction {
  CQK_COMPACT_OFF = 0,      /* every pass reads all n indices (the paper's GPU form) */
  CQK_COMPACT_AUTO = 1,     /* general CQK: every evaluation after the first
                               writes, for each bracket it can end with
                               ([lam, hi] or [lo, lam]), the indices that
                               bracket leaves unresolved, giving a side up
                               as soon as it would keep more than
                               compact_theta of the indices read; the next
                               pass reads the set of the side that happened.
                               For n >= 2^22 a bracket estimated from two
                               samples (4096 and 1048576 indices: the
                               solution of the sampled equation +- 5
                               estimated standard deviations, widened to
                               the first iterate the sample predicts, or
                               to the second when the first lies far out)
                               lets
                               the first pass, or the lam_0 pass of a warm
                               or formula start, compact too; a set is read
                               only at multipliers strictly inside the
                               bracket its sums hold on, the caller's
                               arrays otherwise, so Algorithm 1's iterates
                               do not depend on the estimate.  Sides an
                               evaluation will not use (by the estimate, or
                               by their share of the set's bracket) are not
                               written.
                               Simplex / l1: compact on y + lam <= 0 */
  CQK_COMPACT_ALWAYS = 2    /* as AUTO with compact_theta = 1 (every side kept) */
} cqk_compaction;

typedef enum cqk_accum {
  CQK_ACCUM_DEFAULT = 0,    /* f64 inputs: f64; f32 inputs: f64 */
  CQK_ACCUM_F32 = 1,        /* f32 inputs only: f32 values and sums, integer counts */
  CQK_ACCUM_F64 = 2
} cqk_accum;

typedef struct cqk_opts {
  int32_t lambda0_mode;     /* cqk_lambda0_mode; default ZERO (CONDAT for simplex/l1) */
  double lambda0_user;      /* used with CQK_LAMBDA0_USER */
  int32_t max_iter;         /* Newton iterations (evaluations of phi); default 100 */
  double tol;               /* <= 0: eps^(3/4) of the working type (Section 5) */
  int32_t compaction;       /* cqk_compaction; default AUTO */
  double compact_theta;     /* <= 0: the context's (0.5 unless set or tuned) */
  int32_t accum;            /* cqk_accum */
  int32_t sync;             /* 1 (default): wait and fill *info */
  int32_t trace;            /* 1: record one cqk_trace_rec per pass */
  int32_t timing;           /* 1: time every pass kernel with HIP events;
                               2 (general CQK): only the first Newton pass
                               and the x-writing pass, so the others run
                               without the gaps the runtime leaves around a
                               timed dispatch (other calls: as 1) */
} cqk_opts;

typedef struct cqk_info {
  int32_t status;           /* cqk_status of the solve */
  int32_t iterations;       /* evaluations of phi (Newton iterations) */
  int32_t passes;           /* kernel passes over the data, incl. breakpoint passes */
  int32_t stop_reason;      /* 0 none, 1/2/3 = stopping criterion of Section 5,
                               4 = exact stop (phi(lam) = r or free set fixed),
                               5 = trivial case (empty, r = 0, inside l1 ball) */
  double lambda;            /* multiplier x was evaluated at */
  double lambda0;           /* initial multiplier actually used */
  double residual;          /* |b^T x - r| of the returned x (device sum) */
  double abs_bx;            /* sum_i |b_i x_i| of the returned x */
  int64_t n_free;           /* #{l_i < x_i < u_i} (simplex: #{x_i > 0}) */
  int64_t n_after_init;     /* simplex/l1 with CONDAT: survivors of Alg. 2 */
  double pass_bytes;        /* algorithmic bytes of the Newton/init passes */
  double pass_ms;           /* their summed kernel time (opts.timing = 1) */
  double finalize_bytes;    /* algorithmic bytes of the x-writing pass */
  double finalize_ms;       /* its kernel time (opts.timing = 1) */
  int64_t rows_spilled;     /* batched: long rows whose survivors of Alg. 2 did
                               not fit the on-chip list (Newton then re-reads
                               the row); 0 otherwise */
  int64_t pass_launches;    /* grid passes queued (pass_ms covers all of them;
                               those queued after the loop stopped return at
                               once and move no bytes) */
} cqk_info;

/* One record per kernel pass (opts.trace = 1). */
typedef struct cqk_trace_rec {
  int32_t iter;             /* Newton iteration the pass belongs to */
  int32_t kind;             /* 0 init, 1 evaluate phi, 2 breakpoint search,
                               3 Newton step taken, 4 secant step taken,
                               5 breakpoint step, 6 bisection (the secant
                               point rounded onto a bracket end), 7 one
                               thread's Algorithm 2 (simplex / l1 start, see
                               below), 8 and 9 the first and second
                               sampled-bracket estimates (general CQK, see
                               CQK_COMPACT_AUTO).  For kinds 3, 4 and 6, lam
                               is the next iterate, phi and slope those it
                               was taken from.  Kinds 8 and 9: lam solves
                               the sampled equation, lo/hi the bracket (NaN
                               when none), phi the estimated standard
                               deviation of lam, slope the share of the
                               sample with a breakpoint in the bracket,
                               compacted (kind 9) 1 when the first pass
                               compacts for it, n_in the sample size, n_out
                               the survivors predicted. */
  int32_t compacted;        /* 1 if the next pass reads a compacted set this
                               pass adopted (written by this pass, or the
                               sampled-bracket set the first pass wrote) */
  int32_t source;           /* 0 original arrays, 1..3 compacted sets */
  double lam;               /* multiplier evaluated by the pass */
  double phi;               /* phi(lam) */
  double slope;             /* slope used for the step (phi'_+ or phi'_-) */
  double lo, hi;            /* Newton bracket after the pass */
  int64_t n_in;             /* indices read by the pass */
  int64_t n_out;            /* indices written (compaction survivors; general
                               CQK: of both sides, the next pass's n_in
                               being the kept side's) */
} cqk_trace_rec;

typedef struct cqk_ctx cqk_ctx;

/* Create a context bound to `hip_stream` (a hipStream_t; NULL = the null
 * stream) on the current HIP device.  Returns CQK_DEVICE_ERROR if no device
 * is usable. */
cqk_status cqk_create(cqk_ctx** ctx, void* hip_stream);
void cqk_destroy(cqk_ctx* ctx);
cqk_status cqk_set_stream(cqk_ctx* ctx, void* hip_stream);
/* Grow the workspace for solves of up to max_n indices and batched calls of
 * up to max_seg rows. */
cqk_status cqk_reserve(cqk_ctx* ctx, int64_t max_n, int32_t max_seg);
const char* cqk_status_string(int32_t status);
void cqk_default_opts(cqk_opts* opts);
/* Outcome of the last call on this context (Section 1: the problem's status,
 * the infeasible exits of Algorithm 1): waits for the context's stream, then
 * reads the device-side status words and fills *info as a call with
 * opts->sync = 1 would have (batched calls: the worst row status, as their
 * return value; the per-row flags are in the caller's status_out /
 * lambda_out arrays).  After a replay of a captured graph it reports that
 * replay, provided no other call ran on the context since the capture.
 * Returns info->status, or CQK_INVALID_ARG when no call has run yet (or the
 * last one failed its host-side checks, or was the SPG driver), or while the
 * stream is capturing. */
cqk_status cqk_ctx_last_info(cqk_ctx* ctx, cqk_info* info);

/* Copy up to `cap` trace records of the last call into host memory `out`;
 * *count receives the number recorded.
 * A simplex / l1 call with the CONDAT start and opts->trace = 1 writes one
 * kind-7 record first: lane 0 of the first sample wave ran Algorithm 2
 * (Section 2.2, the per-chunk form of Section 4) on the values of the tile at
 * index 0 it holds, value e (e = 0..15, ascending in y) being y[(e / V) * 64 * V +
 * e % V] with V = 16 / sizeof(element).  Fields: n_in = mask of the values
 * above the wave's filter (those Algorithm 2 scanned, in order of e), n_out =
 * mask of its final set J, compacted = |J|, phi = sum of J (of |y| for l1),
 * lam = (r - phi) / |J| (Algorithm 2's bound), slope = the filter threshold,
 * lo = the wave's bound after merging and refining, source = mask of the
 * values of J that bound keeps (v + min(lam, lo) > 0; every other value of
 * the tile is zero at the solution), hi = 0 (the tile's index). */
cqk_status cqk_last_trace(cqk_ctx* ctx, cqk_trace_rec* out, int32_t cap, int32_t* count);
/* Kernel time in milliseconds of each grid pass of the last single-instance
 * call made with opts->timing = 1 and sync = 1 (cqk_solve_*,
 * cqk_project_*), in the order the passes were queued: the lambda_0 pass,
 * the two sampled-bracket kernels or the Algorithm 2 sample and filtering
 * passes if any, then the Newton passes, including those queued after the
 * loop had stopped, which return at once.  With opts->timing = 2 a general
 * solve lists its first Newton pass only.  The x-writing pass is not
 * included (info->finalize_ms).  Copies min(cap, count) values; *count
 * receives the number of passes.  The list is refilled whenever a
 * single-instance call's info is filled (sync = 1, or cqk_ctx_last_info) and
 * is empty unless that call had opts->timing set and sync = 1; batched calls
 * and the SPG driver leave it as it was. */
cqk_status cqk_last_pass_ms(cqk_ctx* ctx, float* ms, int32_t cap, int32_t* count);

/* General CQK (Section 1 eq. (CQK), Algorithm 1).
 * d, a, b, l, u: n inputs each; x: n outputs.  r: right-hand side.
 * INVALID_ARG: n < 0, a null pointer with n > 0, non-finite r, or (found on
 * the device in the first pass) d_i <= 0, b_i <= 0, l_i > u_i, l_i = +inf,
 * u_i = -inf, or a NaN / infinite value in d, a, b.
 * INFEASIBLE: r outside [b^T l, b^T u].  n = 0: OK iff r = 0. */
cqk_status cqk_solve_f64(cqk_ctx* ctx, int64_t n, const double* d, const double* a,
                         const double* b, const double* l, const double* u, double r,
                         double* x, const cqk_opts* opts, cqk_info* info);
cqk_status cqk_solve_f32(cqk_ctx* ctx, int64_t n, const float* d, const float* a,
                         const float* b, const float* l, const float* u, double r,
                         float* x, const cqk_opts* opts, cqk_info* info);

/* Projection onto the r-simplex {x >= 0, sum x = r} (Section 1 (proj_Delta),
 * Section 3 Algorithm 4 with Algorithm 2 as the start).
 * y: n inputs; x: n outputs.  INVALID_ARG: n < 0, null pointers, r < 0 or
 * non-finite, a NaN/inf in y (device check); n = 0 with r > 0 is INFEASIBLE;
 * r = 0 gives x = 0. */
cqk_status cqk_project_simplex_f32(cqk_ctx* ctx, int64_t n, const float* y, double r,
                                   float* x, const cqk_opts* opts, cqk_info* info);
cqk_status cqk_project_simplex_f64(cqk_ctx* ctx, int64_t n, const double* y, double r,
                                   double* x, const cqk_opts* opts, cqk_info* info);

/* Projection onto the l1 ball {x : sum |x_i| <= radius} (Section 3.2,
 * Lemma 1): x = y if y is inside, else sgn(y) * P_Delta(|y|).  Same errors
 * as the simplex call, with `radius` for r. */
cqk_status cqk_project_l1_f32(cqk_ctx* ctx, int64_t n, const float* y, double radius,
                              float* x, const cqk_opts* opts, cqk_info* info);
cqk_status cqk_project_l1_f64(cqk_ctx* ctx, int64_t n, const double* y, double radius,
                              double* x, const cqk_opts* opts, cqk_info* info);

/* Warm starts from a primal estimate xbar (n DEVICE values, same type as x,
 * read only; it must not overlap x).  They return what the calls above
 * return; only lambda_0 (info->lambda0) and the indices dropped before the
 * first Newton pass change.  opts->lambda0_mode is ignored.
 *
 * General CQK (Section 2.1, the estimate's variant of eq. (CQKlambda0)):
 * J = {l_i < xbar_i < u_i} is taken as free and every other index as fixed
 * at the bound xbar reaches (xbar_i <= l_i: l_i, xbar_i >= u_i: u_i):
 *   lambda_0 = (r - sum_{xbar<=l} b l - sum_{xbar>=u} b u - sum_J b a/d)
 *              / sum_J b^2/d,
 * plain eq. (CQKlambda0) over all indices when J is empty.  One extra read
 * of d, a, b, l, u, xbar.  A NaN in xbar counts as fixed at neither bound
 * and outside J.
 *
 * Simplex / l1 (Section 3.1): I = {xbar_i > 0} (l1: {xbar_i != 0}).  The
 * start pass runs Algorithm 2 as the cold call does (its bounds fix values
 * at zero whatever set they come from) and reads xbar beside y: the
 * estimate's bound is lam_J over the kept values of I (every value of I that
 * is free at the solution is kept), or r - max_I v when none is kept
 * (v = y, l1: |y|).  lambda_0 is the smallest of it and the cold bounds, all
 * upper bounds of lam*.  If I is empty, lambda_0 = max{r/n, -max_i v_i} and
 * Newton's first step may come from below.
 * INVALID_ARG: as the cold calls, plus xbar null or overlapping x. */
cqk_status cqk_solve_warm_f64(cqk_ctx* ctx, int64_t n, const double* d, const double* a,
                              const double* b, const double* l, const double* u,
                              const double* xbar, double r, double* x, const cqk_opts* opts,
                              cqk_info* info);
cqk_status cqk_solve_warm_f32(cqk_ctx* ctx, int64_t n, const float* d, const float* a,
                              const float* b, const float* l, const float* u, const float* xbar,
                              double r, float* x, const cqk_opts* opts, cqk_info* info);
cqk_status cqk_project_simplex_warm_f32(cqk_ctx* ctx, int64_t n, const float* y,
                                        const float* xbar, double r, float* x,
                                        const cqk_opts* opts, cqk_info* info);
cqk_status cqk_project_simplex_warm_f64(cqk_ctx* ctx, int64_t n, const double* y,
                                        const double* xbar, double r, double* x,
                                        const cqk_opts* opts, cqk_info* info);
cqk_status cqk_project_l1_warm_f32(cqk_ctx* ctx, int64_t n, const float* y, const float* xbar,
                                   double radius, float* x, const cqk_opts* opts,
                                   cqk_info* info);
cqk_status cqk_project_l1_warm_f64(cqk_ctx* ctx, int64_t n, const double* y, const double* xbar,
                                   double radius, double* x, const cqk_opts* opts,
                                   cqk_info* info);

/* Sparse output of the simplex / l1 projections (Sec. 5.2: the support of x
 * returned as (index, value) pairs instead of a dense x, so no n-sized
 * write).  The support S = {i : x_i != 0} is written in ascending index
 * order: idx[k] (DEVICE int64) and val[k] (DEVICE, the type of y) for
 * k < |S|; *nnz (HOST, may be NULL) receives |S|.  No dense x is written at
 * any point (the start pass's zero fill is skipped).
 * xbar: NULL for the cold start opts->lambda0_mode chooses, else a warm-start
 * estimate as in the _warm calls.
 * cap: entries idx and val hold.  BUFFER_TOO_SMALL: |S| > cap; nothing is
 * written to idx / val and *nnz holds |S| (cap = 0 with NULL idx / val only
 * counts).  INVALID_ARG: the cold calls' cases, cap < 0, idx or val NULL
 * with cap > 0, or idx, val and y overlapping.  y inside the l1 ball gives
 * S = {y_i != 0} and val = y there; r = 0 gives S empty.
 * The context keeps a bitmap of n bits (n/8 bytes) for these calls. */
cqk_status cqk_project_simplex_sparse_f32(cqk_ctx* ctx, int64_t n, const float* y,
                                          const float* xbar, double r, int64_t cap,
                                          int64_t* idx, float* val, int64_t* nnz,
                                          const cqk_opts* opts, cqk_info* info);
cqk_status cqk_project_simplex_sparse_f64(cqk_ctx* ctx, int64_t n, const double* y,
                                          const double* xbar, double r, int64_t cap,
                                          int64_t* idx, double* val, int64_t* nnz,
                                          const cqk_opts* opts, cqk_info* info);
cqk_status cqk_project_l1_sparse_f32(cqk_ctx* ctx, int64_t n, const float* y, const float* xbar,
                                     double radius, int64_t cap, int64_t* idx, float* val,
                                     int64_t* nnz, const cqk_opts* opts, cqk_info* info);
cqk_status cqk_project_l1_sparse_f64(cqk_ctx* ctx, int64_t n, const double* y,
                                     const double* xbar, double radius, int64_t cap,
                                     int64_t* idx, double* val, int64_t* nnz,
                                     const cqk_opts* opts, cqk_info* info);

/* Spectral projected gradient on the l1-constrained least-squares problem
 * of Section 5.2 (basis pursuit):
 *     min 1/2 ||A x - b||^2   s.t.  ||x||_1 <= radius,
 * every projection by the l1 projection above, warm-started from the
 * current iterate (Section 3.1) unless opts->warm = 0.  Steps of SPG2
 * (Birgin, Martinez, Raydan): x_0 = 0, spectral step clipped to
 * [1e-30, 1e30], non-monotone line search over the last `memory` values
 * with sufficient-decrease constant 1e-4 and safeguarded quadratic
 * interpolation in [0.1, 0.9] t; stops when ||P(x - g) - x||_inf <= tol.
 * A: DEVICE float64 m x n row-major; b: DEVICE float64[m]; x: DEVICE
 * float64[n] output (must not overlap A or b).  Two products with A and
 * two projections per iteration; the host reads a few scalars per step.
 * NOT_CONVERGED: max_iter reached (x is the last iterate).  A projection's
 * failure status is returned as is. */
typedef struct cqk_spg_opts {
  double tol;               /* projected-gradient tolerance; default 1e-4 */
  int32_t max_iter;         /* default 10000 */
  int32_t memory;           /* non-monotone line search memory; default 10 */
  int32_t warm;             /* 1 (default): warm-started projections */
  int32_t pad_;
} cqk_spg_opts;

typedef struct cqk_spg_info {
  int32_t status;
  int32_t iterations;       /* SPG iterations */
  int64_t projections;      /* l1 projections made */
  int64_t newton_iterations;/* Newton iterations summed over the projections */
  double objective;         /* 1/2 ||A x - b||^2 at the returned x */
  double pg;                /* ||P(x - g) - x||_inf there */
  double total_ms;          /* host wall time of the call */
  double proj_ms;           /* of which in the projections */
} cqk_spg_info;

void cqk_spg_default_opts(cqk_spg_opts* opts);
cqk_status cqk_spg_l1_lasso_f64(cqk_ctx* ctx, int64_t m, int64_t n, const double* A,
                                const double* b, double radius, double* x,
                                const cqk_spg_opts* opts, cqk_spg_info* info);

/* Many simplex projections in one launch: row s is y[offsets[s] ..
 * offsets[s+1]) (Section 3 Algorithms 2 and 4 applied per row).
 * offsets: int64[nseg+1] DEVICE array, non-decreasing, offsets[0] = 0.
 * r: DEVICE float64[nseg] radii, or NULL to use r_scalar for every row.
 * lambda_out: optional DEVICE float64[nseg], the row multipliers.
 * nfree_out: optional DEVICE int32[nseg], #{x_i > 0} per row.
 * INVALID_ARG: nseg < 0, null y/x/offsets with nseg > 0, r_scalar < 0 or
 * non-finite (when r is NULL); on the device, a row radius < 0 or NaN marks
 * that row's lambda_out as NaN and its x as 0 and sets the call status.
 * An empty row with r > 0 is infeasible and is reported the same way. */
cqk_status cqk_project_simplex_batched_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                           const float* y, const double* r, double r_scalar,
                                           float* x, double* lambda_out, int32_t* nfree_out,
                                           const cqk_opts* opts, cqk_info* info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture without a prior cqk_reserve, serving loops and harnesses that
 * forbid hipMalloc): cqk_project_simplex_batched_f32 with the same arguments,
 * kernels, results and statuses, whose planning buffers (row list, row
 * extents, length histogram, counters) live in a fixed device array of the
 * library instead of the context's workspace.  That array holds the buffers
 * for CQK_NOALLOC_MAX_SEG rows (about 1.3 MB); each GPU the library runs on
 * keeps its own copy until the process ends.  The call allocates nothing:
 * nseg > CQK_NOALLOC_MAX_SEG returns CQK_BUFFER_TOO_SMALL before anything is
 * enqueued, and opts->timing is ignored.  Every call on one GPU, from any
 * context, shares that GPU's array (the kernels clear their counters
 * themselves): calls that overlap in time on one GPU (different streams or
 * host threads) race and give undefined results.  cqk_ctx_last_info reads the
 * last such call on the context as long as no later call on the GPU has
 * reused the array. */
#define CQK_NOALLOC_MAX_SEG 65536
cqk_status cqk_project_simplex_batched_noalloc_f32(cqk_ctx* ctx, int32_t nseg,
                                                   const int64_t* offsets, const float* y,
                                                   const double* r, double r_scalar, float* x,
                                                   double* lambda_out, int32_t* nfree_out,
                                                   const cqk_opts* opts, cqk_info* info);

/* Many general CQK instances in one launch (Section 2.1, Algorithm 1 per
 * row, each row with its own bracket, breakpoint and secant state): row s
 * is (d, a, b, l, u)[offsets[s] .. offsets[s+1]) with right-hand side r[s].
 * offsets: int64[nseg+1] DEVICE array, non-decreasing, offsets[0] = 0.
 * d, a, b, l, u, x: DEVICE float64 arrays of offsets[nseg] values (float32
 * in the _f32 variant, which loads and stores float32 and computes every
 * sum, the multiplier and the clamp in float64).
 * r: DEVICE float64[nseg] (required, both variants).
 * lambda_out: optional DEVICE float64[nseg], the row multipliers (NaN for a
 * row without one).  status_out: optional DEVICE int32[nseg], each row's
 * cqk_status.
 * opts: lambda0_mode ZERO, FORMULA (eq. (CQKlambda0) per row) or USER (the
 * same lambda0_user for every row); compaction is not used.
 * Returns the worst row status: INVALID_ARG (a row failing the input checks
 * of cqk_solve_f64, or a non-finite r[s]), else INFEASIBLE, else
 * NOT_CONVERGED, else OK; x of a row without a multiplier is NaN.
 * An empty row is OK iff r[s] = 0.  info->iterations: the largest row
 * iteration count; info->passes: the iterations summed over rows. */
cqk_status cqk_solve_batched_f64(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                 const double* d, const double* a, const double* b,
                                 const double* l, const double* u, const double* r, double* x,
                                 double* lambda_out, int32_t* status_out, const cqk_opts* opts,
                                 cqk_info* info);
cqk_status cqk_solve_batched_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                 const float* d, const float* a, const float* b, const float* l,
                                 const float* u, const double* r, float* x, double* lambda_out,
                                 int32_t* status_out, const cqk_opts* opts, cqk_info* info);

/* Vector-Jacobian product of the batched CQK solution w.r.t. a and r on each
 * row's free set F = {l_i < x_i < u_i} (eq. (xopt) on F, eq. (opt)
 * differentiated):  q = sum_F b^2/d,  mu = (sum_F g b/d)/q,
 *   grad_a_i = [i in F](g_i - b_i mu)/d_i,   grad_r[s] = mu   (0 if F empty).
 * x: forward output, g: upstream gradient, grad_a: output, all DEVICE
 * float64 in the forward layout (float32 in the _f32 variant, sums in
 * float64); grad_r: optional DEVICE float64[nseg]. */
cqk_status cqk_solve_batched_backward_f64(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                          const double* x, const double* g, const double* d,
                                          const double* b, const double* l, const double* u,
                                          double* grad_a, double* grad_r, const cqk_opts* opts);
cqk_status cqk_solve_batched_backward_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                          const float* x, const float* g, const float* d,
                                          const float* b, const float* l, const float* u,
                                          float* grad_a, double* grad_r, const cqk_opts* opts);

/* Vector-Jacobian product of the batched simplex projection w.r.t. y and r
 * on each row's support S = {x_i > 0} (derived from eq. (lambdaJ)):
 *   grad_y_i = [i in S] (g_i - mean_S g),   grad_r[s] = mean_S g.
 * x: forward output, g: upstream gradient, grad_y: output (same layout);
 * grad_r: optional DEVICE float64[nseg]. */
cqk_status cqk_project_simplex_batched_backward_f32(cqk_ctx* ctx, int32_t nseg,
                                                    const int64_t* offsets, const float* x,
                                                    const float* g, float* grad_y,
                                                    double* grad_r, const cqk_opts* opts);

/* How a batched call maps rows onto the GPU.  Rows of at most
 * 64 * small_per values are solved by one wave each (their values stay in
 * registers), longer rows by a workgroup of four waves.  blocks_per_cu
 * persistent workgroups per compute unit pull rows from a device queue;
 * short_first = 1 hands out the one-wave rows before the workgroup rows
 * (which always go longest first). */
typedef struct cqk_batch_schedule {
  int32_t small_per;        /* 4 or 8: rows of at most 64 * small_per values are
                               solved by one wave from its registers */
  int32_t blocks_per_cu;    /* 1 .. 8: persistent workgroups per compute unit */
  int32_t short_first;      /* 0 or 1: one-wave rows handed out first */
  int32_t medium_tiles;     /* 0 .. 64, batched simplex (forward and
                               backward) only: rows of at most 1024 *
                               medium_tiles values (and more than 64 *
                               small_per) are solved by one wave, tile after
                               tile, four rows per workgroup; 0: every longer
                               row gets a whole workgroup.  Ignored by the
                               batched general CQK. */
} cqk_batch_schedule;

/* The schedule the context uses for one kind of batched call: which = 0
 * batched simplex forward, 1 its backward, 2 batched general CQK forward,
 * 3 its backward; a new context starts with {8, 4, 1, 16} for the batched
 * simplex forward and {8, 4, 0, 0} for the others.  Set
 * returns INVALID_ARG for a schedule outside the ranges above or another
 * `which`. */
cqk_status cqk_get_batch_schedule(cqk_ctx* ctx, int32_t which, cqk_batch_schedule* out);
cqk_status cqk_set_batch_schedule(cqk_ctx* ctx, int32_t which,
                                  const cqk_batch_schedule* sched);

/* Autotuner: runs cqk_project_simplex_batched_f32 on these rows under every
 * candidate schedule (small_per in {4, 8} x blocks_per_cu in {2, 3, 4, 6} x
 * short_first in {0, 1} x medium_tiles in {0, 4, 8, 16, 32, 64}), `repeats` timed
 * runs each after one warm-up, keeps the fastest as the context's forward
 * schedule and returns it with its time in milliseconds (either pointer may
 * be NULL).  x is overwritten.  Synchronises the stream; not for use under
 * graph capture. */
cqk_status cqk_tune_batched_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                const float* y, const double* r, double r_scalar, float* x,
                                int32_t repeats, cqk_batch_schedule* best, double* best_ms);
/* The same for the backward call (x: forward output, g: upstream gradient,
 * grad_y overwritten; the same candidates); sets the context's backward
 * schedule. */
cqk_status cqk_tune_batched_backward_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                         const float* x, const float* g, float* grad_y,
                                         int32_t repeats, cqk_batch_schedule* best,
                                         double* best_ms);

/* Autotuner of the batched general CQK: runs cqk_solve_batched_f64
 * (backward = 0: needs d, a, b, l, u, r, x; x is overwritten) or
 * cqk_solve_batched_backward_f64 (backward = 1: needs x, g, d, b, l, u,
 * grad_a; grad_a is overwritten) on these rows under every candidate
 * schedule, as cqk_tune_batched_f32 does, from lambda = 0 with the default
 * options, and keeps the fastest as the context's schedule of that kind
 * (which = 2 or 3 above; one schedule of each kind serves both element
 * types).  The _f32 variant times the float32 calls.  Synchronises; not under
 * graph capture. */
cqk_status cqk_tune_batched_cqk_f64(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                    const double* d, const double* a, const double* b,
                                    const double* l, const double* u, const double* r,
                                    double* x, const double* g, double* grad_a,
                                    int32_t backward, int32_t repeats, cqk_batch_schedule* best,
                                    double* best_ms);
cqk_status cqk_tune_batched_cqk_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                    const float* d, const float* a, const float* b,
                                    const float* l, const float* u, const double* r, float* x,
                                    const float* g, float* grad_a, int32_t backward,
                                    int32_t repeats, cqk_batch_schedule* best,
                                    double* best_ms);

/* The compaction threshold theta that AUTO calls of the general CQK use when
 * opts->compact_theta <= 0 (Section 2.2 variable fixing: a side is written
 * only while it keeps at most theta of the indices read).  A new context
 * starts at 0.5; set takes 0 < theta <= 1, else INVALID_ARG. */
cqk_status cqk_get_compact_theta(cqk_ctx* ctx, double* theta);
cqk_status cqk_set_compact_theta(cqk_ctx* ctx, double theta);

/* Candidates of the theta tuner, in this order. */
#define CQK_THETA_CANDIDATES 7   /* 0.2, 0.3, 0.4, 0.5, 0.6, 0.75, 1.0 */

/* Autotuner of theta (Section 2.2; when compaction pays is an empirical
 * question there): solves this instance with cqk_solve_f64 (_f32: with
 * cqk_solve_f32) at every candidate theta, with AUTO compaction and the rest
 * of *opts (NULL: defaults; sync, trace and timing are ignored), `repeats`
 * timed solves each after one warm-up, keeps the fastest as the context's
 * theta and returns it with its time in milliseconds (host clock around the
 * synchronised call, median of the repeats).  times_ms, if not NULL, receives
 * the CQK_THETA_CANDIDATES times in candidate order.  x is overwritten.  Any
 * solve that does not return CQK_OK ends the tuning with its status and the
 * context's theta unchanged.  Synchronises; not under graph capture
 * (INVALID_ARG). */
cqk_status cqk_tune_theta_f64(cqk_ctx* ctx, int64_t n, const double* d, const double* a,
                              const double* b, const double* l, const double* u, double r,
                              double* x, const cqk_opts* opts, int32_t repeats,
                              double* best_theta, double* best_ms, double* times_ms);
cqk_status cqk_tune_theta_f32(cqk_ctx* ctx, int64_t n, const float* d, const float* a,
                              const float* b, const float* l, const float* u, double r,
                              float* x, const cqk_opts* opts, int32_t repeats,
                              double* best_theta, double* best_ms, double* times_ms);

#ifdef __cplusplus
}
#endif

#endif /* CQK_H */
