/*
 * spline_solve.h -- C ABI of the MI355X (gfx950) cubic-spline library.
 *
 * The library implements the hot path of Hornbeck, "Fast Cubic Spline
 * Interpolation" (arXiv 2001.09253) on the GPU, in FP64:
 *
 *   build    the knot second derivatives y''[n]: the tridiagonal system of the
 *            section "Generating Second Derivatives" (equation eqn:init_val and
 *            the rows a_j, b_j, c_j, d_j after it), with the end rows of the
 *            section "Start and End Derivatives", solved by a parallel form of
 *            Thomas' algorithm (section "Implementation");
 *   evaluate m uniformly spaced queries between the first and the last knot
 *            (section "Curve Interpolation", step 8 of the methodology), each
 *            bracketed to its interval and evaluated with the rewritten
 *            interpolant of the section "Fast Interpolation" (the routine the
 *            paper calls newint).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Knots x[n] and values y[n] are FP64, contiguous, x strictly increasing,
 *    n >= 3 (the paper's routine asserts both).  A NaN knot counts as not
 *    increasing.
 *  - An end is natural (y'' = 0 there) iff its derivative argument is
 *    > 0.99e30, the paper's sentinel; otherwise it is clamped to that first
 *    derivative.  Each end is decided on its own.  NaN values or derivatives
 *    are not rejected: they propagate as NaN.
 *  - Uniform query k of m is x[0] + k*h with h = (x[n-1]-x[0])/(m-1), one
 *    multiply then one add (never fused), and query m-1 is x[n-1] itself;
 *    with m == 1 the only query is x[0].
 *  - The interval of query q is clip(#{j : x_j < q} - 1, 0, n-2): at an
 *    interior knot the left interval, as the paper's bracketing loop picks.
 *    Explicit queries outside [x[0], x[n-1]] use the end intervals (cubic
 *    extrapolation).
 *  - Return values: SOLVE_OK (0) or a negative SOLVE_E_* code.  No entry
 *    point aborts the process.
 *  - "device pointer" means memory the GPU can read or write (hipMalloc,
 *    torch CUDA tensors); "stream" is a hipStream_t passed as void* (NULL =
 *    the legacy default stream).  The device-level calls are asynchronous on
 *    that stream and never allocate device memory.
 */
#ifndef SPLINE_SOLVE_H
#define SPLINE_SOLVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------------- */
#define SOLVE_OK 0
#define SOLVE_E_ARG (-1)     /* null pointer, bad config or option            */
#define SOLVE_E_SIZE (-2)    /* n < 3, m < 1, or sizes beyond the limits      */
#define SOLVE_E_ORDER (-3)   /* knots not strictly increasing (or NaN)        */
#define SOLVE_E_BUDGET (-4)  /* one instance exceeds the whole HBM budget     */
#define SOLVE_E_DEVICE (-5)  /* a HIP runtime call failed                     */
#define SOLVE_E_TICKET (-6)  /* unknown or already reaped ticket              */
#define SOLVE_E_STATE (-7)   /* context shutting down or in a failed state    */

/* ---- request status (solve_poll) ------------------------------------------ */
#define SOLVE_PENDING 0
#define SOLVE_DONE 1
#define SOLVE_ERROR 2

/* ---- precision modes -------------------------------------------------------- */
#define SOLVE_FP64 0          /* every step in FP64                              */
#define SOLVE_FP32_REFINE 1   /* FP32 bulk solve + FP64 residual/correction      */

/* ---- solve_config.flags ------------------------------------------------------ */
#define SOLVE_PLAIN 1u        /* one instance per synchronous launch, no batching */
#define SOLVE_NO_GRAPH 2u     /* launch kernels directly instead of a hipGraph    */

/* ---- limits ------------------------------------------------------------------- */
#define SOLVE_MAX_N_BLOCK 16384   /* largest n of spline_build (one workgroup)   */
#define SOLVE_MAX_N_BATCH 2048    /* largest n of an instance in a fused batch   */
#define SOLVE_MAX_N_SOLVE 1073741824  /* largest n of spline_solve_uniform and of a */
                                      /* request (2^30)                            */

typedef struct solve_ctx solve_ctx;
typedef uint64_t solve_ticket;

typedef struct {
    int device;                /* HIP device ordinal                                */
    uint64_t hbm_budget_bytes; /* budget for the device buffers of resident requests */
    uint32_t max_slots;        /* max requests resident on the device at once       */
    uint32_t precision;        /* SOLVE_FP64 or SOLVE_FP32_REFINE                    */
    uint32_t flags;            /* SOLVE_PLAIN, SOLVE_NO_GRAPH                        */
    uint32_t max_inflight;     /* batches in flight on the device (>= 1; 0 = 2)     */
    void *stream;              /* the caller's hipStream_t (NULL = the legacy        */
                               /* default stream): solve_submit orders its reads of */
                               /* device inputs and writes of device outputs after  */
                               /* the work queued there when it is called           */
} solve_config;

/* ============================================================================
 * Request API (the method's problem statement: knots, values, start and end
 * derivative as in the paper's routine new_second_derivative(knots, values,
 * start_deriv, end_deriv), plus the points to interpolate at).
 * ========================================================================== */

/* Every call below but solve_destroy may be made from several host threads
 * at once on one context (submissions, polls and waits are serialised
 * internally); solve_destroy must not overlap another call on its context. */

/* Create a context on cfg->device.  *out receives an owned handle that must be
 * released with solve_destroy.  A background scheduler thread admits
 * requests against hbm_budget_bytes / max_slots and launches them in fused
 * batches (continuous batching) unless SOLVE_PLAIN is set, in which case
 * solve_submit runs the request synchronously.  Admission keeps the summed
 * footprints of the requests on the device (plus 4096 bytes per batch) within
 * hbm_budget_bytes; each in-flight batch's device buffers are sized within
 * what the budget leaves beside the other slots' buffers (idle slots give
 * theirs up when needed), and are allocated and freed in stream order on the
 * slot's own stream, so resizing never waits for other batches.  The device
 * bytes actually held are reported by solve_memory.  Errors: E_ARG (null or
 * bad config), E_DEVICE. */
int solve_create(const solve_config *cfg, solve_ctx **out);

/* Submit one curve.  knots/values: n doubles each (host or device pointers,
 * detected per pointer); they are copied before the call returns, so the
 * caller may free them at once.  Device inputs are read after the work queued
 * on cfg->stream when the call is made (so a kernel that produces them there
 * just before the call is waited for).  start_deriv/end_deriv: see the
 * conventions.  xq: m explicit query points, or NULL for m uniform queries.
 * yq_out: m results, ypp_out: n second derivatives or NULL; both
 * caller-owned, device, pinned host (written by the device directly) or
 * pageable host (copied from the library's pinned staging), and written only
 * when the request completes -- they must stay valid until solve_poll reports
 * DONE/ERROR or until solve_destroy.  Device outputs are written after the
 * work queued on cfg->stream when the call is made.  Curves of up to
 * SOLVE_MAX_N_BATCH knots join the fused batches; longer ones (and every
 * SOLVE_PLAIN request) run on the kernels of spline_solve_uniform (with
 * explicit queries: its y'' and then spline_eval_points).  *ticket_out
 * receives the request's ticket.  Errors: E_ARG, E_SIZE (n < 3, m < 1,
 * n > SOLVE_MAX_N_SOLVE), E_ORDER (the copied knots are checked before the
 * call returns), E_BUDGET (the request's footprint, 8*(3n + m [+ m for
 * explicit queries]) + 40 bytes plus 48 bytes per work item (at most
 * 2*((n-2)/255 + 1) + m/queries_per_tile + 1 items), plus one batch's 4096,
 * exceeds hbm_budget_bytes), E_STATE (context
 * shutting down), E_DEVICE.  With SOLVE_PLAIN the request has completed when
 * the call returns (its ticket then polls DONE or ERROR). */
int solve_submit(solve_ctx *ctx, const double *knots, const double *values, int64_t n,
                 double start_deriv, double end_deriv, const double *xq, int64_t m,
                 double *yq_out, double *ypp_out, solve_ticket *ticket_out);

/* Non-blocking status of a ticket: *status = SOLVE_PENDING, SOLVE_DONE or
 * SOLVE_ERROR.  A ticket reported DONE or ERROR is reaped: a later poll of it
 * returns E_TICKET.  Errors: E_ARG, E_TICKET. */
int solve_poll(solve_ctx *ctx, solve_ticket ticket, int *status);

/* Waits until the ticket is DONE or ERROR (or timeout_ms elapses, < 0 =
 * forever; then *status = SOLVE_PENDING) and reports its status.  Does not
 * reap the ticket: solve_ticket_info still works, and the solve_poll that
 * reports it finished reaps it.  Errors: E_ARG, E_TICKET. */
int solve_wait(solve_ctx *ctx, solve_ticket ticket, int *status, int64_t timeout_ms);

/* Times of a completed or pending ticket in seconds on the library's
 * monotonic clock (solve_clock): t[0] submit, t[1] admitted, t[2] launched,
 * t[3] completed (0 where not reached yet); *error_code receives the ticket's
 * own code (SOLVE_OK or E_ORDER).  Does not reap the ticket. */
int solve_ticket_info(solve_ctx *ctx, solve_ticket ticket, double t[4], int *error_code);

/* Library monotonic clock in seconds (the clock solve_ticket_info uses). */
double solve_clock(void);

/* Counters of a context: out[0] requests submitted, [1] completed, [2]
 * failed, [3] batches launched, [4] resident bytes now, [5] peak resident
 * bytes, [6] requests waiting for admission now, [7] peak requests in one
 * batch. */
int solve_stats(solve_ctx *ctx, uint64_t out[8]);

/* Device memory of a context: out[0] bytes its buffers hold now, out[1] the
 * peak.  The held bytes exceed hbm_budget_bytes only by spare capacity an
 * in-flight batch took while the budget had room (at most half of that
 * batch's own buffers).  Errors: E_ARG. */
int solve_memory(solve_ctx *ctx, uint64_t out[2]);

/* Force the next batch launch to fail (host-side fault injection for tests of
 * the error path; no kernel runs for that batch).  Its tickets report ERROR. */
int solve_inject_fault(solve_ctx *ctx);

/* Stop the scheduler, cancel queued work (its tickets report ERROR), wait for
 * work already on the device, and free every device and host resource of the
 * context.  Tickets of a destroyed context are unknown (E_TICKET). */
int solve_destroy(solve_ctx *ctx);

/* ============================================================================
 * Device-level operations: one instance, device pointers, asynchronous on
 * `stream`, no allocation.  These are the kernels the request API uses.
 * ========================================================================== */

/* Steps a1-a4: validate the knots, set up the rows, solve for y''.
 * x, y: n device doubles; ypp: n device doubles (output).  status: nullable
 * device int32, set to SOLVE_OK or SOLVE_E_ORDER (then ypp is all NaN).
 * Host-side errors: E_ARG, E_SIZE (n < 3 or n > SOLVE_MAX_N_BLOCK). */
int spline_build(const double *x, const double *y, int64_t n, double start_deriv,
                 double end_deriv, double *ypp, int32_t *status, void *stream);

/* Steps a5-a6: m uniform queries, bracketed and evaluated.  x, y, ypp: n
 * device doubles (ypp from spline_build); yq: m device doubles (output).
 * Errors: E_ARG, E_SIZE (n < 3 or m < 1). */
int spline_eval_uniform(const double *x, const double *y, const double *ypp, int64_t n,
                        int64_t m, double *yq, void *stream);

/* Steps a1-a6 for one curve in a single launch, with no synchronisation
 * between workgroups: each workgroup (or wavefront) owns a block of knot
 * intervals, solves the paper's rows over that block plus a halo of rows on
 * either side and evaluates the uniform queries that fall in its intervals.
 * The halo is sized from the knots: the shortest (up to 63 rows) for which
 * the dropped coupling, bounded through the paper's recurrences, is below
 * 2^-60 max|y''|, else 128 rows (below 1e-21 max|y''| by the diagonal
 * dominance the paper proves); curves shorter than a block plus both halos
 * are solved whole.  On curves of 2^17 knots or more with fewer than 10
 * queries per interval each wavefront instead sweeps a run of 256-row blocks
 * in order, carrying the forward elimination's state (c', d') exactly from
 * block to block, so that only the run's ends take a halo (one block before
 * it, below (2/3)^256 max|y''|; the back substitution of a block starts from
 * the next block's backward scan, within 2^-256 max|y''|).  The kernel is
 * chosen by the query density m/(n-1) and by n.
 * x, y: n device doubles; yq: m device doubles (output); ypp: nullable, n
 * device doubles (output).  status: nullable device int32 that the call
 * leaves unchanged unless it finds unordered knots, in which case it is set
 * to SOLVE_E_ORDER and the outputs are unspecified (initialise it to
 * SOLVE_OK).  Errors: E_ARG, E_SIZE (n < 3, n > SOLVE_MAX_N_SOLVE, m < 1). */
int spline_solve_uniform(const double *x, const double *y, int64_t n, double start_deriv,
                         double end_deriv, int64_t m, double *yq, double *ypp, int32_t *status,
                         void *stream);

/* spline_solve_uniform that also reports step a5's result: idx[k] (m device
 * int32, output) receives the interval of uniform query k, clip(#{j : x_j <
 * q_k} - 1, 0, n-2), as each kernel decided it.  It runs the same kernels,
 * chosen by the same rule, compiled with one more store per result, so that
 * the bracketing of the path spline_solve_uniform runs can be checked exactly;
 * yq, ypp and status are as for spline_solve_uniform (and bit-identical to
 * it).  Errors: E_ARG (also idx NULL), E_SIZE as spline_solve_uniform. */
int spline_solve_uniform_indexed(const double *x, const double *y, int64_t n, double start_deriv,
                                 double end_deriv, int64_t m, double *yq, double *ypp, int32_t *idx,
                                 int32_t *status, void *stream);

/* The per-query formulas compared in the paper's "Benchmarks" section
 * ("Curve Interpolation": newint, newint__orig, newint__noinv, splint_one__div,
 * splint_one__mul), for spline_solve_uniform_variant. */
#define SOLVE_NEWINT_HOISTED 0 /* newint, 1/(b-a) and (b-a)^2 once per interval */
#define SOLVE_NEWINT_ORIG 1    /* newint with inv_ba = 1/(b-a) formed per query  */
#define SOLVE_NEWINT_NOINV 2   /* newint dividing by (b-a) per query              */
#define SOLVE_SPLINT_DIV 3     /* the A,B,C,D form ("Fast Interpolation"), /6     */
#define SOLVE_SPLINT_MUL 4     /* the same with the /6 as a multiplication        */
#define SOLVE_HORNER 5         /* not the paper's: power-basis coefficients per    */
                               /* interval, Horner's rule in q - x_j              */

/* spline_solve_uniform with the evaluation formula chosen by `variant` (one of
 * the SOLVE_NEWINT_* / SOLVE_SPLINT_* / SOLVE_HORNER values), for comparing the paper's
 * variants on the same build (a1-a5 unchanged).  It always takes the
 * dense-curve kernels (chosen as for spline_solve_uniform's dense
 * path), whatever the query density.  Arguments,
 * layout, ownership and status as for spline_solve_uniform.  The variants
 * agree to rounding (a few ulp of max|y| at the query); SOLVE_NEWINT_HOISTED
 * matches spline_solve_uniform's dense path bit for bit.  Errors: E_ARG (null
 * pointer, unknown variant), E_SIZE as spline_solve_uniform. */
int spline_solve_uniform_variant(const double *x, const double *y, int64_t n, double start_deriv,
                                 double end_deriv, int64_t m, int32_t variant, double *yq, double *ypp,
                                 int32_t *status, void *stream);

/* Step a5 alone: the interval index of each of the m uniform queries
 * (int32, device, output), computed by the same code as spline_eval_uniform. */
int spline_bracket_uniform(const double *x, int64_t n, int64_t m, int32_t *idx, void *stream);

/* The paper's "noop" loop on the GPU: generate and bracket the m uniform
 * queries but store the interval index (as a double) instead of evaluating. */
int spline_noop_uniform(const double *x, int64_t n, int64_t m, double *out, void *stream);

/* Explicit queries (any order): xq[m] device doubles in; yq[m] values out;
 * d1/d2 nullable outputs of the first and second derivative at the queries;
 * idx nullable int32 output of the intervals. */
int spline_eval_points(const double *x, const double *y, const double *ypp, int64_t n,
                       const double *xq, int64_t m, double *yq, double *d1, double *d2,
                       int32_t *idx, void *stream);

/* A curve's knots, values and second derivatives interleaved for explicit
 * queries: packed[3j], packed[3j+1], packed[3j+2] = x[j], y[j], ypp[j] for
 * j < n (packed: 3n device doubles, caller-owned).  An interval's six numbers
 * then share one or two cache lines instead of three, which is what bounds
 * explicit points in random order; pack once, evaluate many point sets.
 * Asynchronous on `stream`; allocates nothing.  Errors: E_ARG (a pointer
 * NULL), E_SIZE (n < 3), E_DEVICE. */
int spline_pack_knots(const double *x, const double *y, const double *ypp, int64_t n, double *packed,
                      void *stream);

/* spline_eval_points on a packed curve (spline_pack_knots): the same kernel
 * reading x, y and y'' from the n interleaved triples; the same intervals bit
 * for bit, the same values and derivatives to rounding (the two compiled
 * instantiations may contract a multiply and an add differently).  Errors: E_ARG
 * (packed, xq or yq NULL), E_SIZE (n < 3 or m < 1), E_DEVICE. */
int spline_eval_points_packed(const double *packed, int64_t n, const double *xq, int64_t m, double *yq,
                              double *d1, double *d2, int32_t *idx, void *stream);

/* Explicit queries over a batch, in one launch (the evaluation of "Fast
 * Interpolation" at any points, for many curves): count curves in CSR layout
 * on the device, koff and qoff (count + 1 int64 each, non-decreasing).  Curve
 * i owns knots koff[i] .. koff[i+1]-1 of x, y and ypp (its second
 * derivatives: from spline_plan_run, a build-only plan, or spline_build) and
 * queries qoff[i] .. qoff[i+1]-1; query k of the offsets is read from
 * xq[k - qoff[0]] and its results are written to yq[k - qoff[0]] (and to d1,
 * d2, the first and second derivative, and idx, the interval within the
 * curve, each nullable).  total_m = qoff[count] - qoff[0] (a host value: it
 * sizes the launch).  The interval of q is clip(#{x_j < q} - 1, 0, n_i - 2),
 * so points outside a curve's range take its end intervals and a NaN point
 * gives NaN.  Every n_i must be >= 3 (a curve of fewer than two knots gets
 * NaN; the sizes are not read on the host); m_i = 0 is allowed.  Asynchronous
 * on `stream`; allocates nothing.  Errors: E_ARG (koff, qoff, x, y, ypp, xq
 * or yq NULL), E_SIZE (count or total_m < 1), E_DEVICE. */
int spline_batch_eval_points(int64_t count, int64_t total_m, const int64_t *koff, const int64_t *qoff,
                             const double *x, const double *y, const double *ypp, const double *xq,
                             double *yq, double *d1, double *d2, int32_t *idx, void *stream);

/* ============================================================================
 * Batched form: many curves in CSR layout, each solved ("Generating Second
 * Derivatives") and evaluated at its own uniform queries ("Fast
 * Interpolation"), in one launch.
 *
 * Every wavefront takes a work item (curve, knot block, share of the
 * block's queries), solves the block's rows for y'' in its own LDS -- the
 * whole curve when n <= 512 (n <= 256 when every curve of the batch is that
 * small), else 255 intervals plus 128 halo rows on either side, whose dropped
 * coupling is below 4.5 (2/3)^128 of max|y''| -- and evaluates its queries;
 * wavefronts never wait on one another.  With tuning.fused = 2 the curves of
 * up to 256 knots are solved by a first launch instead; with tuning.fused = 3
 * a work item is a workgroup of four wavefronts, one of which solves the span
 * while all four evaluate its queries; with tuning.fused = 4 persistent
 * workgroups pipeline the items, one wavefront solving the next item while
 * the others evaluate the current one.
 * ========================================================================== */

typedef struct spline_plan spline_plan;

/* Tuning knobs of a plan: block = 64, 128 or 256 threads (1, 2 or 4
 * independent wavefronts per workgroup); queries_per_tile = largest share of
 * queries per work item (64 .. 2^24); grid_per_cu = 0 for one work item per
 * wavefront (the hardware dispatcher balances), else at most that many
 * persistent workgroups per compute unit (1..64) striding over the items;
 * fused = 1: one launch, every work item solves its own span; fused = 2: two
 * launches, curves of up to 256 knots solved first (16 lanes per curve, four
 * curves per wavefront) and their work items only evaluate; fused = 3: one
 * launch, one workgroup of four wavefronts per work item (block must be 256,
 * grid_per_cu is ignored; queries_per_tile is the largest share of one
 * workgroup), one wavefront solving the span into LDS and all four
 * evaluating a quarter of the share each; fused = 4: persistent workgroups of
 * four wavefronts (block must be 256, grid_per_cu is ignored), one round of
 * them, each taking every G-th work item: while one wavefront solves the next
 * item's span into one of two LDS buffers, the other three evaluate the
 * current item from the other buffer (FP64; mixed precision runs as
 * fused = 1). */
typedef struct {
    int32_t block;
    int32_t queries_per_tile;
    int32_t grid_per_cu;
    int32_t fused;
} spline_tuning;

/* Plan a batch from host-side sizes: count instances, knot offsets koff[count+1]
 * and query offsets qoff[count+1] (host int64, CSR: instance i owns knots
 * koff[i]..koff[i+1]-1 and outputs qoff[i]..qoff[i+1]-1).  Every n_i must be
 * in [3, SOLVE_MAX_N_BATCH] and every m_i >= 1.  qoff NULL plans a build only:
 * the runs compute the second derivatives of every curve and evaluate
 * nothing (their qoff and yq may then be NULL; spline_batch_eval_points
 * evaluates explicit points from the y'' they leave).  precision: SOLVE_FP64 or
 * SOLVE_FP32_REFINE.  tuning: nullable (library defaults).  The plan owns a
 * device copy of its work tables; *out must be released with
 * spline_plan_destroy.  Errors: E_ARG (also an invalid tuning), E_SIZE,
 * E_DEVICE. */
int spline_plan_create(int device, int64_t count, const int64_t *koff, const int64_t *qoff,
                       uint32_t precision, const spline_tuning *tuning, spline_plan **out);

/* Run the plan once on device-resident data: x, y (sum n doubles), sd, ed
 * (count doubles), koff, qoff (count+1 int64, the same offsets as planned),
 * yq (sum m doubles, output), ypp (sum n doubles, output, required: it holds
 * the second derivatives the evaluation reads), status (nullable, count
 * int32: SOLVE_OK or SOLVE_E_ORDER per instance).  Uniform queries only.
 * Asynchronous on `stream`.  Two runs of one plan must not overlap. */
int spline_plan_run(spline_plan *plan, const double *x, const double *y, const double *sd,
                    const double *ed, const int64_t *koff, const int64_t *qoff, double *yq,
                    double *ypp, int32_t *status, void *stream);

/* spline_plan_run that also writes the interval of every query: idx (sum m
 * device int32, output, CSR like yq) receives, for query k of curve i,
 * clip(#{j : x_j < q_k} - 1, 0, n_i - 2), counted within curve i.  The same
 * kernels compiled with one more store per result (yq, ypp and status as
 * spline_plan_run).  Errors: E_ARG (also idx NULL). */
int spline_plan_run_indexed(spline_plan *plan, const double *x, const double *y, const double *sd,
                            const double *ed, const int64_t *koff, const int64_t *qoff, double *yq,
                            double *ypp, int32_t *idx, int32_t *status, void *stream);

/* Capture one spline_plan_run with these pointers into a hipGraph owned by
 * the plan; spline_plan_replay then launches that graph on `stream`. */
int spline_plan_capture(spline_plan *plan, const double *x, const double *y, const double *sd,
                        const double *ed, const int64_t *koff, const int64_t *qoff, double *yq,
                        double *ypp, int32_t *status, void *stream);
int spline_plan_replay(spline_plan *plan, void *stream);

/* Time candidate tunings of the plan on the given data (reps timed launches
 * each), keep the fastest, and record it under `cache_path` (JSON, nullable)
 * keyed by device architecture and size class.  *best receives the choice,
 * *best_ms its mean launch time.  Outputs are overwritten while tuning. */
int spline_plan_autotune(spline_plan *plan, const double *x, const double *y, const double *sd,
                         const double *ed, const int64_t *koff, const int64_t *qoff, double *yq,
                         double *ypp, int reps, const char *cache_path, spline_tuning *best,
                         double *best_ms);

/* The plan's work tables, for inspection (tests walk every index the kernels
 * form from them).  *n_items receives the number of 48-byte work items,
 * *n_lane the number of curves a first launch builds, *wave_rows the rows of
 * the widest span one wavefront holds (64 x rows per lane).  dst (nullable:
 * then only the counts): host memory of dst_bytes >= the tables' size, which
 * receives the work items (each: int64 first knot, first output, query
 * count; int32 curve, knot count; int16 first and end interval; int32 share,
 * shares, padding), then, from the next multiple of 256 bytes, the n_lane
 * int32 curve indices.  Errors: E_ARG, E_SIZE (dst too small). */
int spline_plan_get_tables(const spline_plan *plan, void *dst, uint64_t dst_bytes, int64_t *n_items,
                           int64_t *n_lane, int64_t *wave_rows);

/* The tuning a plan uses now. */
int spline_plan_get_tuning(const spline_plan *plan, spline_tuning *out);

int spline_plan_destroy(spline_plan *plan);

/* ============================================================================
 * Batched form without device allocation.
 * ========================================================================== */

/* Largest work table spline_batch_run_noalloc holds: 48 bytes per work item
 * (a curve takes one item per 8192 queries or so, more past 512 knots), plus
 * 4 bytes per curve when a first launch builds the short curves. */
#define SOLVE_NOALLOC_SCRATCH_BYTES (8u << 20)

/* For callers that cannot allocate device memory (a serving loop with a fixed
 * footprint, a harness that forbids hipMalloc): spline_plan_create followed
 * by spline_plan_run in one call that allocates no device memory.  The work
 * tables are planned on the host from koff_host/qoff_host (count + 1 host
 * int64 each, as for spline_plan_create, with precision and tuning as there;
 * tuning NULL = the library default) and copied into a file-scope device
 * buffer of SOLVE_NOALLOC_SCRATCH_BYTES that each GPU the library runs on
 * holds until the process ends; x, y, sd, ed, koff, qoff, yq, ypp, status and
 * stream as for spline_plan_run, on the current device.  The kernels are
 * those of spline_plan_run, so the results are the same bit for bit.  The
 * call returns once the table copy is done (it waits for the work queued
 * before it on `stream`); the kernels then run asynchronously.  Every call on
 * one GPU uses that GPU's one buffer: calls that overlap on a GPU (from
 * several host threads, or on several streams) race and must be serialised by
 * the caller.  Not for stream capture (the table copy is waited for).
 * Errors: E_ARG, E_SIZE (sizes as spline_plan_create, or the tables beyond
 * SOLVE_NOALLOC_SCRATCH_BYTES), E_DEVICE. */
int spline_batch_run_noalloc(int64_t count, const int64_t *koff_host, const int64_t *qoff_host,
                             uint32_t precision, const spline_tuning *tuning, const double *x, const double *y,
                             const double *sd, const double *ed, const int64_t *koff, const int64_t *qoff,
                             double *yq, double *ypp, int32_t *status, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SPLINE_SOLVE_H */
