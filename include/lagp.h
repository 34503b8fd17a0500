/*
 * lagp.h -- C ABI of the MI355X local approximate Gaussian-process library.
 *
 * The library implements the data-parallel hot path of Gramacy & Apley,
 * "Local Gaussian process approximation for large computer experiments":
 * for each predictive location x it
 *   (1) takes the n0 nearest design points as the starting local design and
 *       the N' nearest design points as the candidate set (Section 3 and the
 *       N' restriction of Section 6);
 *   (2) grows the local design greedily to n points, each step adding the
 *       candidate with the largest reduction in predictive variance at x
 *       (the ALC criterion, eq dxy, Sections 3.2-3.3; partial-correlation form
 *       eq dxy2, SM Section 4), with the O(j^2) partitioned-inverse update of
 *       SM Section 1 carried in Cholesky (whitened) form;
 *   (3) returns the local Student-t predictive mean, scale, degrees of freedom
 *       and variance (eqs predgp and preds2 with N -> n, Section 2).
 * Locations are independent (Section 4.1); a call processes a whole batch.
 *
 * Model: zero-mean GP with isotropic Gaussian correlation
 * K(a,b) = exp(-||a-b||^2 / d) between distinct points and nugget g added to
 * the diagonal of the local design covariance and to the self-covariance of
 * x and of each candidate (Section 2).  Cross-covariances carry no nugget.
 *
 * Conventions for every entry point:
 *   - Indices are 0-based int32 design-row indices.  N < 2^31.
 *   - Matrices are row-major: X is N x p, XX is T x p, sel is T x sel_stride.
 *   - Unless a flag says otherwise, array arguments of lagp_predict /
 *     lagp_knn are DEVICE pointers on the current HIP device; the caller owns
 *     them.  Work is enqueued on `stream` (a hipStream_t, NULL = default
 *     stream) and outputs are valid once that stream has been synchronised.
 *   - Argument errors are detected synchronously, before any launch, and
 *     return LAGP_E_INVAL; lagp_last_error() then describes the problem.
 *   - A location whose local covariance stops being positive definite (a
 *     pivot v_j(x_s) <= 0) gets status LAGP_LOC_NOTPD, NaN outputs and -1 for
 *     its unfilled design slots; other locations are unaffected and the call
 *     still returns LAGP_OK.
 *   - Calls that share one lagp_design share its workspace: issue them from
 *     one host thread on one stream (or serialise them).
 */
#ifndef LAGP_H
#define LAGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LAGP_OK = 0,
    LAGP_E_INVAL = -1,    /* bad argument (sizes, pointers, parameters)         */
    LAGP_E_NOMEM = -2,    /* device allocation for the design or workspace failed */
    LAGP_E_NODEVICE = -3, /* no HIP device is visible                          */
    LAGP_E_HIP = -4,      /* a HIP runtime call failed                          */
    LAGP_E_BUDGET = -5,   /* request larger than the serving memory budget      */
    LAGP_E_NOTPD = -6     /* strict mode only: some location was not positive definite */
} lagp_status;

/* Per-location status codes written to the optional `status` output. */
enum { LAGP_LOC_OK = 0, LAGP_LOC_NOTPD = 1, LAGP_LOC_NOTCAND = 2 /* a saved starting-design index is not
                                                                     among the location's candidates, or repeats */,
       LAGP_LOC_NOCAND = 3 /* the candidate set could not be formed (a kNN consistency check failed; calls
                              that wait on the host return an error instead) */ };

/* Precision of the ALC scoring contraction (eq dxy2 over the whitened tile
 * of the partitioned-inverse step, Supplementary Material Section 1).  The
 * factor of the chosen points, the chosen point's score and the prediction
 * are FP64 in every mode. */
typedef enum {
    LAGP_PREC_FP64 = 0,        /* everything FP64; the prediction reuses the greedy factor */
    LAGP_PREC_SCORE_FP32 = 1,  /* ranking tile stored and contracted in FP32 (v and cov
                                  accumulated in FP64); every step re-scores the FP32 ranking's
                                  best candidates exactly in FP64 -- each one's column of the
                                  whitened tile by forward substitution against the exact FP64
                                  factor -- and takes the exact argmax; the factor grows by the
                                  exact row and the prediction is FP64 from it (n <= 128).  Where
                                  the FP64 argmax is among the re-scored candidates, the design
                                  and outputs are bitwise those of LAGP_PREC_FP64.  A location
                                  whose short list holds no candidate with a positive exact
                                  variance is redone entirely in FP64 on the device */
    LAGP_PREC_SCORE_BF16 = 2   /* as LAGP_PREC_SCORE_FP32 with the ranking tile stored as
                                  bfloat16 (rounded to nearest even) and contracted with FP32
                                  accumulation: half the tile bytes, a coarser ranking */
} lagp_precision;

/* Flags. */
#define LAGP_PTR_HOST 1u   /* lagp_design_create: X and y are host pointers        */
#define LAGP_STRICT 2u     /* lagp_predict: return LAGP_E_NOTPD if any location failed */

typedef struct {
    int32_t n0;        /* starting nearest-neighbour design size, 1 <= n0 <= n     */
    int32_t n;         /* final local design size, n <= ncand                     */
    int32_t ncand;     /* candidate-set size N' (nearest design points), <= N     */
    double d;          /* lengthscale theta > 0                                    */
    double g;          /* nugget eta >= 0                                          */
    int32_t precision; /* lagp_precision                                           */
    uint32_t flags;    /* LAGP_STRICT                                              */
} lagp_params;

typedef struct lagp_design lagp_design;

/* Copy a design (X: N x p row-major, y: N) to the current device in the
 * layouts the kernels read (coordinate-major and row-major copies).  X and y
 * are device pointers unless flags has LAGP_PTR_HOST.  The caller keeps
 * ownership of X and y; the design owns its copies until
 * lagp_design_destroy.  Section 2: the design D = (X, Y). */
int lagp_design_create(const double *X, const double *y, int64_t N, int32_t p, uint32_t flags,
                       void *stream, lagp_design **out);

/* Free the design and its workspace.  NULL is ignored. */
void lagp_design_destroy(lagp_design *design);

/* Candidate sets (Section 3 nearest neighbours; Section 6 N' restriction):
 * for each of the T locations XX (device, T x p), write the indices of its M
 * nearest design points, ordered by (squared distance, index), into
 * idx[t * idx_stride + m] (device int32).  Squared distances are summed over
 * coordinates left to right without fused multiply-add. */
int lagp_knn(const lagp_design *design, const double *XX, int64_t T, int32_t M, int32_t *idx,
             int64_t idx_stride, void *stream);

/* Greedy ALC local designs and local GP prediction for T locations.
 *   XX        device T x p predictive locations;
 *   n_per     optional device int32[T]: per-location n (overrides params->n);
 *   ncand_per optional device int32[T]: per-location N' (overrides params->ncand);
 *   mean, s2  device double[T]: predictive mean k'K^{-1}Y and Student-t scale
 *             psi * v_n(x) / n (eqs predgp, preds2);
 *   df        optional device int32[T]: degrees of freedom n;
 *   var       optional device double[T]: variance psi * v_n(x) / (n-2) (NaN if n <= 2);
 *   sel       optional device int32 T x sel_stride: chosen design indices in
 *             selection order (first n0 are the nearest neighbours);
 *   status    optional device int8[T]: LAGP_LOC_OK / LAGP_LOC_NOTPD.
 * Requires 1 <= n0 <= n <= ncand <= N for every location; sel_stride >= max n.
 * With n_per or ncand_per the call is not asynchronous: the planner groups
 * the locations by size on the host, so it copies those arrays to the host
 * and waits for the copy on `stream`.  Uneven batches that must not wait
 * (graph capture, serving loops) use lagp_batch_*, whose sizes are host
 * arrays given at creation. */
int lagp_predict(const lagp_design *design, const double *XX, int64_t T, const lagp_params *params,
                 const int32_t *n_per, const int32_t *ncand_per, double *mean, double *s2,
                 int32_t *df, double *var, int32_t *sel, int64_t sel_stride, int8_t *status,
                 void *stream);

/* Options of lagp_predict_ex (Section 6's discussion of augmenting saved
 * local designs and of a stopping rule; Section 4.2's per-location
 * lengthscales).  Zero-initialise and set what is used. */
typedef struct {
    const double *d_per;     /* optional device double[T]: lengthscale per location (replaces params->d) */
    const int32_t *start;    /* optional device int32 T x start_stride: saved local designs; location t's
                                first start_n[t] (or params->n0) entries replace its n0 nearest
                                neighbours as the starting design, so the greedy search picks up
                                where an earlier one left off.  Each index must be one of the
                                location's ncand candidates and appear once, else the location
                                gets status LAGP_LOC_NOTCAND and NaN outputs */
    int64_t start_stride;    /* >= the largest starting-design size                              */
    const int32_t *start_n;  /* optional device int32[T]: starting-design sizes, 1 <= start_n <= n */
    double vratio;           /* 0: off.  Otherwise stop the greedy search before step j once the
                                best candidate's variance ratio v_j(x) / (v_j(x) - ALC_j), i.e.
                                V_j(x) / V_{j+1}(x) with psi cancelled, is below vratio; the
                                design then has df[t] <= n points (df is required; sel entries
                                past df[t] are -1) */
} lagp_options;

/* lagp_predict with the options above; opts may be NULL. */
int lagp_predict_ex(const lagp_design *design, const double *XX, int64_t T, const lagp_params *params,
                    const lagp_options *opts, const int32_t *n_per, const int32_t *ncand_per, double *mean,
                    double *s2, int32_t *df, double *var, int32_t *sel, int64_t sel_stride, int8_t *status,
                    void *stream);

/* lagp_predict with a lengthscale per location (Section 4.2: after local
 * inference each location has its own theta_x, possibly smoothed over the
 * locations): d_per is a device double[T] that replaces params->d, which must
 * still be a valid lengthscale.  A location whose d_per entry is not a
 * positive finite number gets status LAGP_LOC_NOTPD, NaN outputs and sel
 * entries -1. */
int lagp_predict_theta(const lagp_design *design, const double *XX, int64_t T, const lagp_params *params,
                       const double *d_per, const int32_t *n_per, const int32_t *ncand_per, double *mean,
                       double *s2, int32_t *df, double *var, int32_t *sel, int64_t sel_stride, int8_t *status,
                       void *stream);

/* Local GP prediction from given local designs (eqs predgp, preds2 with
 * N -> n): for each location t, K_n = K(D_t, D_t) + g I over the n (or n_per[t])
 * design indices sel[t * sel_stride + 0 .. n-1] is factorised afresh in FP64
 * and mean, s2, df, var written as in lagp_predict.  d_per (nullable, device
 * double[T]) gives each location its own lengthscale in place of d.  A
 * location with an index outside [0, N), a lengthscale that is not a positive
 * finite number, or a non-positive pivot gets status LAGP_LOC_NOTPD and NaN
 * outputs.  Device pointers; n is limited by LDS (about 190 on gfx950). */
int lagp_predict_designs(const lagp_design *design, const double *XX, int64_t T, const int32_t *sel,
                         int64_t sel_stride, const int32_t *n_per, int32_t n, double d, const double *d_per,
                         double g, double *mean, double *s2, int32_t *df, double *var, int8_t *status,
                         void *stream);

/* Greedy local designs by the MSPE criterion (Section 3.1, eq mspe) in place
 * of ALC, at the fixed lengthscale params->d (Section 3.2):
 *   J(c) = V_j(x|c) + (dmu_j(x)/dtheta)^2 / G_{j+1}(c),
 * the reduced predictive variance plus the theta-uncertainty term with the
 * expected Fisher information G of eq G (F_j = -l''(theta), eq d2l, plus the
 * candidate's expected information); the next point minimises J (ties to the
 * smaller design index).  The derivative of V_j(c) is that of psi v_j(c)/(j-2)
 * (dpsi/dtheta = -Y'K^{-1} dK K^{-1}Y).  Sizes and outputs as in lagp_predict
 * (n_per, ncand_per optional device arrays).  FP64 only; 3 <= n0 <= n <= ncand
 * <= min(N, 2048); n is limited by LDS (about 96 at p = 8). */
int lagp_predict_mspe(const lagp_design *design, const double *XX, int64_t T, const lagp_params *params,
                      const int32_t *n_per, const int32_t *ncand_per, double *mean, double *s2, int32_t *df,
                      double *var, int32_t *sel, int64_t sel_stride, int8_t *status, void *stream);

/* ---- Local inference of the lengthscale (Sections 3.2 and 4.2).
 *
 * The concentrated log likelihood of a local design (eq gpk of Section 2,
 * constants dropped) l(theta) = -1/2 log|K| - n/2 log(Y'K^{-1}Y), with
 * K = K(D, D) + g I, is maximised over theta by Newton's method with its
 * analytic first and second derivatives (eqs dl, d2l of SM Section 2).  The
 * paper leaves the controls of the search open; these are the ones taken: where l'' < 0 the step is -l'/l'', elsewhere
 * it is theta in the direction of l'; a step that would leave (tmin, tmax)
 * goes half way to the bound instead; the search starts from theta0 (from
 * sqrt(tmin tmax) when theta0 is outside the interval) and stops when a step
 * moves theta by at most tol * theta, or after maxit iterates. */
typedef struct {
    double tmin, tmax;  /* search interval, 0 < tmin < tmax, finite          */
    int32_t maxit;      /* Newton iterates, >= 1 (100 is ample)               */
    double tol;         /* relative step that ends the search, > 0 (1e-10)    */
} lagp_mle_params;

/* Maximum-likelihood lengthscale of T given local designs.
 *   sel       device int32 T x sel_stride design indices (first n, or n_per[t]);
 *   n_per     optional device int32[T] per-location design size (else n);
 *   d0_per    optional device double[T] starting lengthscales (else d0);
 *   d_hat     device double[T] estimates;
 *   iters     optional device int32[T] Newton iterates taken;
 *   status    optional device int8[T]: LAGP_LOC_NOTPD where a design index is
 *             outside [0, N), the design has fewer than 2 points, or K was
 *             not positive definite at some iterate (d_hat is then NaN).
 * The designs are held in LDS: n up to about 128 on gfx950 (p = 8). */
int lagp_mle(const lagp_design *design, int64_t T, const int32_t *sel, int64_t sel_stride, const int32_t *n_per,
             int32_t n, const double *d0_per, double d0, double g, const lagp_mle_params *mle, double *d_hat,
             int32_t *iters, int8_t *status, void *stream);

/* The two-stage scheme of Section 4.2 with one repetition ("alc2"), on the
 * device end to end: greedy ALC designs at params->d (or d_per), the local
 * MLE theta1 of each design, designs again at theta1, the local MLE theta2 of
 * the new designs (Newton started from theta1), and the prediction from the
 * second designs at theta2.  The candidate sets are computed once.  Outputs
 * as in lagp_predict, sel holding the second designs; d1 and d2 (optional
 * device double[T]) receive theta1 and theta2.  A location that fails at any
 * stage gets status LAGP_LOC_NOTPD and NaN outputs.  Requires n >= 2 for every
 * location; the mixed precision mode applies to both design passes. */
int lagp_predict_alc2(const lagp_design *design, const double *XX, int64_t T, const lagp_params *params,
                      const lagp_mle_params *mle, const double *d_per, const int32_t *n_per,
                      const int32_t *ncand_per, double *mean, double *s2, int32_t *df, double *var, int32_t *sel,
                      int64_t sel_stride, int8_t *status, double *d1, double *d2, void *stream);

/* ---- Fixed-shape batches (uneven sizes, HIP-graph replay).
 *
 * A batch fixes T and the per-location sizes once.  lagp_batch_create checks
 * them (as lagp_predict does), groups the locations into buckets of similar
 * (n, N') -- candidate-set size rounded up to a power of two >= 256 and
 * design size to a power of two >= 32 -- orders each bucket by decreasing
 * modelled cost n^2 N' (longest first, so that the persistent workgroups of
 * a launch finish together), chooses each bucket's kernel variant (the tuned
 * table shipped with the library, else the traffic model), and allocates all
 * device memory the batch will use.  The work is that of lagp_predict on
 * every location (Sections 3-4.1); results are identical to lagp_predict's.
 *
 *   n_per, ncand_per  HOST int32[T] arrays (nullable: params->n / ->ncand),
 *                     copied at creation;
 *   flags             LAGP_BATCH_SEL / LAGP_BATCH_STATUS when the calls will
 *                     pass sel / status (they are required exactly then);
 *   params->flags     must not contain LAGP_STRICT (it needs a host wait).
 * A batch belongs to its design and must be destroyed before it. */
#define LAGP_BATCH_SEL 1u
#define LAGP_BATCH_STATUS 2u
typedef struct lagp_batch lagp_batch;
int lagp_batch_create(const lagp_design *design, int64_t T, const lagp_params *params, const int32_t *n_per,
                      const int32_t *ncand_per, uint32_t flags, lagp_batch **out);

/* Enqueue the batch for the locations XX (device T x p) with outputs as in
 * lagp_predict.  Only kernel launches are enqueued -- no allocation, host
 * synchronisation or memset -- so a caller may capture this call into its
 * own HIP graph.  Calls on one batch share its workspace: do not overlap them. */
int lagp_batch_enqueue(lagp_batch *batch, const double *XX, double *mean, double *s2, int32_t *df, double *var,
                       int32_t *sel, int64_t sel_stride, int8_t *status, void *stream);

/* As lagp_batch_enqueue, through a HIP graph the batch records on its own
 * stream at the first call (and again whenever a pointer argument changes)
 * and then launches on `stream` as a single graph launch. */
int lagp_batch_launch_graph(lagp_batch *batch, const double *XX, double *mean, double *s2, int32_t *df,
                            double *var, int32_t *sel, int64_t sel_stride, int8_t *status, void *stream);

/* Number of buckets (design-kernel launches per replay) and workspace bytes. */
int lagp_batch_info(const lagp_batch *batch, int32_t *buckets, size_t *workspace_bytes);

/* Wait for the batch's work, free its memory and graph.  NULL is ignored. */
void lagp_batch_destroy(lagp_batch *batch);

/* Kernel-variant override for the greedy-design kernel, for tuning runs:
 * threads 0 (tuned table or model), 256 or 512 (a candidate set above 2048
 * always uses 512); coords -1 (table or model), 0 candidate coordinates in
 * global memory, 1 in LDS when they fit.  Applies to later calls on `design`. */
int lagp_design_set_variant(lagp_design *design, int32_t threads, int32_t coords);
/* As lagp_design_set_variant, and the share of the LDS left after the fixed
 * part that holds rows of the whitened candidate tile L^-1 K(X_j, candidates)
 * (the factor form of the partitioned-inverse step, Supplementary Material
 * Section 1): rows beyond those in registers go to LDS up to that share and
 * the rest stream from global memory.  lds_rows_pct -1 (table, else 100) or
 * 0..100; threads 0, coords -1 and lds_rows_pct -1 restore the table. */
int lagp_design_set_variant_ex(lagp_design *design, int32_t threads, int32_t coords, int32_t lds_rows_pct);

/* ---- Serving: continuous batching of requests under an HBM budget.
 *
 * A server owns a device arena of hbm_budget_bytes, `slots` HIP streams
 * (default priority) and host threads that feed and drain them.  Submitted
 * requests wait in a FIFO queue.  Their locations are cut into pieces of at
 * most `piece_locations` locations of one model (n0, d, g, precision), taken
 * in arrival order; a request may span pieces and a piece may hold several
 * requests.  Up to `slots` pieces run at once, each on its own stream in its
 * own first-fit region of the arena, so requests that arrive while others run
 * are admitted as soon as a slot and memory are free and run beside them.  The
 * last slot only takes requests that have not started, so a short request
 * does not wait behind the rest of a long one.  A request completes when its
 * last location's results are in (its own completion time).  Each location's
 * arithmetic is independent of the piece it runs in (locations are
 * independent, Section 4.1): a request's results are bitwise the same alone
 * or mixed with other traffic.  Pieces in flight share no device memory:
 * each has its own workspace.
 * All server arrays are HOST memory; inputs are copied at submission.
 * Calls are thread-safe.  The server must be destroyed before its design.
 * slots: 0 (3) or 2..8; piece_locations: 0 (1024) or 1..131072; other
 * values give LAGP_E_INVAL.  lagp_server_create uses the defaults. */
typedef struct lagp_server lagp_server;
int lagp_server_create(const lagp_design *design, size_t hbm_budget_bytes, lagp_server **out);
int lagp_server_create_ex(const lagp_design *design, size_t hbm_budget_bytes, int32_t slots,
                          int32_t piece_locations, lagp_server **out);

/* Queue T locations XX (host, T x p) with per-location n / N' (host int32[T],
 * nullable: params values).  Checks as lagp_predict; params->flags must be 0.
 * Returns LAGP_E_BUDGET when the request alone cannot fit the arena.  Does
 * not wait for the device; *ticket identifies the request. */
int lagp_server_submit(lagp_server *server, const double *XX, int32_t T, const lagp_params *params,
                       const int32_t *n_per, const int32_t *ncand_per, uint64_t *ticket);

/* Returns 1 and copies the results (host arrays, each nullable; sel is
 * T x sel_stride with sel_stride >= the request's largest n) when the request
 * is done, releasing the ticket; 0 while it is pending.  wait_ms: 0 polls,
 * > 0 waits at most that long, < 0 waits for completion.  times (nullable)
 * receives [submission, completion] in seconds on the monotonic clock of
 * lagp_monotonic_seconds.  A request a failed piece held returns its error code. */
int lagp_server_poll(lagp_server *server, uint64_t ticket, int32_t wait_ms, double *mean, double *s2, int32_t *df,
                     double *var, int32_t *sel, int64_t sel_stride, int8_t *status, double *times);

/* Pieces dispatched, locations and requests completed, and seconds during
 * which at least one piece was in flight, since creation. */
int lagp_server_stats(lagp_server *server, int64_t *pieces, int64_t *locations, int64_t *requests,
                      double *busy_seconds);

/* Finish the queued requests, stop the threads and free the arena.  NULL is ignored. */
void lagp_server_destroy(lagp_server *server);

/* Seconds on the steady (monotonic) clock the server's timestamps use. */
double lagp_monotonic_seconds(void);

/* ---- An entry point that allocates nothing.
 *
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * lagp_predict with uniform sizes (params->n, params->ncand for every
 * location) whose workspace is a fixed device array of
 * LAGP_NOALLOC_SCRATCH_BYTES inside the library instead of memory allocated
 * on the design.  Each device holds its own copy of the array from the first
 * call there until the process ends.  Locations run in chunks small enough
 * for a chunk's workspace to fit the array; a configuration whose single
 * location does not fit returns LAGP_E_BUDGET.  Arguments, outputs and
 * results are those of lagp_predict (device pointers; params->flags must be
 * 0); the kNN runs its fixed pass budget without host waits, and a location
 * whose candidate set fails the kNN's consistency check gets status
 * LAGP_LOC_NOCAND.  Every call on a device shares that device's array: calls
 * that overlap on one device (two host threads, two streams) race, so
 * serialise them.  No memory is allocated or freed by this call. */
#define LAGP_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int lagp_predict_noalloc(const lagp_design *design, const double *XX, int64_t T, const lagp_params *params,
                         double *mean, double *s2, int32_t *df, double *var, int32_t *sel, int64_t sel_stride,
                         int8_t *status, void *stream);
/* The size of that array in bytes (LAGP_NOALLOC_SCRATCH_BYTES). */
size_t lagp_noalloc_scratch_bytes(void);

/* Device bytes of workspace lagp_predict needs for a batch of T locations
 * with the given maxima (for admission control by callers). */
int lagp_workspace_bytes(const lagp_design *design, int64_t T, int32_t nmax, int32_t ncand_max,
                         size_t *out);

/* Per-phase device timing.  While enabled, the prediction entry points record
 * HIP events on their stream between the phases of each chunk of locations:
 * the candidate-set (kNN) kernels; each design pass (the greedy-design kernel
 * launches, one per size bucket, plus in the mixed mode the FP64 prediction
 * kernel and the FP64 redo launch); in the two-stage scheme each likelihood
 * pass and the final prediction.  lagp_phase_times waits for the recorded
 * events, writes the summed milliseconds per phase into ms[LAGP_PHASES]
 * (indexed by LAGP_PHASE_*) and the number of design-kernel bucket launches
 * since the last call, and clears the record. */
enum { LAGP_PHASE_KNN = 0, LAGP_PHASE_DESIGN = 1, LAGP_PHASE_MLE = 2, LAGP_PHASE_PREDICT = 3, LAGP_PHASES = 4 };
int lagp_timing_enable(lagp_design *design, int enable);
int lagp_phase_times(lagp_design *design, double *ms, int64_t *design_launches);

/* Number of HIP devices visible (0 when none); never fails. */
int lagp_device_count(void);

/* Thread-local description of the last non-OK status returned on this thread. */
const char *lagp_last_error(void);

/* ABI version (major * 100 + minor). */
int lagp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LAGP_H */
