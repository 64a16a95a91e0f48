/*
 * pcv.h -- C ABI of the MI355X parallel cross-validation library.
 *
 * Computes the parallel CV loss of Gerber & Nychka, "Parallel
 * cross-validation: a scalable fitting method for Gaussian process models"
 * (arXiv:1912.13132) on one AMD Instinct MI355X (gfx950), and kriging
 * predictions from the resulting per-subset factors.
 *
 *   model            Sec. 2.1, eq. (1):  y ~ N(0, sigma^2 Sigma(theta) + tau I)
 *   kriging          Sec. 2.1, eq. (3):  yhat = Sigma_p^T (Sigma + lambda I)^{-1} y,
 *                                        lambda = tau / sigma^2
 *   hold-out loss    Sec. 2.2, eq. (4):  SSPE = sum_v (yhat_v - y_v)^2
 *   parallel CV      Sec. 2.3, eq. (7) and Algorithm 1:
 *                                        CV~ = sum_i CV(y~^i_T, y^i_V, zeta)
 *   covariance       Sec. 3:             c(d) = exp(-d / theta)
 *
 * Conventions shared by every call
 *   - Every call returns a pcv_status; PCV_OK (0) is success.  On failure
 *     pcv_last_error() returns a thread-local message naming the offending
 *     argument / subset.
 *   - All validation happens before any device work: a call that returns
 *     PCV_ERR_INVALID has had no side effects.
 *   - Host arrays are owned by the caller and only read (inputs) or written
 *     (outputs) during the call.  pcv_problem_create copies its inputs to
 *     device memory; the problem owns those copies.
 *   - Locations are row-major (x, y) pairs in float64.  Index arrays are
 *     0-based.  A subset's training and validation points are given as CSR:
 *     subset i trains on train_idx[train_ptr[i] .. train_ptr[i+1]) and
 *     validates on val_idx[val_ptr[i] .. val_ptr[i+1]).
 *   - One caller thread per pcv_problem.  Different problems may be used
 *     from different threads.
 *   - The library runs on the HIP device that is current when the problem
 *     is created and uses that device for the problem's lifetime.
 */
#ifndef PCV_H
#define PCV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PCV_OK = 0,
  PCV_ERR_INVALID = 1, /* bad argument; nothing was done                      */
  PCV_ERR_OOM = 2,     /* device or pinned memory exhausted / over the cap     */
  PCV_ERR_NOT_PD = 3,  /* a subset matrix is not positive definite in FP64     */
  PCV_ERR_DEVICE = 4,  /* a HIP runtime call failed                            */
  PCV_ERR_STATE = 5,   /* call out of order (e.g. predict before factor)       */
  PCV_ERR_BUSY = 6     /* a wait timed out / the server is shutting down       */
} pcv_status;

/* Covariance family.  PCV_COV_EXP is the paper's exponential covariance
 * (Sec. 3).  PCV_COV_MATERN32 is the Matern nu = 3/2 member of the same
 * parametrisation, c(d) = (1 + d/theta) exp(-d/theta). */
typedef enum { PCV_COV_EXP = 0, PCV_COV_MATERN32 = 1 } pcv_cov;

/* Arithmetic of a theta-evaluation.
 * PCV_PREC_FP64:  covariance, Cholesky, solves, prediction and loss in FP64
 *                 (the factorisation's tile updates on FP64 MFMA).
 * PCV_PREC_MIXED: covariance tiles and the bulk of the Cholesky in FP32
 *                 (FP32 MFMA, FP32 accumulation); diagonal blocks factored in
 *                 FP64; solves accumulate in FP64; iterative refinement with
 *                 an FP64 residual regenerated from FP64 coordinates; FP64
 *                 prediction and loss. */
typedef enum { PCV_PREC_FP64 = 0, PCV_PREC_MIXED = 1 } pcv_prec;

/* zeta of Sec. 2.1: range theta > 0 and noise-to-signal ratio
 * lambda = tau / sigma^2 >= 0.  sigma2 > 0 only scales kriging variances
 * (it cancels from eq. (3) and eq. (4)). */
typedef struct {
  int32_t cov;   /* pcv_cov */
  double range;  /* theta  */
  double lambda; /* lambda */
  double sigma2; /* sigma^2 */
} pcv_theta;

typedef struct {
  int32_t prec;           /* pcv_prec; default PCV_PREC_MIXED                        */
  int32_t max_refine;     /* mixed: refinement sweeps, at most (default 2, max 8).
                             Every subset takes the first; a later one only where
                             the residual the previous sweep measured has
                             ||r||_2 > refine_tol * ||y_T||_2                    */
  double refine_tol;      /* mixed: a subset whose residual before its last correction
                             has ||r||_2 > tol * ||y_T||_2 is re-run in FP64 (1e-4)  */
  void* hip_stream;       /* hipStream_t to run on; NULL = library-owned stream      */
  size_t mem_cap_bytes;   /* device workspace cap, 0 = no cap                         */
  int32_t profile;        /* nonzero: time each kernel phase with HIP events          */
  int32_t debug_flags;    /* testing hook, 0 in production.  Bit 0: in mixed mode
                             treat every FP32 factorisation as broken down, so the
                             FP64 fallback path runs for every subset.  Bit 1:
                             pcv_eval behaves as if another evaluation's shared
                             launch held the device (see max_wg_per_subset)    */
  int32_t graph;          /* nonzero (default): capture the theta-evaluation once as a
                             HIP graph and replay it; 0: launch kernel by kernel  */
  int32_t inputs_on_device; /* nonzero: every array argument of pcv_problem_create
                             and pcv_predict (inputs and outputs) is a device
                             pointer on the current device, e.g. a torch tensor's
                             data_ptr().  Each must lie inside one device (or
                             managed) allocation, else PCV_ERR_INVALID.  The
                             library reads the inputs on hip_stream (with no
                             hip_stream, after a device-wide synchronisation),
                             so writes the caller queued there come first;
                             nothing is kept after the call returns.  The
                             other calls always take host arrays.  Default 0 */
  int32_t max_wg_per_subset; /* work-groups that may factor one subset together
                             in pcv_eval's first factorisation launch: a subset
                             whose padded size n is at least 2,048 and whose
                             n^3 exceeds the launch's average n^3 per compute
                             unit gets round(n^3 / average) of them, within
                             [2, this], as long as the launch's shared
                             work-groups fit one per compute unit.  Same
                             factor bit for bit.  1 = one work-group per
                             subset; 0 = default (8); at most 8.  Not used by
                             a served problem or by the multi-theta launches
                             of pcv_eval_batch.  The work-groups of a shared
                             subset wait for each other with a bounded wait,
                             so at most one evaluation per device and process
                             runs a shared launch at a time: an evaluation
                             that finds one in flight on its device (another
                             problem evaluated concurrently from another
                             thread) factors with one work-group per subset,
                             the same bits, and reports n_coop_subsets = 0.
                             Shared launches of other processes on the same
                             device are not seen; two of them side by side can
                             hold each other's compute units until a wait runs
                             out, and the subsets concerned are then re-run in
                             FP64 (mixed) or the evaluation fails with
                             PCV_ERR_DEVICE (FP64): set 1 when several
                             processes evaluate on one device */
  int32_t est_error;      /* mixed, nonzero: pcv_eval estimates its loss error
                             against the FP64 path (est_rel_err of the report):
                             one more refinement sweep is applied to a copy of
                             every FP32-factored subset's alpha and the loss
                             recomputed from it; the refinement contracts the
                             solve error by a large factor per sweep, so the
                             loss change is the current loss error up to that
                             factor.  Costs about one sweep and one
                             prediction pass per pcv_eval that asks for a
                             report.  Default 0 */
  int32_t reserved[2];
} pcv_options;

/* Per-evaluation report.  Arrays are optional, caller-owned, length S. */
typedef struct {
  double sspe;               /* = *loss                                             */
  int64_t n_val;             /* validation points over non-skipped subsets          */
  double mse;                /* sspe / n_val                                        */
  int32_t n_subsets_used;    /* subsets with >= 1 validation point                  */
  int32_t n_fallback_fp64;   /* mixed: subsets re-run in FP64                       */
  int32_t max_refine_iters;  /* mixed: largest number of sweeps any subset used     */
  int32_t pad0;
  double max_rel_residual;   /* mixed: max_i ||r_i|| / ||y_i|| of the residual the
                                last refinement sweep corrected                     */
  double seconds;            /* wall time of the call                               */
  /* phase times in ms (HIP events on the evaluation stream), when profiling */
  double ms_factor, ms_solve, ms_refine, ms_predict, ms_reduce;
  double* per_subset_sspe;   /* optional out [S]: z_i (0 for skipped subsets)       */
  double* per_subset_logdet; /* optional out [S]: log det(Sigma_i + lambda I)       */
  int32_t* per_subset_iters; /* optional out [S]: refinement sweeps used (0 for a
                                subset re-run in FP64); pcv_eval only            */
  /* Composite likelihood over the evaluated subsets (Sec. 2.1, eq. (2) applied
   * to each subset's training data, tau = lambda sigma^2):
   *   -2 l_i = n_i log(2 pi) + n_i log sigma^2 + log det(Sigma_i + lambda I)
   *            + y_i^T (Sigma_i + lambda I)^{-1} y_i / sigma^2.
   * In mixed precision the log det comes from the FP32 factor (relative
   * error ~1e-6 of |log det|); the quadratic term uses the refined alpha. */
  double neg2loglik;              /* sum of -2 l_i                                  */
  double* per_subset_neg2loglik;  /* optional out [S] (0 for skipped subsets)       */
  /* Schedule (pcv_eval).  When there are more evaluated subsets than compute
   * units and not a whole number of rounds of them, the largest
   * n_factor_first subsets are factored first (whole rounds) and the rest
   * beside their solves.  When profiling, ms_factor is that first
   * factorisation launch alone, ms_solve / ms_refine / ms_predict the first
   * group's later phases and ms_factor_all the factorisation of every subset
   * on its stream.  With one group n_factor_first = S evaluated subsets and
   * ms_factor_all = ms_factor.  n_coop_subsets of the first launch's
   * largest subsets were each factored by several work-groups together
   * (see max_wg_per_subset). */
  int32_t n_factor_first;
  int32_t n_coop_subsets;
  double ms_factor_all;
  /* pcv_eval's estimated relative error of the loss against the FP64 path:
   * |loss - loss'| / |loss|, loss' the loss after one more refinement sweep
   * (see est_error).  0 in FP64 mode, -1 when not estimated. */
  double est_rel_err;
} pcv_eval_report;

typedef struct pcv_problem pcv_problem;

void pcv_default_options(pcv_options* opt);

/* Make a problem resident on the current device (Algorithm 1, steps 2-5:
 * the data are divided and read once, then evaluated for many zeta).
 *   n          number of locations (>= 1)
 *   locs       host float64 [n][2]
 *   y          host float64 [n]
 *   S          number of subsets (>= 1)
 *   train_ptr  host int64 [S+1], nondecreasing, train_ptr[0] = 0
 *   train_idx  host int32 [train_ptr[S]], each in [0, n)
 *   val_ptr    host int64 [S+1], nondecreasing, val_ptr[0] = 0
 *   val_idx    host int32 [val_ptr[S]], each in [0, n)
 *   core_rect  host float64 [S][4] (xlo, ylo, xhi, yhi) of each core, used to
 *              route prediction queries; may be NULL (then pcv_predict routes
 *              every query to the subset whose training centroid is nearest)
 *   opt        may be NULL (defaults)
 * All arrays are device arrays instead when opt->inputs_on_device is set.
 * Subsets without validation points are kept but never evaluated (they
 * contribute 0, as in Sec. 4.3.1).  A subset larger than the library's
 * maximum (PCV_MAX_SUBSET training points) is rejected with PCV_ERR_INVALID.
 * Errors: PCV_ERR_INVALID (sizes, NaN/Inf, index range, ptr order),
 * PCV_ERR_OOM, PCV_ERR_DEVICE. */
#define PCV_MAX_SUBSET 16320
pcv_status pcv_problem_create(pcv_problem** out, int64_t n, const double* locs,
                              const double* y, int32_t S, const int64_t* train_ptr,
                              const int32_t* train_idx, const int64_t* val_ptr,
                              const int32_t* val_idx, const double* core_rect,
                              const pcv_options* opt);

/* One theta-evaluation: *loss = CV~ of eq. (7) (the SSPE summed over all
 * subsets with validation data).  Synchronous: returns after the loss is
 * on the host.  report may be NULL.
 * Errors: PCV_ERR_INVALID (theta), PCV_ERR_NOT_PD (an FP64 factorisation
 * broke down; pcv_last_error names the subset), PCV_ERR_DEVICE. */
pcv_status pcv_eval(pcv_problem* p, const pcv_theta* theta, double* loss,
                    pcv_eval_report* report);

/* n_theta evaluations; losses[k] for thetas[k], bit-identical to n_theta
 * calls of pcv_eval.  Up to 64 theta values run together, one launch per
 * kernel over all (theta, subset) pairs (the per-theta workspace is sized
 * from the memory cap, else at most 16 GiB; when one slot does not fit twice,
 * the values run one by one).  A theta whose subsets need the FP64 re-run
 * is evaluated again on its own. */
pcv_status pcv_eval_batch(pcv_problem* p, int32_t n_theta, const pcv_theta* thetas,
                          double* losses);

/* As pcv_eval_batch; report (may be NULL) receives the wall time, the phase
 * times summed over the launches (when profiling), n_val, n_subsets_used and
 * in n_fallback_fp64 the number of theta values evaluated again on their own.
 * The per-subset arrays of the report are not written. */
pcv_status pcv_eval_batch_ex(pcv_problem* p, int32_t n_theta, const pcv_theta* thetas,
                             double* losses, pcv_eval_report* report);

/* Local losses over a set of theta values (Sec. 4.4: local RMSPE and the
 * best local zeta of each subset, the basis of non-stationary fits),
 * evaluated by the multi-theta launches of pcv_eval_batch.
 * losses[k] as pcv_eval for thetas[k] (bit for bit); per_subset_sspe (may be NULL) receives
 * z_i(theta_k) at [k * S + i]; best (may be NULL) receives, per subset, the k
 * with the smallest z_i (lowest k on ties; -1 for subsets without
 * validation points). */
pcv_status pcv_eval_grid(pcv_problem* p, int32_t n_theta, const pcv_theta* thetas, double* losses,
                         double* per_subset_sspe, int32_t* best);

/* Launch shapes and schedule picked by measurement.  pcv_autotune times
 * pcv_eval at theta under the candidate choices that change a launch of this
 * problem and keeps the fastest for every later evaluation of the problem
 * (pcv_eval, pcv_eval_batch, served evaluations):
 *   small_npad         FP32 factorisations whose schedule group's largest
 *                      subset pads to at most this many rows use 4-wave
 *                      work-groups with 64-column panels, the others 8-wave
 *                      ones with 128-column panels (candidates 0, 1,024,
 *                      1,408 = the default, 1,536, 2,048, 3,072, 4,096;
 *                      FP64 always uses 8-wave ones);
 *   max_wg_per_subset  work-groups sharing one large subset in the first
 *                      launch (1, 2, 3, 4, 6, 8; see pcv_options);
 *   two_groups         1: the largest subsets in whole rounds of one
 *                      work-group per compute unit, the rest in a second
 *                      launch beside the first group's solves; 0: one launch.
 * Coordinate search (small_npad, then max_wg_per_subset, then two_groups),
 * candidates that launch the same shapes are timed once; each candidate is
 * one warm-up evaluation (its graph is captured) and `reps` timed ones
 * (median).  Sharing, the schedule groups and the graph change no bits; the
 * shape threshold changes the factor's rounding (both shapes are within the
 * mixed path's tolerance), so losses after tuning may differ from the
 * defaults' in the last bits, and pcv_eval and pcv_eval_batch stay
 * bit-identical to each other.
 * cache_path (may be NULL): a text file of earlier choices, one line per
 * problem shape, keyed by the device architecture, the HIP runtime version,
 * this library's build, the precision and the padded sizes of the evaluated
 * subsets in schedule order; a matching line is applied without timing
 * (report->from_cache = 1), a new choice is appended.  reps in [1, 20].
 * The problem must not be held by a server.  report may be NULL.
 * Errors: PCV_ERR_INVALID (theta, reps), PCV_ERR_STATE (served),
 * PCV_ERR_NOT_PD / PCV_ERR_DEVICE as pcv_eval. */
typedef struct {
  int32_t small_npad, max_wg_per_subset, two_groups;
  int32_t from_cache;        /* 1: taken from the cache file, nothing timed     */
  int32_t n_timed;           /* configurations timed                             */
  int32_t pad0;
  double default_s;          /* seconds per evaluation with the defaults         */
  double best_s;             /* with the chosen configuration                    */
  double tuning_s;           /* wall time of the call                            */
} pcv_tune_report;
pcv_status pcv_autotune(pcv_problem* p, const pcv_theta* theta, const char* cache_path, int32_t reps,
                        pcv_tune_report* report);

/* Factor every subset at theta in FP64 and keep L_i and
 * alpha_i = (Sigma_i + lambda I)^{-1} y_i resident for pcv_predict. */
pcv_status pcv_factor(pcv_problem* p, const pcv_theta* theta);

/* As pcv_factor, but subset i at its own thetas[i] (host array [S]): local
 * zeta, so that pcv_predict gives the non-stationary predictions the paper
 * suggests in Sec. 5 (each query uses its owning subset's parameters). */
pcv_status pcv_factor_local(pcv_problem* p, const pcv_theta* thetas);

/* Kriging at q query locations (host float64 [q][2]) from the factors of
 * the last pcv_factor: each query is routed to its core (half-open
 * rectangles, edges on the domain maximum closed, nearest core if outside
 * all), mean = k^T alpha (eq. (3)) and
 * var = sigma^2 (1 - k^T (Sigma + lambda I)^{-1} k) (+ sigma^2 lambda when
 * obs_noise != 0).  var may be NULL.  owner (may be NULL) receives each
 * query's subset.  With the problem's inputs_on_device option, qlocs, mean,
 * var and owner are device arrays and the results are in them when the call
 * returns.  Errors: PCV_ERR_STATE before pcv_factor. */
pcv_status pcv_predict(pcv_problem* p, int64_t q, const double* qlocs, double* mean,
                       double* var, int32_t obs_noise, int32_t* owner);

/* For callers that cannot allocate device memory (code running beside a HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * pcv_predict with every work buffer (grouped queries, work items, means,
 * variances and the variance's per-item panels) in a fixed device array of
 * PCV_NOALLOC_SCRATCH_MIB MiB inside the library, one per device, held from
 * the first call on that device until the process ends.  The caller passes
 * inputs and outputs as for pcv_predict (host arrays, or device arrays with
 * inputs_on_device); results are bit for bit those of pcv_predict.  Calls no
 * hipMalloc / hipFree; routing and the item plan on the host reuse buffers
 * the problem keeps (grown by the first calls).  At most
 * PCV_NOALLOC_MAX_QUERIES queries per call, else PCV_ERR_INVALID with
 * nothing launched; items whose panels do not fit the array together run in
 * consecutive launches.  Calls on one device share the array: the library
 * serialises them inside a process (a per-device lock held until the call's
 * stream has drained), and unsynchronised calls from outside that lock would
 * race on it.  Errors as pcv_predict. */
#define PCV_NOALLOC_SCRATCH_MIB 128
#define PCV_NOALLOC_MAX_QUERIES 262144
pcv_status pcv_predict_noalloc(pcv_problem* p, int64_t q, const double* qlocs, double* mean,
                               double* var, int32_t obs_noise, int32_t* owner);

/* Generalised least squares estimate of a linear mean in each subset (Sec. 5,
 * eq. (8)): beta_i = (X_i^T M_i^{-1} X_i)^{-1} X_i^T M_i^{-1} y_i through the
 * FP64 factors of the last pcv_factor / pcv_factor_local.
 *   X       host float64 [n][n_cov], covariates of every location (row-major),
 *           1 <= n_cov <= 8
 *   beta    host float64 [S][n_cov] out; NaN for subsets without training
 *           points or whose normal matrix is not positive definite
 *   status  host int32 [S] out (may be NULL): 0 fine, j + 1 normal matrix not
 *           positive definite at column j, -1 no training points
 * Errors: PCV_ERR_INVALID, PCV_ERR_STATE (before pcv_factor). */
pcv_status pcv_gls(pcv_problem* p, int32_t n_cov, const double* X, double* beta, int32_t* status);

pcv_status pcv_problem_destroy(pcv_problem* p);

/* Sizes of the problem: subsets, total training memberships, largest
 * subset, device bytes held. */
pcv_status pcv_problem_info(const pcv_problem* p, int32_t* S, int64_t* nnz_train,
                            int32_t* max_train, size_t* device_bytes);

const char* pcv_status_string(pcv_status s);
const char* pcv_last_error(void);

/* Testing hook for the FP64 device arithmetic of the refinement residual and
 * the kriging of validation points: on the current device,
 * e[i] = e^{-t[i]} (t[i] >= 0; t above 740 is taken as 740) and
 * r[i] = sqrt(x[i]) (x[i] >= 0), for i < n.  Host arrays of n doubles.
 * Errors: PCV_ERR_INVALID (n < 0, NULL arrays, negative or non-finite
 * input), PCV_ERR_OOM, PCV_ERR_DEVICE. */
pcv_status pcv_selftest_math(int64_t n, const double* t, const double* x, double* e, double* r);

/* -------------------------------------------------------- partitioning --
 * The division of Sec. 2.3 / 2.4 (Algorithm 1, steps 2-3) on the device: the
 * input preparation for pcv_problem_create.  Rectangles are (xlo, ylo, xhi,
 * yhi), half-open [lo, hi) per axis with edges on the domain maximum closed
 * (the domain is the bounding box of the cores).  A core's shell is its
 * rectangle widened by delta on every side, clipped to the domain, minus the
 * core; shells add training points only.  Temporary device memory is
 * allocated and freed inside each call.  Results are deterministic. */

/* Recursive balanced division of `domain` (float64 [4]) into m cores
 * (Sec. 2.4): the x-range is split first and the axes alternate; a
 * rectangle with k cores is cut into floor(k/2) : ceil(k/2) cores where the
 * point counts of the two halves, each with its shell of width delta, are in
 * that ratio (64 bisection steps on the cut; without shells the cut is moved
 * midway between the neighbouring coordinates).  core_rect: host float64
 * [m][4] out, in depth-first order (lower / left half first). */
pcv_status pcv_part_divide(int64_t n, const double* locs, const double* domain, int32_t m, double delta,
                           double* core_rect);

/* Total memberships sum_i |core_i + shell_i| of all n points for the cores
 * and delta (the quantity the overlap of a division is set by). */
pcv_status pcv_part_count(int64_t n, const double* locs, int32_t S, const double* core_rect, double delta,
                          int64_t* memberships);

/* Subsets of the cores: owner (host int32 [n] out, may be NULL) is the core
 * of every point (lowest index on shared edges); subset i trains on the
 * points of core i and of its shell that are not held out (is_val: host
 * uint8 [n], nonzero = held out, may be NULL = none) and validates on the
 * held-out points of core i.  train_ptr / val_ptr: host int64 [S+1] out
 * (may be NULL); train_idx / val_idx: host int32 out of train_ptr[S] /
 * val_ptr[S] entries, increasing within each subset (may be NULL: call once
 * for the sizes, then again for the lists).
 * Errors: PCV_ERR_INVALID (arguments; a point outside every core). */
pcv_status pcv_part_subsets(int64_t n, const double* locs, int32_t S, const double* core_rect, double delta,
                            const uint8_t* is_val, int32_t* owner, int64_t* train_ptr, int32_t* train_idx,
                            int64_t* val_ptr, int32_t* val_idx);

/* ------------------------------------------------------------ serving --
 * A server owns a resident problem while it exists (do not call the
 * pcv_problem functions on it meanwhile) and accepts, from any number of
 * threads, kriging requests (from the factors of the last pcv_factor, as in
 * pcv_predict) and theta-evaluation requests (as in pcv_eval), so that the
 * factored subsets stay in device memory between requests (the data are read
 * once and evaluated for many zeta, Algorithm 1).
 *
 * Continuous batching: kriging requests are routed in the submitting thread
 * and queued; a batcher packs queued queries, first come first served and
 * grouped by subset across requests, into the next free workspace slot and
 * launches it while earlier batches are still on the device; a request
 * larger than a slot spans several batches.  Evaluations run concurrently
 * on their own stream.  Each query's result is independent of the batch it
 * shares (the same bits as pcv_predict).
 *
 * Memory-gated admission: the workspace (mem_budget bytes of device memory,
 * split over 3 slots, plus the same amount of pinned host memory for the
 * query and result buffers) bounds the queries and kriging items of one
 * batch; at most max_inflight requests are admitted and unfinished at any
 * time, and a submit call blocks until a place is free.
 *
 * Pointers passed to a submit call (query locations, outputs) must stay
 * valid until pcv_server_wait for its ticket has returned. */
typedef struct pcv_server pcv_server;
typedef int64_t pcv_ticket;

/* mem_budget: workspace bytes, 0 = 8 GiB.  max_inflight >= 1.
 * Errors: PCV_ERR_INVALID (budget below one kriging item per slot),
 * PCV_ERR_OOM, PCV_ERR_DEVICE. */
pcv_status pcv_server_create(pcv_server** out, pcv_problem* p, size_t mem_budget,
                             int32_t max_inflight);

/* Queue kriging of q query locations (host float64 [q][2]); mean (host
 * [q]) and var (host [q], may be NULL) are written before pcv_server_wait
 * returns PCV_OK for *ticket.  obs_noise as in pcv_predict.
 * Errors: PCV_ERR_INVALID, PCV_ERR_STATE (no pcv_factor before the server
 * was created). */
pcv_status pcv_server_submit_predict(pcv_server* s, int64_t q, const double* qlocs, double* mean,
                                     double* var, int32_t obs_noise, pcv_ticket* ticket);

/* Queue one theta-evaluation; *loss is written before pcv_server_wait
 * returns PCV_OK for *ticket. */
pcv_status pcv_server_submit_eval(pcv_server* s, const pcv_theta* theta, double* loss,
                                  pcv_ticket* ticket);

/* Batching window for kriging while evaluations are active (default 0.03 s).
 * Reading the resident factors dominates a kriging batch (a batch touching
 * every subset reads all of them), so batches launched back to back would
 * keep the device from the evaluations.  While evaluation requests are
 * queued or running, a kriging batch is launched only once its oldest query
 * has waited `seconds`, or the queue holds a full batch; with no evaluation
 * active a batch is launched as soon as a workspace slot is free.  0 turns
 * the window off.  Errors: PCV_ERR_INVALID (seconds outside [0, 10]). */
pcv_status pcv_server_set_batch_window(pcv_server* s, double seconds);

/* Wait for a request (timeout_s < 0: no limit) and collect it: returns the
 * request's own status, after which the ticket is no longer valid.
 * PCV_ERR_BUSY: not finished within timeout_s (the ticket stays valid).
 * PCV_ERR_INVALID: unknown or already collected ticket. */
pcv_status pcv_server_wait(pcv_server* s, pcv_ticket ticket, double timeout_s);

/* Latency of finished kriging requests (submit to results written, nearest-
 * rank percentiles, seconds), kriging queries and evaluations per second
 * from the first submit to the last completion. */
pcv_status pcv_server_stats(pcv_server* s, double* p50_s, double* p99_s, double* qps,
                            double* evals_per_s);

typedef struct {
  int64_t n_predict, n_eval, n_queries;  /* finished requests / queries     */
  int64_t n_batches;                     /* kriging launches                */
  double mean_batch_queries;
  double p50_s, p99_s, max_s;            /* kriging request latency          */
  double eval_p50_s, eval_p99_s;         /* evaluation request latency       */
  double elapsed_s, qps, evals_per_s;
  int64_t admission_waits;               /* submits that had to wait         */
  int64_t workspace_bytes;               /* device bytes of the slots        */
  int64_t batch_query_cap, batch_item_cap;
} pcv_server_report;
pcv_status pcv_server_report_get(pcv_server* s, pcv_server_report* out);

/* Finish every queued request, then stop and free the server.  Tickets not
 * collected become invalid.  The problem stays usable. */
pcv_status pcv_server_destroy(pcv_server* s);

#ifdef __cplusplus
}
#endif
#endif /* PCV_H */
