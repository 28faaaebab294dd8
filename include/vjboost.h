/*
 * vjboost.h -- C ABI of the MI355X (gfx950) Viola-Jones AdaBoost round engine.
 *
 * The library trains discrete AdaBoost over Haar-feature decision stumps as
 * described in arXiv 1306.1467, Section 2 (integral image, Section 2.1; the five
 * Haar feature types and the decision stump, Section 2.2; weights,
 * normalisation, best-stump search, update and the strong classifier,
 * Section 2.3).  Each boosting round searches every feature and every window
 * for the stump with the smallest weighted error, then updates the weights.
 *
 * General rules for every entry point:
 *  - Plain C types only; every "d_" pointer is HIP device memory, every other
 *    pointer is host memory.  Nothing is retained from a host pointer after the
 *    call returns.
 *  - Return value: BOOST_OK (0) or a negative status below; details are in
 *    boost_last_error() (a thread-local string, valid until the next call on
 *    that thread).  No exception crosses this boundary.
 *  - Work is enqueued on boost_options.stream (a hipStream_t; NULL is the
 *    legacy default stream).  A call returns once its work is enqueued, except
 *    where it says it synchronises (any call that writes a host output does).
 *  - Sample indices seen through this interface are the caller's order; the
 *    library internally keeps positives first.
 *  - One context must not be used from two threads at once.
 */
#ifndef VJBOOST_H
#define VJBOOST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define BOOST_OK            0
#define BOOST_E_INVALID    (-1)  /* bad argument (see each call) */
#define BOOST_E_NOMEM      (-2)  /* workspace too small */
#define BOOST_E_DEVICE     (-3)  /* a HIP runtime error */
#define BOOST_E_DEGENERATE (-4)  /* eps = 0 (or below the floor) with BOOST_ON_PERFECT_STOP */

/* ------------------------------------------------------------ feature set
 * Section 2.2: five Haar feature types.  Bit t of type_mask enables type t:
 *   0 three-rectangle horizontal [white | dark | white]
 *   1 three-rectangle vertical   (the same stacked)
 *   2 two-rectangle horizontal   [white | dark]
 *   3 two-rectangle vertical     [white / dark]
 *   4 four-rectangle             [white dark / dark white]
 * A feature's value is (sum over dark cells) - (sum over white cells), exact
 * int32.  Each cell is cell_w x cell_h pixels (both >= 1, scaled
 * independently) and the feature sits at every (x, y) where it fits in the
 * window.  Global index order: type (in the order above), cell_w, cell_h, y,
 * x (x fastest).  For a 24x24 window this gives 27,600 + 27,600 + 43,200 +
 * 43,200 + 20,736 = 162,336 features, the counts printed in Section 2.2.
 * Windows are 1..32 pixels on each side. */
#define BOOST_TYPE_3H 0
#define BOOST_TYPE_3V 1
#define BOOST_TYPE_2H 2
#define BOOST_TYPE_2V 3
#define BOOST_TYPE_4  4
#define BOOST_ALL_TYPES 0x1Fu

typedef struct {
    int32_t  window_w;
    int32_t  window_h;
    uint32_t type_mask;
} boost_feature_set;

typedef struct {
    int32_t type, x, y, cell_w, cell_h;
} boost_feature;

/* ------------------------------------------------------------ options
 * precision: arithmetic of the per-round weighted-error scan.
 *   BOOST_PREC_FP32        FP32 weights, FP32 running sums (plain).
 *   BOOST_PREC_FP32_KAHAN  FP32 weights, a compensated FP32 running sum:
 *                          Fast2Sum (the sum is biased so that it always
 *                          dominates the added weight) collects each
 *                          addition's exact rounding error in an FP32
 *                          compensation term, folded back into the sum every
 *                          16 keys; candidates are compared in FP64 (the
 *                          prefix s + c at the last key of each 8-key unit,
 *                          and for each earlier key the next key's candidate
 *                          minus the next key's weight).
 *   BOOST_PREC_FP64        FP64 weights and FP64 running sums (n <= 20000:
 *                          the table must fit in LDS).
 *   BOOST_PREC_FP32_WIDE   FP32 weights accumulated in FP64.  For weights
 *                          above ~1e-9 every sum is exact, so the only
 *                          difference from FP64 weights is the FP32 rounding
 *                          of each weight (<= 2^-24 relative on every error).
 * Normalisation, the update, beta and alpha are always FP64.
 * on_perfect: what a round with eps_raw <= eps_floor does.  Section 2.3 leaves
 *   eps = 0 undefined (beta = 0, alpha infinite).  CLAMP uses
 *   eps' = max(eps, eps_floor) for beta and alpha and goes on; STOP records
 *   the stump, leaves the weights unchanged and makes every later round a
 *   no-op (its record has feature = -1), returning BOOST_E_DEGENERATE.
 * eps_floor: > 0 and < 0.5 (default 1e-10).
 * schedule_id: 0 picks the default launch shape (512-thread workgroups, 8
 *   key units per load batch, 16 lanes per feature); 1 .. count-1 select
 *   other shapes (see boost_schedule_count), among them 9 and 10, which keep
 *   4 key units per lane in flight all the time (rotating loads at 512 and
 *   1024 threads); BOOST_SCHEDULE_AUTO lets init time every shape that
 *   shares the default's 16-lane key layout on the job's own keys and keep
 *   the fastest (batches: per key format, by successive halving, then also
 *   the work-queue granularity).  Choices are cached per process by device
 *   and workload shape, and also in the file named by the environment
 *   variable VJBOOST_TUNE_CACHE when it is set (read on the first miss,
 *   appended on each new choice; entries that do not fit are re-tuned);
 *   boost_get_schedule / boost_batch_get_schedule report them.
 * flags: BOOST_FLAG_TIMING records per-kernel device times (boost_get_timing);
 *   BOOST_FLAG_NO_GRAPH launches kernels directly instead of replaying a
 *   captured HIP graph in boost_train. */
#define BOOST_PREC_FP32        0
#define BOOST_PREC_FP32_KAHAN  1
#define BOOST_PREC_FP64        2
#define BOOST_PREC_FP32_WIDE   3

#define BOOST_ON_PERFECT_CLAMP 0
#define BOOST_ON_PERFECT_STOP  1

#define BOOST_SCHEDULE_AUTO (-1)

#define BOOST_FLAG_TIMING   1
#define BOOST_FLAG_NO_GRAPH 2

typedef struct {
    int32_t precision;
    int32_t on_perfect;
    double  eps_floor;
    int32_t schedule_id;
    int32_t flags;
    void   *stream;
} boost_options;

/* Fills *o with the defaults: FP32_WIDE, CLAMP, 1e-10, schedule 0, no flags,
 * NULL stream.  Returns BOOST_E_INVALID if o is NULL. */
int boost_options_default(boost_options *o);

/* ------------------------------------------------------------ stump record
 * One weak classifier, Section 2.2 / 2.3: h(x) = 1 iff p * f(x) < p * theta.
 * polarity p is +1 or -1; threshold theta is an integer that realises the
 * chosen split exactly.  split_rank k: the number of windows, in ascending
 * feature-value order, on the side below the threshold.  error_raw is the
 * minimum weighted error eps_t under the normalised weights; error is
 * max(error_raw, eps_floor); beta = error / (1 - error); alpha =
 * ln(1 / beta).  round is the 0-based round index.  Ties: smaller error, then
 * smaller feature index, then p = +1, then smaller split_rank. */
typedef struct {
    int64_t feature;
    int32_t type, x, y, cell_w, cell_h;
    int32_t polarity;
    int32_t threshold;
    int32_t split_rank;
    int32_t round;
    int32_t pad;
    double  error_raw;
    double  error;
    double  beta;
    double  alpha;
} boost_stump;

typedef struct boost_ctx boost_ctx;

/* ------------------------------------------------------------ host-only queries */

/* Number of features of a feature set (closed form of the Section 2.2
 * enumeration).  Returns -1 for an invalid set (window outside 1..32, empty or
 * out-of-range mask, NULL). */
int64_t boost_feature_count(const boost_feature_set *fs);

/* Descriptor of feature j (0 <= j < count) in the global order. */
int boost_feature_desc(const boost_feature_set *fs, int64_t j, boost_feature *out);

/* Device workspace bytes boost_init needs for n windows; 0 for invalid
 * arguments (n < 2, n > 32767, invalid feature set or options). */
size_t boost_workspace_bytes(int64_t n, const boost_feature_set *fs, const boost_options *o);

/* Number of launch schedules (schedule_id values 0 .. count-1) for a precision. */
int boost_schedule_count(int32_t precision);

/* Forgets every BOOST_SCHEDULE_AUTO choice cached in this process's memory
 * (a VJBOOST_TUNE_CACHE file is left as it is and read again on the next
 * miss). */
void boost_tune_cache_clear(void);

/* ------------------------------------------------------------ training
 * boost_init: ingest n windows and prepare every feature once (Section 3.3.1's
 * one-time "upload" of the feature values): copy labels and a positives-first
 * order, integral images (Section 2.1), the int32 value of every feature on
 * every window (Section 2.2) and, per feature, the windows in ascending value
 * order with the ends of runs of equal values marked.  Then the Table 2
 * initial weights 1/(2l) and 1/(2m), normalised.
 *   d_images  n x window_h x window_w uint8, row-major per window (device).
 *   d_labels  n uint8, 1 = positive (face), 0 = negative (device).
 *   d_workspace / workspace_bytes  caller-owned device memory of at least
 *             boost_workspace_bytes(n, fs, o) bytes; it must outlive the
 *             context.  Inputs may be freed once boost_init returns.
 * Errors: BOOST_E_INVALID for NULL pointers, n outside 2..32767, an invalid
 * feature set or options, a label other than 0/1, or a class with no
 * windows (1/(2l) or 1/(2m) undefined); BOOST_E_NOMEM if the workspace is too
 * small; BOOST_E_DEVICE on a HIP error.  Synchronises.  On success *out holds
 * a context owned by the library (free with boost_destroy). */
int boost_init(boost_ctx **out, const uint8_t *d_images, const uint8_t *d_labels, int64_t n,
               const boost_feature_set *fs, const boost_options *o,
               void *d_workspace, size_t workspace_bytes);

/* Incremental retraining: a new context over the union of c's windows (in
 * c's caller order) and m new ones (after them), as boost_init would prepare
 * it from the concatenated images and labels -- bit for bit the same
 * integral images, feature values, sorted keys and initial weights (Table 2
 * over the union), so training continues as from a fresh boost_init.  The
 * paper's case for a distributed trainer is fast retraining when the
 * training set changes (Abstract, Section 1.1).  The old windows' integral
 * images are copied.  For m <= 256 new windows and a union of 7,169 to
 * 15,360, the old windows' value order is reused: only the new windows are
 * put in order and merged into each feature's order.  Any other union is
 * sorted in full, which is faster there (the merge still evaluates every
 * window).
 *   c              a prepared context (not modified; it stays valid).
 *   d_images       m new windows, window_h x window_w uint8 row-major (device).
 *   d_labels       m labels 0/1 (device).
 *   d_workspace    caller-owned device memory of at least
 *                  boost_extend_workspace_bytes(c, m) bytes (that of
 *                  boost_workspace_bytes for n + m windows), distinct from c's.
 * The new context has c's feature set and options (precision, schedule
 * policy, stream, ...).  Errors as boost_init, and BOOST_E_INVALID for m < 1
 * or n + m > 32767.  Synchronises.
 * boost_extend_merged: 1 if the context's keys were merged from an extended
 * context's, 0 if they were sorted in full. */
size_t boost_extend_workspace_bytes(const boost_ctx *c, int64_t m);
int boost_extend(boost_ctx **out, const boost_ctx *c, const uint8_t *d_images, const uint8_t *d_labels,
                 int64_t m, void *d_workspace, size_t workspace_bytes);
int boost_extend_merged(const boost_ctx *c);

/* One boosting round (Section 2.3 steps 1-4; Section 3.3.2 master steps 1-4):
 * the normalised weights' best stump over all features and thresholds, its
 * beta and alpha, and the weight update w_i <- w_i beta^(1 - e_i) followed by
 * normalisation.
 *   out_host       NULL, or a host record that receives the stump (synchronises).
 *   d_feature_err  NULL, or device double[F][2] receiving each feature's
 *                  minimum error for p = +1 ([j][0]) and p = -1 ([j][1]).
 * Returns BOOST_E_DEGENERATE when the STOP policy has triggered (checked only
 * when the call synchronises). */
int boost_round(boost_ctx *c, boost_stump *out_host, double *d_feature_err);

/* rounds consecutive rounds; out_host (NULL or host array of rounds records)
 * receives every stump (synchronises).  Rounds are replayed from a captured
 * HIP graph unless BOOST_FLAG_NO_GRAPH or BOOST_FLAG_TIMING is set. */
int boost_train(boost_ctx *c, int32_t rounds, boost_stump *out_host);

/* Current normalised weights, device double[n], caller's sample order. */
int boost_get_weights(boost_ctx *c, double *d_w);

/* Replace the weights (device double[n], caller's order; finite, >= 0, not all
 * zero; normalised by the library).  Synchronises to validate;
 * BOOST_E_INVALID if the check fails (the previous weights are kept). */
int boost_set_weights(boost_ctx *c, const double *d_w);

/* Rounds completed so far. */
int boost_rounds_done(boost_ctx *c, int32_t *out_rounds);

/* Accumulated device time of the rounds run with BOOST_FLAG_TIMING:
 * out[0] scan-kernel ms, out[1] finalize-kernel ms, out[2] rounds timed,
 * out[3] scan launches timed.  Synchronises.  boost_reset_timing clears it. */
int boost_get_timing(boost_ctx *c, double out[4]);
int boost_reset_timing(boost_ctx *c);

/* Diagnostic: the memory-system ceiling of this context's scan.  Launches
 * reps + 1 times (the first untimed) a kernel that reads every key exactly as
 * the scan does (same grid, workgroup size, lane segments and load batches)
 * with no LDS gathers or sums, and returns in *best_ms the fastest launch
 * (HIP events on the context's stream; synchronises).  Key bytes (features x
 * windows x 2) over *best_ms is the bandwidth the scan would reach if its
 * arithmetic were free.  Weights and results are not changed.
 * BOOST_E_INVALID for a NULL context or output or reps < 1. */
int boost_probe_stream(boost_ctx *c, int32_t reps, double *best_ms);

/* Launch schedule in use (the tuner's choice under BOOST_SCHEDULE_AUTO).
 * ms_out NULL or host double[cap]: ms_out[k] = the fastest of the timed scan
 * launches of schedule k during tuning, -1 where schedule k was not timed
 * (not a candidate, a fixed schedule, or a choice taken from the cache).
 * Returns the schedule id, or BOOST_E_INVALID for a NULL context. */
int boost_get_schedule(const boost_ctx *c, double *ms_out, int32_t cap);

/* ------------------------------------------------------------ inspection (parity checks)
 * Values of features j0 .. j0+nf-1 on every window: device int32[nf][n],
 * caller's order (Section 2.2). */
int boost_get_feature_values(boost_ctx *c, int64_t j0, int64_t nf, int32_t *d_out);

/* Integral images, device int32[n][window_h+1][window_w+1], caller's order,
 * zero first row and column (Section 2.1). */
int boost_get_integral(boost_ctx *c, int32_t *d_out);

/* The per-feature value order built by boost_init: for features j0 ..
 * j0+nf-1, d_order int32[nf][n] = window index (caller's order) at each rank
 * of ascending value, d_run_end uint8[nf][n] = 1 where the value at that rank
 * differs from the next (or it is the last rank). */
int boost_get_sorted(boost_ctx *c, int64_t j0, int64_t nf, int32_t *d_order, uint8_t *d_run_end);

/* Strong classifier of Section 2.3: C(x) = 1 iff sum_t alpha_t h_t(x) >=
 * 1/2 sum_t alpha_t, for the context's training windows.
 *   stumps  host array of T records (only feature, polarity, threshold, alpha are read).
 *   d_out   device uint8[n] decisions; d_score NULL or device double[n] with
 *           sum_t alpha_t h_t(x) (caller's order). */
int boost_classify_train(boost_ctx *c, const boost_stump *stumps, int32_t T,
                         uint8_t *d_out, double *d_score);

/* Training-error curve of the Section 2.3 strong classifier: d_err_curve
 * (device int32[T]) receives, for t = 1..T, the number of the context's
 * training windows that the classifier built from the first t stumps
 * (C_t(x) = 1 iff sum_{u<=t} alpha_u h_u(x) >= 1/2 sum_{u<=t} alpha_u)
 * misclassifies, in one launch.  stumps as for boost_classify_train.
 * Synchronises.  BOOST_E_INVALID for NULL pointers, T outside 0..4096 or an
 * invalid record. */
int boost_classify_train_curve(boost_ctx *c, const boost_stump *stumps, int32_t T, int32_t *d_err_curve);

/* The Section 2.3 strong classifier on any windows (held-out or new ones),
 * with no training context: C(x) = 1 iff sum_t alpha_t h_t(x) >= 1/2 sum_t
 * alpha_t, h_t(x) = 1 iff p_t f_t(x) < p_t theta_t (Section 2.2), where f_t
 * is the Haar feature the record describes (type, x, y, cell_w, cell_h).
 *   d_images     n x window_h x window_w uint8, row-major per window (device).
 *   d_labels     NULL or device uint8[n] (1 = positive); needed for the curve.
 *   stumps       host array of T records (0 <= T <= 4096; type, x, y, cell_w,
 *                cell_h, polarity, threshold and alpha are read).
 *   d_out        NULL or device uint8[n]: decisions of the classifier of all T stumps.
 *   d_score      NULL or device double[n]: sum_t alpha_t h_t(x).
 *   d_err_curve  NULL or device int32[T]: for t = 1..T, the windows whose
 *                label differs from the decision of the first t stumps
 *                (a label other than 0 / 1 counts as an error).
 *   stream       hipStream_t (NULL: the legacy default stream).
 *   d_workspace  caller-owned device memory of at least
 *                boost_classify_workspace_bytes(n, window_w, window_h) bytes
 *                (the windows' integral images and the stump table).
 * Sums run in stump order in FP64, so each decision equals the definition
 * evaluated in that order.  Synchronises.  BOOST_E_INVALID for NULL images,
 * n < 1, a window outside 1..32, T outside 0..4096, a curve without labels,
 * or a record whose polarity is not +-1, whose alpha is not finite or whose
 * feature does not fit the window; BOOST_E_NOMEM for a short workspace. */
size_t boost_classify_workspace_bytes(int64_t n, int32_t window_w, int32_t window_h);
int boost_classify(const uint8_t *d_images, int64_t n, int32_t window_w, int32_t window_h,
                   const uint8_t *d_labels, const boost_stump *stumps, int32_t T,
                   uint8_t *d_out, double *d_score, int32_t *d_err_curve,
                   void *stream, void *d_workspace, size_t workspace_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * boost_classify with no workspace argument.  The integral images and the
 * stump table live in a 32 MiB device buffer of the library's own, a
 * file-scope array that each GPU the library runs on holds from the
 * library's load until the process ends; the call allocates nothing.
 * Arguments, results, errors and synchronisation as boost_classify; in
 * addition BOOST_E_INVALID when the windows do not fit the buffer
 * (boost_classify_noalloc_max_windows(window_w, window_h) per call: 13,248
 * windows of 24x24, 7,552 of 32x32; split larger sets).  Every call on a GPU
 * shares that GPU's buffer, which keeps the last call's contents: calls that
 * overlap on one GPU (two streams, two host threads) race, so serialise
 * them.
 * boost_classify_noalloc_max_windows: the largest n one call accepts for that
 * window size; 0 for a window outside 1..32. */
size_t boost_classify_noalloc_max_windows(int32_t window_w, int32_t window_h);
int boost_classify_noalloc(const uint8_t *d_images, int64_t n, int32_t window_w, int32_t window_h,
                           const uint8_t *d_labels, const boost_stump *stumps, int32_t T,
                           uint8_t *d_out, double *d_score, int32_t *d_err_curve, void *stream);

void boost_destroy(boost_ctx *c);

/* ------------------------------------------------------------ batched jobs
 * Many independent training jobs (each its own windows, labels and feature
 * set) advanced one round at a time: one persistent scan launch per key
 * format present (jobs of at most 16,383 windows use 14-bit keys, larger ones
 * 15-bit keys), whose workgroups take (job, feature range) segments from a
 * work queue, then one update launch for all jobs.  Each job's results equal
 * those of the same job run alone through boost_init/boost_round with the
 * same options. */
typedef struct {
    const uint8_t    *d_images;
    const uint8_t    *d_labels;
    int64_t           n;
    boost_feature_set fs;
} boost_job;

typedef struct boost_batch boost_batch;

/* Workspace for a batch; 0 for invalid arguments. */
size_t boost_batch_workspace_bytes(int32_t n_jobs, const boost_job *jobs, const boost_options *o);

/* As boost_init for every job (host array jobs[n_jobs], 1..4096 jobs). */
int boost_batch_init(boost_batch **out, int32_t n_jobs, const boost_job *jobs,
                     const boost_options *o, void *d_workspace, size_t workspace_bytes);

/* One round of every job; out_host NULL or host boost_stump[n_jobs]
 * (synchronises). */
int boost_batch_round(boost_batch *b, boost_stump *out_host);

/* rounds rounds of every job; out_host NULL or host boost_stump[rounds][n_jobs]. */
int boost_batch_train(boost_batch *b, int32_t rounds, boost_stump *out_host);

/* Weights of job k, device double[n_k], caller's order. */
int boost_batch_get_weights(boost_batch *b, int32_t job, double *d_w);

/* Schedule of the scan launch for key format key_format (0: 14-bit keys,
 * 1: 15-bit keys): *schedule = its schedule id, or -1 when no job of the
 * batch uses that format; *segs_per_wg (if not NULL) = work-queue segments
 * per workgroup (0 when absent).  BOOST_E_INVALID for a NULL batch or
 * schedule pointer or a format other than 0 and 1. */
int boost_batch_get_schedule(const boost_batch *b, int32_t key_format, int32_t *schedule, int32_t *segs_per_wg);

/* As boost_get_timing, summed over the batch's launches. */
int boost_batch_get_timing(boost_batch *b, double out[4]);

void boost_batch_destroy(boost_batch *b);

/* ------------------------------------------------------------ misc */
const char *boost_last_error(void);
int boost_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VJBOOST_H */
