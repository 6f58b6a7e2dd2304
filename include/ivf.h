/*
 * ivf.h - C ABI of the MI355X (gfx950) inverted-file spherical k-means library.
 *
 * The method is the inverted-file Lloyd iteration of Aoyama, Saito and Ikeda,
 * "Inverted-File k-Means Clustering: Performance Analysis" (Algorithm 3):
 *   assignment: every L2-normalised sparse object x_i is scored against all k
 *     sparse unit-norm means by walking the term-major inverted file of the
 *     means (term t -> ascending list of (cluster j, mean value m_jt)),
 *     rho_j += x_it * m_jt; the object joins the argmax cluster (rho_max starts
 *     at 0, strict ">", ascending j: the lowest j wins exact ties; an object
 *     sharing no term with any mean keeps its previous cluster);
 *   update: every mean is the member sum divided by |C_j| and then by its
 *     2-norm; the inverted file is rebuilt from the new means with every list
 *     in ascending cluster order.
 * The problem statement (object set, k, initial state, iterations) follows the
 * paper's Section "Lloyd-Type k-Means Clustering Algorithm".
 *
 * Conventions shared by every entry point
 *  - Pointers marked "device" are HIP device pointers; all work is enqueued
 *    on ivf_options.stream.  Entry points that fill an ivf_stats synchronise
 *    that stream before returning.
 *  - Ownership: the caller owns every buffer it passes.  The object set given
 *    to ivf_build is BORROWED: it must stay alive and unchanged until
 *    ivf_destroy.  The handle owns the means, the inverted file and scratch.
 *  - Ids are 0-based; an assignment of -1 means "unassigned" (the object has
 *    not yet shared a term with any mean).
 *  - Errors: every call returns an ivf_status; nothing throws across the ABI.
 *    Argument checks happen before any launch; ivf_last_error(h) gives text.
 *  - Concurrency: one handle must not be used from two host threads at once.
 */
#ifndef IVF_H
#define IVF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ivf_handle ivf_handle;

typedef enum {
    IVF_OK = 0,
    IVF_ERR_ARG = -1,        /* bad sizes, null pointers, k out of [1, n] */
    IVF_ERR_UNSORTED = -2,   /* term ids not strictly ascending in a row, or out of [0, d) */
    IVF_ERR_NONFINITE = -3,  /* NaN or infinite value */
    IVF_ERR_NEGATIVE = -4,   /* a value <= 0 (stored nonzeros must be positive) */
    IVF_ERR_CAPACITY = -5,   /* sizes beyond the library's limits (nnz >= 2^31, ...) */
    IVF_ERR_OOM = -6,        /* device allocation failed */
    IVF_ERR_HIP = -7,        /* a HIP runtime call failed (text in ivf_last_error) */
    IVF_ERR_STATE = -8       /* call order: e.g. ivf_assign before any means exist */
} ivf_status;

/* Precision of the mean values stored in the inverted file used by the
 * assignment walk.  Scores are always accumulated in FP32 (a rounded product
 * then a rounded sum for FP32 values, one fused multiply-add for 16-bit ones;
 * the stated bound covers both); objects whose top-1/top-2 margin is inside
 * that error bound are re-scored in FP64. */
typedef enum { IVF_VAL_F32 = 0, IVF_VAL_BF16 = 1, IVF_VAL_F16 = 2 } ivf_valtype;

/* Object set, CSR (the paper's sparse expression of Fig. "fig:str"(a)).
 * indptr[n+1] (int64, indptr[0] == 0, non-decreasing, indptr[n] == nnz),
 * indices[nnz] (int32, strictly ascending within a row, in [0, d)),
 * values[nnz] (float32, finite, > 0).  All device pointers. */
typedef struct {
    int64_t n;
    int64_t d;
    int64_t nnz;
    const int64_t* indptr;
    const int32_t* indices;
    const float* values;
} ivf_csr;

/* k means, mean-major CSR in FP64: row j lists (term, value) of mean j with
 * strictly ascending terms.  All device pointers.  For ivf_get_means the
 * caller allocates indptr[k+1], indices[nnz], values[nnz]. */
typedef struct {
    int32_t k;
    int64_t d;
    int64_t nnz;
    int64_t* indptr;
    int32_t* indices;
    double* values;
} ivf_means;

typedef struct {
    int32_t valtype;        /* ivf_valtype of the inverted-file values */
    int32_t certify;        /* 1: certify every argmax, re-score uncertified objects in
                               FP64 (assignments equal the FP64 reference); 0: take the
                               FP32 argmax as is (for timing studies only) */
    int32_t cluster_range;  /* clusters per range (one score tile per wave: FP32 values in
                               ranges of at most 1,024 clusters keep it in registers, other
                               ranges in LDS); 0: planner's choice (1,024 for FP32 values,
                               1,280 for 16-bit ones) */
    int32_t waves_per_wg;   /* waves (each owning one tile) per workgroup; 0: planner */
    int32_t objects_per_item; /* objects per work-queue item; 0: planner */
    int32_t force_rescore;  /* test hook: 1 = treat every object as uncertified */
    float dense_threshold;  /* a (term, range) slice holding at least this fraction of the
                               range's clusters is stored as a dense slab (zeros for absent
                               clusters, no ids); 0: default, 0.45 for FP32 values in ranges
                               of at most 1,024 clusters (the register walk), else 0.35;
                               > 1: never dense */
    void* stream;           /* hipStream_t; NULL = the null stream */
    int32_t full_update;    /* 1: every ivf_update runs the full reduction over all object
                               entries; 0 (default): when few objects changed cluster since
                               the previous update, only their entries are reduced and merged
                               into the stored exact member sums (same result bit for bit) */
} ivf_options;

/* Fills *o with the defaults (F32, certify on, planner's choices, null stream). */
void ivf_default_options(ivf_options* o);

typedef struct {
    /* assignment step */
    double objective;        /* sum_i rho_{i,a_i}: certified objects contribute their
                                FP32 score, re-scored ones their FP64 score */
    double objective_bound;  /* relative error bound of `objective` w.r.t. the FP64
                                objective (largest per-object bound used) */
    int64_t changed;         /* objects whose cluster changed */
    int64_t certified;       /* objects whose FP32 argmax was certified by the bound */
    int64_t rescored;        /* objects re-scored in FP64 */
    int64_t zero_overlap;    /* objects sharing no term with any mean */
    int64_t mult_adds;       /* M = sum_i sum_h (nc)_{t(i,h)} (the paper's Eq. ivf_mult) */
    double max_rel_err_rescored; /* max |rho~ - rho64| / rho64 of the FP32 winner, over the
                                objects re-scored in FP64 (certified objects are not
                                scored in FP64, so they do not enter it) */
    float assign_ms;         /* device time of the assignment step */
    float walk_ms;           /* device time of its inverted-file walk kernel alone */
    /* update step */
    double objective_exact;  /* sum_j mu_j(old) . s_j(new member sum), FP64: the same J
                                as `objective` computed from the update's exact sums */
    int64_t empty_clusters;  /* clusters without members (their means are kept) */
    int64_t nnz_means;       /* sum_j (ntm)_j after the call */
    int64_t inexact_terms;   /* terms whose fixed-point member sums were rounded */
    float update_ms;         /* device time of the update step */
    int64_t update_delta_entries; /* the update was incremental: object entries of the
                                objects that changed cluster, reduced and merged into the
                                stored sums; -1: the full reduction ran */
} ivf_stats;

/*
 * ivf_build: validate the object set, derive its term-major view and plan the
 * launch shapes.  No means exist yet: call ivf_set_means or ivf_init_seeds.
 * This is the problem statement of the paper's Section "Lloyd-Type k-Means
 * Clustering Algorithm" (an object set X of N points in D dimensions and a
 * positive integer k); the initial state is given separately, as the method
 * starts from a given initial state (Section "Proposed algorithm: IVF": IVF
 * keeps the standard Lloyd solution under an identical initial state).  The
 * caller gives k here and the initial means later (ivf_set_means, or
 * ivf_init_seeds for k seed objects), so one validated object set can be
 * clustered from several initial states.
 *   X     object set (device pointers, borrowed, see ivf_csr)
 *   k     number of clusters, 1 <= k <= n, k < 2^24
 *   opts  NULL for defaults
 *   out   receives the handle (NULL on failure)
 * Errors: IVF_ERR_ARG, IVF_ERR_UNSORTED, IVF_ERR_NONFINITE, IVF_ERR_NEGATIVE,
 * IVF_ERR_CAPACITY, IVF_ERR_OOM, IVF_ERR_HIP.  Synchronises the stream.
 */
ivf_status ivf_build(const ivf_csr* X, int32_t k, const ivf_options* opts, ivf_handle** out);

/*
 * ivf_set_means: replace the means with caller-given FP64 means (mean-major,
 * device pointers; copied) and rebuild the inverted file (Alg. 3's M-breve).
 * M->k must equal the handle's k and M->d its d.  Rows must hold strictly
 * ascending terms in [0, d) and finite values.  Synchronises the stream.
 */
ivf_status ivf_set_means(ivf_handle* h, const ivf_means* M);

/*
 * ivf_init_seeds: initial state from k seed objects: mean j is object
 * seeds[j] (device int32 [k], each in [0, n)) renormalised in FP64, i.e. the
 * update step applied to the partition {seeds[j]} -> j.  Synchronises.
 */
ivf_status ivf_init_seeds(ivf_handle* h, const int32_t* seeds);

/*
 * ivf_assign: one assignment step (Alg. 3, assignment part) under the current
 * means.  assign (device int32 [n]) holds the previous assignment on entry
 * (-1 = unassigned) and the new one on return.  stats may be NULL (then the
 * call does not synchronise); when given, its assignment fields are filled.
 */
ivf_status ivf_assign(ivf_handle* h, int32_t* assign, ivf_stats* stats);

/*
 * ivf_assign_static: ivf_assign for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  The same step with the same results, bit for bit; its
 * per-call scratch (the previous assignment, the FP64 re-score queue and the
 * walk's per-(object, cluster range) records: n * (16 * ranges + 8) bytes,
 * each part rounded up to 256 bytes) lives in a fixed 64 MiB array the library
 * holds on every GPU it runs on until the process ends, instead of in the
 * handle's buffers.  Calls no allocating routine.
 *   h, assign, stats  as for ivf_assign; the handle's device must be current.
 * Errors: as ivf_assign; IVF_ERR_CAPACITY (nothing launched) when the step
 * needs more than the 64 MiB; IVF_ERR_STATE when another device is current.
 * Every call on one GPU shares that GPU's array and leaves its contents there:
 * calls that overlap on one GPU (any handles, any streams, without stats so
 * that they do not synchronise) race; order them, e.g. on one stream.
 */
ivf_status ivf_assign_static(ivf_handle* h, int32_t* assign, ivf_stats* stats);

/*
 * ivf_update: one update step (Alg. 3, update part) from the assignment
 * (device int32 [n], -1 entries ignored): exact member sums, FP64 norms and
 * renormalisation, clusters without members keep their mean, then the
 * inverted-file rebuild.  stats may be NULL; the update fields are filled when
 * given.  Synchronises the stream (the new means' size sets later launches).
 */
ivf_status ivf_update(ivf_handle* h, const int32_t* assign, ivf_stats* stats);

/*
 * ivf_iterate: `iters` Lloyd iterations (assignment then update), the
 * two-step repetition of the paper's Section "Lloyd-Type k-Means Clustering
 * Algorithm" run to a predetermined termination condition (a fixed count);
 * each iteration is Algorithm 3 at iteration r.  assign as in ivf_assign.
 * per_iter (host, [iters]) may be NULL; it receives each iteration's
 * assignment and update fields.  Synchronises (as ivf_update does).
 */
ivf_status ivf_iterate(ivf_handle* h, int32_t iters, int32_t* assign, ivf_stats* per_iter);

/*
 * ivf_converge: Lloyd iterations until an assignment step changes no object's
 * cluster (the partition, and hence the means, are then a fixed point of the
 * iteration), or max_iters assignment steps.  This is the "until the
 * convergence" of the paper's Section "Lloyd-Type k-Means Clustering
 * Algorithm", which leaves convergence undefined; here it means no change of
 * cluster.  The converged step's update is
 * skipped: it would return the same means.  assign as in ivf_assign;
 * per_iter (host, [max_iters]) may be NULL; *iters_done receives the number
 * of assignment steps run (the last has changed == 0 unless max_iters was
 * reached).  Synchronises.
 */
ivf_status ivf_converge(ivf_handle* h, int32_t max_iters, int32_t* assign, ivf_stats* per_iter,
                        int32_t* iters_done);

/*
 * ivf_assign_ivfd: the assignment step of IVFD (the paper's Algorithm 4,
 * Section "IVFD and IVF"): the OBJECTS are inverted and every mean, in
 * ascending j, is a query whose scores for all objects are compared with each
 * object's running maximum (strict ">" from 0, so the lowest j wins ties; an
 * object sharing no term with any mean keeps its cluster).  It computes the
 * same partition as ivf_assign (the two differ only in loop order) and is
 * provided to measure which side is better inverted on this hardware.
 *   objects_per_range  objects per LDS score tile: 4096, 8192 or 16384
 *                      (0: 16384).  The objects' inverted file, range-major,
 *                      is built on the first call (and again when this
 *                      changes) and kept with the object set: nnz * 8 bytes
 *                      plus (ranges * d + 1) * 4 bytes of device memory.
 *   assign, stats      as for ivf_assign.  stats->mult_adds is the number of
 *                      inverted-file entries the IVFD walk met, which equals
 *                      M (the paper notes the two algorithms multiply equally
 *                      often).  walk_ms times the IVFD walk kernel.
 * Scores are summed in fixed point (each FP32 product scaled by 2^F and
 * rounded to an integer, F set from the largest object and mean norms so
 * that no sum overflows 32 bits), certified with a bound for that rounding,
 * and uncertified objects re-scored in FP64 as in ivf_assign (the re-score
 * reads the means' inverted file the handle keeps).  Synchronises once to
 * read the means' largest norm.  Requires an FP32 handle (IVF_ERR_ARG otherwise), not a
 * batch member (IVF_ERR_STATE), ranges x d < 2^32 (IVF_ERR_CAPACITY).
 */
ivf_status ivf_assign_ivfd(ivf_handle* h, int32_t objects_per_range, int32_t* assign,
                           ivf_stats* stats);

/*
 * ivf_get_means: two-call copy of the current means: the content of the
 * inverted mean file M-breve that Algorithm 3 returns (Section "Proposed
 * algorithm: IVF"), given mean-major in FP64 (per cluster j its ascending
 * (term p, u_p = w_p / ||w||) entries) rather than term-major.  With
 * out->indptr NULL only out->k, out->d and out->nnz are filled; otherwise the caller's device
 * buffers (indptr[k+1], indices[nnz], values[nnz], nnz from the first call)
 * receive the mean-major FP64 means.  Synchronises.
 */
ivf_status ivf_get_means(ivf_handle* h, ivf_means* out);

/*
 * ivf_get_scores: per-object results of the last ivf_assign (device outputs,
 * any may be NULL): best[n] FP32 top-1 score of the tile walk, best_id[n] its
 * cluster (-1 if no term is shared), second[n] FP32 best score of any other
 * cluster, rho[n] the score used for the objective (FP64; the FP64 re-score
 * where one was made), flags[n] (bit 0: certified, bit 1: re-scored in FP64,
 * bit 2: no shared term).  Synchronises.
 */
ivf_status ivf_get_scores(ivf_handle* h, float* best, int32_t* best_id, float* second,
                          double* rho, uint8_t* flags);

/*
 * ivf_get_plan: the launch plan chosen by ivf_build: plan[0] clusters per
 * range (k_r), plan[1] number of ranges, plan[2] waves per workgroup,
 * plan[3] objects per work item, plan[4] and plan[5] clusters per range and
 * ranges of the FP64 re-score's FP32 candidate walk (the walk's own),
 * plan[6] LDS bytes per workgroup.
 */
ivf_status ivf_get_plan(const ivf_handle* h, int32_t plan[7]);

/*
 * ivf_plan_shape: the planner alone (host only, no GPU needed): for k
 * clusters and the given options, fills plan[7] as ivf_get_plan would.
 * Returns IVF_ERR_ARG for k < 1 or requests beyond the LDS budget.
 */
ivf_status ivf_plan_shape(int32_t k, const ivf_options* opts, int32_t plan[7]);

/*
 * ivf_cert_bound: the certification constants for an object of `nt`
 * nonzeros, the given value type and objects whose values are all <= vmax
 * (host only).  The bound is the recursive-summation error bound of a sum of
 * non-negative products (the FP64 reference's own rounding is c[2]).
 *   c[0] relative bound of an FP32 tile score against the exact score:
 *        ((1 + u_s)(1 + gamma_nt) - 1) * 1.01 + 1e-15, with u_s the unit
 *        roundoff of the stored mean value (FP32 2^-24; BF16 and FP16 their
 *        own plus the FP32 step) and gamma_nt = nt 2^-24 / (1 - nt 2^-24);
 *   c[1] absolute term for results below the normal range:
 *        nt (vmax eta_m + 2 eta) (1 + gamma_nt) * 1.01, eta = 2^-126 (one FP32
 *        rounding of a tiny result, kept subnormal or flushed), eta_m = eta for
 *        FP32 and BF16 values, 2^-25 + eta for FP16 values (FP16 subnormals);
 *   c[2] relative bound of the FP64 reference's rounding (gamma_nt in FP64).
 * The test certifying cluster a over every other cluster b is
 *   (s_a - c[1]) (1 - c[2]) / (1 + c[0])  >  (s_b + c[1]) (1 + c[2]) / (1 - c[0]).
 * The library uses vmax = the largest value of the handle's object set.
 * IVF_ERR_ARG for an unknown valtype, nt < 0 or vmax not finite and >= 0.
 */
ivf_status ivf_cert_bound(int32_t valtype, int64_t nt, double vmax, double c[3]);

/*
 * ivf_cert_bound_fixed: the same constants for the fixed-point scores of
 * ivf_assign_ivfd (host only): each FP32 product of the FP32-rounded mean
 * value and the object value, times `scale` (a power of two), rounded to the
 * nearest integer; the integers summed exactly; the sum converted to FP32 and
 * divided by scale.  c[0] = ((1 + 2^-24)^3 - 1) * 1.01 + 1e-15, c[1] =
 * nt * (1/(2 scale) + (vmax + 1) 2^-126) * (1 + 2^-24) * 1.01, c[2] as above.
 * IVF_ERR_ARG for nt < 0, a scale that is not a positive finite number, or
 * vmax not finite and >= 0.
 */
ivf_status ivf_cert_bound_fixed(int64_t nt, double scale, double vmax, double c[3]);

/*
 * ivf_read_ceiling: a measurement utility, not a step of the method: the
 * read bandwidth of a plain 16-byte-per-lane streaming read kernel over the
 * caller's device buffer `buf` of `bytes` bytes (>= 16 KiB; its contents are
 * irrelevant), the roof against which the assignment walk's cache and memory
 * traffic is placed.  mode 0: every workgroup reads the whole buffer (a few
 * MB stay resident in each L2); mode 1: the workgroups split the buffer and
 * sweep it `passes` times (a buffer between the L2s' and the Infinity
 * Cache's sizes is served by the latter, GBs by HBM).  unroll (4, 8 or 16)
 * loads per lane are in flight before any is used; wgs_per_cu (1 .. 32)
 * workgroups of 256 threads per compute unit.  One untimed launch warms the
 * caches, one launch is timed with HIP events on `stream` (hipStream_t, NULL
 * = null stream); *gbps receives bytes read / time in GB/s.  Allocates and
 * frees a small sink buffer; synchronises the stream.  IVF_ERR_ARG for bad
 * arguments, IVF_ERR_HIP / IVF_ERR_OOM on HIP failures.
 */
ivf_status ivf_read_ceiling(const void* buf, int64_t bytes, int32_t mode, int32_t passes,
                            int32_t unroll, int32_t wgs_per_cu, void* stream, double* gbps);

/* Frees the handle and everything it owns (NULL is a no-op). */
void ivf_destroy(ivf_handle* h);

/* Text of the last error on h (or of the last ivf_build failure if h is NULL). */
const char* ivf_last_error(const ivf_handle* h);

/* Static name of a status code. */
const char* ivf_status_str(int32_t status);

/* ------------------------------------------------------------------ batches
 * Many independent clustering instances (different object sets, k, or seeds
 * of one set: restarts) advanced together.  Every iteration walks ALL
 * instances in one persistent launch of the assignment kernel (work items of
 * every instance in one queue, one LDS tile width for all), then runs each
 * instance's merge, FP64 re-score and update.  Each instance computes exactly
 * what a single handle of the same options computes (Alg. 3 per instance):
 * assignments and means are bit-identical to one ivf_handle per instance.
 *
 * Execution: the first two iterations run eagerly and size every buffer;
 * then capacities are fixed (1.5x what was needed) and one iteration of the
 * whole batch is recorded as a HIP graph (two graphs: the means' double
 * buffer alternates) and replayed.  A replay whose new means would exceed a
 * fixed capacity is detected from device flags after the replay, that
 * instance's update is redone eagerly with larger buffers and the graphs are
 * recorded again, so results never depend on the capacities.
 * Tiles: with opts->cluster_range == 0 an autotuner times the batched walk
 * over a few (clusters per tile, waves per workgroup) shapes on the means of
 * the second iteration and keeps the fastest; otherwise the given shape is used.
 * The shapes are timed at each instance's default dense-slab threshold.  When
 * the tuner runs and opts->dense_threshold is 0, it then times the thresholds
 * 0.35, 0.45, 0.5 and 0.65 on the chosen shape and keeps the fastest.
 * After the walk, the instances' merges and updates run on 4 streams the
 * batch creates (default priority), forked from and joined back into the
 * batch stream within every iteration, so work the caller enqueues on the
 * batch stream after a call is ordered after all of it.
 */
typedef struct ivf_batch ivf_batch;

/*
 * ivf_batch_build: count instances; X[i] (host array of count ivf_csr, device
 * pointers inside, borrowed until ivf_batch_destroy) and k[i] (host int32).
 * Instances whose X[i] names the same device arrays share one term-major view.
 * opts applies to every instance (NULL: defaults); opts->stream NULL makes the
 * batch create a stream of its own (graph capture cannot use the null stream).
 * Errors as ivf_build; text from ivf_batch_last_error(NULL).
 */
ivf_status ivf_batch_build(int32_t count, const ivf_csr* X, const int32_t* k,
                           const ivf_options* opts, ivf_batch** out);

/* Seeds of every instance: seeds[i] is a device int32 [k[i]] array (host
 * array of count pointers).  As ivf_init_seeds per instance.  Synchronises. */
ivf_status ivf_batch_init_seeds(ivf_batch* b, const int32_t* const* seeds);

/* Caller-given means of instance `inst` (as ivf_set_means).  Only before the
 * first ivf_batch_iterate; all instances need means before iterating. */
ivf_status ivf_batch_set_means(ivf_batch* b, int32_t inst, const ivf_means* M);

/*
 * ivf_batch_iterate: `iters` Lloyd iterations of every instance.  assign is a
 * host array of count device pointers, assign[i] int32 [n_i] (previous
 * assignment in, new one out, -1 = unassigned); the same pointers should be
 * passed on every call (new pointers force the graphs to be recorded again).
 * stats (host, [iters * count], iteration-major) may be NULL; when given, each
 * entry holds that instance's assignment and update fields, assign_ms the
 * device time of the whole batch iteration and walk_ms that of its one walk
 * launch, read from the device real-time clock just before and after it
 * (both the same for every instance).  Synchronises before returning.
 */
ivf_status ivf_batch_iterate(ivf_batch* b, int32_t iters, int32_t* const* assign,
                             ivf_stats* stats);

/* Means of instance `inst`, two-call form as ivf_get_means.  Synchronises. */
ivf_status ivf_batch_get_means(ivf_batch* b, int32_t inst, ivf_means* out);

/*
 * ivf_batch_set_slack: the fixed capacities become need * (1 + frac) + abs
 * entries (defaults 0.5 and 1024), need being what the eager iterations used.
 * Less slack saves memory across many instances at the price of more graph
 * re-recordings after overflows; results do not depend on it.  0 <= frac <= 64,
 * abs >= 0, else IVF_ERR_ARG.
 */
ivf_status ivf_batch_set_slack(ivf_batch* b, double frac, int64_t abs_entries);

/*
 * ivf_batch_get_plan: plan[0] clusters-per-tile limit, plan[1] waves per
 * workgroup, plan[2] floats per tile (the widest range of any instance),
 * plan[3] workgroups of the persistent walk, plan[4] 1 once the iteration is
 * recorded as graphs, plan[5] 1 once the autotuner has run, plan[6] times the
 * iteration was recorded, plan[7] replays redone after a capacity overflow.
 */
ivf_status ivf_batch_get_plan(const ivf_batch* b, int32_t plan[8]);

/*
 * ivf_batch_get_tuning: what the autotuner measured (host outputs).  *count
 * receives the number of candidates timed (0 before it ran or when the tile
 * shape was given); the first min(cap, *count) entries are written:
 * shapes[2i], shapes[2i+1] = clusters per tile, waves per workgroup, and
 * ms[i] = the batched walk's device time with that shape.
 */
ivf_status ivf_batch_get_tuning(const ivf_batch* b, int32_t cap, int32_t* shapes, float* ms,
                                int32_t* count);

/*
 * ivf_batch_get_threshold_tuning: the dense-slab thresholds the autotuner
 * timed on its chosen shape (host outputs), as ivf_batch_get_tuning: *count
 * receives how many (0 before it ran, when the shape was given or when
 * opts->dense_threshold was set), thetas[i] the threshold, ms[i] the batched
 * walk's device time with it, in the order timed (0.35, 0.45, 0.5, 0.65).
 */
ivf_status ivf_batch_get_threshold_tuning(const ivf_batch* b, int32_t cap, float* thetas,
                                          float* ms, int32_t* count);

/* Frees the batch, its instances and its stream if it created one. */
void ivf_batch_destroy(ivf_batch* b);

/* Text of the last error on b (or of the last ivf_batch_build failure if b is NULL). */
const char* ivf_batch_last_error(const ivf_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* IVF_H */
