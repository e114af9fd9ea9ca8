/*
 * leafi.h -- C ABI of the MI355X (gfx950) LeaFi search library.
 *
 * LeaFi (Wang, Ileana, Palpanas, SIGMOD 2025) speeds up exact tree-based
 * data-series k-NN search by placing small learned models ("filters") in leaf
 * nodes.  A filter predicts the node-wise nearest-neighbour distance d^L of a
 * query; after a conformal offset is subtracted the prediction acts as an
 * extra lower bound that prunes leaves the summaries cannot prune.
 *
 * Conventions shared by every entry point:
 *   - Return value: LEAFI_OK (0) or a negative LEAFI_E* code.  The message of
 *     the last failure on the calling thread is available from
 *     leafi_last_error().  No C++ exception crosses this boundary.  On error
 *     no output buffer is guaranteed to have been written.
 *   - Pointers named *_dev are device pointers (HIP global memory on the
 *     current device); pointers named *_host are host memory.  The caller owns
 *     every buffer it passes; the library never frees or keeps them.  Input
 *     buffers are only read.  The library owns the index handle and all
 *     resident device memory it allocates (leaf store, filters, tables); it
 *     is released by leafi_destroy().
 *   - `stream` is a hipStream_t (NULL = the default stream).  Kernels are
 *     enqueued on it; calls return once their results are on the device
 *     (they may synchronise the stream to read small control values).
 *   - Matrices are row-major.  Series and queries are raw fp32; the library
 *     z-normalises them itself (mean and population standard deviation in
 *     FP64; a series whose deviation is below 1e-8 becomes all zeros).
 *   - Distances are Euclidean distances between z-normalised series (not
 *     squared).  Result rows are sorted by (distance, id) ascending; ids are
 *     row indices of the series array given to leafi_build_index.
 *   - One index handle must not be used by two threads at the same time.
 */
#ifndef LEAFI_H
#define LEAFI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LEAFI_OK 0
#define LEAFI_EINVAL (-1)   /* invalid argument (shape, range, null pointer) */
#define LEAFI_ENOMEM (-2)   /* device or host allocation failed */
#define LEAFI_ESTATE (-3)   /* call out of order (e.g. search before build) */
#define LEAFI_EHIP (-4)     /* a HIP runtime call failed */
#define LEAFI_EAGAIN (-5)   /* serving: request not admitted now, retry later */
#define LEAFI_EINTERNAL (-6)

typedef struct leafi_index leafi_index;

/* ------------------------------------------------------------------------
 * Handle management
 * ---------------------------------------------------------------------- */

/* Device memory allocator supplied by the caller (e.g. a framework's caching
 * allocator).  alloc stores a device pointer of at least `bytes` bytes (256-
 * byte aligned) in *dptr and returns 0, or returns nonzero when it cannot;
 * free releases a pointer alloc returned.  The library calls free only after
 * every piece of work it queued on the device has finished (it synchronises
 * the device first), so a pool may hand the block out again at once. */
typedef int (*leafi_alloc_fn)(void *ctx, size_t bytes, void **dptr);
typedef void (*leafi_free_fn)(void *ctx, void *dptr);

/*
 * Create an empty index handle bound to the current HIP device.  Every
 * device allocation the handle makes (leaf store, filters, calibration
 * tables, search workspace, serving state) goes through alloc / free with
 * `alloc_ctx`, which must stay valid until leafi_destroy returns; with both
 * NULL the library uses hipMalloc / hipFree.  Giving only one of them is
 * LEAFI_EINVAL.  A refused allocation makes the call that needed it return
 * LEAFI_ENOMEM; the handle stays valid (an index build that failed leaves it
 * unbuilt).
 */
int leafi_create(leafi_alloc_fn alloc, leafi_free_fn free_fn, void *alloc_ctx, leafi_index **out);

/* Release the handle and every device allocation it owns.  NULL is a no-op. */
void leafi_destroy(leafi_index *index);

/* Message of the last failure on this thread ("" if none).  The pointer stays
 * valid until the next failing call on the same thread. */
const char *leafi_last_error(void);

/* Library version string. */
const char *leafi_version(void);

/* ------------------------------------------------------------------------
 * Index building (paper: Section "Preliminaries", tree-based indexes; the
 * DSTree backbone of Section "Evaluation Setup")
 * ---------------------------------------------------------------------- */

typedef struct {
  int32_t leaf_capacity; /* split nodes holding more series than this (>= 1) */
  int32_t n_segments;    /* S: equal segments of the node summaries, 1..64, <= m */
  int32_t split_rule;    /* 0 = median split, 1 = midpoint of the range, 2 = iSAX (the MESSI
                            backbone; n_segments <= 32) */
  int32_t reserved;
} leafi_build_opts;

/*
 * Build the index over n raw fp32 series of length m (series_dev [n, m]).
 * Steps: z-normalisation, per-segment mean/std summaries, a tree split until
 * every leaf holds <= leaf_capacity series, then a device-resident leaf
 * store: the normalised series grouped leaf by leaf in fp32 and in a bf16
 * copy, with per-leaf summaries.  Split rules 0 and 1 (DSTree-style binary
 * tree): a node splits on the segment statistic with the largest
 * seg_len * range^2, at the median or the range midpoint; summaries are per
 * segment the min/max of the members' mean and std.  Split rule 2 (iSAX, the
 * MESSI backbone of Section "Evaluation Setup"): each segment mean becomes a
 * SAX symbol of up to 8 bits (breakpoints at the N(0, 1) quantiles j / 256);
 * the root's children are the words of one bit per segment, and a node over
 * capacity takes the next bit of the segment that divides its members most
 * evenly (a node whose members agree in all 8 bits of every segment stays
 * whole); summaries are each leaf's SAX intervals (the lower bound is then
 * MINDIST(PAA(q), iSAX word)).  Any previous
 * index, filters and calibration in the handle are discarded.
 * Limits: 1 <= n < 2^31; at most 16384 leaves; 32 <= m <= 512, m a
 * multiple of 32.  The BF16 scan needs m <= 256, the FP32 scan m <= 256 or
 * m in {384, 512}; a search with a scan that does not support m fails with
 * LEAFI_EINVAL.
 */
int leafi_build_index(leafi_index *index, const float *series_dev, int64_t n, int32_t m,
                      const leafi_build_opts *opts, void *stream);

typedef struct {
  int64_t n_series;
  int32_t m;
  int32_t n_leaves;
  int32_t n_segments;
  int32_t n_filters;   /* 0 until filters are trained or set */
  int32_t hidden;      /* filter hidden width h (MLP) or channel count (CNN) */
  int32_t n_calibrated;/* number of calibrated (k, target) pairs */
  int64_t padded_rows; /* rows of the leaf store including per-leaf padding */
  int64_t device_bytes;/* resident device memory owned by the handle */
  int32_t filter_arch; /* LEAFI_FILTER_MLP or LEAFI_FILTER_CNN */
  int32_t reserved;
} leafi_info;

int leafi_get_info(const leafi_index *index, leafi_info *out);

/* Leaf partition: leaf_offsets_host [n_leaves + 1] (prefix sums of the leaf
 * sizes) and member_ids_host [n_series] (ids of each leaf's members, leaf by
 * leaf, ascending within a leaf).  Leaves are numbered depth-first, left child
 * first.  Either pointer may be NULL. */
int leafi_export_leaves(const leafi_index *index, int64_t *leaf_offsets_host, int64_t *member_ids_host);

/* Leaf summaries: boxes_host [n_leaves, n_segments, 4] = (mean lo, mean hi,
 * std lo, std hi) per segment, widened outward by one fp32 ulp. */
int leafi_export_boxes(const leafi_index *index, float *boxes_host);

/* ------------------------------------------------------------------------
 * Learned filters (paper: Section "The LeaFi Framework", Algorithms 1 and 3,
 * Section "Training Data Generation", Section "Evaluation Setup")
 * ---------------------------------------------------------------------- */

typedef struct {
  int32_t n_global;      /* global training queries, incl. validation (paper: 3/4 of 2,000) */
  int32_t n_local;       /* local training queries per filtered leaf (paper: 1/4 of 2,000) */
  float noise_lo;        /* training noise level range: each query draws its */
  float noise_hi;        /*   level uniformly in [noise_lo, noise_hi] */
  float a;               /* Algorithm 3 hyperparameter a = 1 / p^F (paper: 2) */
  float val_fraction;    /* share of the global queries held out for validation (0.2) */
  double th_override;    /* < 0: th = a * t^F / t^S measured on this GPU; >= 0: use as th */
  int64_t mem_budget;    /* c^M: device bytes available for filter weights */
  int32_t hidden;        /* h (MLP) or channels (CNN); 0 = m (paper: width = series length) */
  int32_t max_epochs;    /* paper: 1,000 */
  float lr0;             /* paper: 0.01 */
  float lr_min;          /* paper: 1e-5 (training stops below it) */
  int32_t batch;         /* SGD mini-batch size */
  int32_t patience;      /* epochs without validation improvement before lr /= 10 */
  uint64_t seed;
  int32_t keep_examples; /* 1: keep the training queries and targets for leafi_get_examples */
  int32_t selection;     /* LEAFI_SELECT_SIZE (Algorithm 3) or LEAFI_SELECT_KNAPSACK (Equations 1-2) */
  int32_t arch;          /* LEAFI_FILTER_MLP (default) or LEAFI_FILTER_CNN */
  int32_t reserved;
} leafi_train_opts;

/* Filter architectures (paper: Section "Evaluation Setup" for the MLP,
 * Section "Varying Model Type" for the CNN).
 * MLP: d^f(q) = w2 . ReLU(W1 q + b1) + b2, hidden width h; packed as
 *   [W1 (input-major: element (i, j) at i*h + j) | b1 (h) | w2 (h) | b2],
 *   P = h*m + 2h + 1 floats.
 * CNN: two cross-correlations of kernel 3 over the series positions with one
 *   zero of padding at each end (tap t reads position p + t - 1), 1 -> C then
 *   C -> C channels, ReLU after each, the second layer's channels averaged
 *   over the positions and read out linearly:
 *   d^f(q) = b3 + sum_c w3[c] mean_p ReLU(z2[c][p]); packed as
 *   [W1 (C, 3) | b1 (C) | W2 (C_out, C_in, 3) | b2 (C) | w3 (C) | b3],
 *   P = 3C^2 + 6C + 1 floats.  m and C multiples of 4 whose inference fits
 *   the 160 KiB LDS (C = m = 96 does); else LEAFI_EINVAL.  Inference and
 *   training are plain FP32 (no matrix cores): t^F, and so Algorithm 3's
 *   size threshold, is far larger than the MLP's. */
#define LEAFI_FILTER_MLP 0
#define LEAFI_FILTER_CNN 1

/* Leaf selection rules of leafi_train_filters (opts.selection).
 * SIZE: Algorithm 3 - leaves of size >= th = a t^F / t^S, largest first,
 *   while the filters fit in mem_budget (th_override replaces th).
 * KNAPSACK: Equation 1 with the benefit of Equation 2 estimated per leaf on
 *   the global training queries, as leafi_select_knapsack computes it, with
 *   t^F and t^S measured, or, when th_override >= 0, with the ratio
 *   t^F / t^S = th_override / a (the benefits' signs and order depend on the
 *   ratio alone). */
#define LEAFI_SELECT_SIZE 0
#define LEAFI_SELECT_KNAPSACK 1

/* Fill opts with the defaults listed above (n_global 1500, n_local 500,
 * noise 0.1..0.4, a 2, val 0.2, th measured, budget 8 GiB, h = m, 1000
 * epochs, lr 0.01 -> 1e-5, batch 64, patience 10, seed 1, examples not
 * kept, selection SIZE). */
void leafi_default_train_opts(leafi_train_opts *opts);

typedef struct {
  double t_filter_s;     /* measured t^F: seconds per (query, filter) inference */
  double t_series_s;     /* measured t^S: seconds per (query, series) distance */
  double th;             /* size threshold used */
  int32_t n_filters;
  int32_t epochs_max_run;/* largest epoch count any filter ran */
  double ms_collect;     /* training-target collection (scan) time */
  double ms_train;       /* SGD time */
  double mean_val_mse;   /* mean final validation MSE over filters */
} leafi_train_report;

/*
 * Algorithm 1: select leaves (Algorithm 3, or the knapsack of Equations 1-2
 * per opts.selection), generate global and local
 * training queries (collection series plus Gaussian noise), compute their
 * node-wise nearest-neighbour distances d^L with the leaf scan, and train one
 * MLP per selected leaf by SGD on the mean squared error.  `report` may be
 * NULL.  Replaces any previous filters and clears calibration.
 */
int leafi_train_filters(leafi_index *index, const leafi_train_opts *opts, leafi_train_report *report,
                        void *stream);

/*
 * The training set of the last leafi_train_filters call that had
 * keep_examples = 1 (paper: Algorithm 1 and Section "Training Data
 * Generation").  The training queries are raw (before z-normalisation): the
 * n_global global queries first (collection series drawn uniformly, plus
 * noise), then n_local local queries per filter, filter by filter (series of
 * the filter's leaf, plus noise).  Per filter f the n_examples examples are
 * [global training | local | global validation]: example e pairs query
 * ex_query[f * n_examples + e] with target ex_target[f * n_examples + e] =
 * d^L(query, leaf of f), the node-wise nearest-neighbour distance.
 * Outputs (each may be NULL): *n_queries, *n_examples, *n_train (training
 * examples per filter, the rest validate), queries_dev [n_queries, m] fp32,
 * ex_query_host [n_filters, n_examples] int32, ex_target_dev [n_filters,
 * n_examples] fp32.  LEAFI_ESTATE if no training set was kept.
 */
int leafi_get_examples(const leafi_index *index, int64_t *n_queries, int32_t *n_examples, int32_t *n_train,
                       float *queries_dev, int32_t *ex_query_host, float *ex_target_dev, void *stream);

/*
 * The schedule of the same kept training run: *max_epochs, epochs_run_host
 * [n_filters] (epochs each filter trained) and val_mse_host [n_filters,
 * max_epochs] (validation mean squared error after each epoch, NaN after the
 * filter's last epoch).  Each may be NULL.  LEAFI_ESTATE if no run was kept.
 */
int leafi_get_train_trace(const leafi_index *index, int32_t *max_epochs, int32_t *epochs_run_host,
                          float *val_mse_host);

/*
 * Install given filters instead of training them: n_filters filters on the
 * leaves leaf_ids_host[n_filters] (distinct), weights_dev [n_filters, P] with
 * P = h*m + 2h + 1 packed as [W1 (input-major: element (i, j) at i*h + j) |
 * b1 (h) | w2 (h) | b2].  A filter predicts d^f(q) = w2 . ReLU(W1 q + b1) + b2
 * for the z-normalised query q.  Clears calibration.
 */
int leafi_set_filters(leafi_index *index, int32_t n_filters, int32_t hidden, const int32_t *leaf_ids_host,
                      const float *weights_dev, void *stream);

/* Install given CNN filters (LEAFI_FILTER_CNN packing, `channels` C) on the
 * leaves leaf_ids_host[n_filters] (distinct).  Clears calibration. */
int leafi_set_cnn_filters(leafi_index *index, int32_t n_filters, int32_t channels, const int32_t *leaf_ids_host,
                          const float *weights_dev, void *stream);

/* Copy the filters out: leaf_ids_host [n_filters] and weights_dev [n_filters, P]
 * (the packing of the installed architecture).  Either pointer may be NULL. */
int leafi_get_filters(const leafi_index *index, int32_t *leaf_ids_host, float *weights_dev, void *stream);

/* ------------------------------------------------------------------------
 * Conformal auto-tuning (paper: Section "Filter Conformal Auto-tuning",
 * Algorithm 4; Section "Preliminaries", conformal regression)
 * ---------------------------------------------------------------------- */

#define LEAFI_CALIB_STEP 0         /* offsets of the first sorted position reaching the target */
#define LEAFI_CALIB_STEFFEN 1      /* Steffen monotone interpolation of offset vs. recall */
#define LEAFI_CALIB_NO_CORRECTION 2/* flag: use the raw target, not ceil((n_c+1) t) / n_c */

/*
 * Fit the auto-tuners on n_calib raw calibration queries (calib_dev [n_calib, m]):
 * absolute prediction errors alpha = |d^f - d^L| per filter, sorted; for each
 * sorted position j the offsets o_i = alpha_{i,(j)} and the recall of the
 * simulated search on the calibration set (a true neighbour in a filtered
 * leaf is lost iff d^f - o > d^bsf, the exact best-so-far before that leaf);
 * then, for every (k, target) pair of ks_host[n_ks] x targets_host[n_targets],
 * the offsets whose recall reaches the target.  `flags` = LEAFI_CALIB_STEP or
 * LEAFI_CALIB_STEFFEN, optionally | LEAFI_CALIB_NO_CORRECTION.  Targets must
 * lie in (0, 1]; ks in [1, 256].
 */
int leafi_calibrate(leafi_index *index, const float *calib_dev, int32_t n_calib, const int32_t *ks_host,
                    int32_t n_ks, const float *targets_host, int32_t n_targets, int32_t flags, void *stream);

/* Offsets of calibrated pair p (pairs are ordered k-major: p = ik * n_targets
 * + it): offsets_host [n_pairs, n_filters]; +inf disables a filter. */
int leafi_get_offsets(const leafi_index *index, float *offsets_host);

/* Install offsets directly for the given (k, target) pairs (offsets_host
 * [n_ks * n_targets, n_filters], k-major as above).  Replaces calibration. */
int leafi_set_offsets(leafi_index *index, const int32_t *ks_host, int32_t n_ks, const float *targets_host,
                      int32_t n_targets, const float *offsets_host);

/* ------------------------------------------------------------------------
 * Search (paper: Algorithm 2)
 * ---------------------------------------------------------------------- */

#define LEAFI_SCAN_BF16 0   /* batched: BF16 MFMA scan, FP32 rerank + FP64 band */
#define LEAFI_SCAN_FP32 1   /* plain: FP32 direct-difference scan, one query at a time */

typedef struct {
  int32_t k_max;           /* width of the output rows, 1..256 */
  int32_t scan;            /* LEAFI_SCAN_BF16 or LEAFI_SCAN_FP32 */
  int32_t use_filters;     /* 0: summaries only (exact search) */
  int32_t n_schedule;      /* entries used in schedule[] (>= 1) */
  int32_t schedule[8];     /* leaves searched per query per round; the last entry
                              repeats; 0 = every leaf that survives.  {1} is the
                              paper's sequential loop. */
  int32_t kprime;          /* BF16 candidates kept per (query, leaf); 0 = 4k */
  int32_t flags;           /* LEAFI_SEARCH_* bits below; 0 = automatic */
  int32_t reserved[2];
} leafi_search_opts;

#define LEAFI_SEARCH_NO_GRAPH 1     /* planned sequence as plain launches, never captured */
#define LEAFI_SEARCH_HOST_ROUNDS 2  /* host-driven rounds (counts read back every round) */
/* Filter inference tiles: by default a batch with at least one 32-query tile
 * per compute unit uses 64-query tiles (filter weights read half as often),
 * else 32-query tiles.  These flags force one size; values never depend on
 * it (every (query, filter) sum runs in the same order). */
#define LEAFI_SEARCH_FILTER_TILE_SMALL 4
#define LEAFI_SEARCH_FILTER_TILE_LARGE 8

void leafi_default_search_opts(leafi_search_opts *opts);

typedef struct {
  int64_t leaves_scanned;
  int64_t leaves_lb_pruned;
  int64_t leaves_filter_pruned;
  int64_t series_scanned;   /* real series in scanned leaves */
  int64_t fallback_items;   /* (query, leaf) pairs whose candidates could not certify the
                               top k: rescanned by the next round's scan when the schedule
                               ends in 0 and has one, else exactly in FP32 (each rescan
                               counts once) */
  int32_t rounds;           /* regular rounds that scanned at least one leaf */
  int32_t path;             /* how the batch ran: 0 host-driven rounds (counts read back
                               every round), 1 planned launch sequence, 2 replay of a
                               captured graph, 3 captured in this call and replayed,
                               4 a planned sequence (or replay) one of whose rounds held more
                               items than its buffers' capacity, then run again with
                               host-driven rounds (the counts given are that run's) */
  double ms_total;
  double ms_scan;           /* time in the BF16 leaf-scan kernels (HIP events on the stream) */
  double scan_bytes;        /* unique leaf-store bytes the scan kernels had to read */
  int64_t filter_evals;     /* (query, leaf) pairs whose learned filter was evaluated */
} leafi_search_stats;

/*
 * k-NN search for nq raw queries (queries_dev [nq, m]).  k_dev [nq] (int32,
 * 1 <= k <= k_max) and target_dev [nq] (float) give each query's k and recall
 * target; a query whose (k, target) pair is not calibrated, or whose target is
 * >= 1, runs without filters (exact).  Outputs ids_dev [nq, k_max] (int64) and
 * dists_dev [nq, k_max] (fp32); slots beyond a query's k hold id -1 and +inf.
 * `stats` (host) may be NULL; when given, the call synchronises the stream.
 *
 * Execution: with the BF16 scan and a schedule that contains a 0 (so every
 * query ends within that many rounds), the batch runs as a fixed launch
 * sequence (a planned batch).  Each pass's item buffers are sized from its
 * upper bound nq * min(R, n_leaves) plus the previous round's rescans (at
 * most nq * n_leaves) when the bound-sized buffers fit 16 GiB, else from the
 * largest item count that fits (or the capacity set by
 * leafi_set_plan_capacity, if smaller).  A batch whose passes all fit their
 * bounds reads nothing back.  Otherwise each round's layout compares its
 * item count with the capacity on the device; a round with more items lays
 * out nothing and raises an overflow word, which the call reads back (one
 * synchronisation of the stream) before returning; after an overflow the
 * batch runs again with host-driven rounds (stats->path 4), and later calls
 * of the same shape, options and buffers run host-driven rounds at once
 * (path 0).  The second call
 * with the same shape, options and buffer addresses captures the sequence in
 * a HIP graph, and later identical calls replay it (the graph reads the
 * current contents of the caller's buffers).  Other cases run host-driven
 * rounds.  Results are identical on every path.
 */
int leafi_search_knn(leafi_index *index, const float *queries_dev, int64_t nq, const int32_t *k_dev,
                     const float *target_dev, const leafi_search_opts *opts, int64_t *ids_dev,
                     float *dists_dev, leafi_search_stats *stats, void *stream);

/*
 * The same search for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * It allocates nothing: every per-batch buffer is carved from one fixed
 * device array of LEAFI_NOALLOC_SCRATCH_BYTES per GPU, owned by the library
 * until the process ends; the caller still passes the inputs and outputs.
 * Arguments, layouts and results are those of leafi_search_knn (results are
 * bit-identical to it), with these limits:
 *   - the batch must run as a planned launch sequence: BF16 scan, a schedule
 *     containing a 0, neither LEAFI_SEARCH_HOST_ROUNDS nor statistics; it is
 *     enqueued as plain launches (never captured by the library, no events);
 *   - its buffers must fit the scratch array: a batch that needs more is
 *     rejected with LEAFI_EINVAL before anything is enqueued (the message
 *     states both sizes); fewer queries per call fit.
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (each batch's first kernel zeroes the counters and control
 * words a batch starts from): calls that overlap on one GPU -- from two
 * threads, or on two streams without ordering between them -- race.  The
 * array's device address is looked up on the first call on each device.  The
 * call returns once the work is enqueued on `stream`.
 */
#define LEAFI_NOALLOC_SCRATCH_BYTES (256u << 20)
int leafi_search_knn_noalloc(leafi_index *index, const float *queries_dev, int64_t nq, const int32_t *k_dev,
                             const float *target_dev, const leafi_search_opts *opts, int64_t *ids_dev,
                             float *dists_dev, void *stream);

/* ------------------------------------------------------------------------
 * Scan tiling auto-tuner (no counterpart in the paper: it picks the BF16 leaf
 * scan's tile shape for this GPU and workload)
 * ---------------------------------------------------------------------- */

#define LEAFI_TUNE_MAX 16

typedef struct {
  int32_t n_candidates;                 /* tile shapes timed */
  int32_t chosen;                       /* index of the fastest, now in use */
  int32_t chunk_rows[LEAFI_TUNE_MAX];   /* leaf rows per scan tile */
  int32_t queries_per_tile[LEAFI_TUNE_MAX];
  double ms[LEAFI_TUNE_MAX];            /* median time of one search of the sample batch */
} leafi_tune_report;

/*
 * Time the sample batch (queries_dev [nq, m], k_dev, target_dev and opts as
 * for leafi_search_knn, BF16 scan) once per candidate tile shape -- rows per
 * tile in {512, 1024, 2048} times 16, 32, 48 or 64 queries per tile --
 * `repeats` times each after one warm-up, and keep the shape with the
 * smallest median for all later searches of this index.  Results of every search are identical under every shape.
 * The stream is synchronised.  `report` (host) may be NULL.
 */
int leafi_autotune(leafi_index *index, const float *queries_dev, int64_t nq, const int32_t *k_dev,
                   const float *target_dev, const leafi_search_opts *opts, int32_t repeats,
                   leafi_tune_report *report, void *stream);

/* Set the BF16 scan's tile shape directly (what leafi_autotune chooses):
 * chunk_rows in {128, 256, ..., 4096}; queries_per_tile 16, 32, 48 or 64.
 * The default is 1024 rows and 32 queries.  Results do not depend on the
 * shape. */
int leafi_set_tiling(leafi_index *index, int32_t chunk_rows, int32_t queries_per_tile);

/* Item capacity of a planned batch's passes (see leafi_search_knn): at most
 * max_items (query, leaf) items per pass, which bounds the planned batch's
 * device buffers; 0 (the default) means as many as 16 GiB of buffers hold.
 * A batch whose round exceeds it still returns exact results (it runs again
 * with host-driven rounds).  Does not change any result. */
int leafi_set_plan_capacity(leafi_index *index, int64_t max_items);

/* Why this index stopped capturing planned batches into HIP graphs (the
 * first capture that failed), or "" while capture works.  The string is
 * owned by the index and valid until its next search or destroy. */
const char *leafi_graph_note(const leafi_index *index);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of k-NN requests (Algorithm 2 for a stream of
 * queries with mixed k and recall targets)
 *
 * A server keeps the index, filters and offsets resident and runs engine
 * rounds on its own HIP stream from a worker thread.  Every admitted request
 * owns a slot of per-query device state; a round prepares the requests
 * admitted since the previous round, advances every active request by one
 * round of its own schedule (requests are grouped by surviving leaf across
 * the whole mix for the leaf scan) and retires finished requests, freeing
 * their slots.  A request's result does not depend on which other requests
 * shared its rounds.  Admission is by memory: the number of slots is
 * max_slots, or fewer if mem_budget cannot hold that many slots' state.
 * While a server exists, its index must not be used by any other call.
 * ---------------------------------------------------------------------- */

typedef struct leafi_server leafi_server;

typedef struct {
  int32_t max_slots;      /* requests on the GPU at once (0 = as many as mem_budget holds) */
  int32_t k_max;          /* largest k of any request, 1..256 (k is clamped to it) */
  int32_t scan;           /* LEAFI_SCAN_BF16 or LEAFI_SCAN_FP32 */
  int32_t use_filters;
  int32_t n_schedule;     /* per-request round schedule, as in leafi_search_opts */
  int32_t schedule[8];
  int32_t queue_capacity; /* requests waiting for a slot before submit returns LEAFI_EAGAIN */
  int64_t mem_budget;     /* device bytes for per-slot state (0 = unlimited) */
  int32_t reserved[4];
} leafi_server_opts;

typedef struct {
  int64_t completed;      /* requests finished during the replay */
  int64_t rounds;         /* engine rounds run during the replay */
  double wall_s;          /* first arrival to last completion */
  double mean_active;     /* mean requests per round */
  int32_t max_active;
  int32_t reserved;
} leafi_server_report;

/* Defaults: 1024 slots, k_max 1, BF16 scan, filters on, schedule {1, 0},
 * queue capacity 2^20, mem_budget 4 GiB. */
void leafi_default_server_opts(leafi_server_opts *opts);

/* Start a server on a built index (calibrated if it should use filters). */
int leafi_server_create(leafi_index *index, const leafi_server_opts *opts, leafi_server **out);

/* Stop the worker after it has finished every submitted request; release all. */
void leafi_server_destroy(leafi_server *server);

/* Number of slots the server admitted (after the memory budget). */
int leafi_server_info(const leafi_server *server, int32_t *max_slots);

/* Queue one raw query (query_host [m]) with its k and recall target; returns
 * a ticket.  LEAFI_EAGAIN when queue_capacity requests are already waiting. */
int leafi_server_submit(leafi_server *server, const float *query_host, int32_t k, float target, uint64_t *ticket);

/* done = 1 once the request has finished; then ids_host / dists_host [k_max]
 * (either may be NULL) receive its result, latency_ms (nullable) the time from
 * submission to completion, and the ticket is released. */
int leafi_server_poll(leafi_server *server, uint64_t ticket, int64_t *ids_host, float *dists_host,
                      double *latency_ms, int32_t *done);

/* Replay an arrival trace: query i (queries_host [n, m]) is submitted at
 * arrival_s[i] seconds after the call starts (a full queue delays it); waits
 * for every result.  Outputs ids_host / dists_host [n, k_max] and latency_ms
 * [n] (scheduled arrival to completion).  `report` may be NULL. */
int leafi_server_replay(leafi_server *server, const float *queries_host, int64_t n, const double *arrival_s,
                        const int32_t *ks, const float *targets, int64_t *ids_host, float *dists_host,
                        double *latency_ms, leafi_server_report *report);

/* ------------------------------------------------------------------------
 * Building blocks, exposed for checking and for callers that compose them
 * ---------------------------------------------------------------------- */

/* z-normalise n rows of length m: out_dev [n, m] fp32 (may alias x_dev). */
int leafi_znorm(const float *x_dev, int64_t n, int32_t m, float *out_dev, void *stream);

/* Summary lower bounds d^lb for raw queries: lb_dev [nq, n_leaves] fp32. */
int leafi_lower_bounds(leafi_index *index, const float *queries_dev, int64_t nq, float *lb_dev, void *stream);

/* Filter predictions for already z-normalised inputs x_dev [nq, m]:
 * out_dev [nq, n_filters] = d^f (before any offset), fp32.  m is a multiple
 * of 4 in [4, 1024], hidden a multiple of 4 in [4, 1024]; x_dev is 16-byte
 * aligned.  Returns -1 otherwise. */
int leafi_mlp_infer(const float *weights_dev, int32_t n_filters, int32_t m, int32_t hidden, const float *x_dev,
                    int64_t nq, float *out_dev, void *stream);

/* One plain SGD step per filter on its own batch: x_dev [n_filters, batch, m],
 * y_dev [n_filters, batch]; weights_dev [n_filters, P] is updated in place with
 * w -= lr * grad of mean((d^f - y)^2).  loss_dev [n_filters] receives the
 * batch loss before the step (may be NULL). */
int leafi_mlp_sgd_step(float *weights_dev, int32_t n_filters, int32_t m, int32_t hidden, const float *x_dev,
                       const float *y_dev, int32_t batch, float lr, float *loss_dev, void *stream);

/* CNN filter predictions for z-normalised inputs x_dev [nq, m]: out_dev
 * [nq, n_filters] = d^f, fp32 (LEAFI_FILTER_CNN packing, C channels). */
int leafi_cnn_infer(const float *weights_dev, int32_t n_filters, int32_t m, int32_t channels, const float *x_dev,
                    int64_t nq, float *out_dev, void *stream);

/* One plain SGD step per CNN filter on its own batch (as leafi_mlp_sgd_step):
 * x_dev [n_filters, batch, m], y_dev [n_filters, batch]; loss_dev
 * [n_filters] receives the batch loss before the step. */
int leafi_cnn_sgd_step(float *weights_dev, int32_t n_filters, int32_t m, int32_t channels, const float *x_dev,
                       const float *y_dev, int32_t batch, float lr, float *loss_dev, void *stream);

/* Node-wise k nearest neighbours of raw queries in every leaf (the scan in
 * all-pairs mode, used for the filters' training targets): d_dev
 * [nq, n_leaves, k] fp32 and ids_dev [nq, n_leaves, k] int64, sorted by
 * (distance, id), empty slots -1 / +inf.  d_dev[q, L, 0] is d^L(q, L). */
int leafi_leaf_knn(leafi_index *index, const float *queries_dev, int64_t nq, int32_t k, float *d_dev,
                   int64_t *ids_dev, void *stream);

/*
 * Leaf selection as a knapsack (paper: Section "Leaf Node Selection",
 * Equations 1-2; the per-leaf rates are the estimates that section leaves
 * open).  For n_queries raw training queries (device, [n_queries, m] fp32)
 * each query's exact 1-NN search (no filters) is followed in its visit
 * order, with the index's summary bounds d^lb and the node-wise 1-NN
 * distances d^L from the leaf scan; d^bsf is the best distance over the
 * leaves ahead of leaf i.  Per leaf i:
 *   p_lb[i] = share of queries with d^lb > d^bsf (the bound prunes leaf i);
 *   p_f[i]  = share of the remaining visits with d^L > d^bsf (what a filter
 *             predicting d^L exactly prunes; 0 if no query reaches leaf i);
 *   benefit[i] = b_i = (1 - p_lb[i]) (p_f[i] / a * t^S * |N_i| - t^F).
 * The knapsack (capacity mem_budget bytes, one filter of the hidden width
 * weighs 4 (h m + 2 h + 1) bytes, hidden 0 = m) takes the leaves with
 * b_i > 0, largest first (ties by leaf id), at most floor(mem_budget /
 * weight) of them: with equal weights that is the exact optimum.
 * t_filter_s / t_series_s: t^F and t^S in seconds; either <= 0: both are
 * measured on this GPU as leafi_train_filters measures them.
 * Outputs (host, each may be NULL): leaf_ids [n_leaves capacity] the
 * selection in that order, *n_selected its length, benefit, p_lb and p_f
 * [n_leaves].  Installs nothing.
 */
int leafi_select_knapsack(leafi_index *index, const float *queries_dev, int64_t n_queries, float a,
                          double t_filter_s, double t_series_s, int32_t hidden, int64_t mem_budget,
                          int32_t *leaf_ids_host, int32_t *n_selected, double *benefit_host, double *p_lb_host,
                          double *p_f_host, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LEAFI_H */
