// Launch wrappers for the gfx950 kernels of libleafi.  Every wrapper enqueues
// on `st` and checks the launch; sizes are validated by the caller.
#pragma once

#include "common.h"

namespace leafi {

// ---- ingest and query preparation (k_prep.hip) ---------------------------

// Per series: mean and population std in FP64 (sd < 1e-8 marks a constant
// series), and per-segment mean/std of the stored fp32 normalised values.
void launch_series_stats(const float *raw, int64_t n, int m, int S, double *mean, double *sd, float *seg_mu,
                         float *seg_sd, hipStream_t st);

// Build the leaf store: output row r takes raw series src_of_row[r] (-1 =
// padding) and writes the normalised fp32 row, its bf16 copy, ||x~||^2, the
// original id, and raises leaf_eps[leaf_of_row[r]] to ||x - x~||.
void launch_pack(const float *raw, const int64_t *src_of_row, const int32_t *leaf_of_row, int64_t rows, int m,
                 const double *mean, const double *sd, float *x32, uint16_t *x16, float *xn16, int64_t *rowid,
                 float *leaf_eps, hipStream_t st);

// Plain z-normalisation (out may alias x).
void launch_znorm(const float *x, int64_t n, int m, float *out, hipStream_t st);

// Query preparation: normalised fp32 and bf16 rows, ||q~||^2, ||q - q~||, and
// per-segment (mean, std) pairs qstat [., S, 2].  With `slots`, raw row i
// goes to output row slots[i] (the serving engine's per-query slots).
void launch_qprep(const float *raw, int64_t nq, int m, int S, float *q32, uint16_t *q16, float *qn16, float *qeps,
                  float *qstat, hipStream_t st, const int32_t *slots = nullptr);

// Summary lower bounds lb [., N] for rows i (or slots[i]).
void launch_lb(const float *qstat, int64_t nq, const float *boxes, int N, int S, int m, float *lb, hipStream_t st,
               const int32_t *slots = nullptr);

// Visit order: per query, leaves sorted by (lb, leaf id); lbs receives the
// bounds in that order.
void launch_order(const float *lb, int64_t nq, int N, int32_t *order, float *lbs, hipStream_t st,
                  const int32_t *slots = nullptr);

// Training queries: q_j = x32[row_j] + sigma_j * N(0, 1) noise from a
// counter-based generator keyed by (seed, j, t).
void launch_make_queries(const float *x32, const int64_t *rows, const float *sigma, int64_t nq, int m,
                         uint64_t seed, float *out, hipStream_t st);

// ---- round machinery (k_rounds.hip) ---------------------------------------

struct RoundBufs {
  // per query
  int32_t *cursor;      // next position in the visit order
  float *tau;           // k-th best distance so far (+inf until k results)
  int32_t *kq;          // k of each query
  int32_t *pair;        // calibrated (k, target) row of the offset table, -1 = filters off
  int32_t *res_cnt;     // results held
  double *res_d2;       // [nq, kmax] squared FP64 distances, sorted
  int32_t *res_row;     // [nq, kmax] leaf-store rows
  int32_t *qitem_cnt;   // items emitted this round
  int32_t *qitem_leaf;  // [nq, N] leaves emitted this round
  int32_t *qitem_idx;   // [nq, N] their item slots
  // per leaf
  int32_t *leaf_cnt;    // [N] items per leaf this round
  int32_t *leaf_fill;   // [N]
  int32_t *leaf_istart; // [N + 1]
  int32_t *tile_start;  // [N + 1]
  // per item
  int32_t *item_q;
  int32_t *item_leaf;
  double *item_d2;      // [items, kmax]
  int32_t *item_row;    // [items, kmax]
  int32_t *item_cnt;
  float *item_bound;    // lower bound on any row of the item that is not a candidate
  int32_t *item_live;   // a search round's items that its bounds did not certify (ctl[kCtlLive] of them)
  // fallback list of (query, leaf) pairs
  int32_t *fb_q;
  int32_t *fb_leaf;
  // control: see Ctl
  int64_t *ctl;
  // [N] real (unpadded) series per leaf: the algorithmic bytes of a round
  const int32_t *leaf_n;
  // rows per scan tile of the pass in flight (a multiple of kRowAlign)
  int32_t chunk;
  // 1: a search round, whose BF16 scan may skip rows provably farther than
  // the query's tau; 0: per-item exact top-k (all-pairs passes)
  int32_t use_tau;
  // 1: each query keeps its own number of candidates, item_kprime(k) of the
  // pass's kprime (a batch of mixed k); 0: every query keeps kprime
  int32_t kp_query;
  // > 0: the item buffers hold this many items (a planned round sized below
  // its worst case).  A layout that finds more sets ctl[kCtlOverflow] and
  // lays out nothing; from then on every round of the batch is empty and
  // the kernels that read item lists return at once (the host then runs
  // the batch again with host-driven rounds).  0: buffers fit every layout.
  // The overflow word is zeroed at the start of every batch (query setup)
  // and by every round reset (host-driven and served rounds).  cap_tiles
  // (> 0) bounds the round's scan tiles the same way.
  int64_t cap_items;
  int64_t cap_tiles;
};

// Candidates a query of k results keeps per (query, leaf) in a pass whose
// lists have kprime slots: 4k for the BF16 scan, k + 8 for the FP32 scan
// (never fewer than k, never more than kprime), or kprime for all.
__host__ __device__ inline int item_kprime(int kp_query, int kprime, int k, bool bf16) {
  if (!kp_query) return kprime;
  const int kp = bf16 ? 4 * k : k + 8;
  return kp < kprime ? kp : kprime;
}

// Tile of item group g (queries g*mq ..) and row chunk c of leaf L: chunk-major
// (the groups of one chunk are consecutive tiles, so work-groups that read
// the same rows run side by side on one XCD and share its L2).
__host__ __device__ inline int64_t tile_of(const int32_t *tile_start, int L, int g, int c, int G) {
  return static_cast<int64_t>(tile_start[L]) + static_cast<int64_t>(c) * G + g;
}

// Control words: each on its own 128-byte line (kCtlStride int64 apart), so
// that atomics on different counters do not serialise on one L2 line.
constexpr int kCtlStride = 16;
enum Ctl : int {
  kCtlItems = 0 * kCtlStride,       // items this round
  kCtlTiles = 1 * kCtlStride,       // scan tiles this round
  kCtlActive = 2 * kCtlStride,      // queries with leaves left
  kCtlFallback = 3 * kCtlStride,    // uncertified items queued for an exact rescan
  kCtlLbPruned = 4 * kCtlStride,
  kCtlFPruned = 5 * kCtlStride,
  kCtlSeries = 6 * kCtlStride,      // real series in scanned items
  kCtlScanned = 7 * kCtlStride,     // items (leaves) scanned, excluding rescans
  kCtlFbTotal = 8 * kCtlStride,     // uncertified items rescanned, over the batch
  kCtlScanBytes = 9 * kCtlStride,   // unique leaf-store bytes the regular rounds read
  kCtlRounds = 10 * kCtlStride,     // regular rounds with at least one item
  kCtlFEvals = 11 * kCtlStride,     // (query, leaf) pairs queued for filter inference
  kCtlOverflow = 12 * kCtlStride,   // nonzero: a round's items exceeded the buffers' capacity (cap_items)
  kCtlLive = 13 * kCtlStride,       // a search round's items left to rerank (item_live)
  kCtlCount = 14 * kCtlStride,
  kCtlRoundWords = kCtlFallback + 1  // words a round starts from zero (items .. fallback)
};

struct StoreView {
  const float *x32;
  const uint16_t *x16;
  const float *xn16;
  const int64_t *leaf_off;  // padded row offsets [N + 1]
  const int32_t *leaf_n;    // real rows per leaf
  const float *leaf_eps;
  int m;
  int N;
};

struct QueryView {
  const float *q32;
  const uint16_t *q16;
  const float *qn16;
  const float *qeps;
};

// All of a batch's per-query preparation in one launch (one work-group per
// query): the results of launch_qprep, launch_lb, launch_order and
// launch_select_pairs plus the search state (cursor 0, tau +inf, no results,
// no items); work-group 0 zeroes the control words, leaf counts and (pcnt
// non-null) F filter-pair counts.  boxes_t holds the boxes as [S][4][N].
void launch_query_setup(const float *raw, int64_t nq, int m, int S, const float *boxes, const float *boxes_t, int N, float *q32,
                        uint16_t *q16, float *qn16, float *qeps, float *qstat, float *lb, int32_t *order, float *lbs, const int32_t *k_dev, const float *t_dev,
                        int n_pairs, const int32_t *pair_k, const float *pair_t, int kmax, RoundBufs b, int F,
                        int32_t *pcnt, hipStream_t st);

// Round schedule: leaves per query in round r = r_[min(r, n - 1)] (0 = all survivors).
struct Schedule {
  int n;
  int r[8];
};

// Emit this round's (query, leaf) pairs from the visit order (Algorithm 2's
// prune cascade).  want = leaves per query this round (0 = all survivors);
// with qround (serving), each query instead takes sched.r at its own round
// count, which the kernel advances.
// lbs and dfo are [nq, N] in visit order: the summary bound and (filters
// active) the filter's pruning value d^f - o, -inf where no filter applies.
// With `append` the emitted leaves follow the rescans the last merge queued
// in each query's item list (counted in qitem_cnt and leaf_cnt), so this
// round's scan also rescans them.
void launch_worklist(int64_t nq, int N, const float *lbs, const int32_t *order, const float *dfo,
                     const int32_t *leaf_n, int want, RoundBufs b, hipStream_t st, const Schedule *sched = nullptr,
                     int32_t *qround = nullptr, bool append = false);

// (query, visit position) pairs whose filter test a later round can reach,
// grouped by filter into plist [F, nq] (entries q * N + position) with counts
// pcnt [F] (zeroed by the caller).  Every other position ahead of the cursor
// gets dfo = -inf (never pruned by a filter).
void launch_filter_pairs(int64_t nq, int N, const float *lbs, const int32_t *order, const int32_t *filt_of_leaf,
                         RoundBufs b, int64_t *plist, int32_t *pcnt, float *dfo, hipStream_t st,
                         const int32_t *qround = nullptr);

// Serving: retire finished active slots (state 1 -> 2) into a compact done list.
void launch_collect_done(int64_t n_slots, int N, int kmax, const int64_t *rowid, RoundBufs b, int32_t *state,
                         int32_t *done_slot, int64_t *done_ids, float *done_d, int32_t *n_done, hipStream_t st);

// Emit pairs from the fallback list instead.  The count is read on the device
// (ctl[kCtlFallback]); `bound` >= that count sizes the grid.
void launch_emit_fallback(int64_t bound, int N, RoundBufs b, hipStream_t st);

// Items CSR by leaf and tile ranges (single work-group).  row_bytes > 0 adds
// the padded rows of every leaf with items times row_bytes to
// ctl[kCtlScanBytes] and counts a round in ctl[kCtlRounds] if it has items.
void launch_leaf_scan(int N, const int64_t *leaf_off, int mq, int64_t row_bytes, RoundBufs b, hipStream_t st);

// Zero the first n_ctl control words, leaf_cnt[0..N) and qitem_cnt[0..nq)
// (either count may be 0) in one launch.  A kernel, not a memset, so that the
// sequence can be captured in a graph.
void launch_round_reset(RoundBufs b, int n_ctl, int N, int64_t nq, hipStream_t st);

// Place each query's emitted leaves into item slots.
void launch_scatter(int64_t nq, int N, RoundBufs b, hipStream_t st);

// launch_leaf_scan then launch_scatter in one launch of the scatter's grid
// (every work-group recomputes the leaf scan into LDS), for N <=
// kLayoutLdsMax.  leaf_fill must be zero on entry (launch_worklist zeroes it);
// leaf_cnt is left for launch_item_rerank to zero.
constexpr int kLayoutLdsMax = 4096;
void launch_layout_scatter(int64_t nq, int N, const int64_t *leaf_off, int mq, int64_t row_bytes, RoundBufs b,
                           hipStream_t st);

// The first round of a batch when it takes one leaf per query: each query's
// item is the first leaf of its visit order (nothing can be pruned yet);
// replaces launch_worklist, launch_leaf_scan and launch_scatter for that
// round (single work-group, N <= kLayoutLdsMax).
void launch_first_round_layout(int64_t nq, int N, const int32_t *order, const int64_t *leaf_off,
                               const int32_t *leaf_n, int mq, int64_t row_bytes, RoundBufs b, hipStream_t st);

// launch_leaf_scan then launch_scatter in one single-work-group launch, for
// passes with few items (its placement loop is serial per query).
void launch_leaf_scan_scatter(int64_t nq, int N, const int64_t *leaf_off, int mq, int64_t row_bytes, RoundBufs b,
                              hipStream_t st);

// Leaf scan over all tiles; keeps the kprime best (key = dist^2 bits, row)
// per (tile, query slot) in cand.
void launch_scan_bf16(StoreView s, QueryView q, RoundBufs b, int mq, int kprime, uint64_t *cand, int grid,
                      hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_scan_fp32(StoreView s, QueryView q, RoundBufs b, int mq, int kprime, uint64_t *cand, int grid,
                      hipStream_t st);

// Per query of a search round after its BF16 scan: qbound[q] = an upper bound
// of the query's k-th distance after the round (from the k-th smallest key
// over all its candidate lists, and its tau), for the rerank to skip
// candidates that cannot enter its top k.  With the bound known, each of the
// query's items whose every row is provably farther gets no results and that
// bound as its certificate; the others are listed in item_live
// (ctl[kCtlLive] of them) for the rerank.  cmax = chunks of the largest leaf;
// eps_max = the largest leaf rounding radius.
void launch_query_bound(StoreView s, QueryView q, RoundBufs b, int64_t nq, int mq, int kprime, int kmax, int cmax,
                        float eps_max, const uint64_t *cand, float *qbound, hipStream_t st);
// Per item: merge its tiles' candidates, rerank in FP32 (FP64 for the band
// around the k-th), write the item's top-k and its certificate bound.  With
// qbound (a search round) only the items launch_query_bound listed are
// reranked.
void launch_item_rerank(StoreView s, QueryView q, RoundBufs b, int mq, int kprime, int kmax, bool bf16,
                        const uint64_t *cand, int grid, int max_chunks, hipStream_t st, const float *qbound = nullptr);

// Candidate-list geometry for kprime kept keys: queries per tile and list
// capacity.  BF16: mq_pref queries per tile (16, 32, 48 or 64; others mean
// 32).  FP32: 32 queries per tile when kprime <= 32 and mq_pref != 16, else 16.
void scan_geometry(bool bf16, int kprime, int mq_pref, int m, int *mq, int *cap);

// Per query: merge the round's items into the running top-k, update tau,
// queue uncertified items (check_cert) and count active queries.  With ids
// non-null (the batch's last merge) also write every query's output row, as
// launch_finalize does.
// With fp.plist non-null the merge also selects each query's filter pairs
// from its new tau, as launch_filter_pairs does (no separate launch).
struct FilterPairArgs {
  const float *lbs = nullptr;
  const int32_t *order = nullptr;
  const int32_t *filt_of_leaf = nullptr;
  int64_t *plist = nullptr;
  int32_t *pcnt = nullptr;
  float *dfo = nullptr;
};
void launch_query_merge(int64_t nq, int N, int kmax, bool check_cert, bool dedupe, RoundBufs b, hipStream_t st,
                        const int64_t *rowid = nullptr, int64_t *ids = nullptr, float *dists = nullptr,
                        const FilterPairArgs &fp = FilterPairArgs());

// Final outputs: ids (original series ids) and Euclidean distances.
void launch_finalize(int64_t nq, int kmax, const int64_t *rowid, RoundBufs b, int64_t *ids, float *dists,
                     hipStream_t st);

// Per-leaf top-k for all (query, leaf) items (all-pairs mode): copies item
// results into d [nq, N, k] / ids [nq, N, k].
void launch_items_to_leaf_knn(int64_t n_items, int N, int k, int kmax, const int64_t *rowid, RoundBufs b,
                              float *d, int64_t *ids, hipStream_t st);

// ---- learned filters (k_mlp.hip) -------------------------------------------

// d^f for every (query, filter): out [nq, F].
void launch_mlp_infer(const float *w, int F, int m, int h, const float *x, int64_t nq, float *out, hipStream_t st);

// Pruning values for listed pairs only: filter f evaluates the entries
// plist[f * stride + 0 .. pcnt[f]) (q * N + visit position) and writes
// dfo[entry] = d^f(x[q]) - offsets[pair[q] * F + f].  A persistent grid walks
// the non-empty query tiles of all filters; their prefix over the filters
// is computed by every work-group itself for F <= 4096, else by a first
// launch into tile_prefix [F + 1] (scratch).  tile_mode: 0 = 32-query tiles,
// or 64-query tiles when the batch has at least one 32-query tile per CU
// (F <= 4096); 1 = always 32; 2 = always 64.  Values never depend on it.
void launch_mlp_infer_pairs(const float *w, int F, int m, int h, const float *x, const int64_t *plist,
                            const int32_t *pcnt, int64_t stride, int N, const int32_t *pair, const float *offsets,
                            int32_t *tile_prefix, float *dfo, hipStream_t st, int tile_mode = 0);

// Per-query offset row lookup for (k, target) pairs.
// k is clamped to [1, kmax].
void launch_select_pairs(int64_t nq, const int32_t *k_dev, const float *t_dev, int n_pairs, const int32_t *pair_k,
                         const float *pair_t, int kmax, int32_t *pair, int32_t *kq, hipStream_t st,
                         const int32_t *slots = nullptr);

struct TrainArgs {
  float *w;              // [F, P] weights (updated)
  float *w_best;         // [F, P] best-validation copy
  const float *xq;       // query pool [*, m] (normalised)
  const int32_t *ex_q;   // [F, n_ex] query index of each example
  const float *ex_y;     // [F, n_ex] target
  int n_train;           // first n_train examples of each filter train
  int n_ex;              // remaining n_ex - n_train validate
  int F, m, h;
  int batch;
  int max_epochs;
  int patience;
  float lr0, lr_min;
  uint64_t seed;
  float *val_mse;        // [F] best validation MSE
  int32_t *epochs_run;   // [F]
  float *val_trace;      // [F, max_epochs] validation MSE after each epoch run (may be null)
};

// Full SGD training, one work-group per filter.
void launch_mlp_train(const TrainArgs &a, hipStream_t st);

// One SGD step per filter on explicit batches.
void launch_mlp_sgd_step(float *w, int F, int m, int h, const float *x, const float *y, int batch, float lr,
                         float *loss, hipStream_t st);

// ---- CNN filters (k_cnn.hip) -------------------------------------------------

// Floats of a packed CNN filter with C channels (3C^2 + 6C + 1).
int64_t cnn_param_count(int C);
// LEAFI_EINVAL unless length m and C channels are multiples of 4 whose
// inference fits in LDS.
void cnn_check(int m, int C);
// d^f of every (query, filter): out [nq, F].
void launch_cnn_infer(const float *w, int F, int m, int C, const float *x, int64_t nq, float *out, hipStream_t st);
// Listed pairs, as launch_mlp_infer_pairs: dfo[e] = d^f - offsets[pair[q] F + f].
void launch_cnn_infer_pairs(const float *w, int F, int m, int C, const float *x, const int64_t *plist,
                            const int32_t *pcnt, int64_t stride, int N, const int32_t *pair, const float *offsets,
                            float *dfo, hipStream_t st);
// Full SGD training, one work-group per filter (a.h = channels); gbuf [F, P]
// is gradient scratch.
void launch_cnn_train(const TrainArgs &a, float *gbuf, hipStream_t st);
// One SGD step per filter on explicit batches; gbuf [F, P] scratch.
void launch_cnn_sgd_step(float *w, int F, int m, int C, const float *x, const float *y, int batch, float lr,
                         float *loss, float *gbuf, hipStream_t st);

}  // namespace leafi
