// Host-side state of an index handle and the host algorithms (tree build,
// leaf selection, calibration) of libleafi.
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace leafi {

// ---- tree (tree.cpp) ------------------------------------------------------

struct TreeResult {
  std::vector<std::vector<int64_t>> leaves;  // member ids per leaf (ascending), depth-first order
  // iSAX trees only: per leaf and segment the symbol's bits and the symbol
  // at those bits, [N, S] each (empty for the binary trees)
  std::vector<uint8_t> isax_bits, isax_sym;
};

// Split until every leaf holds <= capacity series.  seg_mu / seg_sd are
// [n, S] fp32 summaries; rule 0 = median, 1 = range midpoint, 2 = iSAX
// (build_isax_tree; S <= 32).
TreeResult build_tree(const std::vector<float> &seg_mu, const std::vector<float> &seg_sd, int64_t n, int S, int m,
                      int capacity, int rule);

// iSAX symbols of up to this many bits per segment.
constexpr int kIsaxMaxBits = 8;
// SAX breakpoints of cardinality 2^bits as fp32: the N(0, 1) quantiles j / 2^bits.
std::vector<float> isax_breakpoints(int bits);
// The iSAX tree over the segment means (see tree.cpp).
TreeResult build_isax_tree(const std::vector<float> &seg_mu, int64_t n, int S, int capacity);

// Per-leaf boxes [N, S, 4] (mu lo, mu hi, sd lo, sd hi), widened by one fp32
// ulp: the members' ranges, or for an iSAX tree each leaf's SAX intervals
// (the deviation unconstrained).
std::vector<float> leaf_boxes(const std::vector<float> &seg_mu, const std::vector<float> &seg_sd, int S,
                              const TreeResult &t);

// ---- leaf selection (tree.cpp) -----------------------------------------------

// Algorithm 3: leaves by size (largest first, ties by id) with size >= th
// while the filters fit in cM bytes.
std::vector<int32_t> select_leaves(const std::vector<int64_t> &sizes, double th, double w, double cM);

// Equations 1-2: the benefit b_i = (1 - p^lb_i) (p^F_i t^S |N_i| - t^F) with
// p^F_i = p_f[i] / a (p_f: the ideal filter rate), and the 0/1 knapsack of
// capacity cM over filters of w bytes each: the leaves with b_i > 0 by
// benefit (largest first, ties by id), at most floor(cM / w) of them.
// benefit (optional) receives b [N].
std::vector<int32_t> select_knapsack(const std::vector<int64_t> &sizes, const std::vector<double> &p_lb,
                                     const std::vector<double> &p_f, double a, double tS, double tF, double w,
                                     double cM, std::vector<double> *benefit);

// ---- calibration (calib.cpp) ---------------------------------------------------

struct CalibInput {
  int nc = 0;        // calibration queries
  int N = 0;         // leaves
  int F = 0;         // filters
  int kmax = 0;      // entries per (query, leaf) list
  std::vector<int32_t> order;       // [nc, N] visit order
  std::vector<double> leaf_d;       // [nc, N, kmax] per-leaf sorted distances (+inf padding)
  std::vector<int64_t> leaf_ids;    // [nc, N, kmax] ids (-1 padding)
  std::vector<float> dfilt;         // [nc, F] filter predictions
  std::vector<int32_t> leaf_of_filter;  // [F]
};

// Algorithm 4 for one k: offsets [n_targets, F] for the given targets.
// mapping 0 = step, 1 = Steffen; corrected = finite-sample target correction.
std::vector<float> calibrate_k(const CalibInput &in, int k, const std::vector<float> &targets, int mapping,
                               bool corrected);

// Steffen (1990) monotone interpolant evaluation through (x, y) (x strictly
// increasing), clamped to the end values outside [x0, xn].
double steffen_eval(const std::vector<double> &x, const std::vector<double> &y, double t);

// ---- index handle -----------------------------------------------------------------

struct Filters {
  int F = 0;
  int arch = LEAFI_FILTER_MLP;         // LEAFI_FILTER_MLP or LEAFI_FILTER_CNN
  int h = 0;                           // MLP hidden width, or CNN channels
  int64_t P = 0;                       // floats per filter
  DevBuf<float> w;                     // [F, P]
  std::vector<int32_t> leaf_of_filter; // [F]
  DevBuf<int32_t> filt_of_leaf;        // [N], -1 = no filter
};

struct Calibration {
  std::vector<int32_t> ks;
  std::vector<float> targets;
  std::vector<float> h_offsets;   // [pairs, F]
  DevBuf<float> offsets;          // [pairs, F]
  DevBuf<int32_t> pair_k;         // [pairs]
  DevBuf<float> pair_t;           // [pairs]
  int pairs() const { return static_cast<int>(ks.size() * targets.size()); }
};

// Scratch buffers of one search / all-pairs pass, grown on demand.
// Planned batch searches have at most this many regular rounds.
constexpr int kMaxPlannedRounds = 8;
// Executable graphs kept per index (least recently used evicted).
constexpr int kGraphCacheSize = 8;

struct GraphEntry {
  std::vector<uint64_t> key;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;
};

// Captured planned searches, keyed by everything baked into their launches.
struct GraphCache {
  std::vector<GraphEntry> entries;
  std::vector<std::vector<uint64_t>> pending;  // keys of recent uncaptured planned batches
  // keys of recent planned batches that overflowed their item capacity: the
  // same shape runs host-driven rounds right away from then on
  std::vector<std::vector<uint64_t>> overflowed;
  hipStream_t cap = nullptr;      // capture stream (default priority)
  bool off = false, off_timed = false;  // capture failed once: do not retry
  std::string why;
  uint64_t tick = 0;
  void clear() {
    for (auto &e : entries)
      if (e.exec) (void)hipGraphExecDestroy(e.exec);
    entries.clear();
    pending.clear();
    overflowed.clear();
  }
};

// Training set kept by leafi_train_filters (keep_examples): raw queries and
// the per-filter example table.
struct Examples {
  int64_t nq = 0;
  int n_ex = 0, n_train = 0;
  DevBuf<float> q;              // [nq, m] raw
  std::vector<int32_t> ex_q;    // [F, n_ex] query of each example
  DevBuf<float> ex_y;           // [F, n_ex] d^L targets
  int max_epochs = 0;
  std::vector<int32_t> epochs;  // [F] epochs each filter ran
  std::vector<float> val_trace; // [F, max_epochs] validation MSE after each epoch (NaN after the last)
};

struct Workspace {
  // queries
  DevBuf<float> q32, qn16, qeps, qstat, lb, dfilt, tau;
  DevBuf<uint16_t> q16;
  DevBuf<int32_t> order, cursor, kq, pair, res_cnt, res_row, qitem_cnt, qitem_leaf, qitem_idx;
  DevBuf<double> res_d2;
  // leaves
  DevBuf<int32_t> leaf_cnt, leaf_fill, leaf_istart, tile_start;
  // items
  DevBuf<int32_t> item_q, item_leaf, item_row, item_cnt, item_live, fb_q, fb_leaf;
  DevBuf<double> item_d2;
  DevBuf<float> item_bound;
  DevBuf<uint64_t> cand;
  DevBuf<int64_t> plist;        // filter pairs to evaluate (q * N + visit position)
  DevBuf<int32_t> pcnt;
  DevBuf<float> lbs, dfo;       // [nq, N] in visit order: summary bound, filter pruning value
  DevBuf<float> qbound;         // [nq] a search round's bound on each query's k-th distance (rerank)
  DevBuf<int32_t> ptile;        // prefix of the filters' 16-query inference tiles [F + 1]
  DevBuf<int64_t> ctl;
  std::vector<int64_t> h_ctl;
  const int32_t *leaf_n = nullptr;  // the index's leaf sizes (device), for views()
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<hipEvent_t> sev;  // per planned round: scan begin / end
  GraphCache graphs;
};

}  // namespace leafi

struct leafi_index {
  leafi::AllocFns alloc;  // the caller's allocator (both NULL: hipMalloc / hipFree)
  int device = 0;
  bool built = false;
  int64_t n = 0;
  int m = 0;
  int S = 0;
  int N = 0;
  int64_t rows = 0;     // padded rows
  // per scan chunk size kRowAlign << j: chunks of the largest leaf, and over all leaves
  int chunks_max[leafi::kChunkSizes] = {};
  int64_t chunks_total[leafi::kChunkSizes] = {};
  int max_chunks_for(int chunk) const { return chunks_max[leafi::chunk_log(chunk)]; }
  int64_t total_chunks_for(int chunk) const { return chunks_total[leafi::chunk_log(chunk)]; }
  // leaf store (device)
  leafi::DevBuf<float> x32, xn16, boxes, leaf_eps;
  float leaf_eps_max = 0.0f;  // the largest leaf_eps
  leafi::DevBuf<float> boxes_t;  // the boxes as [S][4][N]: one value of every leaf, contiguous
  leafi::DevBuf<uint16_t> x16;
  leafi::DevBuf<int64_t> rowid, leaf_off;
  leafi::DevBuf<int32_t> leaf_n;
  // host copies
  std::vector<int64_t> h_leaf_off, h_leaf_n, h_members;
  std::vector<float> h_boxes;
  leafi::Filters filt;
  leafi::Examples examples;
  leafi::Calibration cal;
  leafi::Workspace ws;
  int num_cus = 256;
  // Item capacity of a planned batch's passes (leafi_set_plan_capacity);
  // 0: as many as the planned buffer limit holds.
  int64_t plan_cap_items = 0;
  // The largest round item and tile counts a planned batch that overflowed
  // met (in its host-driven rerun): later planned batches are sized for them.
  int64_t plan_items_seen = 0;
  int64_t plan_tiles_seen = 0;
  double dev_mem = 0.0;  // the device's memory (bytes)
  // BF16 scan tiling (set by leafi_autotune or leafi_set_tiling): rows and
  // queries per tile
  int tune_chunk = leafi::kChunkRows;
  int tune_mq = 32;
  ~leafi_index();
};
