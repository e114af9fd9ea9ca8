// Host orchestration helpers shared by the C ABI entry points (api.hip) and
// the serving engine (serve.hip).
#pragma once

#include <string>
#include <vector>

#include "index.h"

namespace leafi {

extern thread_local std::string g_last_error;

// Device allocations made while this is in scope go through the handle's allocator.
#define INDEX_ALLOC_SCOPE(ix) ::leafi::AllocScope leafi_alloc_scope_((ix) ? &(ix)->alloc : nullptr)

// Run fn, turning exceptions into LEAFI_E* codes and the thread's message.
template <typename Fn>
int guarded(Fn &&fn) {
  try {
    fn();
    return LEAFI_OK;
  } catch (const Error &e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return LEAFI_ENOMEM;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return LEAFI_EINTERNAL;
  } catch (...) {
    g_last_error = "unknown failure";
    return LEAFI_EINTERNAL;
  }
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

template <typename T>
void h2d(T *dst, const T *src, size_t n, hipStream_t st) {
  if (n) HIP_OK(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, st));
}
template <typename T>
void d2h(T *dst, const T *src, size_t n, hipStream_t st) {
  if (n) HIP_OK(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, st));
}

struct Timing {
  double scan_ms = 0.0;
  double scan_bytes = 0.0;
};

void require_built(const leafi_index *ix);
void fill_f32(float *p, int64_t n, float v, hipStream_t st);
void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
RoundBufs views(Workspace &w);
StoreView store_view(const leafi_index *ix);
QueryView query_view(Workspace &w);
// Grow the per-query workspace for nq queries of up to kmax results.
void ensure_queries(leafi_index *ix, int64_t nq, int kmax);
void ensure_items(leafi_index *ix, int64_t items, int kmax);
// Copy the control words to the host (synchronises the stream).
void read_ctl(leafi_index *ix, hipStream_t st);
// Zero the per-round control words (items, tiles, active, fallback) and the
// per-leaf item counts.
void reset_round(leafi_index *ix, hipStream_t st);
// Zero the per-leaf and per-query item counts before a fallback pass.
void reset_for_fallback(leafi_index *ix, int64_t nq, hipStream_t st);

struct RoundOpts {
  bool may_read = true;         // false: never read counts back (planned / captured sequences)
  int64_t row_bytes = 0;        // > 0: account the round's unique leaf bytes in ctl[kCtlScanBytes]
  hipEvent_t ev_begin = nullptr;  // recorded around the scan kernel when set
  hipEvent_t ev_end = nullptr;
  bool small = false;           // a pass expected to hold few items (rescans): small persistent grids
  bool use_tau = false;         // a search round: the BF16 scan skips rows provably farther than tau
  bool first_leaf = false;      // the batch's first round of one leaf per query, emitted by the layout
                                // itself from the visit order (no prune cascade launch; may_read false)
  bool kp_query = false;        // each query keeps item_kprime(its k) candidates (mixed-k batches)
  bool one_leaf = false;        // at most one leaf per query (a first round of schedule 1): BF16 tiles
                                // of 16 queries, whatever the tuned size (few queries share a leaf)
  int64_t cap_items = 0;        // > 0: the buffers hold this many items and cap_tiles scan tiles,
  int64_t cap_tiles = 0;        // checked on the device (RoundBufs::cap_items); 0: the bound holds
                                // every layout
};

// Capacity of one pass of a planned batch (see planned_cap in api.hip).
struct PassCap {
  int64_t items = 0;
  int64_t tiles = 0;
  bool checked = false;  // below the pass's bound: the layout checks its counts on the device
};
// Lay out the round's items, scan and rerank them (see api.hip).
int64_t scan_round(leafi_index *ix, int64_t nq, bool bf16, int kprime, int kmax, hipStream_t st, Timing *tm,
                   int64_t items_bound = -1, const RoundOpts *ro = nullptr);
void add_scan_time(leafi_index *ix, Timing *tm);
// Upper bound of the bound-sized buffers of a round that reads nothing back.
constexpr double kPlannedLimit = 16.0 * (1 << 30);
// Device bytes a scan pass of items_bound items needs (items and candidate lists).
double round_bytes_bound(const leafi_index *ix, int64_t nq, int64_t items_bound, bool bf16, int kprime, int kmax);
// Queries per scan tile and list capacity of a pass (one_leaf: see RoundOpts).
void pass_geometry(const leafi_index *ix, bool bf16, int kprime, int *mq, int *cap, bool one_leaf = false);
int default_kprime(int kmax, bool bf16);
// d^f - offset for the (query, visit position) pairs listed per filter
// (plist / pcnt, nq queries) with the installed filters, MLP or CNN.
void infer_filter_pairs(leafi_index *ix, int64_t nq, int ftile, hipStream_t st);

// How a batch search runs (from leafi_search_opts).
struct SearchPlan {
  int kmax = 1;
  bool bf16 = true;
  bool filters = false;
  std::vector<int> schedule{1};
  int kprime = 4;
  bool graph = true;  // planned batches may be captured and replayed
  int ftile = 0;      // filter inference tiles: 0 by batch size, 1 small, 2 large
  bool kp_query = true;  // per-query candidate counts (the default kprime); false: kprime for every query
};
SearchPlan make_plan(const leafi_index *ix, const leafi_search_opts *o);
void check_queries(const leafi_index *ix, const float *q, int64_t nq);
// Whether the batch can run as a planned launch sequence (no read-back).
bool can_plan(const leafi_index *ix, int64_t nq, const SearchPlan &p);
// Whether a planned batch has a pass sized below its bound (its overflow
// word must be read back before the results are used).
bool plan_checked(const leafi_index *ix, int64_t nq, const SearchPlan &p);
// Reserve every buffer of a planned batch at its bound (no allocation after).
void prepare_planned(leafi_index *ix, int64_t nq, const SearchPlan &p, bool use_f);
// Enqueue the planned launch sequence of a batch on `st`.
void enqueue_planned(leafi_index *ix, const float *raw, int64_t nq, const int32_t *k_dev, const float *t_dev,
                     const SearchPlan &p, bool use_f, int64_t *ids, float *dists, bool timed, hipStream_t st);

}  // namespace leafi
