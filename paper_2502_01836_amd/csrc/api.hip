// C ABI of libleafi and the host orchestration of its device kernels:
// index build, filter training (Algorithms 1 and 3), auto-tuner fitting
// (Algorithm 4) and the batched round-based search (Algorithm 2).
#include <algorithm>
#include <mutex>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <random>
#include <string>

#include "engine.h"

using namespace leafi;

leafi_index::~leafi_index() {
  if (ws.ev0) (void)hipEventDestroy(ws.ev0);
  if (ws.ev1) (void)hipEventDestroy(ws.ev1);
  for (hipEvent_t e : ws.sev) (void)hipEventDestroy(e);
  ws.graphs.clear();
  if (ws.graphs.cap) (void)hipStreamDestroy(ws.graphs.cap);
}

namespace leafi {

thread_local std::string g_last_error;
thread_local const AllocFns *t_alloc = nullptr;
thread_local Arena *t_arena = nullptr;

void *dev_alloc(size_t bytes, AllocFns *how, bool *from_arena) {
  *how = AllocFns();
  *from_arena = false;
  if (t_arena) {
    const size_t off = (t_arena->used + 255) & ~static_cast<size_t>(255);
    if (off > t_arena->cap || bytes > t_arena->cap - off)
      fail(LEAFI_ENOMEM, "scratch area of " + std::to_string(t_arena->cap) + " bytes exhausted");
    t_arena->used = off + bytes;
    *from_arena = true;
    // a measuring arena (no base) hands out distinct non-null stand-ins
    return t_arena->base ? t_arena->base + off : reinterpret_cast<char *>(off + 256);
  }
  void *p = nullptr;
  if (t_alloc && t_alloc->alloc) {
    if (t_alloc->alloc(t_alloc->ctx, bytes, &p) != 0 || p == nullptr)
      fail(LEAFI_ENOMEM, "the caller's allocator refused " + std::to_string(bytes) + " bytes");
    *how = *t_alloc;
    return p;
  }
  HIP_OK(hipMalloc(&p, bytes));
  return p;
}

void dev_free(void *p, const AllocFns &how, bool from_arena) noexcept {
  if (from_arena || p == nullptr) return;
  if (how.alloc) {
    // like hipFree, wait until no queued work can still touch the block: a
    // caching pool may hand it out again at once
    (void)hipDeviceSynchronize();
    how.free(how.ctx, p);
    return;
  }
  (void)hipFree(p);
}

void require_built(const leafi_index *ix) {
  if (!ix) fail(LEAFI_EINVAL, "index handle is NULL");
  if (!ix->built) fail(LEAFI_ESTATE, "index not built (call leafi_build_index first)");
}

// ---- small kernels of the orchestration --------------------------------------

__global__ void k_fill_f32(float *p, int64_t n, float v) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
// Every query searches the same leaves list[0..cnt).
__global__ void k_fill_allpairs(int32_t *qitem_leaf, int32_t *qitem_cnt, int32_t *leaf_cnt, int64_t nq, int N,
                                const int32_t *list, int cnt) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nq * cnt) return;
  int64_t q = i / cnt;
  int r = static_cast<int>(i - q * cnt);
  qitem_leaf[q * N + r] = list[r];
  if (r == 0) qitem_cnt[q] = cnt;
  if (q == 0) leaf_cnt[list[r]] = static_cast<int32_t>(nq);
}
// Per-query explicit lists (CSR): query q searches list[off[q] .. off[q+1]).
__global__ void k_fill_lists(int32_t *qitem_leaf, int32_t *qitem_cnt, int32_t *leaf_cnt, int64_t nq, int N,
                             const int64_t *off, const int32_t *list) {
  int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  int c = static_cast<int>(off[q + 1] - off[q]);
  for (int r = 0; r < c; ++r) {
    int L = list[off[q] + r];
    qitem_leaf[q * N + r] = L;
    atomicAdd(leaf_cnt + L, 1);
  }
  qitem_cnt[q] = c;
}
// All-pairs mode: queue every item whose certificate does not exceed its own
// k-th distance (each item stands alone).
__global__ void k_item_cert(int64_t n_items, int kmax, RoundBufs b) {
  int64_t it = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (it >= n_items) return;
  int k = b.kq[b.item_q[it]];
  double kth = b.item_cnt[it] >= k ? sqrt(b.item_d2[it * kmax + k - 1]) : __builtin_inf();
  if (!(static_cast<double>(b.item_bound[it]) > kth)) {
    unsigned long long slot = atomicAdd(reinterpret_cast<unsigned long long *>(b.ctl + kCtlFallback), 1ull);
    b.fb_q[slot] = b.item_q[it];
    b.fb_leaf[slot] = b.item_leaf[it];
  }
}
// Training examples from items: d^L of (query, filtered leaf); item query
// indices are relative to the chunk starting at training query q_off.
__global__ void k_items_to_examples(int64_t n_items, int kmax, RoundBufs b, const int32_t *filt_of_leaf, int n_g,
                                    int n_gt, int n_l, int n_ex, float *ex_y, int64_t q_off) {
  int64_t it = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (it >= n_items) return;
  int64_t q = b.item_q[it] + q_off;
  int f = filt_of_leaf[b.item_leaf[it]];
  if (f < 0) return;
  int64_t e;
  if (q < n_gt) e = q;
  else if (q < n_g) e = n_gt + n_l + (q - n_gt);
  else e = n_gt + (q - n_g - static_cast<int64_t>(f) * n_l);
  ex_y[static_cast<int64_t>(f) * n_ex + e] = static_cast<float>(sqrt(b.item_d2[it * kmax]));
}

void fill_f32(float *p, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f32, dim3(ceil_div(n, 256)), dim3(256), 0, st, p, n, v);
  LAUNCH_OK("fill_f32");
}
void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(ceil_div(n, 256)), dim3(256), 0, st, p, n, v);
  LAUNCH_OK("fill_i32");
}

// ---- workspace ----------------------------------------------------------------

void allow_lds(const void *kernel, size_t lds) {
  if (lds <= 65536) return;
  static std::mutex mu;
  static std::vector<std::pair<const void *, size_t>> set;  // the largest limit set per kernel
  std::lock_guard<std::mutex> lk(mu);
  auto it = std::find_if(set.begin(), set.end(), [&](const auto &e) { return e.first == kernel; });
  if (it != set.end() && it->second >= lds) return;
  HIP_OK(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  if (it != set.end()) it->second = lds;
  else set.emplace_back(kernel, lds);
}

RoundBufs views(Workspace &w) {
  // zeroed first, padding included: plan_key copies the struct's bytes
  RoundBufs b;
  std::memset(&b, 0, sizeof b);
  b.cursor = w.cursor.get();
  b.tau = w.tau.get();
  b.kq = w.kq.get();
  b.pair = w.pair.get();
  b.res_cnt = w.res_cnt.get();
  b.res_d2 = w.res_d2.get();
  b.res_row = w.res_row.get();
  b.qitem_cnt = w.qitem_cnt.get();
  b.qitem_leaf = w.qitem_leaf.get();
  b.qitem_idx = w.qitem_idx.get();
  b.leaf_cnt = w.leaf_cnt.get();
  b.leaf_fill = w.leaf_fill.get();
  b.leaf_istart = w.leaf_istart.get();
  b.tile_start = w.tile_start.get();
  b.item_q = w.item_q.get();
  b.item_leaf = w.item_leaf.get();
  b.item_d2 = w.item_d2.get();
  b.item_row = w.item_row.get();
  b.item_cnt = w.item_cnt.get();
  b.item_bound = w.item_bound.get();
  b.item_live = w.item_live.get();
  b.fb_q = w.fb_q.get();
  b.fb_leaf = w.fb_leaf.get();
  b.chunk = kChunkRows;
  b.use_tau = 0;
  b.kp_query = 0;
  b.ctl = w.ctl.get();
  b.leaf_n = w.leaf_n;
  b.cap_items = 0;
  b.cap_tiles = 0;
  return b;
}

StoreView store_view(const leafi_index *ix) {
  StoreView s;
  std::memset(&s, 0, sizeof s);
  s.x32 = ix->x32.get();
  s.x16 = ix->x16.get();
  s.xn16 = ix->xn16.get();
  s.leaf_off = ix->leaf_off.get();
  s.leaf_n = ix->leaf_n.get();
  s.leaf_eps = ix->leaf_eps.get();
  s.m = ix->m;
  s.N = ix->N;
  return s;
}

QueryView query_view(Workspace &w) {
  QueryView q;
  std::memset(&q, 0, sizeof q);
  q.q32 = w.q32.get();
  q.q16 = w.q16.get();
  q.qn16 = w.qn16.get();
  q.qeps = w.qeps.get();
  return q;
}

void ensure_queries(leafi_index *ix, int64_t nq, int kmax) {
  Workspace &w = ix->ws;
  const int64_t m = ix->m, N = ix->N, S = ix->S;
  const int64_t F = std::max(ix->filt.F, 1);
  nq = std::max<int64_t>(nq, 1);
  w.q32.reserve(nq * m);
  w.q16.reserve(nq * m);
  w.qn16.reserve(nq);
  w.qeps.reserve(nq);
  w.qstat.reserve(nq * S * 2);
  w.lb.reserve(nq * N);
  w.order.reserve(nq * N);
  w.lbs.reserve(nq * N);
  w.dfo.reserve(nq * N);
  w.qbound.reserve(nq);
  w.dfilt.reserve(nq * F);
  w.tau.reserve(nq);
  w.cursor.reserve(nq);
  w.kq.reserve(nq);
  w.pair.reserve(nq);
  w.res_cnt.reserve(nq);
  w.res_d2.reserve(nq * kmax);
  w.res_row.reserve(nq * kmax);
  w.qitem_cnt.reserve(nq);
  w.qitem_leaf.reserve(nq * N);
  w.qitem_idx.reserve(nq * N);
  w.leaf_cnt.reserve(N);
  w.leaf_fill.reserve(N);
  w.leaf_istart.reserve(N + 1);
  w.tile_start.reserve(N + 1);
  w.ctl.reserve(kCtlCount);
  w.leaf_n = ix->leaf_n.get();
  if (w.h_ctl.size() < static_cast<size_t>(kCtlCount)) w.h_ctl.resize(kCtlCount);
  if (!w.ev0 && !t_arena) {
    // timing-only events: no system-scope fence (no cache write-back) around the kernels they bracket
    HIP_OK(hipEventCreateWithFlags(&w.ev0, hipEventDisableSystemFence));
    HIP_OK(hipEventCreateWithFlags(&w.ev1, hipEventDisableSystemFence));
  }
}

void ensure_items(leafi_index *ix, int64_t items, int kmax) {
  Workspace &w = ix->ws;
  if (items <= 0) return;
  if (static_cast<int64_t>(w.item_q.size()) < items || static_cast<int64_t>(w.item_d2.size()) < items * kmax) {
    int64_t cap = std::max<int64_t>(items, static_cast<int64_t>(w.item_q.size()) * 3 / 2);
    w.item_q.alloc(cap);
    w.item_leaf.alloc(cap);
    w.item_cnt.alloc(cap);
    w.item_bound.alloc(cap);
    w.item_live.alloc(cap);
    w.fb_q.alloc(cap);
    w.fb_leaf.alloc(cap);
    w.item_d2.alloc(cap * kmax);
    w.item_row.alloc(cap * kmax);
  }
}

void read_ctl(leafi_index *ix, hipStream_t st) {
  Workspace &w = ix->ws;
  d2h(w.h_ctl.data(), w.ctl.get(), kCtlCount, st);
  HIP_OK(hipStreamSynchronize(st));
}

// Zero the per-round control words (items, tiles, active, fallback) and the
// per-leaf item counts; the statistics words keep accumulating.
void reset_round(leafi_index *ix, hipStream_t st) {
  launch_round_reset(views(ix->ws), kCtlRoundWords, ix->N, 0, st);
}

// Before a fallback pass: zero the per-leaf and per-query item counts.  The
// fallback count itself stays: the emit kernel reads it.
void reset_for_fallback(leafi_index *ix, int64_t nq, hipStream_t st) {
  launch_round_reset(views(ix->ws), 0, ix->N, nq, st);
}

// Prepare nq raw queries: normalised copies, lower bounds and visit order.
void prep_queries(leafi_index *ix, const float *raw, int64_t nq, hipStream_t st) {
  Workspace &w = ix->ws;
  launch_qprep(raw, nq, ix->m, ix->S, w.q32.get(), w.q16.get(), w.qn16.get(), w.qeps.get(), w.qstat.get(), st);
  launch_lb(w.qstat.get(), nq, ix->boxes.get(), ix->N, ix->S, ix->m, w.lb.get(), st);
  launch_order(w.lb.get(), nq, ix->N, w.order.get(), w.lbs.get(), st);
}

// Upper bound of scan work-groups per CU; the launch clamps the persistent
// grid to what can be resident at once.
constexpr int kScanBlocksPerCU = 8;
// Device bytes above which a round's item buffers are sized from the actual
// counts (one host read-back) instead of from an upper bound.
constexpr double kPreallocLimit = 1.0 * (1 << 30);


// With the round's item lists in place (qitem_leaf / qitem_cnt / leaf_cnt)
// and the round control words zeroed: lay out items and tiles, scan, rerank.
// items_bound >= 0 is an upper bound of the round's items: buffers are sized
// from it and nothing is read back.  Otherwise the counts are read back
// first.  Returns the item count when it was read back, else -1.
// Rows per scan tile for a pass: the preferred size, doubled while the
// per-item merge of the chunk candidate lists (chunks x kprime keys) would
// exceed kMaxRerankKeys.
constexpr int kMaxRerankKeys = 4096;
constexpr int kFp32ChunkRows = 128;  // the FP32 scan streams 4 m bytes per row: finer tiles
int pick_chunk(const leafi_index *ix, int kprime, int pref) {
  int chunk = pref;
  while (chunk < (kRowAlign << (kChunkSizes - 1)) &&
         static_cast<int64_t>(ix->max_chunks_for(chunk)) * kprime > kMaxRerankKeys)
    chunk *= 2;
  return chunk;
}
int pass_chunk(const leafi_index *ix, bool bf16, int kprime) {
  return pick_chunk(ix, kprime, bf16 ? ix->tune_chunk : kFp32ChunkRows);
}
void pass_geometry(const leafi_index *ix, bool bf16, int kprime, int *mq, int *cap, bool one_leaf) {
  scan_geometry(bf16, kprime, bf16 ? (one_leaf ? 16 : ix->tune_mq) : 32, ix->m, mq, cap);
}

int64_t tiles_bound(const leafi_index *ix, int64_t nq, int64_t items_bound, int mq, int chunk) {
  // every leaf has at most nq items, and at most items_bound in all
  const int64_t a = ceil_div(items_bound, mq) * ix->max_chunks_for(chunk) + ix->total_chunks_for(chunk);
  const int64_t b = ceil_div(nq, mq) * ix->total_chunks_for(chunk);
  return std::min(a, b);
}

double round_bytes_bound(const leafi_index *ix, int64_t nq, int64_t items_bound, bool bf16, int kprime, int kmax) {
  int mq, cap;
  pass_geometry(ix, bf16, kprime, &mq, &cap);
  const int chunk = pass_chunk(ix, bf16, kprime);
  return static_cast<double>(items_bound) * (kmax * 12.0 + 32.0) +
         static_cast<double>(tiles_bound(ix, nq, items_bound, mq, chunk)) * mq * kprime * 8.0;
}

int64_t scan_round(leafi_index *ix, int64_t nq, bool bf16, int kprime, int kmax, hipStream_t st, Timing *tm,
                   int64_t items_bound, const RoundOpts *ro) {
  Workspace &w = ix->ws;
  RoundOpts def;
  if (!ro) ro = &def;
  int mq, cap;
  pass_geometry(ix, bf16, kprime, &mq, &cap, ro->one_leaf);
  (void)cap;
  const int chunk = pass_chunk(ix, bf16, kprime);
  RoundBufs b0 = views(w);
  b0.chunk = chunk;
  b0.use_tau = ro->use_tau ? 1 : 0;
  b0.kp_query = ro->kp_query ? 1 : 0;
  b0.cap_items = ro->cap_items;
  b0.cap_tiles = ro->cap_tiles;
  // a pass with few items (rescans, a first round of one leaf per query)
  // and preallocated buffers lays out and places its items in one
  // single-work-group launch (below, once the buffers are final)
  constexpr int64_t kFusedItems = 8192;
  const bool fused = !ro->may_read && (ro->small || (items_bound >= 0 && items_bound <= kFusedItems));
  // otherwise, with up to kLayoutLdsMax leaves, every work-group of the
  // placement recomputes the leaf scan itself (one launch instead of two)
  const bool fused_grid = !ro->may_read && !fused && ix->N <= kLayoutLdsMax;
  if (ro->first_leaf && (ro->may_read || ix->N > kLayoutLdsMax))
    fail(LEAFI_EINTERNAL, "scan_round: first-leaf layout needs a planned round and at most 4096 leaves");
  if (!ro->first_leaf && !fused && !fused_grid) launch_leaf_scan(ix->N, ix->leaf_off.get(), mq, ro->row_bytes, b0, st);
  int64_t items = -1, tiles;
  const int64_t tb = items_bound < 0        ? -1
                     : ro->cap_tiles > 0 ? std::min(ro->cap_tiles, tiles_bound(ix, nq, items_bound, mq, chunk))
                                         : tiles_bound(ix, nq, items_bound, mq, chunk);
  const double bytes = items_bound >= 0 ? static_cast<double>(items_bound) * (kmax * 12.0 + 32.0) +
                                              static_cast<double>(tb) * mq * kprime * 8.0
                                        : 0.0;
  if (!ro->may_read && (items_bound < 0 || bytes > std::max(kPlannedLimit, 0.4 * ix->dev_mem)))
    fail(LEAFI_EINTERNAL, "scan_round: planned round exceeds its preallocation bound");
  if (ro->may_read && (items_bound < 0 || bytes > kPreallocLimit)) {
    read_ctl(ix, st);
    items = w.h_ctl[kCtlItems];
    tiles = w.h_ctl[kCtlTiles];
    if (items == 0) return 0;
  } else {
    items = -1;
    tiles = tb;
  }
  ensure_items(ix, items >= 0 ? items : std::max<int64_t>(items_bound, 1), kmax);
  w.cand.reserve(static_cast<size_t>(std::max<int64_t>(tiles, 1)) * mq * kprime);
  RoundBufs b = views(w);
  b.chunk = chunk;
  b.use_tau = ro->use_tau ? 1 : 0;
  b.kp_query = ro->kp_query ? 1 : 0;
  b.cap_items = ro->cap_items;
  b.cap_tiles = ro->cap_tiles;
  StoreView s = store_view(ix);
  QueryView q = query_view(w);
  if (ro->first_leaf)
    launch_first_round_layout(nq, ix->N, w.order.get(), ix->leaf_off.get(), ix->leaf_n.get(), mq, ro->row_bytes, b,
                              st);
  else if (fused) launch_leaf_scan_scatter(nq, ix->N, ix->leaf_off.get(), mq, ro->row_bytes, b, st);
  else if (fused_grid) launch_layout_scatter(nq, ix->N, ix->leaf_off.get(), mq, ro->row_bytes, b, st);
  else launch_scatter(nq, ix->N, b, st);
  int grid_scan = static_cast<int>(std::min<int64_t>(std::max<int64_t>(tiles, 1),
                                                     static_cast<int64_t>(ix->num_cus) * (ro->small ? 1 : kScanBlocksPerCU)));
  hipEvent_t e0 = ro->ev_begin ? ro->ev_begin : (tm ? w.ev0 : nullptr);
  hipEvent_t e1 = ro->ev_end ? ro->ev_end : (tm ? w.ev1 : nullptr);
  // Outside graph capture the BF16 scan's own dispatch carries the timing
  // events (start and stop of the kernel itself); under capture they are
  // separate event-record nodes around it.
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (e0 || e1) HIP_OK(hipStreamIsCapturing(st, &cs));
  const bool ext = bf16 && cs == hipStreamCaptureStatusNone;
  if (e0 && !ext) HIP_OK(hipEventRecord(e0, st));
  if (bf16) launch_scan_bf16(s, q, b, mq, kprime, w.cand.get(), grid_scan, st, ext ? e0 : nullptr, ext ? e1 : nullptr);
  else launch_scan_fp32(s, q, b, mq, kprime, w.cand.get(), grid_scan, st);
  if (e1 && !ext) HIP_OK(hipEventRecord(e1, st));
  int64_t ib = items >= 0 ? items : std::max<int64_t>(items_bound, 1);
  // one wavefront per item, a persistent grid of what is resident at once
  // (three four-wavefront work-groups per CU)
  int grid_r = static_cast<int>(std::min<int64_t>(ib, static_cast<int64_t>(ix->num_cus) * (ro->small ? 1 : 12)));
  // a search round's rerank skips candidates that cannot enter their query's
  // top k; not in a round of one leaf per query, whose bound comes from that
  // one item's own keys: it certifies no item and trims few candidates
  const bool bound = bf16 && ro->use_tau && !ro->one_leaf;
  if (bound) {
    launch_query_bound(s, q, b, nq, mq, kprime, kmax, ix->max_chunks_for(chunk), ix->leaf_eps_max, w.cand.get(),
                       w.qbound.get(), st);
  }
  launch_item_rerank(s, q, b, mq, kprime, kmax, bf16, w.cand.get(), grid_r, ix->max_chunks_for(chunk), st,
                     bound ? w.qbound.get() : nullptr);
  return items;
}

void add_scan_time(leafi_index *ix, Timing *tm) {
  if (!tm) return;
  float ms = 0.0f;
  HIP_OK(hipEventSynchronize(ix->ws.ev1));
  HIP_OK(hipEventElapsedTime(&ms, ix->ws.ev0, ix->ws.ev1));
  tm->scan_ms += ms;
}

int default_kprime(int kmax, bool bf16) {
  int kp = bf16 ? 4 * kmax : kmax + 8;
  kp = std::min(kp, 128);
  kp = std::max(kp, kmax);
  return std::min(kp, 256);
}

// Bytes of one leaf-store row as the scan of that precision reads it.
int64_t scan_row_bytes(const leafi_index *ix, bool bf16) { return bf16 ? 2LL * ix->m + 4 : 4LL * ix->m; }

// Queries, lower bounds, visit order, (k, target) pair, batch state.
void begin_batch(leafi_index *ix, const float *raw, int64_t nq, const int32_t *k_dev, const float *t_dev,
                 const SearchPlan &p, bool use_f, hipStream_t st) {
  Workspace &w = ix->ws;
  launch_query_setup(raw, nq, ix->m, ix->S, ix->boxes.get(), ix->boxes_t.get(), ix->N, w.q32.get(), w.q16.get(), w.qn16.get(),
                     w.qeps.get(), w.qstat.get(), w.lb.get(),
                     w.order.get(), w.lbs.get(), k_dev, t_dev, use_f ? ix->cal.pairs() : 0,
                     use_f ? ix->cal.pair_k.get() : nullptr, use_f ? ix->cal.pair_t.get() : nullptr, p.kmax,
                     views(w), ix->filt.F, use_f ? w.pcnt.get() : nullptr, st);
}

// After the first round has set tau: d^f for every (query, filtered leaf)
// pair a later round can still test.  tau only decreases, so this covers all
// later rounds (filter-pair counts were zeroed by begin_batch).
void infer_filter_pairs(leafi_index *ix, int64_t nq, int ftile, hipStream_t st) {
  Workspace &w = ix->ws;
  if (ix->filt.arch == LEAFI_FILTER_CNN)
    launch_cnn_infer_pairs(ix->filt.w.get(), ix->filt.F, ix->m, ix->filt.h, w.q32.get(), w.plist.get(), w.pcnt.get(),
                           nq, ix->N, w.pair.get(), ix->cal.offsets.get(), w.dfo.get(), st);
  else
    launch_mlp_infer_pairs(ix->filt.w.get(), ix->filt.F, ix->m, ix->filt.h, w.q32.get(), w.plist.get(),
                           w.pcnt.get(), nq, ix->N, w.pair.get(), ix->cal.offsets.get(), w.ptile.get(), w.dfo.get(), st,
                           ftile);
}

// d^f of every (query, filter) with the installed filters: out [nq, F].
void infer_filters_dense(leafi_index *ix, const float *x, int64_t nq, float *out, hipStream_t st) {
  if (ix->filt.arch == LEAFI_FILTER_CNN) launch_cnn_infer(ix->filt.w.get(), ix->filt.F, ix->m, ix->filt.h, x, nq, out, st);
  else launch_mlp_infer(ix->filt.w.get(), ix->filt.F, ix->m, ix->filt.h, x, nq, out, st);
}

void eval_filters(leafi_index *ix, int64_t nq, int ftile, hipStream_t st) {
  Workspace &w = ix->ws;
  launch_filter_pairs(nq, ix->N, w.lbs.get(), w.order.get(), ix->filt.filt_of_leaf.get(), views(w), w.plist.get(),
                      w.pcnt.get(), w.dfo.get(), st);
  infer_filter_pairs(ix, nq, ftile, st);
}

// The filter-pair selection done by a merge (see launch_query_merge).
FilterPairArgs filter_pair_args(leafi_index *ix) {
  Workspace &w = ix->ws;
  FilterPairArgs fp;
  fp.lbs = w.lbs.get();
  fp.order = w.order.get();
  fp.filt_of_leaf = ix->filt.filt_of_leaf.get();
  fp.plist = w.plist.get();
  fp.pcnt = w.pcnt.get();
  fp.dfo = w.dfo.get();
  return fp;
}

void launch_round_worklist(leafi_index *ix, int64_t nq, int want, bool f_now, hipStream_t st, bool append) {
  Workspace &w = ix->ws;
  launch_worklist(nq, ix->N, w.lbs.get(), w.order.get(), f_now ? w.dfo.get() : nullptr, ix->leaf_n.get(), want,
                  views(w), st, nullptr, nullptr, append);
}

void stats_from_ctl(const leafi_index *ix, leafi_search_stats *stats) {
  const std::vector<int64_t> &c = ix->ws.h_ctl;
  stats->leaves_scanned += c[kCtlScanned];
  stats->leaves_lb_pruned += c[kCtlLbPruned];
  stats->leaves_filter_pruned += c[kCtlFPruned];
  stats->series_scanned += c[kCtlSeries];
  stats->fallback_items += c[kCtlFbTotal];
  stats->rounds += static_cast<int32_t>(c[kCtlRounds]);
  stats->scan_bytes += static_cast<double>(c[kCtlScanBytes]);
  stats->filter_evals += c[kCtlFEvals];
}

int planned_rounds(const SearchPlan &p);

// Batched search of nq raw queries (Algorithm 2 in rounds), host-driven: the
// counts of every round are read back, which sizes the buffers from actual
// counts and ends the loop as soon as no query has leaves left.  Serves any
// schedule, including open-ended ones such as the paper's one leaf per round.
// max_items (optional, two entries) receives the largest item and tile
// counts of a round's BF16 scan.
void search_batch(leafi_index *ix, const float *raw, int64_t nq, const int32_t *k_dev, const float *t_dev,
                  const SearchPlan &p, int64_t *ids, float *dists, leafi_search_stats *stats, hipStream_t st,
                  int64_t *max_items = nullptr) {
  Workspace &w = ix->ws;
  const int N = ix->N;
  ensure_queries(ix, nq, p.kmax);
  const int F = ix->filt.F;
  const bool use_f = p.filters && F > 0 && ix->cal.pairs() > 0;
  if (use_f) {
    w.plist.reserve(static_cast<size_t>(F) * nq);
    w.pcnt.reserve(F);
    w.ptile.reserve(F + 1);
  }
  begin_batch(ix, raw, nq, k_dev, t_dev, p, use_f, st);
  const int kprime_fb = default_kprime(p.kmax, false);
  Timing tm;
  RoundOpts ro;
  ro.row_bytes = scan_row_bytes(ix, p.bf16);
  ro.use_tau = true;
  ro.kp_query = p.kp_query;
  RoundOpts rfb;  // the exact FP32 rescan pass
  rfb.kp_query = p.kp_query;
  bool filters_ready = false;
  // A schedule that ends in 0 has a known last round: uncertified items of an
  // earlier round are rescanned by the next round's scan, as the planned
  // sequence does; otherwise (and after the last round) by an exact FP32 pass
  // right away.
  const int R = planned_rounds(p);
  int64_t deferred = 0;  // rescans the last merge left queued for this round
  for (int r = 0;; ++r) {
    if (use_f && r > 0 && !filters_ready) {
      eval_filters(ix, nq, p.ftile, st);
      filters_ready = true;
    }
    if (r > 0 && deferred == 0) reset_round(ix, st);
    const int want = p.schedule[std::min<size_t>(r, p.schedule.size() - 1)];
    launch_round_worklist(ix, nq, want, use_f && filters_ready, st, deferred > 0);
    const int64_t bound = nq * static_cast<int64_t>(want == 0 ? N : std::min(want, N)) + deferred;
    ro.one_leaf = r == 0 && want == 1;
    int64_t items = scan_round(ix, nq, p.bf16, p.kprime, p.kmax, st, stats ? &tm : nullptr, bound, &ro);
    if (items == 0) break;
    launch_query_merge(nq, N, p.kmax, true, r > 0, views(w), st);
    read_ctl(ix, st);
    if (w.h_ctl[kCtlItems] == 0) break;
    if (max_items) {
      max_items[0] = std::max(max_items[0], w.h_ctl[kCtlItems]);
      max_items[1] = std::max(max_items[1], w.h_ctl[kCtlTiles]);
    }
    add_scan_time(ix, stats ? &tm : nullptr);
    const int64_t active = w.h_ctl[kCtlActive];
    const int64_t n_fb = w.h_ctl[kCtlFallback];
    deferred = 0;
    if (n_fb > 0) {
      // the merge left each query's rescan list in its item list
      if (R > 0 && r < R - 1) {
        deferred = n_fb;
      } else if (scan_round(ix, nq, false, kprime_fb, p.kmax, st, nullptr, n_fb, &rfb) != 0) {
        launch_query_merge(nq, N, p.kmax, false, true, views(w), st);
      }
    }
    if (active == 0 && deferred == 0) break;
  }
  launch_finalize(nq, p.kmax, ix->rowid.get(), views(w), ids, dists, st);
  if (stats) {
    read_ctl(ix, st);
    stats_from_ctl(ix, stats);
    stats->ms_scan += tm.scan_ms;
    stats->path = 0;
  }
}

// Regular rounds of a schedule that ends in 0 (every survivor): the round
// with the first 0 takes all remaining leaves of every query, so the batch
// has at most that many rounds.  0 if the schedule is open-ended.
int planned_rounds(const SearchPlan &p) {
  for (size_t r = 0; r < p.schedule.size(); ++r)
    if (p.schedule[r] == 0) return static_cast<int>(r) + 1;
  return 0;
}

// Items of round r: its own leaves plus the rescans the previous round left
// (at most that round's items), never more than one per (query, leaf).
int64_t planned_bound(const leafi_index *ix, int64_t nq, const SearchPlan &p, int r) {
  const int want = p.schedule[r];
  const int64_t own = nq * static_cast<int64_t>(want == 0 ? ix->N : std::min(want, ix->N));
  return std::min(nq * static_cast<int64_t>(ix->N), own + (r > 0 ? planned_bound(ix, nq, p, r - 1) : 0));
}

// Capacity of a planned pass (bf16: round r's scan; else the exact rescan
// pass after round r): items and scan tiles.  Its bound, with tiles from
// tiles_bound, when buffers of that size fit the planned limit.  Else the
// largest item count whose bound-sized buffers fit the limit; or, for a
// round's scan after a planned batch of this index overflowed, a quarter
// more items and tiles than the largest round its host-driven rerun met
// (plan_items_seen, plan_tiles_seen), as long as those buffers fit 40 % of
// the device's memory; never more items than the index's plan_cap_items when
// that is set.  A pass below its bound checks both counts on the device
// (RoundBufs::cap_items, cap_tiles).
PassCap planned_cap(const leafi_index *ix, int64_t nq, const SearchPlan &p, int r, bool bf16) {
  const int64_t bnd = planned_bound(ix, nq, p, r);
  const int kp = bf16 ? p.kprime : default_kprime(p.kmax, false);
  // one first-leaf round per query is sized with its one-leaf tiles
  const bool one = bf16 && r == 0 && p.schedule[0] == 1;
  int mq, lcap;
  pass_geometry(ix, bf16, kp, &mq, &lcap, one);
  const int chunk = pass_chunk(ix, bf16, kp);
  auto bytes = [&](int64_t items, int64_t tiles) {
    return static_cast<double>(items) * (p.kmax * 12.0 + 32.0) + static_cast<double>(tiles) * mq * kp * 8.0;
  };
  auto tb = [&](int64_t items) { return tiles_bound(ix, nq, items, mq, chunk); };
  PassCap c{bnd, tb(bnd), false};
  if (bytes(c.items, c.tiles) > kPlannedLimit) {
    int64_t lo = 0, hi = bnd;  // fits(lo), !fits(hi)
    while (hi - lo > 1) {
      const int64_t mid = lo + (hi - lo) / 2;
      (bytes(mid, tb(mid)) <= kPlannedLimit ? lo : hi) = mid;
    }
    c = PassCap{lo, tb(lo), true};
    if (bf16 && ix->plan_items_seen > 0) {
      const int64_t it = std::min(bnd, ix->plan_items_seen + ix->plan_items_seen / 4);
      const int64_t tl = std::min(tb(it), ix->plan_tiles_seen + ix->plan_tiles_seen / 4);
      if (it > c.items && bytes(it, tl) <= 0.4 * ix->dev_mem) c = PassCap{it, tl, true};
    }
  }
  if (ix->plan_cap_items > 0 && ix->plan_cap_items < c.items)
    c = PassCap{ix->plan_cap_items, std::min(c.tiles, tb(ix->plan_cap_items)), true};
  c.checked = c.items < bnd || c.tiles < tb(bnd);
  return c;
}

// Every pass's capacity of a planned batch (the rounds' scans, then the rescan pass).
std::vector<int64_t> plan_caps(const leafi_index *ix, int64_t nq, const SearchPlan &p) {
  std::vector<int64_t> v;
  const int R = planned_rounds(p);
  for (int r = 0; r <= R; ++r) {
    if (R == 0) break;
    const PassCap c = r < R ? planned_cap(ix, nq, p, r, true) : planned_cap(ix, nq, p, R - 1, false);
    v.push_back(c.items);
    v.push_back(c.tiles);
  }
  return v;
}

// Whether any pass of a planned batch is sized below its bound (its results
// are then valid only if no round overflowed: the host checks, see
// search_planned).
bool plan_checked(const leafi_index *ix, int64_t nq, const SearchPlan &p) {
  const int R = planned_rounds(p);
  for (int r = 0; r < R; ++r)
    if (planned_cap(ix, nq, p, r, true).checked) return true;
  return R > 0 && planned_cap(ix, nq, p, R - 1, false).checked;
}

// Whether a batch can run as a planned sequence: a bounded number of rounds,
// each pass holding at least one item within the planned limit.
bool can_plan(const leafi_index *ix, int64_t nq, const SearchPlan &p) {
  const int R = planned_rounds(p);
  if (R == 0 || R > kMaxPlannedRounds || !p.bf16) return false;
  for (int r = 0; r < R; ++r)
    if (planned_cap(ix, nq, p, r, true).items < 1) return false;
  return planned_cap(ix, nq, p, R - 1, false).items >= 1;
}

// Reserve every buffer a planned sequence touches at its bound, so that
// enqueueing it allocates nothing (a requirement of graph capture).
void prepare_planned(leafi_index *ix, int64_t nq, const SearchPlan &p, bool use_f) {
  Workspace &w = ix->ws;
  ensure_queries(ix, nq, p.kmax);
  const int F = ix->filt.F;
  if (use_f) {
    w.plist.reserve(static_cast<size_t>(F) * nq);
    w.pcnt.reserve(F);
    w.ptile.reserve(F + 1);
  }
  const int kprime_fb = default_kprime(p.kmax, false);
  int64_t items = 1;
  size_t cand = 1;
  const int R = planned_rounds(p);
  for (int r = 0; r < R; ++r) {
    for (bool bf : {true, false}) {
      if (!bf && r != R - 1) continue;  // the exact rescan pass follows the last round only
      const PassCap c = planned_cap(ix, nq, p, r, bf);
      items = std::max(items, c.items);
      const int kp = bf ? p.kprime : kprime_fb;
      int mq, cap;
      pass_geometry(ix, bf, kp, &mq, &cap, bf && r == 0 && p.schedule[0] == 1);
      cand = std::max(cand, static_cast<size_t>(std::max<int64_t>(c.tiles, 1)) * mq * kp);
    }
  }
  ensure_items(ix, items, p.kmax);
  w.cand.reserve(cand);
  if (w.sev.empty() && !t_arena) {
    w.sev.resize(2 * kMaxPlannedRounds);
    for (auto &e : w.sev) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  }
}

// The whole batch as a fixed launch sequence with no host read-back: each
// round is the prune cascade, scan, rerank and merge; the items a merge
// could not certify are rescanned by the next round's scan (its cascade
// appends the round's own leaves after them), and after the last round by an
// exact FP32 pass whose size is read on the device (an empty pass exits at
// once).  With `timed`, per-round events bracket the scan.  Launches saved
// against that plain sequence (results are the same):
//  * a first round of one leaf per query takes each query's first leaf in
//    its visit order (tau is +inf, no filter is evaluated yet): its layout
//    emits it, with no prune cascade launch;
//  * the filter pairs need only an upper bound of tau (a larger tau selects
//    a superset, and every pair it adds is pruned by its bound anyway), so
//    the first round's merge selects them from its own new tau, and their
//    inference runs right after it.
void enqueue_planned(leafi_index *ix, const float *raw, int64_t nq, const int32_t *k_dev, const float *t_dev,
                     const SearchPlan &p, bool use_f, int64_t *ids, float *dists, bool timed, hipStream_t st) {
  Workspace &w = ix->ws;
  const int N = ix->N;
  const int kprime_fb = default_kprime(p.kmax, false);
  begin_batch(ix, raw, nq, k_dev, t_dev, p, use_f, st);
  const int R = planned_rounds(p);
  // No reset launches: the prune cascade zeroes the round's control words and
  // every merge leaves the per-leaf item counts at its queued rescans.
  for (int r = 0; r < R; ++r) {
    const bool first_leaf = r == 0 && p.schedule[0] == 1 && ix->N <= kLayoutLdsMax;
    if (r == 0 && !first_leaf) launch_round_worklist(ix, nq, p.schedule[r], false, st, false);
    const PassCap pc = planned_cap(ix, nq, p, r, true);
    const int64_t bnd = pc.items;
    RoundOpts ro;
    ro.cap_items = pc.checked ? pc.items : 0;
    ro.cap_tiles = pc.checked ? pc.tiles : 0;
    ro.may_read = false;
    ro.first_leaf = first_leaf;
    ro.one_leaf = r == 0 && p.schedule[0] == 1;
    ro.use_tau = true;
    ro.kp_query = p.kp_query;
    ro.row_bytes = scan_row_bytes(ix, true);
    if (timed) {
      ro.ev_begin = w.sev[2 * r];
      ro.ev_end = w.sev[2 * r + 1];
    }
    scan_round(ix, nq, true, p.kprime, p.kmax, st, nullptr, bnd, &ro);
    const bool last = r == R - 1;
    const bool filters_next = use_f && r == 0 && !last;
    // rounds after the first may rescan a row the previous round merged
    launch_query_merge(nq, N, p.kmax, true, r > 0, views(w), st, nullptr, nullptr, nullptr,
                       filters_next ? filter_pair_args(ix) : FilterPairArgs());
    if (filters_next) infer_filter_pairs(ix, nq, p.ftile, st);
    if (!last) {
      launch_round_worklist(ix, nq, p.schedule[r + 1], use_f, st, true);
      continue;
    }
    // exact rescan pass over the lists the last merge left, then the output rows
    RoundOpts rf;
    rf.may_read = false;
    rf.small = true;
    rf.kp_query = p.kp_query;
    const PassCap fc = planned_cap(ix, nq, p, r, false);
    rf.cap_items = fc.checked ? fc.items : 0;
    rf.cap_tiles = fc.checked ? fc.tiles : 0;
    scan_round(ix, nq, false, kprime_fb, p.kmax, st, nullptr, fc.items, &rf);
    launch_query_merge(nq, N, p.kmax, false, true, views(w), st, ix->rowid.get(), ids, dists);
  }
}

// Identity of a planned sequence: every value and device address baked into
// its launches.  A graph is replayed only for an identical key.
std::vector<uint64_t> plan_key(leafi_index *ix, const float *raw, int64_t nq, const int32_t *k_dev,
                               const float *t_dev, const SearchPlan &p, bool use_f, const int64_t *ids,
                               const float *dists, bool timed) {
  Workspace &w = ix->ws;
  std::vector<uint64_t> k;
  auto put = [&](const void *ptr, size_t bytes) {
    const size_t n0 = k.size();
    k.resize(n0 + (bytes + 7) / 8, 0);
    std::memcpy(k.data() + n0, ptr, bytes);
  };
  auto ptr = [&](const void *q) { k.push_back(reinterpret_cast<uintptr_t>(q)); };
  RoundBufs b = views(w);
  QueryView q = query_view(w);
  StoreView s = store_view(ix);
  put(&b, sizeof b);
  put(&q, sizeof q);
  put(&s, sizeof s);
  for (int64_t v : {nq, static_cast<int64_t>(p.kmax), static_cast<int64_t>(p.kprime), static_cast<int64_t>(use_f),
                    static_cast<int64_t>(timed), static_cast<int64_t>(ix->N), static_cast<int64_t>(ix->m),
                    static_cast<int64_t>(ix->S), static_cast<int64_t>(ix->filt.F), static_cast<int64_t>(ix->filt.h),
                    static_cast<int64_t>(ix->filt.arch), static_cast<int64_t>(ix->cal.pairs()), ix->rows,
                    static_cast<int64_t>(ix->tune_chunk), static_cast<int64_t>(ix->tune_mq),
                    static_cast<int64_t>(p.ftile), static_cast<int64_t>(p.kp_query), ix->plan_cap_items,
                    ix->plan_items_seen, ix->plan_tiles_seen,
                    static_cast<int64_t>(__builtin_bit_cast(uint32_t, ix->leaf_eps_max))})
    k.push_back(static_cast<uint64_t>(v));
  for (int r : p.schedule) k.push_back(static_cast<uint64_t>(r));
  for (const void *a : {static_cast<const void *>(raw), static_cast<const void *>(k_dev),
                        static_cast<const void *>(t_dev), static_cast<const void *>(ids),
                        static_cast<const void *>(dists), static_cast<const void *>(w.cand.get()),
                        static_cast<const void *>(w.plist.get()), static_cast<const void *>(w.pcnt.get()),
                        static_cast<const void *>(w.dfo.get()), static_cast<const void *>(w.lbs.get()),
                        static_cast<const void *>(w.order.get()), static_cast<const void *>(w.qstat.get()),
                        static_cast<const void *>(ix->boxes.get()), static_cast<const void *>(ix->boxes_t.get()),
                        static_cast<const void *>(ix->rowid.get()),
                        static_cast<const void *>(ix->filt.w.get()), static_cast<const void *>(ix->filt.filt_of_leaf.get()),
                        static_cast<const void *>(ix->cal.offsets.get()), static_cast<const void *>(ix->cal.pair_k.get()),
                        static_cast<const void *>(ix->cal.pair_t.get()), static_cast<const void *>(w.ptile.get()),
                        static_cast<const void *>(w.qbound.get())})
    ptr(a);
  if (timed)
    for (hipEvent_t e : w.sev) ptr(e);
  return k;
}

// Capture the planned sequence into an executable graph; nullptr (and the
// cache disabled for this kind, with the reason kept) if capture fails.
hipGraphExec_t capture_planned(leafi_index *ix, const std::vector<uint64_t> &key, const float *raw, int64_t nq,
                               const int32_t *k_dev, const float *t_dev, const SearchPlan &p, bool use_f,
                               int64_t *ids, float *dists, bool timed) {
  GraphCache &g = ix->ws.graphs;
  if (!g.cap) HIP_OK(hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HIP_OK(hipStreamBeginCapture(g.cap, hipStreamCaptureModeRelaxed));
  try {
    enqueue_planned(ix, raw, nq, k_dev, t_dev, p, use_f, ids, dists, timed, g.cap);
  } catch (const Error &e) {
    (void)hipStreamEndCapture(g.cap, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    (timed ? g.off_timed : g.off) = true;
    g.why = e.what();
    return nullptr;
  }
  hipError_t e1 = hipStreamEndCapture(g.cap, &graph);
  hipError_t e2 = e1 == hipSuccess ? hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) : e1;
  if (graph) (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) {
    (void)hipGetLastError();
    (timed ? g.off_timed : g.off) = true;
    g.why = std::string("graph capture: ") + hipGetErrorString(e2);
    return nullptr;
  }
  // nothing may have been reallocated while capturing
  if (plan_key(ix, raw, nq, k_dev, t_dev, p, use_f, ids, dists, timed) != key) {
    (void)hipGraphExecDestroy(exec);
    return nullptr;
  }
  return exec;
}

// Planned batch search.  The first batch of a given shape runs the sequence
// as ordinary launches; from the second identical batch on it is captured
// once into a graph and replayed (up to kGraphCacheSize shapes are kept).
void search_planned(leafi_index *ix, const float *raw, int64_t nq, const int32_t *k_dev, const float *t_dev,
                    const SearchPlan &p, int64_t *ids, float *dists, leafi_search_stats *stats, hipStream_t st) {
  Workspace &w = ix->ws;
  const bool use_f = p.filters && ix->filt.F > 0 && ix->cal.pairs() > 0;
  const bool timed = stats != nullptr;
  prepare_planned(ix, nq, p, use_f);
  GraphCache &g = w.graphs;
  const std::vector<uint64_t> key = plan_key(ix, raw, nq, k_dev, t_dev, p, use_f, ids, dists, timed);
  if (std::find(g.overflowed.begin(), g.overflowed.end(), key) != g.overflowed.end()) {
    // this shape overflowed its planned capacity before: host-driven rounds
    search_batch(ix, raw, nq, k_dev, t_dev, p, ids, dists, stats, st);
    return;
  }
  hipGraphExec_t exec = nullptr;
  int path = 1;
  ++g.tick;
  for (auto &e : g.entries)
    if (e.key == key) {
      exec = e.exec;
      e.last_use = g.tick;
      path = 2;
    }
  const bool allowed = !(timed ? g.off_timed : g.off);
  const bool seen = std::find(g.pending.begin(), g.pending.end(), key) != g.pending.end();
  if (!exec && allowed && p.graph && seen) {
    exec = capture_planned(ix, key, raw, nq, k_dev, t_dev, p, use_f, ids, dists, timed);
    if (exec) {
      if (g.entries.size() >= static_cast<size_t>(kGraphCacheSize)) {
        auto old = std::min_element(g.entries.begin(), g.entries.end(),
                                    [](const GraphEntry &a, const GraphEntry &b) { return a.last_use < b.last_use; });
        (void)hipGraphExecDestroy(old->exec);
        g.entries.erase(old);
      }
      g.entries.push_back(GraphEntry{key, exec, g.tick});
      path = 3;
    }
  }
  if (exec) {
    HIP_OK(hipGraphLaunch(exec, st));
  } else {
    if (!seen) {
      if (g.pending.size() >= static_cast<size_t>(kGraphCacheSize)) g.pending.erase(g.pending.begin());
      g.pending.push_back(key);
    }
    enqueue_planned(ix, raw, nq, k_dev, t_dev, p, use_f, ids, dists, timed, st);
  }
  // A pass sized below its bound: the results stand only if no round held
  // more items than its buffers (the device laid out nothing from then on);
  // otherwise the batch runs again with host-driven rounds, whose buffers
  // follow the actual counts.
  if (stats || plan_checked(ix, nq, p)) {
    read_ctl(ix, st);
    if (w.h_ctl[kCtlOverflow] != 0) {
      // The host-driven run records its largest round; later planned
      // batches of this index are sized for a quarter more (a new shape
      // key).  Where that does not grow any pass's capacity (a set
      // capacity, or the memory limit), the shape runs host-driven rounds at
      // once from now on.
      const std::vector<int64_t> before = plan_caps(ix, nq, p);
      int64_t seen[2] = {0, 0};
      search_batch(ix, raw, nq, k_dev, t_dev, p, ids, dists, stats, st, seen);
      if (stats) stats->path = 4;
      ix->plan_items_seen = std::max(ix->plan_items_seen, seen[0]);
      ix->plan_tiles_seen = std::max(ix->plan_tiles_seen, seen[1]);
      if (plan_caps(ix, nq, p) == before) {
        if (g.overflowed.size() >= static_cast<size_t>(kGraphCacheSize)) g.overflowed.erase(g.overflowed.begin());
        g.overflowed.push_back(plan_key(ix, raw, nq, k_dev, t_dev, p, use_f, ids, dists, timed));
      }
      return;
    }
  }
  if (stats) {
    stats_from_ctl(ix, stats);
    for (int r = 0; r < planned_rounds(p); ++r) {
      float ms = 0.0f;
      HIP_OK(hipEventElapsedTime(&ms, w.sev[2 * r], w.sev[2 * r + 1]));
      stats->ms_scan += ms;
    }
    stats->path = path;
  }
}

// All-pairs leaf scan: items = (query, leaf) for the lists already in place;
// each item's exact top-k (bf16 scan, certificate, FP32 rescan of the
// uncertified).  `consume` is called with the item count after the bf16 pass
// and again after the rescan pass (rescanned items overwrite).
template <typename Consume>
void allpairs_items(leafi_index *ix, int64_t nq, int k, hipStream_t st, Consume consume, Timing *tm,
                    int64_t *n_fallback = nullptr) {
  Workspace &w = ix->ws;
  const bool bf16 = ix->m <= 256;
  int kprime = default_kprime(k, bf16);
  int64_t items = scan_round(ix, nq, bf16, kprime, k, st, tm);
  if (items == 0) return;
  RoundBufs b = views(w);
  hipLaunchKernelGGL(k_item_cert, dim3(ceil_div(items, 256)), dim3(256), 0, st, items, k, b);
  LAUNCH_OK("item_cert");
  consume(items);
  read_ctl(ix, st);
  add_scan_time(ix, tm);
  int64_t n_fb = w.h_ctl[kCtlFallback];
  if (n_fallback) *n_fallback = n_fb;
  if (n_fb > 0) {
    reset_for_fallback(ix, nq, st);
    launch_emit_fallback(n_fb, ix->N, views(w), st);
    int64_t it2 = scan_round(ix, nq, false, default_kprime(k, false), k, st, nullptr);
    if (it2 > 0) consume(it2);
  }
}

// Lay out "every query searches every leaf" item lists.
void lists_all_leaves(leafi_index *ix, int64_t nq, DevBuf<int32_t> &tmp, hipStream_t st) {
  Workspace &w = ix->ws;
  std::vector<int32_t> all(ix->N);
  for (int L = 0; L < ix->N; ++L) all[L] = L;
  tmp.reserve(ix->N);
  h2d(tmp.get(), all.data(), all.size(), st);
  reset_round(ix, st);
  hipLaunchKernelGGL(k_fill_allpairs, dim3(ceil_div(nq * ix->N, 256)), dim3(256), 0, st, w.qitem_leaf.get(),
                     w.qitem_cnt.get(), w.leaf_cnt.get(), nq, ix->N, tmp.get(), ix->N);
  LAUNCH_OK("fill_allpairs");
}

// Per-leaf exact top-k of nq prepared queries over all leaves.  Outputs
// (device) d [nq, N, k] float and ids [nq, N, k] int64.
void leaf_knn_prepared(leafi_index *ix, int64_t nq, int k, float *d_out, int64_t *ids_out, hipStream_t st,
                       Timing *tm) {
  Workspace &w = ix->ws;
  DevBuf<int32_t> tmp;
  fill_i32(w.kq.get(), nq, k, st);
  lists_all_leaves(ix, nq, tmp, st);
  allpairs_items(ix, nq, k, st, [&](int64_t items) {
    launch_items_to_leaf_knn(items, ix->N, k, k, ix->rowid.get(), views(w), d_out, ids_out, st);
  }, tm);
  HIP_OK(hipStreamSynchronize(st));
}

void check_queries(const leafi_index *ix, const float *q, int64_t nq) {
  LEAFI_CHECK_ARG(nq >= 0, "nq must be >= 0");
  LEAFI_CHECK_ARG(nq == 0 || q != nullptr, "queries pointer is NULL");
  LEAFI_CHECK_ARG(nq < (int64_t(1) << 31), "too many queries in one call");
  (void)ix;
}

}  // namespace leafi

namespace leafi {
SearchPlan make_plan(const leafi_index *ix, const leafi_search_opts *o) {
  LEAFI_CHECK_ARG(o != nullptr, "opts is NULL");
  LEAFI_CHECK_ARG(o->k_max >= 1 && o->k_max <= 256, "k_max must be in [1, 256]");
  LEAFI_CHECK_ARG(o->scan == LEAFI_SCAN_BF16 || o->scan == LEAFI_SCAN_FP32, "unknown scan kind");
  LEAFI_CHECK_ARG(o->n_schedule >= 1 && o->n_schedule <= 8, "n_schedule must be in [1, 8]");
  for (int i = 0; i < o->n_schedule; ++i) LEAFI_CHECK_ARG(o->schedule[i] >= 0, "schedule entries must be >= 0");
  LEAFI_CHECK_ARG(o->kprime >= 0 && o->kprime <= 256, "kprime must be in [0, 256]");
  LEAFI_CHECK_ARG((o->flags & ~(LEAFI_SEARCH_NO_GRAPH | LEAFI_SEARCH_HOST_ROUNDS | LEAFI_SEARCH_FILTER_TILE_SMALL |
                                 LEAFI_SEARCH_FILTER_TILE_LARGE)) == 0,
                  "unknown search flags");
  LEAFI_CHECK_ARG((o->flags & LEAFI_SEARCH_FILTER_TILE_SMALL) == 0 || (o->flags & LEAFI_SEARCH_FILTER_TILE_LARGE) == 0,
                  "FILTER_TILE_SMALL and FILTER_TILE_LARGE exclude each other");
  LEAFI_CHECK_ARG(o->scan != LEAFI_SCAN_BF16 || ix->m <= 256, "the bf16 scan supports m <= 256");
  SearchPlan p;
  p.kmax = o->k_max;
  p.bf16 = o->scan == LEAFI_SCAN_BF16;
  p.filters = o->use_filters != 0;
  p.schedule.assign(o->schedule, o->schedule + o->n_schedule);
  p.kprime = o->kprime > 0 ? std::max<int>(o->kprime, p.kmax) : default_kprime(p.kmax, p.bf16);
  p.kp_query = o->kprime == 0;
  p.graph = (o->flags & LEAFI_SEARCH_NO_GRAPH) == 0;
  p.ftile = (o->flags & LEAFI_SEARCH_FILTER_TILE_SMALL) ? 1 : (o->flags & LEAFI_SEARCH_FILTER_TILE_LARGE) ? 2 : 0;
  return p;
}
}  // namespace leafi

// =============================================================================
// C ABI
// =============================================================================

extern "C" {

const char *leafi_last_error(void) { return g_last_error.c_str(); }

const char *leafi_version(void) { return "leafi-gfx950 0.1"; }

int leafi_create(leafi_alloc_fn alloc, leafi_free_fn free_fn, void *alloc_ctx, leafi_index **out) {
  return guarded([&] {
    LEAFI_CHECK_ARG(out != nullptr, "out is NULL");
    LEAFI_CHECK_ARG((alloc == nullptr) == (free_fn == nullptr), "give both alloc and free, or neither");
    auto *ix = new leafi_index();
    ix->alloc.alloc = alloc;
    ix->alloc.free = free_fn;
    ix->alloc.ctx = alloc_ctx;
    HIP_OK(hipGetDevice(&ix->device));
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ix->device) == hipSuccess && cus > 0)
      ix->num_cus = cus;
    size_t mem = 0;
    if (hipDeviceTotalMem(&mem, ix->device) == hipSuccess && mem > 0) ix->dev_mem = static_cast<double>(mem);
    *out = ix;
  });
}

void leafi_destroy(leafi_index *index) { delete index; }

int leafi_build_index(leafi_index *ix, const float *series, int64_t n, int32_t m, const leafi_build_opts *opts,
                      void *stream) {
  return guarded([&] {
    INDEX_ALLOC_SCOPE(ix);
    LEAFI_CHECK_ARG(ix != nullptr, "index is NULL");
    LEAFI_CHECK_ARG(series != nullptr, "series is NULL");
    LEAFI_CHECK_ARG(opts != nullptr, "opts is NULL");
    LEAFI_CHECK_ARG(n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    LEAFI_CHECK_ARG(m >= 32 && m <= 512 && m % 32 == 0, "m must be a multiple of 32 in [32, 512]");
    LEAFI_CHECK_ARG(opts->leaf_capacity >= 1, "leaf_capacity must be >= 1");
    LEAFI_CHECK_ARG(opts->n_segments >= 1 && opts->n_segments <= 64 && opts->n_segments <= m,
                    "n_segments must be in [1, min(64, m)]");
    LEAFI_CHECK_ARG(opts->split_rule >= 0 && opts->split_rule <= 2, "split_rule must be 0, 1 or 2");
    LEAFI_CHECK_ARG(opts->split_rule != 2 || opts->n_segments <= 32, "the iSAX tree takes at most 32 segments");
    hipStream_t st = as_stream(stream);
    const int S = opts->n_segments;
    // discard previous state
    ix->built = false;
    ix->filt = Filters();
    ix->examples = Examples();
    ix->cal = Calibration();
    // 1. statistics
    DevBuf<double> mean(n), sd(n);
    DevBuf<float> smu(static_cast<size_t>(n) * S), ssd(static_cast<size_t>(n) * S);
    launch_series_stats(series, n, m, S, mean.get(), sd.get(), smu.get(), ssd.get(), st);
    std::vector<float> hmu(static_cast<size_t>(n) * S), hsd(static_cast<size_t>(n) * S);
    d2h(hmu.data(), smu.get(), hmu.size(), st);
    d2h(hsd.data(), ssd.get(), hsd.size(), st);
    HIP_OK(hipStreamSynchronize(st));
    smu.release();
    ssd.release();
    // 2. tree
    TreeResult tree = build_tree(hmu, hsd, n, S, m, opts->leaf_capacity, opts->split_rule);
    const int N = static_cast<int>(tree.leaves.size());
    LEAFI_CHECK_ARG(N <= 16384, "more than 16384 leaves; raise leaf_capacity");
    // 3. padded leaf-contiguous layout
    std::vector<int64_t> off(N + 1, 0), lsz(N);
    for (int L = 0; L < N; ++L) {
      lsz[L] = static_cast<int64_t>(tree.leaves[L].size());
      off[L + 1] = off[L] + round_up(lsz[L], kRowAlign);
    }
    const int64_t rows = off[N];
    std::vector<int64_t> src(rows, -1);
    std::vector<int32_t> leaf_of_row(rows);
    std::vector<int64_t> members;
    members.reserve(n);
    for (int L = 0; L < N; ++L) {
      for (int64_t r = off[L]; r < off[L + 1]; ++r) leaf_of_row[r] = L;
      for (size_t i = 0; i < tree.leaves[L].size(); ++i) src[off[L] + i] = tree.leaves[L][i];
      members.insert(members.end(), tree.leaves[L].begin(), tree.leaves[L].end());
    }
    int max_chunks[kChunkSizes];
    int64_t total_chunks[kChunkSizes];
    for (int j = 0; j < kChunkSizes; ++j) {
      max_chunks[j] = 1;
      total_chunks[j] = 0;
      for (int L = 0; L < N; ++L) {
        const int64_t c = ceil_div(off[L + 1] - off[L], static_cast<int64_t>(kRowAlign) << j);
        max_chunks[j] = std::max<int>(max_chunks[j], static_cast<int>(c));
        total_chunks[j] += c;
      }
    }
    std::vector<float> boxes = leaf_boxes(hmu, hsd, S, tree);
    // 4. device leaf store
    ix->x32.alloc(static_cast<size_t>(rows) * m);
    ix->x16.alloc(static_cast<size_t>(rows) * m);
    ix->xn16.alloc(rows);
    ix->rowid.alloc(rows);
    ix->leaf_off.alloc(N + 1);
    ix->leaf_n.alloc(N);
    ix->boxes.alloc(boxes.size());
    ix->boxes_t.alloc(boxes.size());
    ix->leaf_eps.alloc(N);
    DevBuf<int64_t> dsrc(rows);
    DevBuf<int32_t> dleaf(rows);
    h2d(dsrc.get(), src.data(), rows, st);
    h2d(dleaf.get(), leaf_of_row.data(), rows, st);
    HIP_OK(hipMemsetAsync(ix->leaf_eps.get(), 0, N * sizeof(float), st));
    launch_pack(series, dsrc.get(), dleaf.get(), rows, m, mean.get(), sd.get(), ix->x32.get(), ix->x16.get(),
                ix->xn16.get(), ix->rowid.get(), ix->leaf_eps.get(), st);
    {
      std::vector<float> eps(N);
      d2h(eps.data(), ix->leaf_eps.get(), N, st);
      HIP_OK(hipStreamSynchronize(st));
      ix->leaf_eps_max = *std::max_element(eps.begin(), eps.end());
    }
    std::vector<int32_t> ln32(N);
    for (int L = 0; L < N; ++L) ln32[L] = static_cast<int32_t>(lsz[L]);
    h2d(ix->leaf_off.get(), off.data(), N + 1, st);
    h2d(ix->leaf_n.get(), ln32.data(), N, st);
    h2d(ix->boxes.get(), boxes.data(), boxes.size(), st);
    std::vector<float> boxes_t(boxes.size());
    for (int L = 0; L < N; ++L)
      for (int j = 0; j < 4 * S; ++j) boxes_t[static_cast<size_t>(j) * N + L] = boxes[(static_cast<size_t>(L) * S) * 4 + j];
    h2d(ix->boxes_t.get(), boxes_t.data(), boxes_t.size(), st);
    HIP_OK(hipStreamSynchronize(st));
    ix->n = n;
    ix->m = m;
    ix->S = S;
    ix->N = N;
    ix->rows = rows;
    for (int j = 0; j < kChunkSizes; ++j) {
      ix->chunks_max[j] = max_chunks[j];
      ix->chunks_total[j] = total_chunks[j];
    }
    ix->h_leaf_off = std::move(off);
    ix->h_leaf_n = std::move(lsz);
    ix->h_members = std::move(members);
    ix->h_boxes = std::move(boxes);
    ix->built = true;
  });
}

int leafi_get_info(const leafi_index *ix, leafi_info *out) {
  return guarded([&] {
    LEAFI_CHECK_ARG(ix != nullptr && out != nullptr, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->n_series = ix->n;
    out->m = ix->m;
    out->n_leaves = ix->N;
    out->n_segments = ix->S;
    out->n_filters = ix->filt.F;
    out->hidden = ix->filt.h;
    out->filter_arch = ix->filt.arch;
    out->n_calibrated = ix->cal.pairs();
    out->padded_rows = ix->rows;
    out->device_bytes = static_cast<int64_t>(ix->x32.bytes() + ix->x16.bytes() + ix->xn16.bytes() + ix->rowid.bytes() +
                                             ix->leaf_off.bytes() + ix->leaf_n.bytes() + ix->boxes.bytes() + ix->boxes_t.bytes() +
                                             ix->leaf_eps.bytes() + ix->filt.w.bytes() + ix->cal.offsets.bytes());
  });
}

int leafi_export_leaves(const leafi_index *ix, int64_t *leaf_offsets, int64_t *member_ids) {
  return guarded([&] {
    require_built(ix);
    if (leaf_offsets) {
      leaf_offsets[0] = 0;
      for (int L = 0; L < ix->N; ++L) leaf_offsets[L + 1] = leaf_offsets[L] + ix->h_leaf_n[L];
    }
    if (member_ids) std::memcpy(member_ids, ix->h_members.data(), ix->h_members.size() * sizeof(int64_t));
  });
}

int leafi_export_boxes(const leafi_index *ix, float *boxes) {
  return guarded([&] {
    require_built(ix);
    LEAFI_CHECK_ARG(boxes != nullptr, "boxes is NULL");
    std::memcpy(boxes, ix->h_boxes.data(), ix->h_boxes.size() * sizeof(float));
  });
}

void leafi_default_train_opts(leafi_train_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->n_global = 1500;
  o->n_local = 500;
  o->noise_lo = 0.1f;
  o->noise_hi = 0.4f;
  o->a = 2.0f;
  o->val_fraction = 0.2f;
  o->th_override = -1.0;
  o->mem_budget = int64_t(8) << 30;
  o->hidden = 0;
  o->max_epochs = 1000;
  o->lr0 = 0.01f;
  o->lr_min = 1e-5f;
  o->batch = 64;
  o->patience = 10;
  o->seed = 1;
}

// Floats of one packed filter of the architecture.
static int64_t filter_params(int arch, int m, int h) {
  return arch == LEAFI_FILTER_CNN ? cnn_param_count(h) : static_cast<int64_t>(h) * m + 2 * h + 1;
}

// Algorithm 3's measured costs: t^F, the amortised time of one (query,
// filter) inference in a batch, and t^S, of one (query, series) distance in
// the batched scan with one query group per leaf (the search regime).  The
// probe queries' rows are drawn from rng.
static void measure_costs(leafi_index *ix, int arch, int h, uint64_t seed, std::mt19937_64 &rng, hipStream_t st,
                          double *t_filter, double *t_series) {
  const int m = ix->m, N = ix->N;
  const bool cnn = arch == LEAFI_FILTER_CNN;
  const int64_t P = filter_params(arch, m, h);
  // a CNN filter costs thousands of MLP ones: fewer queries, a filter per CU
  const int qf = cnn ? 64 : 1024, ff = cnn ? 256 : std::min(N, 64);
  DevBuf<float> wp(static_cast<size_t>(ff) * P), xp(static_cast<size_t>(qf) * m), outp(static_cast<size_t>(qf) * ff);
  fill_f32(wp.get(), wp.size(), 0.01f, st);
  fill_f32(xp.get(), xp.size(), 0.5f, st);
  auto infer = [&] {
    if (cnn) launch_cnn_infer(wp.get(), ff, m, h, xp.get(), qf, outp.get(), st);
    else launch_mlp_infer(wp.get(), ff, m, h, xp.get(), qf, outp.get(), st);
  };
  infer();  // warm-up
  hipEvent_t a, b;
  HIP_OK(hipEventCreate(&a));
  HIP_OK(hipEventCreate(&b));
  HIP_OK(hipEventRecord(a, st));
  infer();
  HIP_OK(hipEventRecord(b, st));
  HIP_OK(hipEventSynchronize(b));
  float msf = 0;
  HIP_OK(hipEventElapsedTime(&msf, a, b));
  *t_filter = msf * 1e-3 / (static_cast<double>(qf) * ff);
  // scan probe: 32 training-like queries against every leaf
  const int qs = 32;
  std::vector<int64_t> prow(qs);
  std::vector<float> psig(qs, 0.1f);
  for (int j = 0; j < qs; ++j) {
    int L = static_cast<int>(rng() % N);
    prow[j] = ix->h_leaf_off[L] + static_cast<int64_t>(rng() % ix->h_leaf_n[L]);
  }
  DevBuf<int64_t> drow(qs);
  DevBuf<float> dsig(qs), qraw(static_cast<size_t>(qs) * m);
  h2d(drow.get(), prow.data(), qs, st);
  h2d(dsig.get(), psig.data(), qs, st);
  launch_make_queries(ix->x32.get(), drow.get(), dsig.get(), qs, m, seed ^ 0x5eed, qraw.get(), st);
  ensure_queries(ix, qs, 1);
  prep_queries(ix, qraw.get(), qs, st);
  DevBuf<float> pd(static_cast<size_t>(qs) * N);
  DevBuf<int64_t> pi(static_cast<size_t>(qs) * N);
  Timing tmp;
  leaf_knn_prepared(ix, qs, 1, pd.get(), pi.get(), st, &tmp);
  *t_series = tmp.scan_ms * 1e-3 / (static_cast<double>(qs) * ix->n);
  HIP_OK(hipEventDestroy(a));
  HIP_OK(hipEventDestroy(b));
}

// Per-leaf rates for the knapsack selection, from nq raw queries (device):
// each query's exact 1-NN search in visit order (bounds and node-wise 1-NN
// distances d^L from the leaf scan); p_lb[i] = share of queries whose bound
// prunes leaf i (d^lb > d^bsf), p_f[i] = share of the other visits with
// d^L > d^bsf (what an exact filter prunes; 0 if no query reaches leaf i).
static void selection_estimates(leafi_index *ix, const float *raw, int64_t nq, hipStream_t st, std::vector<double> *p_lb,
                                std::vector<double> *p_f) {
  const int N = ix->N, m = ix->m;
  std::vector<int64_t> pruned(N, 0), reached(N, 0), ideal(N, 0);
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nq, (int64_t(1) << 22) / N));
  std::vector<float> hlb, hd;
  std::vector<int32_t> hord;
  DevBuf<float> dd;
  DevBuf<int64_t> di;
  for (int64_t q0 = 0; q0 < nq; q0 += chunk) {
    const int64_t nc = std::min(chunk, nq - q0);
    const size_t cells = static_cast<size_t>(nc) * N;
    ensure_queries(ix, nc, 1);
    prep_queries(ix, raw + q0 * m, nc, st);
    hlb.resize(cells);
    hord.resize(cells);
    hd.resize(cells);
    d2h(hlb.data(), ix->ws.lb.get(), cells, st);
    d2h(hord.data(), ix->ws.order.get(), cells, st);
    dd.reserve(cells);
    di.reserve(cells);
    leaf_knn_prepared(ix, nc, 1, dd.get(), di.get(), st, nullptr);
    d2h(hd.data(), dd.get(), cells, st);
    HIP_OK(hipStreamSynchronize(st));
    for (int64_t c = 0; c < nc; ++c) {
      double bsf = INFINITY;
      for (int pos = 0; pos < N; ++pos) {
        const int L = hord[c * N + pos];
        const double lbv = hlb[c * N + L], dl = hd[c * N + L];
        if (lbv > bsf) {
          ++pruned[L];
        } else {
          ++reached[L];
          if (dl > bsf) ++ideal[L];
        }
        bsf = std::min(bsf, dl);
      }
    }
  }
  p_lb->assign(N, 0.0);
  p_f->assign(N, 0.0);
  for (int L = 0; L < N; ++L) {
    (*p_lb)[L] = static_cast<double>(pruned[L]) / static_cast<double>(nq);
    (*p_f)[L] = reached[L] > 0 ? static_cast<double>(ideal[L]) / static_cast<double>(reached[L]) : 0.0;
  }
}

static void install_filters(leafi_index *ix, int arch, int F, int h, const std::vector<int32_t> &leaves,
                            hipStream_t st) {
  ix->examples = Examples();
  ix->filt.F = F;
  ix->filt.arch = arch;
  ix->filt.h = h;
  ix->filt.P = filter_params(arch, ix->m, h);
  ix->filt.leaf_of_filter = leaves;
  std::vector<int32_t> fol(ix->N, -1);
  for (int f = 0; f < F; ++f) fol[leaves[f]] = f;
  ix->filt.filt_of_leaf.alloc(ix->N);
  h2d(ix->filt.filt_of_leaf.get(), fol.data(), ix->N, st);
  ix->cal = Calibration();
}

static void set_filters(leafi_index *ix, int arch, int32_t F, int32_t hidden, const int32_t *leaf_ids,
                        const float *weights, void *stream) {
  {
    require_built(ix);
    LEAFI_CHECK_ARG(F >= 0 && F <= ix->N, "n_filters must be in [0, n_leaves]");
    LEAFI_CHECK_ARG(F == 0 || (leaf_ids && weights), "NULL leaf ids or weights");
    if (arch == LEAFI_FILTER_CNN) cnn_check(ix->m, hidden);
    else LEAFI_CHECK_ARG(hidden >= 4 && hidden <= 1024 && hidden % 4 == 0, "hidden must be a multiple of 4 in [4, 1024]");
    std::vector<int32_t> leaves(leaf_ids, leaf_ids + F);
    std::vector<char> seen(ix->N, 0);
    for (int32_t L : leaves) {
      LEAFI_CHECK_ARG(L >= 0 && L < ix->N, "leaf id out of range");
      LEAFI_CHECK_ARG(!seen[L], "duplicate leaf id");
      seen[L] = 1;
    }
    hipStream_t st = as_stream(stream);
    install_filters(ix, arch, F, hidden, leaves, st);
    ix->filt.w.alloc(static_cast<size_t>(F) * ix->filt.P);
    if (F) HIP_OK(hipMemcpyAsync(ix->filt.w.get(), weights, static_cast<size_t>(F) * ix->filt.P * sizeof(float),
                                 hipMemcpyDeviceToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
  }
}

int leafi_set_filters(leafi_index *ix, int32_t F, int32_t hidden, const int32_t *leaf_ids, const float *weights,
                      void *stream) {
  return guarded([&] {
    INDEX_ALLOC_SCOPE(ix);
    set_filters(ix, LEAFI_FILTER_MLP, F, hidden, leaf_ids, weights, stream);
  });
}

int leafi_set_cnn_filters(leafi_index *ix, int32_t F, int32_t channels, const int32_t *leaf_ids, const float *weights,
                          void *stream) {
  return guarded([&] {
    INDEX_ALLOC_SCOPE(ix);
    set_filters(ix, LEAFI_FILTER_CNN, F, channels, leaf_ids, weights, stream);
  });
}

int leafi_get_filters(const leafi_index *ix, int32_t *leaf_ids, float *weights, void *stream) {
  return guarded([&] {
    require_built(ix);
    if (leaf_ids) std::copy(ix->filt.leaf_of_filter.begin(), ix->filt.leaf_of_filter.end(), leaf_ids);
    if (weights && ix->filt.F) {
      hipStream_t st = as_stream(stream);
      HIP_OK(hipMemcpyAsync(weights, ix->filt.w.get(), ix->filt.w.bytes(), hipMemcpyDeviceToDevice, st));
      HIP_OK(hipStreamSynchronize(st));
    }
  });
}

int leafi_train_filters(leafi_index *ix, const leafi_train_opts *o, leafi_train_report *rep, void *stream) {
  return guarded([&] {
    INDEX_ALLOC_SCOPE(ix);
    require_built(ix);
    LEAFI_CHECK_ARG(o != nullptr, "opts is NULL");
    LEAFI_CHECK_ARG(o->n_global >= 2 && o->n_local >= 0, "need n_global >= 2 and n_local >= 0");
    LEAFI_CHECK_ARG(o->noise_lo >= 0 && o->noise_hi >= o->noise_lo, "bad noise range");
    LEAFI_CHECK_ARG(o->val_fraction > 0 && o->val_fraction < 1, "val_fraction must be in (0, 1)");
    LEAFI_CHECK_ARG(o->batch >= 1 && o->batch <= 64, "batch must be in [1, 64]");
    LEAFI_CHECK_ARG(o->max_epochs >= 1 && o->patience >= 1, "max_epochs and patience must be >= 1");
    LEAFI_CHECK_ARG(o->lr0 > 0 && o->lr_min > 0, "learning rates must be > 0");
    const int h = o->hidden > 0 ? o->hidden : ix->m;
    LEAFI_CHECK_ARG(o->arch == LEAFI_FILTER_MLP || o->arch == LEAFI_FILTER_CNN, "arch must be MLP or CNN");
    const bool cnn = o->arch == LEAFI_FILTER_CNN;
    if (cnn) cnn_check(ix->m, h);
    else LEAFI_CHECK_ARG(h <= 256 && h % 4 == 0, "training supports hidden <= 256, a multiple of 4");
    LEAFI_CHECK_ARG(o->selection == LEAFI_SELECT_SIZE || o->selection == LEAFI_SELECT_KNAPSACK,
                    "selection must be LEAFI_SELECT_SIZE or LEAFI_SELECT_KNAPSACK");
    LEAFI_CHECK_ARG(o->a > 0, "a must be > 0");
    hipStream_t st = as_stream(stream);
    Workspace &w = ix->ws;
    const int m = ix->m, N = ix->N;
    const int64_t P = filter_params(o->arch, m, h);
    leafi_train_report report;
    std::memset(&report, 0, sizeof(report));
    std::mt19937_64 rng(o->seed);

    // ---- leaf selection: Algorithm 3 (size threshold, greedy by size) or
    // the knapsack of Equations 1-2 with per-leaf rates estimated on the
    // global training queries
    const bool knap = o->selection == LEAFI_SELECT_KNAPSACK;
    double th = o->th_override;
    // the knapsack's benefits in units of t^S when th_override fixes the
    // ratio t^F / t^S = th / a (their signs and order depend on it alone)
    double kn_tF = th / o->a, kn_tS = 1.0;
    if (th < 0) {
      measure_costs(ix, o->arch, h, o->seed, rng, st, &report.t_filter_s, &report.t_series_s);
      th = report.t_series_s > 0 ? o->a * report.t_filter_s / report.t_series_s : 0.0;
      kn_tF = report.t_filter_s;
      kn_tS = report.t_series_s;
    }
    report.th = th;
    // the global training queries' rows and noise levels (drawn before the
    // selection: the knapsack estimates its rates on them)
    const int n_g = o->n_global, n_l = o->n_local;
    std::uniform_real_distribution<double> unif(o->noise_lo, o->noise_hi);
    std::vector<int64_t> cum(N + 1, 0);
    for (int L = 0; L < N; ++L) cum[L + 1] = cum[L] + ix->h_leaf_n[L];
    std::vector<int64_t> rows(n_g);
    std::vector<float> sig(n_g);
    for (int j = 0; j < n_g; ++j) {  // uniform over the collection
      int64_t u = static_cast<int64_t>(rng() % static_cast<uint64_t>(ix->n));
      int L = static_cast<int>(std::upper_bound(cum.begin(), cum.end(), u) - cum.begin()) - 1;
      rows[j] = ix->h_leaf_off[L] + (u - cum[L]);
      sig[j] = static_cast<float>(unif(rng));
    }
    std::vector<int32_t> sel;
    if (knap) {
      DevBuf<int64_t> grows(n_g);
      DevBuf<float> gsig(n_g), graw(static_cast<size_t>(n_g) * m);
      h2d(grows.get(), rows.data(), n_g, st);
      h2d(gsig.get(), sig.data(), n_g, st);
      launch_make_queries(ix->x32.get(), grows.get(), gsig.get(), n_g, m, o->seed, graw.get(), st);
      std::vector<double> p_lb, p_f;
      selection_estimates(ix, graw.get(), n_g, st, &p_lb, &p_f);
      sel = select_knapsack(ix->h_leaf_n, p_lb, p_f, o->a, kn_tS, kn_tF, static_cast<double>(P) * 4.0,
                            static_cast<double>(o->mem_budget), nullptr);
    } else {
      sel = select_leaves(ix->h_leaf_n, th, static_cast<double>(P) * 4.0, static_cast<double>(o->mem_budget));
    }
    const int F = static_cast<int>(sel.size());
    install_filters(ix, o->arch, F, h, sel, st);
    ix->filt.w.alloc(static_cast<size_t>(std::max(F, 1)) * P);
    report.n_filters = F;
    if (F == 0) {
      HIP_OK(hipStreamSynchronize(st));
      if (rep) *rep = report;
      return;
    }

    // ---- training queries: global (train + validation) and local per filter
    const int n_gv = std::max(1, static_cast<int>(std::lround(o->val_fraction * n_g)));
    const int n_gt = n_g - n_gv;
    const int64_t nqt = n_g + static_cast<int64_t>(F) * n_l;
    rows.resize(nqt);
    sig.resize(nqt);
    for (int f = 0; f < F; ++f) {  // uniform over the filtered leaf
      int L = sel[f];
      for (int j = 0; j < n_l; ++j) {
        int64_t i = n_g + static_cast<int64_t>(f) * n_l + j;
        rows[i] = ix->h_leaf_off[L] + static_cast<int64_t>(rng() % static_cast<uint64_t>(ix->h_leaf_n[L]));
        sig[i] = static_cast<float>(unif(rng));
      }
    }
    DevBuf<int64_t> drows(nqt);
    DevBuf<float> dsig(nqt), qraw(static_cast<size_t>(nqt) * m);
    h2d(drows.get(), rows.data(), nqt, st);
    h2d(dsig.get(), sig.data(), nqt, st);
    launch_make_queries(ix->x32.get(), drows.get(), dsig.get(), nqt, m, o->seed, qraw.get(), st);

    // ---- targets d^L with the leaf scan: global queries x filtered leaves,
    // local queries x their own leaf.  Queries go in chunks that bound the
    // round's item buffers (about kChunkItems items) and the per-query
    // buffers strided by the leaf count; each chunk's normalised queries are
    // kept as the SGD inputs.
    auto t0 = std::chrono::steady_clock::now();
    const int n_ex = n_g + n_l, n_train = n_gt + n_l;
    DevBuf<float> xq(static_cast<size_t>(nqt) * m);
    DevBuf<float> ex_y(static_cast<size_t>(F) * n_ex);
    Timing tcol;
    constexpr int64_t kChunkItems = int64_t(1) << 22;
    const int64_t per_query_bytes = static_cast<int64_t>(N) * 6 * 4 + static_cast<int64_t>(F) * 4;
    const int64_t max_chunk = std::max<int64_t>(1, std::min<int64_t>(kChunkItems, (int64_t(3) << 30) / per_query_bytes));
    auto collect = [&](int64_t q0, int64_t q1) {
      const int64_t nc = q1 - q0;
      std::vector<int64_t> loff(nc + 1, 0);
      std::vector<int32_t> lst;
      for (int64_t j = q0; j < q1; ++j) {
        if (j < n_g) lst.insert(lst.end(), sel.begin(), sel.end());
        else lst.push_back(sel[(j - n_g) / n_l]);
        loff[j - q0 + 1] = static_cast<int64_t>(lst.size());
      }
      ensure_queries(ix, nc, 1);
      launch_qprep(qraw.get() + q0 * m, nc, m, ix->S, w.q32.get(), w.q16.get(), w.qn16.get(), w.qeps.get(),
                   w.qstat.get(), st);
      HIP_OK(hipMemcpyAsync(xq.get() + q0 * m, w.q32.get(), static_cast<size_t>(nc) * m * sizeof(float),
                            hipMemcpyDeviceToDevice, st));
      DevBuf<int64_t> dloff(nc + 1);
      DevBuf<int32_t> dlst(lst.size());
      h2d(dloff.get(), loff.data(), loff.size(), st);
      h2d(dlst.get(), lst.data(), lst.size(), st);
      fill_i32(w.kq.get(), nc, 1, st);
      reset_round(ix, st);
      hipLaunchKernelGGL(k_fill_lists, dim3(ceil_div(nc, 256)), dim3(256), 0, st, w.qitem_leaf.get(),
                         w.qitem_cnt.get(), w.leaf_cnt.get(), nc, N, dloff.get(), dlst.get());
      LAUNCH_OK("fill_lists");
      allpairs_items(ix, nc, 1, st, [&](int64_t items) {
        hipLaunchKernelGGL(k_items_to_examples, dim3(ceil_div(items, 256)), dim3(256), 0, st, items, 1, views(w),
                           ix->filt.filt_of_leaf.get(), n_g, n_gt, n_l, n_ex, ex_y.get(), q0);
        LAUNCH_OK("items_to_examples");
      }, &tcol);
      HIP_OK(hipStreamSynchronize(st));  // the chunk's lists are freed on return
    };
    const int64_t g_chunk = std::max<int64_t>(1, std::min<int64_t>(max_chunk, kChunkItems / F));
    for (int64_t q0 = 0; q0 < n_g; q0 += g_chunk) collect(q0, std::min<int64_t>(n_g, q0 + g_chunk));
    for (int64_t q0 = n_g; q0 < nqt; q0 += max_chunk) collect(q0, std::min<int64_t>(nqt, q0 + max_chunk));
    if (o->keep_examples) ix->examples.q = std::move(qraw);
    else qraw.release();
    auto t1 = std::chrono::steady_clock::now();
    report.ms_collect = std::chrono::duration<double, std::milli>(t1 - t0).count();

    // ---- example tables: per filter [global train | local | global validation]
    std::vector<int32_t> exq(static_cast<size_t>(F) * n_ex);
    for (int f = 0; f < F; ++f) {
      int32_t *e = &exq[static_cast<size_t>(f) * n_ex];
      for (int j = 0; j < n_gt; ++j) e[j] = j;
      for (int j = 0; j < n_l; ++j) e[n_gt + j] = n_g + f * n_l + j;
      for (int j = 0; j < n_gv; ++j) e[n_gt + n_l + j] = n_gt + j;
    }
    DevBuf<int32_t> dexq(exq.size());
    h2d(dexq.get(), exq.data(), exq.size(), st);

    // ---- initial weights: uniform +-1/sqrt(fan_in) per layer
    std::vector<float> w0(static_cast<size_t>(F) * P);
    for (int f = 0; f < F; ++f) {
      std::mt19937_64 g(o->seed * 0x9e3779b97f4a7c15ull + static_cast<uint64_t>(f) + 1);
      float *wf = &w0[static_cast<size_t>(f) * P];
      // [layer end, fan-in] of each layer's weights and bias, in packed order
      std::vector<std::pair<int64_t, int>> layers;
      if (cnn)  // [W1 | b1] fan-in 3, [W2 | b2] fan-in 3C, [w3 | b3] fan-in C
        layers = {{4LL * h, 3}, {4LL * h + 3LL * h * h + h, 3 * h}, {P, h}};
      else  // [W1 | b1] fan-in m, [w2 | b2] fan-in h
        layers = {{static_cast<int64_t>(h) * m + h, m}, {P, h}};
      int64_t i = 0;
      for (const auto &L : layers) {
        const float bound = 1.0f / std::sqrt(static_cast<float>(L.second));
        std::uniform_real_distribution<float> u(-bound, bound);
        for (; i < L.first; ++i) wf[i] = u(g);
      }
    }
    h2d(ix->filt.w.get(), w0.data(), w0.size(), st);
    DevBuf<float> wbest(static_cast<size_t>(F) * P), vmse(F);
    DevBuf<int32_t> eruns(F);
    TrainArgs ta{};
    ta.w = ix->filt.w.get();
    ta.w_best = wbest.get();
    ta.xq = xq.get();
    ta.ex_q = dexq.get();
    ta.ex_y = ex_y.get();
    ta.n_train = n_train;
    ta.n_ex = n_ex;
    ta.F = F;
    ta.m = m;
    ta.h = h;
    ta.batch = o->batch;
    ta.max_epochs = o->max_epochs;
    ta.patience = o->patience;
    ta.lr0 = o->lr0;
    ta.lr_min = o->lr_min;
    ta.seed = o->seed;
    ta.val_mse = vmse.get();
    ta.epochs_run = eruns.get();
    DevBuf<float> vtrace;
    if (o->keep_examples) {
      vtrace.alloc(static_cast<size_t>(F) * o->max_epochs);
      fill_f32(vtrace.get(), static_cast<int64_t>(vtrace.size()), NAN, st);
      ta.val_trace = vtrace.get();
    }
    auto t2 = std::chrono::steady_clock::now();
    if (cnn) {
      DevBuf<float> gbuf(static_cast<size_t>(F) * P);
      launch_cnn_train(ta, gbuf.get(), st);
      HIP_OK(hipStreamSynchronize(st));  // gbuf is freed on leaving the scope
    } else {
      launch_mlp_train(ta, st);
    }
    std::vector<float> hv(F);
    std::vector<int32_t> he(F);
    d2h(hv.data(), vmse.get(), F, st);
    d2h(he.data(), eruns.get(), F, st);
    HIP_OK(hipStreamSynchronize(st));
    auto t3 = std::chrono::steady_clock::now();
    report.ms_train = std::chrono::duration<double, std::milli>(t3 - t2).count();
    double s = 0.0;
    for (int f = 0; f < F; ++f) {
      s += hv[f];
      report.epochs_max_run = std::max(report.epochs_max_run, he[f]);
    }
    report.mean_val_mse = s / F;
    if (o->keep_examples) {
      Examples &ex = ix->examples;
      ex.nq = nqt;
      ex.n_ex = n_ex;
      ex.n_train = n_train;
      ex.ex_q = std::move(exq);
      ex.ex_y = std::move(ex_y);
      ex.max_epochs = o->max_epochs;
      ex.epochs.assign(he.begin(), he.end());
      ex.val_trace.resize(vtrace.size());
      d2h(ex.val_trace.data(), vtrace.get(), vtrace.size(), st);
      HIP_OK(hipStreamSynchronize(st));
    }
    if (rep) *rep = report;
  });
}

int leafi_get_train_trace(const leafi_index *ix, int32_t *max_epochs, int32_t *epochs_run, float *val_mse) {
  return guarded([&] {
    require_built(ix);
    const Examples &ex = ix->examples;
    if (ex.nq == 0) fail(LEAFI_ESTATE, "no training run kept (train with keep_examples = 1)");
    if (max_epochs) *max_epochs = ex.max_epochs;
    if (epochs_run) std::copy(ex.epochs.begin(), ex.epochs.end(), epochs_run);
    if (val_mse) std::copy(ex.val_trace.begin(), ex.val_trace.end(), val_mse);
  });
}

int leafi_get_examples(const leafi_index *ix, int64_t *n_queries, int32_t *n_examples, int32_t *n_train,
                       float *queries, int32_t *ex_query, float *ex_target, void *stream) {
  return guarded([&] {
    require_built(ix);
    const Examples &ex = ix->examples;
    if (ex.nq == 0) fail(LEAFI_ESTATE, "no training set kept (train with keep_examples = 1)");
    if (n_queries) *n_queries = ex.nq;
    if (n_examples) *n_examples = ex.n_ex;
    if (n_train) *n_train = ex.n_train;
    if (ex_query) std::copy(ex.ex_q.begin(), ex.ex_q.end(), ex_query);
    hipStream_t st = as_stream(stream);
    if (queries) HIP_OK(hipMemcpyAsync(queries, ex.q.get(), ex.q.bytes(), hipMemcpyDeviceToDevice, st));
    if (ex_target) HIP_OK(hipMemcpyAsync(ex_target, ex.ex_y.get(), ex.ex_y.bytes(), hipMemcpyDeviceToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
  });
}

int leafi_calibrate(leafi_index *ix, const float *calib, int32_t nc, const int32_t *ks, int32_t n_ks,
                    const float *targets, int32_t n_targets, int32_t flags, void *stream) {
  return guarded([&] {
    INDEX_ALLOC_SCOPE(ix);
    require_built(ix);
    if (ix->filt.F == 0) fail(LEAFI_ESTATE, "no filters (train or set them first)");
    LEAFI_CHECK_ARG(nc >= 1 && calib != nullptr, "need calibration queries");
    LEAFI_CHECK_ARG(n_ks >= 1 && ks != nullptr && n_targets >= 1 && targets != nullptr, "need ks and targets");
    int kc = 1;
    for (int i = 0; i < n_ks; ++i) {
      LEAFI_CHECK_ARG(ks[i] >= 1 && ks[i] <= 256, "ks must be in [1, 256]");
      kc = std::max(kc, ks[i]);
    }
    for (int i = 0; i < n_targets; ++i) LEAFI_CHECK_ARG(targets[i] > 0 && targets[i] <= 1, "targets must be in (0, 1]");
    const int mapping = flags & 1;
    const bool corrected = (flags & LEAFI_CALIB_NO_CORRECTION) == 0;
    hipStream_t st = as_stream(stream);
    Workspace &w = ix->ws;
    const int N = ix->N, F = ix->filt.F;
    ensure_queries(ix, nc, kc);
    prep_queries(ix, calib, nc, st);
    infer_filters_dense(ix, w.q32.get(), nc, w.dfilt.get(), st);
    CalibInput in;
    in.nc = nc;
    in.N = N;
    in.F = F;
    in.kmax = kc;
    in.order.resize(static_cast<size_t>(nc) * N);
    in.dfilt.resize(static_cast<size_t>(nc) * F);
    in.leaf_of_filter = ix->filt.leaf_of_filter;
    d2h(in.order.data(), w.order.get(), in.order.size(), st);
    d2h(in.dfilt.data(), w.dfilt.get(), in.dfilt.size(), st);
    DevBuf<float> dd(static_cast<size_t>(nc) * N * kc);
    DevBuf<int64_t> di(static_cast<size_t>(nc) * N * kc);
    leaf_knn_prepared(ix, nc, kc, dd.get(), di.get(), st, nullptr);
    std::vector<float> hd(dd.size());
    in.leaf_ids.resize(di.size());
    d2h(hd.data(), dd.get(), hd.size(), st);
    d2h(in.leaf_ids.data(), di.get(), in.leaf_ids.size(), st);
    HIP_OK(hipStreamSynchronize(st));
    in.leaf_d.assign(hd.begin(), hd.end());
    std::vector<float> tg(targets, targets + n_targets);
    Calibration cal;
    cal.ks.assign(ks, ks + n_ks);
    cal.targets = tg;
    cal.h_offsets.assign(static_cast<size_t>(n_ks) * n_targets * F, INFINITY);
    for (int i = 0; i < n_ks; ++i) {
      std::vector<float> o = calibrate_k(in, ks[i], tg, mapping, corrected);
      std::copy(o.begin(), o.end(), cal.h_offsets.begin() + static_cast<size_t>(i) * n_targets * F);
    }
    std::vector<int32_t> pk;
    std::vector<float> pt;
    for (int i = 0; i < n_ks; ++i)
      for (int t = 0; t < n_targets; ++t) {
        pk.push_back(ks[i]);
        pt.push_back(tg[t]);
      }
    cal.offsets.alloc(cal.h_offsets.size());
    cal.pair_k.alloc(pk.size());
    cal.pair_t.alloc(pt.size());
    h2d(cal.offsets.get(), cal.h_offsets.data(), cal.h_offsets.size(), st);
    h2d(cal.pair_k.get(), pk.data(), pk.size(), st);
    h2d(cal.pair_t.get(), pt.data(), pt.size(), st);
    HIP_OK(hipStreamSynchronize(st));
    ix->cal = std::move(cal);
  });
}

int leafi_get_offsets(const leafi_index *ix, float *offsets) {
  return guarded([&] {
    require_built(ix);
    LEAFI_CHECK_ARG(offsets != nullptr, "offsets is NULL");
    std::copy(ix->cal.h_offsets.begin(), ix->cal.h_offsets.end(), offsets);
  });
}

int leafi_set_offsets(leafi_index *ix, const int32_t *ks, int32_t n_ks, const float *targets, int32_t n_targets,
                      const float *offsets) {
  return guarded([&] {
    INDEX_ALLOC_SCOPE(ix);
    require_built(ix);
    if (ix->filt.F == 0) fail(LEAFI_ESTATE, "no filters (train or set them first)");
    LEAFI_CHECK_ARG(n_ks >= 1 && n_targets >= 1 && ks && targets && offsets, "bad arguments");
    const int F = ix->filt.F;
    Calibration cal;
    cal.ks.assign(ks, ks + n_ks);
    cal.targets.assign(targets, targets + n_targets);
    cal.h_offsets.assign(offsets, offsets + static_cast<size_t>(n_ks) * n_targets * F);
    std::vector<int32_t> pk;
    std::vector<float> pt;
    for (int i = 0; i < n_ks; ++i)
      for (int t = 0; t < n_targets; ++t) {
        pk.push_back(ks[i]);
        pt.push_back(targets[t]);
      }
    cal.offsets.alloc(cal.h_offsets.size());
    cal.pair_k.alloc(pk.size());
    cal.pair_t.alloc(pt.size());
    HIP_OK(hipMemcpy(cal.offsets.get(), cal.h_offsets.data(), cal.h_offsets.size() * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(cal.pair_k.get(), pk.data(), pk.size() * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(cal.pair_t.get(), pt.data(), pt.size() * 4, hipMemcpyHostToDevice));
    ix->cal = std::move(cal);
  });
}

void leafi_default_search_opts(leafi_search_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->k_max = 1;
  o->scan = LEAFI_SCAN_BF16;
  o->use_filters = 1;
  o->n_schedule = 2;
  o->schedule[0] = 1;
  o->schedule[1] = 0;
  o->kprime = 0;
}


int leafi_search_knn(leafi_index *ix, const float *queries, int64_t nq, const int32_t *k_dev, const float *t_dev,
                     const leafi_search_opts *o, int64_t *ids, float *dists, leafi_search_stats *stats,
                     void *stream) {
  return guarded([&] {
    INDEX_ALLOC_SCOPE(ix);
    require_built(ix);
    check_queries(ix, queries, nq);
    SearchPlan p = make_plan(ix, o);
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (nq == 0) return;
    LEAFI_CHECK_ARG(k_dev && t_dev && ids && dists, "NULL k, target or output pointer");
    hipStream_t st = as_stream(stream);
    auto t0 = std::chrono::steady_clock::now();
    if (p.bf16 && (o->flags & LEAFI_SEARCH_HOST_ROUNDS) == 0 && can_plan(ix, nq, p)) {
      search_planned(ix, queries, nq, k_dev, t_dev, p, ids, dists, stats, st);
    } else if (p.bf16) {
      search_batch(ix, queries, nq, k_dev, t_dev, p, ids, dists, stats, st);
    } else {
      // plain form: one query at a time
      for (int64_t q = 0; q < nq; ++q)
        search_batch(ix, queries + q * ix->m, 1, k_dev + q, t_dev + q, p, ids + q * p.kmax, dists + q * p.kmax,
                     stats, st);
    }
    if (stats) {
      HIP_OK(hipStreamSynchronize(st));
      stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
  });
}

const char *leafi_graph_note(const leafi_index *ix) {
  if (!ix) return "";
  return ix->ws.graphs.why.c_str();
}

int leafi_set_plan_capacity(leafi_index *ix, int64_t max_items) {
  return guarded([&] {
    require_built(ix);
    LEAFI_CHECK_ARG(max_items >= 0, "max_items must be >= 0");
    ix->plan_cap_items = max_items;
  });
}

int leafi_set_tiling(leafi_index *ix, int32_t chunk_rows, int32_t queries_per_tile) {
  return guarded([&] {
    require_built(ix);
    bool ok = false;
    for (int j = 0; j < kChunkSizes; ++j) ok = ok || chunk_rows == (kRowAlign << j);
    LEAFI_CHECK_ARG(ok, "chunk_rows must be 128 << j, j = 0 .. 5");
    LEAFI_CHECK_ARG(queries_per_tile == 16 || queries_per_tile == 32 || queries_per_tile == 48 ||
                        queries_per_tile == 64,
                    "queries_per_tile must be 16, 32, 48 or 64");
    ix->tune_chunk = chunk_rows;
    ix->tune_mq = queries_per_tile;
  });
}

int leafi_autotune(leafi_index *ix, const float *queries, int64_t nq, const int32_t *k_dev, const float *t_dev,
                   const leafi_search_opts *o, int32_t repeats, leafi_tune_report *report, void *stream) {
  return guarded([&] {
    INDEX_ALLOC_SCOPE(ix);
    require_built(ix);
    check_queries(ix, queries, nq);
    LEAFI_CHECK_ARG(nq > 0 && k_dev && t_dev, "empty sample or NULL k / target");
    LEAFI_CHECK_ARG(repeats >= 1 && repeats <= 100, "repeats must be in [1, 100]");
    SearchPlan p = make_plan(ix, o);
    LEAFI_CHECK_ARG(p.bf16, "the tuner tunes the BF16 scan");
    p.graph = false;
    hipStream_t st = as_stream(stream);
    DevBuf<int64_t> ids(static_cast<size_t>(nq) * p.kmax);
    DevBuf<float> dists(static_cast<size_t>(nq) * p.kmax);
    std::vector<std::pair<int, int>> cand;  // (chunk rows, queries per tile)
    for (int chunk : {512, 1024, 2048})
      for (int mq : {16, 32, 48, 64}) cand.emplace_back(chunk, mq);
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    HIP_OK(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
    std::vector<double> med(cand.size());
    const int old_chunk = ix->tune_chunk, old_mq = ix->tune_mq;
    try {
      for (size_t c = 0; c < cand.size(); ++c) {
        ix->tune_chunk = cand[c].first;
        ix->tune_mq = cand[c].second;
        std::vector<double> t;
        for (int r = 0; r <= repeats; ++r) {
          HIP_OK(hipEventRecord(e0, st));
          if (can_plan(ix, nq, p)) search_planned(ix, queries, nq, k_dev, t_dev, p, ids.get(), dists.get(), nullptr, st);
          else search_batch(ix, queries, nq, k_dev, t_dev, p, ids.get(), dists.get(), nullptr, st);
          HIP_OK(hipEventRecord(e1, st));
          HIP_OK(hipEventSynchronize(e1));
          float ms = 0.0f;
          HIP_OK(hipEventElapsedTime(&ms, e0, e1));
          if (r > 0) t.push_back(ms);  // the first run is the warm-up
        }
        std::sort(t.begin(), t.end());
        med[c] = t[t.size() / 2];
      }
    } catch (...) {
      ix->tune_chunk = old_chunk;
      ix->tune_mq = old_mq;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const size_t best = static_cast<size_t>(std::min_element(med.begin(), med.end()) - med.begin());
    ix->tune_chunk = cand[best].first;
    ix->tune_mq = cand[best].second;
    if (report) {
      std::memset(report, 0, sizeof(*report));
      report->n_candidates = static_cast<int32_t>(cand.size());
      report->chosen = static_cast<int32_t>(best);
      for (size_t c = 0; c < cand.size() && c < LEAFI_TUNE_MAX; ++c) {
        report->chunk_rows[c] = cand[c].first;
        report->queries_per_tile[c] = cand[c].second;
        report->ms[c] = med[c];
      }
    }
  });
}

int leafi_znorm(const float *x, int64_t n, int32_t m, float *out, void *stream) {
  return guarded([&] {
    LEAFI_CHECK_ARG(n >= 0 && (n == 0 || (x && out)), "bad arguments");
    LEAFI_CHECK_ARG(m >= 1 && m <= 1024, "m must be in [1, 1024]");
    if (n) launch_znorm(x, n, m, out, as_stream(stream));
  });
}

int leafi_lower_bounds(leafi_index *ix, const float *queries, int64_t nq, float *lb, void *stream) {
  return guarded([&] {
    INDEX_ALLOC_SCOPE(ix);
    require_built(ix);
    check_queries(ix, queries, nq);
    if (nq == 0) return;
    LEAFI_CHECK_ARG(lb != nullptr, "lb is NULL");
    hipStream_t st = as_stream(stream);
    ensure_queries(ix, nq, 1);
    prep_queries(ix, queries, nq, st);
    HIP_OK(hipMemcpyAsync(lb, ix->ws.lb.get(), static_cast<size_t>(nq) * ix->N * sizeof(float),
                          hipMemcpyDeviceToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
  });
}

int leafi_mlp_infer(const float *w, int32_t F, int32_t m, int32_t h, const float *x, int64_t nq, float *out,
                    void *stream) {
  return guarded([&] {
    LEAFI_CHECK_ARG(F >= 0 && nq >= 0, "bad sizes");
    LEAFI_CHECK_ARG(m >= 4 && m <= 1024 && m % 4 == 0, "m must be a multiple of 4 in [4, 1024]");
    LEAFI_CHECK_ARG(h >= 4 && h <= 1024 && h % 4 == 0, "hidden must be a multiple of 4 in [4, 1024]");
    if (F == 0 || nq == 0) return;
    LEAFI_CHECK_ARG(w && x && out, "NULL pointer");
    LEAFI_CHECK_ARG(reinterpret_cast<uintptr_t>(x) % 16 == 0, "x must be 16-byte aligned");
    LEAFI_CHECK_ARG(F <= 65535 && ceil_div(nq, 64) <= 65535, "grid too large; split the call");
    launch_mlp_infer(w, F, m, h, x, nq, out, as_stream(stream));
  });
}

int leafi_mlp_sgd_step(float *w, int32_t F, int32_t m, int32_t h, const float *x, const float *y, int32_t batch,
                       float lr, float *loss, void *stream) {
  return guarded([&] {
    LEAFI_CHECK_ARG(F >= 0, "bad sizes");
    LEAFI_CHECK_ARG(m >= 4 && m <= 512 && m % 4 == 0, "m must be a multiple of 4 in [4, 512]");
    LEAFI_CHECK_ARG(h >= 1 && h <= 256, "hidden must be in [1, 256]");
    LEAFI_CHECK_ARG(batch >= 1 && batch <= 64, "batch must be in [1, 64]");
    if (F == 0) return;
    LEAFI_CHECK_ARG(w && x && y, "NULL pointer");
    launch_mlp_sgd_step(w, F, m, h, x, y, batch, lr, loss, as_stream(stream));
  });
}

int leafi_cnn_infer(const float *w, int32_t F, int32_t m, int32_t C, const float *x, int64_t nq, float *out,
                    void *stream) {
  return guarded([&] {
    LEAFI_CHECK_ARG(F >= 0 && nq >= 0, "bad sizes");
    cnn_check(m, C);
    if (F == 0 || nq == 0) return;
    LEAFI_CHECK_ARG(w && x && out, "NULL pointer");
    LEAFI_CHECK_ARG(F <= 65535, "too many filters in one call");
    launch_cnn_infer(w, F, m, C, x, nq, out, as_stream(stream));
  });
}

int leafi_cnn_sgd_step(float *w, int32_t F, int32_t m, int32_t C, const float *x, const float *y, int32_t batch,
                       float lr, float *loss, void *stream) {
  return guarded([&] {
    LEAFI_CHECK_ARG(F >= 0, "bad sizes");
    cnn_check(m, C);
    LEAFI_CHECK_ARG(batch >= 1, "batch must be >= 1");
    if (F == 0) return;
    LEAFI_CHECK_ARG(w && x && y && loss, "NULL pointer");
    LEAFI_CHECK_ARG(F <= 65535, "too many filters in one call");
    hipStream_t st = as_stream(stream);
    DevBuf<float> gbuf(static_cast<size_t>(F) * cnn_param_count(C));
    launch_cnn_sgd_step(w, F, m, C, x, y, batch, lr, loss, gbuf.get(), st);
    HIP_OK(hipStreamSynchronize(st));  // gbuf is freed on return
  });
}

int leafi_leaf_knn(leafi_index *ix, const float *queries, int64_t nq, int32_t k, float *d, int64_t *ids,
                   void *stream) {
  return guarded([&] {
    INDEX_ALLOC_SCOPE(ix);
    require_built(ix);
    check_queries(ix, queries, nq);
    LEAFI_CHECK_ARG(k >= 1 && k <= 256, "k must be in [1, 256]");
    if (nq == 0) return;
    LEAFI_CHECK_ARG(d && ids, "NULL output");
    hipStream_t st = as_stream(stream);
    ensure_queries(ix, nq, k);
    prep_queries(ix, queries, nq, st);
    leaf_knn_prepared(ix, nq, k, d, ids, st, nullptr);
  });
}

int leafi_select_knapsack(leafi_index *ix, const float *queries, int64_t nq, float a, double t_filter_s,
                          double t_series_s, int32_t hidden, int64_t mem_budget, int32_t *leaf_ids, int32_t *n_selected,
                          double *benefit, double *p_lb, double *p_f, void *stream) {
  return guarded([&] {
    INDEX_ALLOC_SCOPE(ix);
    require_built(ix);
    check_queries(ix, queries, nq);
    LEAFI_CHECK_ARG(nq >= 1, "need at least one query");
    LEAFI_CHECK_ARG(a > 0, "a must be > 0");
    LEAFI_CHECK_ARG(mem_budget >= 0, "mem_budget must be >= 0");
    const int h = hidden > 0 ? hidden : ix->m;
    LEAFI_CHECK_ARG(h <= 256 && h % 4 == 0, "hidden must be <= 256, a multiple of 4");
    hipStream_t st = as_stream(stream);
    double tF = t_filter_s, tS = t_series_s;
    if (!(tF > 0) || !(tS > 0)) {
      std::mt19937_64 rng(1);
      measure_costs(ix, LEAFI_FILTER_MLP, h, 1, rng, st, &tF, &tS);
    }
    std::vector<double> pl, pf, b;
    selection_estimates(ix, queries, nq, st, &pl, &pf);
    const double wbytes = 4.0 * (static_cast<double>(h) * ix->m + 2 * h + 1);
    std::vector<int32_t> sel = select_knapsack(ix->h_leaf_n, pl, pf, a, tS, tF, wbytes,
                                               static_cast<double>(mem_budget), &b);
    if (n_selected) *n_selected = static_cast<int32_t>(sel.size());
    if (leaf_ids) std::copy(sel.begin(), sel.end(), leaf_ids);
    if (benefit) std::copy(b.begin(), b.end(), benefit);
    if (p_lb) std::copy(pl.begin(), pl.end(), p_lb);
    if (p_f) std::copy(pf.begin(), pf.end(), p_f);
  });
}

}  // extern "C"
