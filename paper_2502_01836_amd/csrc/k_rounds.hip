// Round machinery of the batched search (Algorithm 2 run for many queries at
// once, a few leaves per query per round): the prune cascade that emits the
// round's (query, leaf) items, the items' CSR-by-leaf layout and scan tiles,
// the per-query merge into the running top-k with the best-so-far tau, and
// the final output.
#include <algorithm>

#include "device_util.h"
#include "kernels.h"

namespace leafi {

namespace {

// Algorithm 2's cascade for one query (one wavefront per query): walk the
// visit order from the cursor 64 positions at a time, prune a leaf when
// d^lb > tau or (it has a filter and d^f - o > tau), and emit up to `want`
// surviving leaves in visit order.  All decisions of the round use the tau
// from before the round.  The order is by ascending d^lb, so the first leaf
// the bound prunes ends the walk (every later leaf is pruned too).
constexpr int kListWaves = 16;  // queries (wavefronts) per work-group of the prune cascade

struct CascadeCount {
  int cnt = 0;  // leaves emitted
  int64_t lbp = 0, fp = 0, series = 0;  // pruned by bound / by filter, real series emitted (lane 0: totals)
};

// The cascade of query q (one wavefront) from its cursor with the given tau:
// emits its surviving leaves into qitem_leaf after the `base` entries already
// queued there (rescans of the previous round), counts them per leaf and
// advances its cursor.
__device__ inline CascadeCount cascade_query(int64_t q, int N, const float *__restrict__ lbs,
                                             const int32_t *__restrict__ order, const float *__restrict__ dfo,
                                             const int32_t *__restrict__ leaf_n, int want, float tau, RoundBufs &b,
                                             int lane, int base) {
  CascadeCount c;
  int pos = b.cursor[q];
  if (pos < N) {
    const float tau_lb = tau * (1.0f + kLbSlack);
    const bool use_f = dfo != nullptr && b.pair[q] >= 0;
    const float *lbq = lbs + q * N;
    const float *fq = use_f ? dfo + q * N : nullptr;
    const int32_t *oq = order + q * N;
    const uint64_t lt = (1ull << lane) - 1ull;
    // the loads of kAhead steps of 64 positions are in flight together (the
    // walk is a chain of steps, each otherwise waiting on its own loads)
    constexpr int kAhead = 4;
    bool done = false;
    while (!done && pos < N && (want == 0 || c.cnt < want)) {
      int Lv[kAhead];
      bool badv[kAhead];
      float fvv[kAhead];
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const int p = pos + kWave * u + lane;
        const bool valid = p < N;
        // three independent coalesced loads per position: leaf, bound, filter value
        Lv[u] = valid ? oq[p] : 0;
        badv[u] = valid && lbq[p] > tau_lb;
        fvv[u] = valid && use_f ? fq[p] : -__builtin_inff();
      }
      // the leaves' series counts, all requested before any is used
      int nv[kAhead];
#pragma unroll
      for (int u = 0; u < kAhead; ++u) nv[u] = leaf_n[Lv[u]];
      // step u starts at the iteration's first position + 64 u: every step
      // before it was a full 64 positions, or the walk has ended
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        if (pos >= N || (want != 0 && c.cnt >= want)) {
          done = true;
          break;
        }
        const int L = Lv[u];
        const bool lbbad = badv[u];
        const float fv = fvv[u];
        const uint64_t mbad = __ballot(lbbad);
        const int nvalid = N - pos < kWave ? N - pos : kWave;
        const int s = mbad ? __ffsll(static_cast<unsigned long long>(mbad)) - 1 : kWave;
        const int stop = s < nvalid ? s : nvalid;
        const bool in = lane < stop;
        const bool fpr = in && fv > tau;
        const bool surv = in && !fpr;
        uint64_t msurv = __ballot(surv);
        int end = stop;
        bool cut = false;
        if (want > 0 && __popcll(msurv) > want - c.cnt) {
          const int need = want - c.cnt;
          const int rank = __popcll(msurv & lt);
          const uint64_t mlast = __ballot(surv && rank == need - 1);
          end = __ffsll(static_cast<unsigned long long>(mlast));  // one past the need-th survivor
          msurv &= end >= kWave ? ~0ull : ((1ull << end) - 1ull);
          cut = true;
        }
        const uint64_t mend = end >= kWave ? ~0ull : ((1ull << end) - 1ull);
        if ((msurv >> lane) & 1ull) {
          const int rank = __popcll(msurv & lt);
          b.qitem_leaf[q * N + base + c.cnt + rank] = L;
          atomicAdd(b.leaf_cnt + L, 1);
          c.series += nv[u];
        }
        c.cnt += __popcll(msurv);
        c.fp += __popcll(__ballot(fpr) & mend);
        if (cut) {
          pos += end;
          done = true;
          break;
        }
        if (s < nvalid) {
          c.lbp += N - (pos + s);
          pos = N;
          done = true;
          break;
        }
        pos += nvalid;
      }
    }
  }
  c.series = wave_sum(c.series);
  if (lane == 0) {
    b.cursor[q] = pos;
    b.qitem_cnt[q] = base + c.cnt;
  }
  return c;
}

__global__ void __launch_bounds__(64 * kListWaves) k_worklist(int64_t nq, int N, const float *__restrict__ lbs,
                                                             const int32_t *__restrict__ order,
                                                             const float *__restrict__ dfo,
                                                             const int32_t *__restrict__ leaf_n, int want,
                                                             Schedule sched, int32_t *qround, RoundBufs b,
                                                             int append) {
  __shared__ int64_t stat[4][kListWaves];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  // the round's control words start from zero (nothing reads them during
  // this kernel), and so do the per-leaf fill counters of the placement
  if (blockIdx.x == 0 && threadIdx.x < kCtlRoundWords) b.ctl[threadIdx.x] = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < N;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    b.leaf_fill[i] = 0;
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kListWaves + wave;
  CascadeCount c;
  if (q < nq) {
    if (qround && b.cursor[q] < N) {
      // serving: each query follows its own schedule from its own round count
      const int r = qround[q];
      want = sched.r[r < sched.n ? r : sched.n - 1];
      if (lane == 0) qround[q] = r + 1;
    }
    // with `append`, the rescans the last merge queued stay first in the list
    c = cascade_query(q, N, lbs, order, dfo, leaf_n, want, b.tau[q], b, lane, append ? b.qitem_cnt[q] : 0);
  }
  // one atomic per counter and work-group
  if (lane == 0) {
    stat[0][wave] = c.lbp;
    stat[1][wave] = c.fp;
    stat[2][wave] = c.cnt;
    stat[3][wave] = c.series;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    int64_t v = 0;
    for (int w = 0; w < kListWaves; ++w) v += stat[threadIdx.x][w];
    const int word = threadIdx.x == 0 ? kCtlLbPruned : threadIdx.x == 1 ? kCtlFPruned
                   : threadIdx.x == 2 ? kCtlScanned : kCtlSeries;
    if (v) atomicAdd(reinterpret_cast<unsigned long long *>(b.ctl + word), static_cast<unsigned long long>(v));
  }
}

// Filter pairs worth evaluating once tau is known: every (query, visit
// position) ahead of the cursor whose leaf has a filter and whose bound does
// not prune it.  Later rounds only lower tau, so no other pair can reach the
// filter test, and no cascade reaches a position whose bound prunes it now.
// Filter f collects its entries q * N + position in plist[f * nq + ...]; the
// other positions ahead of the cursor within the bound get dfo = -inf.
__global__ void __launch_bounds__(256) k_filter_pairs(int64_t nq, int N, const float *__restrict__ lbs,
                                                      const int32_t *__restrict__ order,
                                                      const int32_t *__restrict__ filt_of_leaf, RoundBufs b,
                                                      const int32_t *__restrict__ qround, int64_t *plist,
                                                      int32_t *pcnt, float *dfo) {
  __shared__ int fe_sh[4];
  int n_fe = 0;  // pairs this lane queued (counted once per work-group: a per-wavefront atomic on
                 // one control word serialised on its cache line)
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < nq * N;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t q = idx / N;
    const int pos = static_cast<int>(idx - q * N);
    if (qround && qround[q] != 1) continue;  // serving: only queries that just finished their first round
    if (pos < b.cursor[q] || b.pair[q] < 0) continue;
    if (lbs[idx] > b.tau[q] * (1.0f + kLbSlack)) continue;  // pruned by its bound in every later round
    const int f = filt_of_leaf[order[idx]];
    if (f < 0) {
      dfo[idx] = -__builtin_inff();
      continue;
    }
    const int slot = atomicAdd(pcnt + f, 1);
    plist[static_cast<int64_t>(f) * nq + slot] = idx;
    ++n_fe;
  }
  n_fe = wave_sum(n_fe);
  if ((threadIdx.x & (kWave - 1)) == 0) fe_sh[threadIdx.x / kWave] = n_fe;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int e = fe_sh[0] + fe_sh[1] + fe_sh[2] + fe_sh[3];
    if (e) atomicAdd(reinterpret_cast<unsigned long long *>(b.ctl + kCtlFEvals), static_cast<unsigned long long>(e));
  }
}

__global__ void __launch_bounds__(256) k_emit_fallback(int N, RoundBufs b) {
  const int64_t n_fb = b.ctl[kCtlFallback];
  if (blockIdx.x == 0 && threadIdx.x == 0 && n_fb > 0)
    atomicAdd(reinterpret_cast<unsigned long long *>(b.ctl + kCtlFbTotal), static_cast<unsigned long long>(n_fb));
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n_fb;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int q = b.fb_q[i];
    int L = b.fb_leaf[i];
    int r = atomicAdd(b.qitem_cnt + q, 1);
    b.qitem_leaf[static_cast<int64_t>(q) * N + r] = L;
    atomicAdd(b.leaf_cnt + L, 1);
  }
}

__global__ void __launch_bounds__(256) k_round_reset(RoundBufs b, int n_ctl, int N, int64_t nq) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n_ctl) b.ctl[i] = 0;
  if (n_ctl > 0 && i == 0) b.ctl[kCtlOverflow] = 0;  // a fresh round of a host-driven or served sequence
  if (i < N) b.leaf_cnt[i] = 0;
  if (i < nq) b.qitem_cnt[i] = 0;
}

// Exclusive scans over leaves: item starts and tile starts (the whole
// work-group of 1024 threads).  `publish` writes them, the round's control
// words and (with zero_fill) zeroed per-leaf fill counters to global memory;
// `ist` (optional, LDS [N]) receives the item starts.  Returns true when the
// round must lay out nothing: its items or tiles exceed b.cap_items or
// b.cap_tiles, or an earlier round's did (ctl[kCtlOverflow]); the published
// item and tile counts are then zero and the overflow word is set.
__device__ inline bool leaf_scan_body(int N, const int64_t *__restrict__ leaf_off, int mq, int64_t row_bytes,
                                      RoundBufs &b, int64_t *sh, bool publish = true, bool zero_fill = true,
                                      int32_t *ist = nullptr, const int32_t *cnt_src = nullptr) {
  // read before any work-group of this launch can set it (every one decides
  // the same from its own counts)
  const bool earlier = b.ctl[kCtlOverflow] != 0;
  const int32_t *cnt = cnt_src ? cnt_src : b.leaf_cnt;
  const int tid = threadIdx.x;
  const int per = (N + 1023) / 1024;
  const int l0 = min(N, tid * per), l1 = min(N, l0 + per);
  int64_t si = 0, stl = 0, rows = 0;
  for (int L = l0; L < l1; ++L) {
    int c = cnt[L];
    int64_t chunks = (leaf_off[L + 1] - leaf_off[L] + b.chunk - 1) / b.chunk;
    si += c;
    stl += static_cast<int64_t>((c + mq - 1) / mq) * chunks;
    if (c > 0) rows += b.leaf_n[L];
  }
  // item and tile counts share one scan (each total < 2^31: packed as
  // items + tiles * 2^32, the low half never carries), rows a second
  int64_t tot_it, tot_r;
  const int64_t rit = block_scan_excl<1024>(si + (stl << 32), sh, tot_it);
  block_scan_excl<1024>(rows, sh, tot_r);
  int64_t ri = rit & 0xffffffffll, rt = rit >> 32;
  const int64_t tot_i = tot_it & 0xffffffffll, tot_t = tot_it >> 32;
  for (int L = l0; L < l1; ++L) {
    int c = cnt[L];
    int64_t chunks = (leaf_off[L + 1] - leaf_off[L] + b.chunk - 1) / b.chunk;
    if (ist) ist[L] = static_cast<int32_t>(ri);
    if (publish) {
      b.leaf_istart[L] = static_cast<int32_t>(ri);
      b.tile_start[L] = static_cast<int32_t>(rt);
      if (zero_fill) b.leaf_fill[L] = 0;
    }
    ri += c;
    rt += static_cast<int64_t>((c + mq - 1) / mq) * chunks;
  }
  const bool over = earlier || (b.cap_items > 0 && tot_i > b.cap_items) || (b.cap_tiles > 0 && tot_t > b.cap_tiles);
  if (publish && tid == 0) {
    b.leaf_istart[N] = static_cast<int32_t>(tot_i);
    b.tile_start[N] = static_cast<int32_t>(tot_t);
    b.ctl[kCtlItems] = over ? 0 : tot_i;
    b.ctl[kCtlTiles] = over ? 0 : tot_t;
    b.ctl[kCtlLive] = 0;
    if (over) b.ctl[kCtlOverflow] = 1;
    if (!over && row_bytes > 0 && tot_i > 0) {
      b.ctl[kCtlScanBytes] += tot_r * row_bytes;
      b.ctl[kCtlRounds] += 1;
    }
  }
  return over;
}

__global__ void __launch_bounds__(1024) k_leaf_scan(int N, const int64_t *__restrict__ leaf_off, int mq,
                                                    int64_t row_bytes, RoundBufs b) {
  __shared__ int64_t sh[16];
  leaf_scan_body(N, leaf_off, mq, row_bytes, b, sh);
}

// A small pass (the exact rescan of a round's few uncertified items) in one
// launch instead of two: the leaf scan, then every query's items placed by
// one thread each (the placement is k_scatter's).
__global__ void __launch_bounds__(1024) k_leaf_scan_scatter(int64_t nq, int N, const int64_t *__restrict__ leaf_off,
                                                            int mq, int64_t row_bytes, RoundBufs b, int lds_starts) {
  extern __shared__ int32_t s_ist[];  // [N] with lds_starts, else unused
  __shared__ int64_t sh[16];
  // each thread's first query's item count, requested before the leaf scan
  const int n0 = threadIdx.x < nq ? b.qitem_cnt[threadIdx.x] : 0;
  const bool over = leaf_scan_body(N, leaf_off, mq, row_bytes, b, sh, true, true, lds_starts ? s_ist : nullptr);
  __syncthreads();  // item starts written; the per-leaf counts are consumed
  const int32_t *ist = lds_starts ? s_ist : b.leaf_istart;
  for (int i = threadIdx.x; i < N; i += blockDim.x) b.leaf_cnt[i] = 0;
  if (over) return;  // uniform: nothing is placed
  for (int64_t q = threadIdx.x; q < nq; q += blockDim.x) {
    const int n = q == threadIdx.x ? n0 : b.qitem_cnt[q];
    for (int r = 0; r < n; ++r) {
      const int L = b.qitem_leaf[q * N + r];
      const int slot = ist[L] + atomicAdd(b.leaf_fill + L, 1);
      b.item_q[slot] = static_cast<int32_t>(q);
      b.item_leaf[slot] = L;
      b.qitem_idx[q * N + r] = slot;
    }
  }
}

// The leaf scan and the item placement in one launch for up to
// kLayoutLdsMax leaves: every work-group computes the item starts itself into
// LDS (work-group 0 also publishes them), then places its 16 queries' items
// as k_scatter does.  leaf_fill must be zero on entry (the prune cascade
// zeroes it); leaf_cnt is left for the rerank to zero.
__global__ void __launch_bounds__(1024) k_layout_scatter(int64_t nq, int N, const int64_t *__restrict__ leaf_off,
                                                         int mq, int64_t row_bytes, RoundBufs b) {
  extern __shared__ int32_t s_ist[];  // [N]
  __shared__ int64_t sh[16];
  // the wavefront's query's item list is requested before the leaf scan, so
  // its latency hides under the scan's
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t q = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave;
  int n = 0, L0 = 0;
  if (q < nq) {
    n = b.qitem_cnt[q];
    if (lane < n) L0 = b.qitem_leaf[q * N + lane];
  }
  const bool over = leaf_scan_body(N, leaf_off, mq, row_bytes, b, sh, blockIdx.x == 0, false, s_ist);
  __syncthreads();
  if (q >= nq || over) return;
  for (int r = lane; r < n; r += kWave) {
    const int L = r == lane ? L0 : b.qitem_leaf[q * N + r];
    const int slot = s_ist[L] + atomicAdd(b.leaf_fill + L, 1);
    b.item_q[slot] = static_cast<int32_t>(q);
    b.item_leaf[slot] = L;
    b.qitem_idx[q * N + r] = slot;
  }
}

// A first round of one leaf per query (tau is +inf and no filter is
// evaluated yet, so nothing is pruned and each query's item is the first
// leaf of its visit order) laid out in one single-work-group launch instead
// of the prune cascade plus the layout: per-leaf counts in LDS, the leaf
// scan, the placement, the query's cursor and item list, and the cascade's
// statistics (leaves scanned, series).  Work-group 0 of the batch's query
// preparation has zeroed the control words.
__global__ void __launch_bounds__(1024) k_first_round_layout(int64_t nq, int N, const int32_t *__restrict__ order,
                                                             const int64_t *__restrict__ leaf_off,
                                                             const int32_t *__restrict__ leaf_n, int mq,
                                                             int64_t row_bytes, RoundBufs b) {
  // [N] counts (then fill counters), [N] item starts, [N + 1] leaf offsets
  // (int64, 8-byte aligned: 2 N ints before them, N even or padded), [N] leaf sizes
  extern __shared__ int32_t s_lds[];
  int32_t *s_cnt = s_lds, *s_ist = s_lds + N;
  int64_t *s_off = reinterpret_cast<int64_t *>(s_lds + 2 * N + (N & 1));
  int32_t *s_n = reinterpret_cast<int32_t *>(s_off + N + 1);
  __shared__ int64_t sh[16];
  // every global input requested at once: the leaves' offsets and sizes
  // into LDS and each thread's first query's first leaf into a register
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    s_cnt[i] = 0;
    s_off[i] = leaf_off[i];
    s_n[i] = leaf_n[i];
  }
  if (threadIdx.x == 0) s_off[N] = leaf_off[N];
  const int L0 = threadIdx.x < nq ? order[static_cast<int64_t>(threadIdx.x) * N] : 0;
  __syncthreads();
  if (threadIdx.x < nq) atomicAdd(s_cnt + L0, 1);
  for (int64_t q = threadIdx.x + blockDim.x; q < nq; q += blockDim.x) atomicAdd(s_cnt + order[q * N], 1);
  __syncthreads();
  const bool over = leaf_scan_body(N, s_off, mq, row_bytes, b, sh, true, false, s_ist, s_cnt);
  if (over) return;  // uniform (a planned first round is sized for every query)
  // series in the round's items: sum over leaves of count x real rows
  int64_t series = 0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) series += static_cast<int64_t>(s_cnt[i]) * s_n[i];
  int64_t tot_series;
  block_scan_excl<1024>(series, sh, tot_series);
  // the counts are consumed: they become the LDS fill counters of the placement
  for (int i = threadIdx.x; i < N; i += blockDim.x) s_cnt[i] = 0;
  __syncthreads();
  for (int64_t q = threadIdx.x; q < nq; q += blockDim.x) {
    const int L = q == threadIdx.x ? L0 : order[q * N];
    const int slot = s_ist[L] + atomicAdd(s_cnt + L, 1);
    b.item_q[slot] = static_cast<int32_t>(q);
    b.item_leaf[slot] = L;
    b.qitem_leaf[q * N] = L;
    b.qitem_idx[q * N] = slot;
    b.qitem_cnt[q] = 1;
    b.cursor[q] = 1;
  }
  if (threadIdx.x == 0) {
    b.ctl[kCtlScanned] += nq;
    b.ctl[kCtlSeries] += tot_series;
  }
}

// One wavefront per query: place its emitted leaves into item slots.
__global__ void __launch_bounds__(1024) k_scatter(int64_t nq, int N, RoundBufs b) {
  const int lane = threadIdx.x & (kWave - 1);
  // the per-leaf item counts were consumed by the leaf scan: leave them zero
  // for the next pass (the merge counts rescan items into them)
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < N;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    b.leaf_cnt[i] = 0;
  const int64_t q = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (q >= nq || b.ctl[kCtlOverflow] != 0) return;  // an overflowed round places nothing
  const int n = b.qitem_cnt[q];
  for (int r = lane; r < n; r += kWave) {
    int L = b.qitem_leaf[q * N + r];
    int slot = b.leaf_istart[L] + atomicAdd(b.leaf_fill + L, 1);
    b.item_q[slot] = static_cast<int32_t>(q);
    b.item_leaf[slot] = L;
    b.qitem_idx[q * N + r] = slot;
  }
}

// One wavefront per query: merge the round's item results into the running
// top-k (sorted by (FP64 distance, row)), refresh tau and, in a regular
// round, queue every item whose certificate bound does not exceed the new tau
// for a rescan (by the next round's scan, or an exact FP32 pass after the
// last round).  Every list is already sorted (the running top-k and each
// item's exact top-k), so the k smallest of their union are selected by a
// tournament over the list heads (merge_pass_staged), not a sort of
// everything: each round takes the wavefront minimum of the items' heads and
// emits either the run of running-list entries below it (up to 64 at once)
// or that minimum, so a pass costs about as many rounds as item entries
// enter the top k.  A row met twice (a rescan of a leaf already merged)
// carries the same (distance, row) in both lists and is kept once.
constexpr int kMergePreFp = 4;  // visit positions per lane whose filter-pair inputs the merge prefetches
constexpr int kMergeSlots = 4;  // item lists per lane in one tournament pass (256 items per pass)

// Non-negative doubles order like their bit patterns.
__device__ __forceinline__ uint64_t dbl_bits(double v) { return static_cast<uint64_t>(__double_as_longlong(v)); }

// One pass of the tournament: the k smallest distinct (distance, row)
// entries of the sorted list in (in_v, in_t) (n_in entries, LDS) and of the
// item lists qitem_idx[q N + it0 ..] go to (out_v, out_t) in ascending order;
// returns how many.  The pass's lists are staged in LDS first: every entry of
// the (at most 64 kMergeSlots) lists, each cut to k, is loaded at once (all
// loads in flight together, not one dependent load per round), so the
// tournament's rounds read LDS only.  Takes the leading items whose entries
// fit kMergeStage (at least one: an item has at most k <= 256 entries) and
// sets *consumed to their number; the caller passes the rest again.
// stage_v / stage_t hold kMergeStage entries, soff and sidx 64 kMergeSlots + 1
// ints.
constexpr int kMergeStage = 1024;

// LDS of one merge wavefront: the two kmax-entry lists (16-byte multiple),
// the staged entries, their slot offsets and item indexes.
__host__ __device__ inline size_t merge_lists_bytes(int kmax) {
  return (2 * static_cast<size_t>(kmax) * (sizeof(double) + sizeof(uint32_t)) + 15) / 16 * 16;
}
__host__ __device__ inline size_t merge_slice_bytes(int kmax) {
  const size_t stage = static_cast<size_t>(kMergeStage) * (sizeof(double) + sizeof(uint32_t)) +
                       (2 * kWave * kMergeSlots + 1) * sizeof(int);
  return merge_lists_bytes(kmax) + (stage + 15) / 16 * 16;
}

__device__ inline int merge_pass_staged(int64_t q, int N, int kmax, int k, const RoundBufs &b, int it0, int nb,
                                        const double *in_v, const uint32_t *in_t, int n_in, double *out_v,
                                        uint32_t *out_t, int lane, double *stage_v, uint32_t *stage_t, int *soff,
                                        int *sidx, int *consumed) {
  constexpr double kInf = __builtin_inf();
  constexpr int kSlots = kWave * kMergeSlots;
  int cnt[kMergeSlots], off[kMergeSlots];
  int total = 0;
#pragma unroll
  for (int i = 0; i < kMergeSlots; ++i) {
    const int j = lane + kWave * i;
    int idx = 0, c = 0;
    if (j < nb) {
      idx = b.qitem_idx[q * N + it0 + j];
      c = b.item_cnt[idx];
      c = c < k ? c : k;
    }
    // slot 64 i + lane starts after every slot before it
    int x = c;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(x, o, kWave);
      if (lane >= o) x += y;
    }
    off[i] = total + x - c;
    total += __shfl(x, kWave - 1, kWave);
    cnt[i] = c;
    sidx[j] = idx;
  }
  // the leading items whose entries fit the staging area (slot order
  // follows item order, so they are a prefix); the rest wait for the next call
  int used = 0, staged = 0;
#pragma unroll
  for (int i = 0; i < kMergeSlots; ++i) {
    const bool fit = lane + kWave * i < nb && off[i] + cnt[i] <= kMergeStage;
    used += __popcll(__ballot(fit));
    if (!fit) cnt[i] = 0;
    staged = max(staged, wave_max(fit ? off[i] + cnt[i] : 0));
  }
  *consumed = used;
  total = staged;
#pragma unroll
  for (int i = 0; i < kMergeSlots; ++i) soff[lane + kWave * i] = cnt[i] > 0 ? off[i] : min(off[i], total);
  if (lane == 0) soff[kSlots] = total;
  wave_lds_sync();
  // entry e of the staged lists belongs to the last slot s with soff[s] <= e
  // (slots with no entries share their successor's offset)
  constexpr int kU = 4;  // entries per lane in flight together
  for (int e0 = 0; e0 < total; e0 += kWave * kU) {
    double v[kU];
    uint32_t t[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + lane + kWave * u;
      int sl = 0;
      if (e < total) {
        int lo = 0, hi = kSlots;  // soff[lo] <= e < soff[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (soff[mid] <= e) lo = mid;
          else hi = mid;
        }
        sl = lo;
      }
      const int64_t at = static_cast<int64_t>(sidx[sl]) * kmax + (e < total ? e - soff[sl] : 0);
      v[u] = b.item_d2[at];
      t[u] = static_cast<uint32_t>(b.item_row[at]);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + lane + kWave * u;
      if (e < total) {
        stage_v[e] = v[u];
        stage_t[e] = t[u];
      }
    }
  }
  wave_lds_sync();
  double hv[kMergeSlots];
  uint32_t ht[kMergeSlots];
  int pos[kMergeSlots];
#pragma unroll
  for (int i = 0; i < kMergeSlots; ++i) {
    pos[i] = 0;
    hv[i] = cnt[i] > 0 ? stage_v[off[i]] : kInf;
    ht[i] = cnt[i] > 0 ? stage_t[off[i]] : 0xffffffffu;
  }
  int out = 0, rp = 0;
  while (out < k) {
    // smallest head of the staged lists
    double lv = kInf;
    uint32_t lt = 0xffffffffu;
#pragma unroll
    for (int i = 0; i < kMergeSlots; ++i)
      if (hv[i] < lv || (hv[i] == lv && ht[i] < lt)) {
        lv = hv[i];
        lt = ht[i];
      }
    const uint64_t mvb = wave_min_u64(dbl_bits(lv));
    const uint64_t mtb = wave_min_u64(dbl_bits(lv) == mvb ? static_cast<uint64_t>(lt) : ~0ull);
    const double gv = __longlong_as_double(static_cast<long long>(mvb));
    const uint32_t gt = static_cast<uint32_t>(mtb);
    // the running list's entries below it come next, as one run (up to a
    // wavefront's worth per round; lane j checks entry rp + j)
    bool below = false;
    if (rp + lane < n_in && out + lane < k) {
      const double v = in_v[rp + lane];
      const uint32_t t = in_t[rp + lane];
      below = v < gv || (v == gv && t < gt);
    }
    const uint64_t bm = __ballot(below);
    const int run = ~bm == 0 ? kWave : __builtin_ctzll(~bm);
    if (run > 0) {
      if (lane < run) {
        out_v[out + lane] = in_v[rp + lane];
        out_t[out + lane] = in_t[rp + lane];
      }
      out += run;
      rp += run;
      continue;
    }
    if (gt == 0xffffffffu) break;  // every list is exhausted
    // With one staged list left (a query's first round has one item), its
    // entries below the running head come next, as one run likewise.
    int live = 0, owner = 0, oslot = 0;
#pragma unroll
    for (int i = 0; i < kMergeSlots; ++i) {
      const uint64_t bl = __ballot(pos[i] < cnt[i]);
      if (bl != 0 && live == 0) {
        owner = __builtin_ctzll(bl);
        oslot = i;
      }
      live += __popcll(bl);
    }
    if (live == 1) {
      int po = 0, oo = 0, co = 0;
#pragma unroll
      for (int i = 0; i < kMergeSlots; ++i)
        if (i == oslot) {
          po = pos[i];
          oo = off[i];
          co = cnt[i];
        }
      po = __shfl(po, owner, kWave);
      oo = __shfl(oo, owner, kWave);
      co = __shfl(co, owner, kWave);
      const double rv = rp < n_in ? in_v[rp] : kInf;
      const uint32_t rt = rp < n_in ? in_t[rp] : 0xffffffffu;
      bool take = false;
      if (po + lane < co && out + lane < k) {
        const double v = stage_v[oo + po + lane];
        const uint32_t t = stage_t[oo + po + lane];
        take = v < rv || (v == rv && t < rt);
      }
      const uint64_t tm = __ballot(take);
      const int run2 = ~tm == 0 ? kWave : __builtin_ctzll(~tm);
      if (run2 > 0) {
        if (lane < run2) {
          out_v[out + lane] = stage_v[oo + po + lane];
          out_t[out + lane] = stage_t[oo + po + lane];
        }
        out += run2;
        if (lane == owner) {
#pragma unroll
          for (int i = 0; i < kMergeSlots; ++i)
            if (i == oslot) {
              pos[i] += run2;
              const bool more = pos[i] < cnt[i];
              hv[i] = more ? stage_v[off[i] + pos[i]] : kInf;
              ht[i] = more ? stage_t[off[i] + pos[i]] : 0xffffffffu;
            }
        }
        continue;
      }
    }
    // else the staged minimum (the running head too when it is the same row)
    if (lane == 0) {
      out_v[out] = gv;
      out_t[out] = gt;
    }
    ++out;
    if (rp < n_in && in_v[rp] == gv && in_t[rp] == gt) ++rp;
#pragma unroll
    for (int i = 0; i < kMergeSlots; ++i) {
      if (hv[i] == gv && ht[i] == gt) {
        ++pos[i];
        const bool more = pos[i] < cnt[i];
        hv[i] = more ? stage_v[off[i] + pos[i]] : kInf;
        ht[i] = more ? stage_t[off[i] + pos[i]] : 0xffffffffu;
      }
    }
  }
  wave_lds_sync();
  return out;
}

__global__ void __launch_bounds__(256) k_query_merge(int64_t nq, int N, int kmax, int check_cert,
                                                     RoundBufs b, const int64_t *__restrict__ rowid,
                                                     int64_t *out_ids, float *out_d, FilterPairArgs fp) {
  extern __shared__ unsigned char smem_raw[];
  // four wavefronts per work-group, each with its own LDS slice and query:
  // two lists of kmax entries (the tournament's input and output), then the
  // staging area of merge_pass_staged
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  unsigned char *mine = smem_raw + static_cast<size_t>(wave) * merge_slice_bytes(kmax);
  double *buf_v = reinterpret_cast<double *>(mine);
  uint32_t *buf_t = reinterpret_cast<uint32_t *>(mine + sizeof(double) * 2 * kmax);
  double *stage_v = reinterpret_cast<double *>(mine + merge_lists_bytes(kmax));
  uint32_t *stage_t = reinterpret_cast<uint32_t *>(stage_v + kMergeStage);
  int *soff = reinterpret_cast<int *>(stage_t + kMergeStage);
  int *sidx = soff + kWave * kMergeSlots + 1;
  const uint64_t lt = (1ull << lane) - 1ull;
  __shared__ int active_sh[4], fb_sh[4], fe_sh[4];
  // after a capacity overflow the item lists were never placed: nothing to merge
  if (b.ctl[kCtlOverflow] != 0) return;
  int active = 0, n_fb = 0, n_fe = 0;  // n_fe: this lane's queued filter pairs
  for (int64_t q = static_cast<int64_t>(blockIdx.x) * 4 + wave; q < nq; q += static_cast<int64_t>(gridDim.x) * 4) {
    // Loads that do not depend on the merge are issued before it, so that
    // the query's chain of dependent global loads stays short: the filter-pair
    // inputs of this lane's visit positions (N <= 64 kMergePreFp) and the
    // certificate inputs of the query's first 64 items.
    const int n_it = b.qitem_cnt[q];
    const int k = b.kq[q];
    const int have = b.res_cnt[q];
    const bool pre_fp = fp.plist && N <= kMergePreFp * kWave;
    int cur = 0, pq = -1;
    if (fp.plist) {
      cur = b.cursor[q];
      pq = b.pair[q];
    }
    int pf[kMergePreFp];
    float pl[kMergePreFp];
#pragma unroll
    for (int c = 0; c < kMergePreFp; ++c) {
      pf[c] = -1;
      pl[c] = __builtin_inff();
      const int pos = lane + kWave * c;
      if (pre_fp && pos < N) {
        const int64_t idx = q * N + pos;
        pl[c] = fp.lbs[idx];
        pf[c] = fp.filt_of_leaf[fp.order[idx]];
      }
    }
    float cb = __builtin_inff();
    int cl = 0;
    if (check_cert && lane < n_it) {
      const int idx = b.qitem_idx[q * N + lane];
      cb = b.item_bound[idx];
      cl = b.item_leaf[idx];
    }
    float tau_now = __builtin_inff();  // the query's tau after this merge (filter pairs below)
    if (n_it > 0) {
      double *vals = buf_v, *ov = buf_v + kmax;
      uint32_t *tags = buf_t, *ot = buf_t + kmax;
      for (int i = lane; i < kmax; i += kWave) {
        const double v = b.res_d2[q * kmax + i];  // loaded unconditionally, kept below `have`
        const uint32_t t = static_cast<uint32_t>(b.res_row[q * kmax + i]);
        vals[i] = i < have ? v : __builtin_inf();
        tags[i] = i < have ? t : 0xffffffffu;
      }
      wave_lds_sync();
      int n_in = have < k ? have : k;
      for (int it0 = 0; it0 < n_it;) {
        const int nb = n_it - it0 < kWave * kMergeSlots ? n_it - it0 : kWave * kMergeSlots;
        int used = 0;
        n_in = merge_pass_staged(q, N, kmax, k, b, it0, nb, vals, tags, n_in, ov, ot, lane, stage_v, stage_t, soff,
                                 sidx, &used);
        it0 += used;
        double *sv = vals;
        vals = ov;
        ov = sv;
        uint32_t *st = tags;
        tags = ot;
        ot = st;
      }
      for (int i = n_in + lane; i < kmax; i += kWave) {
        vals[i] = __builtin_inf();
        tags[i] = 0xffffffffu;
      }
      wave_lds_sync();
      int cnt = 0;
      for (int i = 0; i < k; ++i) cnt += tags[i] != 0xffffffffu ? 1 : 0;
      for (int i = lane; i < k; i += kWave) {
        b.res_d2[q * kmax + i] = vals[i];
        b.res_row[q * kmax + i] = static_cast<int32_t>(tags[i]);
      }
      float tau = __builtin_inff();
      if (cnt == k) {
        double d = sqrt(vals[k - 1]);
        tau = static_cast<float>(d);
        if (static_cast<double>(tau) < d) tau = nextafterf(tau, __builtin_inff());
      }
      if (lane == 0) {
        b.res_cnt[q] = cnt;
        b.tau[q] = tau;
      }
      tau_now = tau;
      // the query's item list becomes its rescan list: every item whose
      // certificate bound does not exceed the new tau, in item order
      int nr = 0;
      if (check_cert) {
        for (int it0 = 0; it0 < n_it; it0 += kWave) {
          const int it = it0 + lane;
          bool un = false;
          int L = 0;
          if (it < n_it) {
            if (it0 == 0) {
              un = !(cb > tau);
              L = cl;
            } else {
              const int idx = b.qitem_idx[q * N + it];
              un = !(b.item_bound[idx] > tau);
              L = b.item_leaf[idx];
            }
          }
          const uint64_t mu = __ballot(un);
          if (un) {
            b.qitem_leaf[q * N + nr + __popcll(mu & lt)] = L;
            atomicAdd(b.leaf_cnt + L, 1);
          }
          nr += __popcll(mu);
        }
        n_fb += nr;
      }
      if (out_ids) {  // the batch's last merge: write the query's output row
        for (int i = lane; i < kmax; i += kWave) {
          const bool hit = i < cnt;
          out_ids[q * kmax + i] = hit ? rowid[tags[i]] : -1;
          out_d[q * kmax + i] = hit ? static_cast<float>(sqrt(vals[i])) : __builtin_inff();
        }
      }
      wave_lds_sync();
      if (lane == 0) b.qitem_cnt[q] = nr;  // the rescan pass's items of this query (usually none)
    } else if (out_ids) {
      const int cnt = b.res_cnt[q];
      for (int i = lane; i < kmax; i += kWave) {
        const bool hit = i < cnt;
        out_ids[q * kmax + i] = hit ? rowid[b.res_row[q * kmax + i]] : -1;
        out_d[q * kmax + i] = hit ? static_cast<float>(sqrt(b.res_d2[q * kmax + i])) : __builtin_inff();
      }
    }
    if (fp.plist) {
      // the query's filter pairs for the rounds to come (k_filter_pairs'
      // selection, from the tau just merged)
      if (n_it <= 0) tau_now = b.tau[q];
      if (pq >= 0) {
        if (pre_fp) {
#pragma unroll
          for (int c = 0; c < kMergePreFp; ++c) {
            const int pos = lane + kWave * c;
            if (pos >= cur && pos < N) {
              const int64_t idx = q * N + pos;
              const int f = pf[c];
              if (f < 0 || pl[c] > tau_now * (1.0f + kLbSlack)) {
                fp.dfo[idx] = -__builtin_inff();
              } else {
                fp.plist[static_cast<int64_t>(f) * nq + atomicAdd(fp.pcnt + f, 1)] = idx;
                ++n_fe;
              }
            }
          }
        } else {
          // The bounds ascend along the visit order, so the positions within
          // the cutoff are a prefix: the walk ends at the first one past it.
          // No later cascade reaches a position past it (tau only falls), so
          // those keep no filter value.  Four steps of 64 positions have
          // their loads in flight together.
          const float cutoff = tau_now * (1.0f + kLbSlack);
          constexpr int kAhead = 4;
          for (int pos0 = cur; pos0 < N; pos0 += kAhead * kWave) {
            float lv[kAhead];
            int ov[kAhead], fv[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
              const int pos = pos0 + kWave * u + lane;
              const int64_t idx = q * N + pos;
              lv[u] = pos < N ? fp.lbs[idx] : __builtin_inff();
              ov[u] = pos < N ? fp.order[idx] : 0;
            }
#pragma unroll
            for (int u = 0; u < kAhead; ++u) fv[u] = fp.filt_of_leaf[ov[u]];
            bool end = false;
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
              const int pos = pos0 + kWave * u + lane;
              const int64_t idx = q * N + pos;
              const bool within = pos < N && lv[u] <= cutoff;
              if (within) {
                const int f = fv[u];
                if (f < 0) {
                  fp.dfo[idx] = -__builtin_inff();
                } else {
                  fp.plist[static_cast<int64_t>(f) * nq + atomicAdd(fp.pcnt + f, 1)] = idx;
                  ++n_fe;
                }
              }
              if (__ballot(!within) != 0) {  // uniform: every later position is past the cutoff
                end = true;
                break;
              }
            }
            if (end) break;
          }
        }
      }
    }
    if (check_cert && b.cursor[q] < N) ++active;
  }
  // one atomic per work-group for the count of queries with leaves left, for
  // the rescan items and for the queued filter pairs
  if (fp.plist) n_fe = wave_sum(n_fe);
  if (lane == 0) {
    fe_sh[wave] = n_fe;
    active_sh[wave] = active;
    fb_sh[wave] = n_fb;
  }
  __syncthreads();
  if (fp.plist && threadIdx.x == 0) {
    const int e = fe_sh[0] + fe_sh[1] + fe_sh[2] + fe_sh[3];
    if (e) atomicAdd(reinterpret_cast<unsigned long long *>(b.ctl + kCtlFEvals), static_cast<unsigned long long>(e));
  }
  if (check_cert && threadIdx.x == 0) {
    const int a = active_sh[0] + active_sh[1] + active_sh[2] + active_sh[3];
    const int f = fb_sh[0] + fb_sh[1] + fb_sh[2] + fb_sh[3];
    if (a) atomicAdd(reinterpret_cast<unsigned long long *>(b.ctl + kCtlActive), static_cast<unsigned long long>(a));
    if (f) {
      atomicAdd(reinterpret_cast<unsigned long long *>(b.ctl + kCtlFallback), static_cast<unsigned long long>(f));
      atomicAdd(reinterpret_cast<unsigned long long *>(b.ctl + kCtlFbTotal), static_cast<unsigned long long>(f));
    }
  }
}

__global__ void __launch_bounds__(256) k_finalize(int64_t nq, int kmax, const int64_t *__restrict__ rowid,
                                                  RoundBufs b, int64_t *ids, float *dists) {
  int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= nq * kmax) return;
  int64_t q = idx / kmax;
  int i = static_cast<int>(idx - q * kmax);
  if (i < b.res_cnt[q]) {
    ids[idx] = rowid[b.res_row[idx]];
    dists[idx] = static_cast<float>(sqrt(b.res_d2[idx]));
  } else {
    ids[idx] = -1;
    dists[idx] = __builtin_inff();
  }
}

__global__ void __launch_bounds__(256) k_items_to_leaf_knn(int64_t n_items, int N, int k, int kmax,
                                                           const int64_t *__restrict__ rowid, RoundBufs b, float *d,
                                                           int64_t *ids) {
  int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n_items * k) return;
  int64_t it = idx / k;
  int i = static_cast<int>(idx - it * k);
  int64_t q = b.item_q[it];
  int L = b.item_leaf[it];
  int64_t o = (q * N + L) * k + i;
  if (i < b.item_cnt[it]) {
    d[o] = static_cast<float>(sqrt(b.item_d2[it * kmax + i]));
    ids[o] = rowid[b.item_row[it * kmax + i]];
  } else {
    d[o] = __builtin_inff();
    ids[o] = -1;
  }
}

__global__ void __launch_bounds__(256) k_select_pairs(int64_t nq, const int32_t *__restrict__ k_dev,
                                                      const float *__restrict__ t_dev, int n_pairs,
                                                      const int32_t *__restrict__ pair_k,
                                                      const float *__restrict__ pair_t, int kmax, int32_t *pair,
                                                      int32_t *kq, const int32_t *__restrict__ slots) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const int64_t q = slots ? slots[i] : i;
  const int k = min(max(k_dev[i], 1), kmax);
  pair[q] = select_pair_of(k, t_dev[i], n_pairs, pair_k, pair_t);
  kq[q] = k;
}

// Serving: retire every active slot whose search has ended (cursor past the
// last leaf): copy its ids and distances to the compact done list.
__global__ void __launch_bounds__(256) k_collect_done(int64_t n_slots, int N, int kmax,
                                                      const int64_t *__restrict__ rowid, RoundBufs b, int32_t *state,
                                                      int32_t *done_slot, int64_t *done_ids, float *done_d,
                                                      int32_t *n_done) {
  int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n_slots || state[q] != 1 || b.cursor[q] < N) return;
  state[q] = 2;
  int j = atomicAdd(n_done, 1);
  done_slot[j] = static_cast<int32_t>(q);
  int c = b.res_cnt[q];
  for (int i = 0; i < kmax; ++i) {
    int64_t o = static_cast<int64_t>(j) * kmax + i;
    if (i < c) {
      done_ids[o] = rowid[b.res_row[q * kmax + i]];
      done_d[o] = static_cast<float>(sqrt(b.res_d2[q * kmax + i]));
    } else {
      done_ids[o] = -1;
      done_d[o] = __builtin_inff();
    }
  }
}

}  // namespace

void launch_worklist(int64_t nq, int N, const float *lbs, const int32_t *order, const float *dfo,
                     const int32_t *leaf_n, int want, RoundBufs b, hipStream_t st, const Schedule *sched,
                     int32_t *qround, bool append) {
  Schedule sc{};
  if (sched) sc = *sched;
  hipLaunchKernelGGL(k_worklist, dim3(ceil_div(std::max<int64_t>(nq, 1), kListWaves)), dim3(64 * kListWaves), 0, st,
                     nq, N, lbs, order, dfo, leaf_n, want, sc, qround, b, append ? 1 : 0);
  LAUNCH_OK("worklist");
}

void launch_filter_pairs(int64_t nq, int N, const float *lbs, const int32_t *order, const int32_t *filt_of_leaf,
                         RoundBufs b, int64_t *plist, int32_t *pcnt, float *dfo, hipStream_t st,
                         const int32_t *qround) {
  // a grid-stride loop over (query, visit position) with a few work-groups per CU
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>(ceil_div(nq * N, 256), 1), 4096);
  hipLaunchKernelGGL(k_filter_pairs, dim3(static_cast<int>(blocks)), dim3(256), 0, st, nq, N, lbs, order,
                     filt_of_leaf, b, qround, plist, pcnt, dfo);
  LAUNCH_OK("filter_pairs");
}

void launch_emit_fallback(int64_t bound, int N, RoundBufs b, hipStream_t st) {
  if (bound <= 0) return;
  const int64_t blocks = ceil_div(bound, 256);  // grid-stride: rescans are few, a small grid launches fast
  hipLaunchKernelGGL(k_emit_fallback, dim3(static_cast<int>(blocks < 64 ? blocks : 64)), dim3(256), 0, st, N, b);
  LAUNCH_OK("emit_fallback");
}

void launch_round_reset(RoundBufs b, int n_ctl, int N, int64_t nq, hipStream_t st) {
  const int64_t n = std::max<int64_t>(std::max<int64_t>(n_ctl, N), nq);
  if (n <= 0) return;
  hipLaunchKernelGGL(k_round_reset, dim3(static_cast<int>(ceil_div(n, 256))), dim3(256), 0, st, b, n_ctl, N, nq);
  LAUNCH_OK("round_reset");
}

void launch_leaf_scan(int N, const int64_t *leaf_off, int mq, int64_t row_bytes, RoundBufs b, hipStream_t st) {
  hipLaunchKernelGGL(k_leaf_scan, dim3(1), dim3(1024), 0, st, N, leaf_off, mq, row_bytes, b);
  LAUNCH_OK("leaf_scan");
}

void launch_first_round_layout(int64_t nq, int N, const int32_t *order, const int64_t *leaf_off,
                               const int32_t *leaf_n, int mq, int64_t row_bytes, RoundBufs b, hipStream_t st) {
  if (N > kLayoutLdsMax) fail(LEAFI_EINTERNAL, "first_round_layout: too many leaves");
  // counts, starts, (padding,) offsets, sizes: at most 80 KiB for 4,096 leaves
  const size_t lds = (2 * static_cast<size_t>(N) + (N & 1)) * sizeof(int32_t) +
                     (static_cast<size_t>(N) + 1) * sizeof(int64_t) + static_cast<size_t>(N) * sizeof(int32_t);
  allow_lds(reinterpret_cast<const void *>(k_first_round_layout), lds);
  hipLaunchKernelGGL(k_first_round_layout, dim3(1), dim3(1024), lds, st, nq, N, order, leaf_off, leaf_n, mq,
                     row_bytes, b);
  LAUNCH_OK("first_round_layout");
}

void launch_leaf_scan_scatter(int64_t nq, int N, const int64_t *leaf_off, int mq, int64_t row_bytes, RoundBufs b,
                              hipStream_t st) {
  const bool lds = N <= kLayoutLdsMax;  // item starts kept in LDS for the placement
  hipLaunchKernelGGL(k_leaf_scan_scatter, dim3(1), dim3(1024), lds ? static_cast<size_t>(N) * sizeof(int32_t) : 0, st,
                     nq, N, leaf_off, mq, row_bytes, b, lds ? 1 : 0);
  LAUNCH_OK("leaf_scan_scatter");
}

void launch_layout_scatter(int64_t nq, int N, const int64_t *leaf_off, int mq, int64_t row_bytes, RoundBufs b,
                           hipStream_t st) {
  if (N > kLayoutLdsMax) fail(LEAFI_EINTERNAL, "layout_scatter: too many leaves");
  hipLaunchKernelGGL(k_layout_scatter, dim3(ceil_div(std::max<int64_t>(nq, 1), 16)), dim3(1024),
                     static_cast<size_t>(N) * sizeof(int32_t), st, nq, N, leaf_off, mq, row_bytes, b);
  LAUNCH_OK("layout_scatter");
}

void launch_scatter(int64_t nq, int N, RoundBufs b, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter, dim3(ceil_div(nq, 16)), dim3(1024), 0, st, nq, N, b);  // 16 queries per work-group
  LAUNCH_OK("scatter");
}

void launch_query_merge(int64_t nq, int N, int kmax, bool check_cert, bool dedupe, RoundBufs b, hipStream_t st,
                        const int64_t *rowid, int64_t *ids, float *dists, const FilterPairArgs &fp) {
  // LDS slice per wavefront: two lists of kmax entries and the staging area
  size_t lds = 4 * merge_slice_bytes(kmax);
  int64_t blocks = ceil_div(nq, 4);
  int grid = static_cast<int>(blocks < 65536 ? blocks : 65536);
  allow_lds(reinterpret_cast<const void *>(k_query_merge), lds);
  (void)dedupe;  // the tournament keeps a row met twice once in every round
  hipLaunchKernelGGL(k_query_merge, dim3(grid), dim3(256), lds, st, nq, N, kmax, check_cert ? 1 : 0, b, rowid,
                     ids, dists, fp);
  LAUNCH_OK("query_merge");
}

void launch_finalize(int64_t nq, int kmax, const int64_t *rowid, RoundBufs b, int64_t *ids, float *dists,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(ceil_div(nq * kmax, 256)), dim3(256), 0, st, nq, kmax, rowid, b, ids, dists);
  LAUNCH_OK("finalize");
}

void launch_items_to_leaf_knn(int64_t n_items, int N, int k, int kmax, const int64_t *rowid, RoundBufs b, float *d,
                              int64_t *ids, hipStream_t st) {
  if (n_items <= 0) return;
  hipLaunchKernelGGL(k_items_to_leaf_knn, dim3(ceil_div(n_items * k, 256)), dim3(256), 0, st, n_items, N, k, kmax,
                     rowid, b, d, ids);
  LAUNCH_OK("items_to_leaf_knn");
}

void launch_select_pairs(int64_t nq, const int32_t *k_dev, const float *t_dev, int n_pairs, const int32_t *pair_k,
                         const float *pair_t, int kmax, int32_t *pair, int32_t *kq, hipStream_t st,
                         const int32_t *slots) {
  hipLaunchKernelGGL(k_select_pairs, dim3(ceil_div(nq, 256)), dim3(256), 0, st, nq, k_dev, t_dev, n_pairs, pair_k,
                     pair_t, kmax, pair, kq, slots);
  LAUNCH_OK("select_pairs");
}

}  // namespace leafi

namespace leafi {
void launch_collect_done(int64_t n_slots, int N, int kmax, const int64_t *rowid, RoundBufs b, int32_t *state,
                         int32_t *done_slot, int64_t *done_ids, float *done_d, int32_t *n_done, hipStream_t st) {
  if (n_slots <= 0) return;
  hipLaunchKernelGGL(k_collect_done, dim3(ceil_div(n_slots, 256)), dim3(256), 0, st, n_slots, N, kmax, rowid, b,
                     state, done_slot, done_ids, done_d, n_done);
  LAUNCH_OK("collect_done");
}
}  // namespace leafi
