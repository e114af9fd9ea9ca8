// Leaf-scan kernels (SearchNode of Algorithm 2 for many (query, leaf) items at
// once); the per-item rerank of their candidate lists is in k_rerank.hip.
//
// A scan tile is (leaf L, group of up to MQ queries that all search L this
// round, chunk of kChunkRows rows of L).  The persistent grid walks the tiles;
// per tile it streams the chunk's rows once for all the group's queries and
// keeps, per query, the kprime best (squared distance, row) keys.
//
// BF16 form: the squared distance of the bf16-rounded vectors is
// ||q~||^2 + ||x~||^2 - 2 q~.x~ with q~.x~ on v_mfma_f32_16x16x32_bf16 (data
// rows are the A operand, 16 rows per MFMA; queries the B operand, 16 per
// MFMA; FP32 accumulation).  Every lane loads 16 contiguous bytes of its row
// per K step, so the four lanes of a row read 64 contiguous bytes.
//
// FP32 form: direct difference sum_t (q_t - x_t)^2, 16 lanes per row, each
// lane summing m/16 contiguous elements, then a fixed 16-lane tree.
//
// Candidate keeping (both forms): per query an LDS list with a threshold; a
// key below the threshold is appended with an LDS atomic; when a list could
// overflow in the next 64 rows it is sorted (bitonic, one wavefront) and cut
// to kprime, which also tightens the threshold.
//
// The BF16 form keeps 32-bit keys in LDS: the squared distance's float bits
// with the lowest kDropBits cut off (rounded down, so the value a key stands
// for is a lower bound of the computed distance), then the row's index within
// the tile.  Half the LDS of full keys, so twice the queries share one pass
// over a tile's rows.  The tile's lists are written out as full 64-bit keys
// (truncated distance, global row); within a tile both orders agree.
#include <hip/hip_ext.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "device_util.h"
#include "kernels.h"
#include "scan_bounds.h"

namespace leafi {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// 32-bit scan keys (BF16 form, layout in scan_bounds.h); all bits set: empty.
constexpr uint32_t kKey32Max = ~0u;

__device__ __forceinline__ uint32_t make_key32(float d2, uint32_t local) {
  return ((f2u(d2) >> kDropBits) << kLocalBits) | local;
}

// The smallest 32-bit threshold such that every key at or above it stands
// for a squared distance >= T (T >= 0 finite): T's truncated bits, plus one
// step when the truncation dropped anything.
__device__ __forceinline__ uint32_t key32_ceil(float T) {
  const uint32_t u = f2u(T);
  uint32_t h = u >> kDropBits;
  if ((h << kDropBits) != u) ++h;
  return h << kLocalBits;
}

// A tile's LDS key as a candidate key: (truncated squared distance, global row).
__device__ __forceinline__ uint64_t cand_key(uint32_t k, int64_t r0) {
  if (k == kKey32Max) return kKeyMax;
  const float d = u2f((k >> kLocalBits) << kDropBits);
  return make_key(d, static_cast<uint32_t>(r0 + (k & ((1u << kLocalBits) - 1))));
}
__device__ __forceinline__ uint64_t cand_key(uint64_t k, int64_t) { return k; }

// The empty key of either width: all bits set.
template <typename K>
constexpr K key_max() { return static_cast<K>(~static_cast<K>(0)); }

struct TileInfo {
  int L, g, c, C;
  int64_t r0, r1, real_end;
  int p0, nqt;
};

// Work-groups are dispatched to the 8 XCDs round-robin (work-group i runs
// on XCD i mod 8).  With a grid that is a multiple of 8, renumber them so
// that each XCD takes a contiguous range of tiles per pass of the persistent
// loop: neighbouring tiles (other query groups of the same rows) then share
// an L2.
constexpr int kXcds = 8;
constexpr int kXcdRun = 4;  // consecutive tiles kept on one XCD
// j-th tile (j = 0, 1, ...) of the work-groups of XCD x: runs of kXcdRun
// consecutive tiles, dealt to the XCDs in turn, so every XCD gets an equal
// share of the tiles (to within one run) wherever the tile count ends.
__device__ inline int64_t xcd_tile(int64_t j, int x) {
  return ((j / kXcdRun) * kXcds + x) * kXcdRun + j % kXcdRun;
}

// Work-group barrier for LDS traffic only: waits for this wave's LDS
// operations, then s_barrier.  Unlike __syncthreads it does not drain
// outstanding global loads, so prefetched rows stay in flight across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Leaf of tile t, found by the whole work-group: the L with
// tile_start[L] <= t < tile_start[L + 1] (tile_start is non-decreasing and
// tile_start[N] is the tile count, so exactly one L qualifies, and exactly
// one bucket of B consecutive leaves holds it).  One thread per bucket
// finds the bucket, then one thread per leaf of the bucket the leaf: two
// dependent loads where a binary search takes log2 N.  Every thread must
// call it; sh holds two ints of LDS, free when it is called.  (Kernels
// carve sh from their dynamic LDS: a static __shared__ variable would move
// the dynamic block off its 16-byte alignment.)
__device__ inline int tile_leaf(int t, const int32_t *__restrict__ tile_start, int N, int *sh) {
  const int B = (N + blockDim.x - 1) / blockDim.x;
  const int lo = threadIdx.x * B;
  if (lo < N && tile_start[lo] <= t && t < tile_start[lo + B < N ? lo + B : N]) sh[0] = lo;
  lds_barrier();
  // the value is uniform: readfirstlane keeps it (and all that derives from
  // it) in scalar registers
  const int L0 = __builtin_amdgcn_readfirstlane(sh[0]);
  if (B == 1) return L0;
  const int L = L0 + static_cast<int>(threadIdx.x);
  if (static_cast<int>(threadIdx.x) < B && L < N && tile_start[L] <= t && t < tile_start[L + 1]) sh[1] = L;
  lds_barrier();
  return __builtin_amdgcn_readfirstlane(sh[1]);
}

__device__ inline TileInfo decode_tile(int t, const StoreView &s, const RoundBufs &b, int mq, int *sh) {
  const int lo = tile_leaf(t, b.tile_start, s.N, sh);
  TileInfo ti;
  ti.L = lo;
  int64_t off0 = s.leaf_off[lo], off1 = s.leaf_off[lo + 1];
  ti.C = static_cast<int>((off1 - off0 + b.chunk - 1) / b.chunk);
  const int G = (b.leaf_istart[lo + 1] - b.leaf_istart[lo] + mq - 1) / mq;
  int local = t - b.tile_start[lo];  // chunk-major: local = c * G + g (see tile_of)
  ti.c = local / G;
  ti.g = local - ti.c * G;
  ti.r0 = off0 + static_cast<int64_t>(ti.c) * b.chunk;
  ti.r1 = ti.r0 + b.chunk < off1 ? ti.r0 + b.chunk : off1;
  ti.real_end = off0 + s.leaf_n[lo];
  ti.p0 = b.leaf_istart[lo] + ti.g * mq;
  int left = b.leaf_istart[lo + 1] - ti.p0;
  ti.nqt = left < mq ? left : mq;
  return ti;
}

// Candidate list j of a tile occupies keys[j (cap + 1) .. + cap): the one
// spare entry per list staggers the lists across LDS banks (appends of
// different queries at equal slots would otherwise hit one bank).

// Up to this many kept keys, a list is cut by selection instead of a sort.
constexpr int kListSelectMax = 16;

// Keep the kprime best keys of list j, in ascending order at its head, and
// refresh the threshold.  Few wanted (kprime <= kListSelectMax): kprime
// rounds of a wavefront minimum over the keys above the previous round's
// (the keys of one list are distinct: one per row); otherwise a bitonic sort.
template <typename K>
__device__ inline void compact_list(K *keys, int *cnt, K *thr, int j, int cap, int kprime, int lane) {
  constexpr K kMax = key_max<K>();
  K *lst = keys + static_cast<int64_t>(j) * (cap + 1);
  int c = cnt[j];
  if (kprime <= kListSelectMax) {
    K prev = 0, mine = kMax;  // lane r keeps the r-th smallest
    int keep = 0;
    // a list of up to 128 keys is read into registers once (two per lane)
    // instead of once per round
    const bool regs = c <= 2 * kWave;
    const K v0 = regs && lane < c ? lst[lane] : kMax;
    const K v1 = regs && lane + kWave < c ? lst[lane + kWave] : kMax;
    for (int r = 0; r < kprime; ++r) {
      K lo = kMax;
      if (regs) {
        if ((r == 0 || v0 > prev) && v0 < lo) lo = v0;
        if ((r == 0 || v1 > prev) && v1 < lo) lo = v1;
      } else {
        for (int e = lane; e < c; e += kWave) {
          const K v = lst[e];
          if ((r == 0 || v > prev) && v < lo) lo = v;
        }
      }
      lo = wave_min_key(lo);
      if (lo == kMax) break;  // fewer than kprime keys (uniform)
      if (lane == r) mine = lo;
      prev = lo;
      ++keep;
    }
    wave_lds_sync();  // every lane has read the list before its head is rewritten
    if (lane < keep) lst[lane] = mine;
    if (lane == 0) {
      cnt[j] = keep;
      if (keep == kprime) thr[j] = prev;  // else the list is not full: keep the threshold
    }
    wave_lds_sync();
    return;
  }
  wave_sort_keys_n(lst, c, lane);  // in place: the list's capacity need not be a power of two
  int keep = c < kprime ? c : kprime;
  if (lane == 0) {
    cnt[j] = keep;
    if (keep == kprime) thr[j] = lst[kprime - 1];  // else the list is not full: keep the threshold
  }
  wave_lds_sync();
}

__device__ inline void append_key(uint64_t *keys, int *cnt, const uint64_t *thr, int j, int cap, uint64_t key) {
  if (key < thr[j]) {
    int slot = atomicAdd(cnt + j, 1);
    keys[static_cast<int64_t>(j) * (cap + 1) + slot] = key;
  }
}

// The tile's lists to its candidate slots: list j keeps its kpl[j] best keys
// (kpl[j] <= kprime), the rest of its kprime slots are empty.  Slots of lists
// past the tile's queries (j >= nqt) belong to no item and are never read:
// they are not written.
template <typename K>
__device__ inline void finish_tile(K *keys, int *cnt, K *thr, const int *kpl, int t, int mq, int nqt, int cap,
                                   int kprime, int64_t r0, int wave, int nwaves, int lane, uint64_t *cand) {
  for (int j = wave; j < nqt; j += nwaves) {
    uint64_t *out = cand + (static_cast<int64_t>(t) * mq + j) * kprime;
    compact_list(keys, cnt, thr, j, cap, kpl[j], lane);
    // only the first cnt[j] entries are candidates; the list may hold fewer
    // than kprime (a chunk with few real rows) and LDS beyond them is stale
    const K *lst = keys + static_cast<int64_t>(j) * (cap + 1);
    const int keep = cnt[j];
    for (int i = lane; i < kprime; i += kWave) out[i] = i < keep ? cand_key(lst[i], r0) : kKeyMax;
  }
}

// A operand of this wave's 16 rows of the 64-row block at `base`: lane l
// holds row base + 16 wave + (l & 15), elements 32 k + 8 (l >> 4) .. + 8.  In
// the panel layout (panel_index) that is element 512 k + 8 l of the rows'
// panel: each of the KS loads reads 1 KiB of consecutive memory.
template <int KS>
__device__ __forceinline__ void load_rows(const uint16_t *x16, int64_t base, int wave, int lane, int m,
                                          bf16x8 (&a)[KS]) {
  const uint16_t *ap = x16 + (base + 16 * wave) * m + 8 * lane;
#pragma unroll
  for (int k = 0; k < KS; ++k) a[k] = *reinterpret_cast<const bf16x8 *>(ap + 512 * k);
}

// One 64-row block: its squared norms, the prefetch of the next block into
// `nxt`, MFMAs on `cur`, candidate appends, then list maintenance.
template <int KS, int QB>
__device__ __forceinline__ void scan_block(const StoreView &s, const TileInfo &ti, int64_t base, bf16x8 (&cur)[KS],
                                           bf16x8 (&nxt)[KS], int64_t pre, const uint16_t *qs, int qstride,
                                           const float (&qn)[QB], uint32_t *keys, int *cnt, uint32_t *thr, int cap,
                                           const int *kpl, bool check, int room, int wave, int lane) {
  constexpr int kWaves = 4;
  const int64_t rowc = base + 16 * wave + 4 * (lane >> 4);
  const float4 xn = *reinterpret_cast<const float4 *>(s.xn16 + rowc);
  // rows `pre` into nxt, unconditionally (past the tile's last block a valid
  // block is read again, from cache): a branch here would leave the
  // in-flight load count ambiguous and make the compiler drain every load
  // before the MFMAs
  load_rows<KS>(s.x16, pre, wave, lane, s.m, nxt);
  floatx4 acc[QB];
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) acc[qb] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  // B operand from LDS: lane l reads query 16 qb + (l & 15), same k-chunk as A
  const uint16_t *qb0 = qs + (lane & 15) * qstride + 8 * (lane >> 4);
#pragma unroll
  for (int k = 0; k < KS; ++k)
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
      const bf16x8 bq = *reinterpret_cast<const bf16x8 *>(qb0 + 16 * qb * qstride + 32 * k);
      acc[qb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur[k], bq, acc[qb], 0, 0, 0);
    }
  // epilogue: lane holds rows rowc..rowc+3 for query column (lane & 15)
  const float xr[4] = {xn.x, xn.y, xn.z, xn.w};
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const int j = 16 * qb + (lane & 15);
    if (j < ti.nqt) {
      // the lane's (up to 4) appends take one LDS atomic: one round trip per
      // block instead of one per row
      const uint32_t tj = thr[j];
      uint32_t kk[4];
      int n = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = rowc + r;
        const float d2 = fmaxf(qn[qb] + xr[r] - 2.0f * acc[qb][r], 0.0f);
        kk[r] = make_key32(d2, static_cast<uint32_t>(row - ti.r0));
        if (!(row < ti.real_end && kk[r] < tj)) kk[r] = kKey32Max;
        n += kk[r] != kKey32Max;
      }
      if (n > 0) {
        uint32_t *dst = keys + static_cast<int64_t>(j) * (cap + 1) + atomicAdd(cnt + j, n);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (kk[r] != kKey32Max) *dst++ = kk[r];
      }
    }
  }
  // Lists are checked after every block, or with room for two blocks of
  // appends (room = 128) after every second one: between checks the
  // wavefronts need no barrier at all.
  if (!check) return;
  lds_barrier();
  // lists that could overflow before the next check: every count read at
  // once (one lane per list, MQ <= 64), then this wavefront's lists j = wave mod 4
  uint64_t over = __ballot(lane < ti.nqt && cnt[lane < ti.nqt ? lane : 0] > cap - room) &
                  (0x1111111111111111ull << wave);
  while (over) {
    const int j = __ffsll(static_cast<unsigned long long>(over)) - 1;
    over &= over - 1;
    compact_list(keys, cnt, thr, j, cap, kpl[j], lane);
  }
  lds_barrier();
}

template <int KS, int QB>
__global__ void __launch_bounds__(256, QB >= 3 ? 2 : 4) k_scan_bf16(StoreView s, QueryView qv, RoundBufs b,
                                                                   int kprime, int cap, uint64_t *cand) {
  constexpr int MQ = 16 * QB;
  static_assert(MQ <= kWave, "one lane per candidate list");
  constexpr int kWaves = 4;
  extern __shared__ uint64_t smem[];
  // MQ is a multiple of 16, so every array below starts 16-byte aligned
  uint32_t *keys = reinterpret_cast<uint32_t *>(smem);
  uint32_t *thr = keys + MQ * (cap + 1);
  int *cnt = reinterpret_cast<int *>(thr + MQ);
  int *kpl = cnt + MQ;                                     // [MQ] candidates each list keeps
  uint16_t *qs = reinterpret_cast<uint16_t *>(kpl + MQ);  // [MQ][m + 8], 16-byte aligned
  int *s_leaf = reinterpret_cast<int *>(qs + MQ * (s.m + 8));  // [2], after the tile's queries
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int m = s.m;
  const int n_tiles = static_cast<int>(b.ctl[kCtlTiles]);
  // work-group i runs on XCD i % 8; with a grid that is a multiple of 8 it
  // takes the tiles xcd_tile(i / 8 + p * gridDim.x / 8, i % 8), p = 0, 1, ...
  const bool by_xcd = gridDim.x % kXcds == 0;
  const int x = blockIdx.x % kXcds, per = gridDim.x / kXcds;
  for (int64_t j = by_xcd ? blockIdx.x / kXcds : blockIdx.x;; j += by_xcd ? per : gridDim.x) {
    const int64_t tt = by_xcd ? xcd_tile(j, x) : j;
    if (by_xcd ? (j / kXcdRun) * kXcds * kXcdRun >= n_tiles : tt >= n_tiles) break;
    if (tt >= n_tiles) continue;
    const int t = static_cast<int>(tt);
    TileInfo ti = decode_tile(t, s, b, MQ, s_leaf);
    // The tile's first rows are requested before its queries are staged, so
    // the two sets of loads are in flight together.
    // Row buffers: two (ping-pong, the next block in flight), or four
    // (three blocks in flight) for 48 and 64 queries per tile, whose two
    // work-groups per CU leave the registers for them, on rows of up to 128
    // elements: a block of those carries too few products to cover a load's
    // latency, while rows of 256 gain nothing from the deeper pipeline
    // (measured: 25M x 96 +9 %, 10M and 50M x 256 flat or slower).
    constexpr int kBufs = (QB >= 3 && KS <= 4) ? 4 : 2;
    bf16x8 a0[KS], a1[KS], a2[kBufs > 2 ? KS : 1], a3[kBufs > 2 ? KS : 1];
    load_rows<KS>(s.x16, ti.r0, wave, lane, m, a0);
    if constexpr (kBufs > 2) {
      load_rows<KS>(s.x16, ti.r0 + 64 < ti.r1 ? ti.r0 + 64 : ti.r0, wave, lane, m, a1);
      load_rows<KS>(s.x16, ti.r0 + 128 < ti.r1 ? ti.r0 + 128 : ti.r0, wave, lane, m, a2);
    }
    if (threadIdx.x < MQ) {
      const int j = threadIdx.x;
      cnt[j] = 0;
      uint32_t t0 = kKey32Max;
      int kp = kprime;
      if (j < ti.nqt) {
        const int64_t qq = b.item_q[ti.p0 + j];
        if (b.kp_query) kp = item_kprime(1, kprime, b.kq[qq], true);
        if (b.use_tau) {
          const float T = tau_threshold(b.tau[qq], qv.qn16[qq], qv.qeps[qq], s.leaf_eps[ti.L], m);
          if (T < __builtin_inff()) t0 = key32_ceil(T);
        }
      }
      thr[j] = t0;
      kpl[j] = kp;
    }
    // B operand: this lane's query column and k-chunk, all K steps
    // The group's bf16 queries go to LDS (row stride m + 8 elements, so the 16
    // rows one MFMA reads start in different banks); they are the B operand.
    const int qstride = m + 8;
    for (int e = threadIdx.x; e < MQ * (m / 8); e += blockDim.x) {
      const int j = e / (m / 8), c = e - j * (m / 8);
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (j < ti.nqt) v = *reinterpret_cast<const uint4 *>(qv.q16 + static_cast<int64_t>(b.item_q[ti.p0 + j]) * m + 8 * c);
      *reinterpret_cast<uint4 *>(qs + j * qstride + 8 * c) = v;
    }
    float qn[QB];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
      const int j = 16 * qb + (lane & 15);
      qn[qb] = j < ti.nqt ? qv.qn16[b.item_q[ti.p0 + j]] : 0.0f;
    }
    lds_barrier();
    // The A operand of the wave's 16 rows in the next 64-row block is loaded
    // while the current block is processed (ping-pong registers, no copies),
    // so one block of global loads is always in flight; the barriers wait on
    // LDS only.  Loads are issued in the order they are consumed because the
    // hardware's load counter retires in order.
    // Chunks hold an even number of 64-row blocks (leaves are padded to 128
    // rows), so both halves of the unrolled body always run.
    // a list cut back to its kpl[j] <= kprime keys has room for two blocks
    // of appends when the capacity allows (uniform)
    const bool pair = cap - kprime >= 128;
    const int room = pair ? 128 : 64;
    if constexpr (kBufs == 2) {
      for (int64_t base = ti.r0; base < ti.r1; base += 128) {
        scan_block<KS, QB>(s, ti, base, a0, a1, base + 64, qs, qstride, qn, keys, cnt, thr, cap, kpl, !pair, room,
                           wave, lane);
        scan_block<KS, QB>(s, ti, base + 64, a1, a0, base + 128 < ti.r1 ? base + 128 : base + 64, qs, qstride, qn,
                           keys, cnt, thr, cap, kpl, true, room, wave, lane);
      }
    } else {
      // block b is in buffer b mod 4 and requests block b + 3 (a re-read of
      // the tile's first block past its end); blocks come in pairs, so a
      // group of four may end after its second
      auto pre = [&](int64_t row) { return row < ti.r1 ? row : ti.r0; };
      for (int64_t base = ti.r0; base < ti.r1; base += 256) {
        scan_block<KS, QB>(s, ti, base, a0, a3, pre(base + 192), qs, qstride, qn, keys, cnt, thr, cap, kpl, !pair,
                           room, wave, lane);
        scan_block<KS, QB>(s, ti, base + 64, a1, a0, pre(base + 256), qs, qstride, qn, keys, cnt, thr, cap, kpl, true,
                           room, wave, lane);
        if (base + 128 < ti.r1) {  // uniform
          scan_block<KS, QB>(s, ti, base + 128, a2, a1, pre(base + 320), qs, qstride, qn, keys, cnt, thr, cap, kpl,
                             !pair, room, wave, lane);
          scan_block<KS, QB>(s, ti, base + 192, a3, a2, pre(base + 384), qs, qstride, qn, keys, cnt, thr, cap, kpl,
                             true, room, wave, lane);
        }
      }
    }
    finish_tile(keys, cnt, thr, kpl, t, MQ, ti.nqt, cap, kprime, ti.r0, wave, kWaves, lane, cand);
    __syncthreads();
  }
}

template <int EPL>
__global__ void __launch_bounds__(256) k_scan_fp32(StoreView s, QueryView qv, RoundBufs b, int mq, int kprime,
                                                   int cap, uint64_t *cand) {
  constexpr int kWaves = 4;
  extern __shared__ uint64_t smem[];
  uint64_t *keys = smem;
  uint64_t *thr = keys + mq * (cap + 1);
  int *cnt = reinterpret_cast<int *>(thr + mq);
  int *kpl = cnt + mq;  // [mq] candidates each list keeps
  float *qs = reinterpret_cast<float *>(kpl + mq);
  int *s_leaf = reinterpret_cast<int *>(qs + mq * s.m);  // [2], after the tile's queries
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int sub = lane & 15, rsel = lane >> 4;
  const int m = s.m;  // == 16 * EPL
  const int n_tiles = static_cast<int>(b.ctl[kCtlTiles]);
  // work-group i runs on XCD i % 8; with a grid that is a multiple of 8 it
  // takes the tiles xcd_tile(i / 8 + p * gridDim.x / 8, i % 8), p = 0, 1, ...
  const bool by_xcd = gridDim.x % kXcds == 0;
  const int x = blockIdx.x % kXcds, per = gridDim.x / kXcds;
  for (int64_t j = by_xcd ? blockIdx.x / kXcds : blockIdx.x;; j += by_xcd ? per : gridDim.x) {
    const int64_t tt = by_xcd ? xcd_tile(j, x) : j;
    if (by_xcd ? (j / kXcdRun) * kXcds * kXcdRun >= n_tiles : tt >= n_tiles) break;
    if (tt >= n_tiles) continue;
    const int t = static_cast<int>(tt);
    TileInfo ti = decode_tile(t, s, b, mq, s_leaf);
    if (threadIdx.x < mq) {
      const int j = threadIdx.x;
      cnt[j] = 0;
      thr[j] = kKeyMax;
      kpl[j] = j < ti.nqt && b.kp_query ? item_kprime(1, kprime, b.kq[b.item_q[ti.p0 + j]], false) : kprime;
    }
    for (int e = threadIdx.x; e < ti.nqt * m; e += blockDim.x) {
      int j = e / m;
      qs[e] = qv.q32[static_cast<int64_t>(b.item_q[ti.p0 + j]) * m + (e - j * m)];
    }
    __syncthreads();
    for (int64_t base = ti.r0; base < ti.r1; base += 64) {
      float x[4][EPL];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const float *xp = s.x32 + (base + 16 * wave + 4 * st + rsel) * m + sub * EPL;
#pragma unroll
        for (int e = 0; e < EPL; e += 2) {
          float2 v = *reinterpret_cast<const float2 *>(xp + e);
          x[st][e] = v.x;
          x[st][e + 1] = v.y;
        }
      }
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        int64_t row = base + 16 * wave + 4 * st + rsel;
        for (int j = 0; j < ti.nqt; ++j) {
          const float *qp = qs + j * m + sub * EPL;
          float p = 0.0f;
#pragma unroll
          for (int e = 0; e < EPL; ++e) {
            float d = qp[e] - x[st][e];
            p = fmaf(d, d, p);
          }
          p += __shfl_xor(p, 8, 16);
          p += __shfl_xor(p, 4, 16);
          p += __shfl_xor(p, 2, 16);
          p += __shfl_xor(p, 1, 16);
          if (sub == 0 && row < ti.real_end) append_key(keys, cnt, thr, j, cap, make_key(p, static_cast<uint32_t>(row)));
        }
      }
      __syncthreads();
      // every count read at once (mq <= 64), then this wavefront's lists
      uint64_t over =
          __ballot(lane < ti.nqt && cnt[lane < ti.nqt ? lane : 0] > cap - 64) & (0x1111111111111111ull << wave);
      while (over) {
        const int j = __ffsll(static_cast<unsigned long long>(over)) - 1;
        over &= over - 1;
        compact_list(keys, cnt, thr, j, cap, kpl[j], lane);
      }
      __syncthreads();
    }
    finish_tile(keys, cnt, thr, kpl, t, mq, ti.nqt, cap, kprime, ti.r0, wave, kWaves, lane, cand);
    __syncthreads();
  }
}

// Work-groups that can be resident at once for `kern` with `lds` bytes of
// LDS, capped at `want`.  A persistent grid larger than this would leave a
// tail of work-groups that only start after the first ones have finished.
// The occupancy query is cached per (kernel, LDS bytes): it is asked on every
// launch and the answer never changes.
template <typename K>
int resident_grid(K kern, size_t lds, int want) {
  static std::mutex mu;
  static std::map<std::pair<const void *, size_t>, int> cache;
  static int cus = 0;
  const void *fn = reinterpret_cast<const void *>(kern);
  int g = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (cus == 0) {
      int dev = 0;
      HIP_OK(hipGetDevice(&dev));
      HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    }
    auto it = cache.find({fn, lds});
    if (it == cache.end()) {
      int per_cu = 0;
      HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds));
      it = cache.emplace(std::make_pair(fn, lds), cus * (per_cu > 0 ? per_cu : 1)).first;
    }
    g = it->second;
  }
  g = want < g ? (want > 0 ? want : 1) : g;
  return g >= kXcds ? g / kXcds * kXcds : g;  // a multiple of the XCD count (see xcd_tile)
}

constexpr int kLdsPerCu = 160 * 1024;

// LDS of a BF16 scan work-group: 32-bit lists, thresholds, counts, per-list
// candidate counts, the queries (row stride m + 8), two ints.
size_t scan_bf16_lds(int mq, int cap, int m) {
  return static_cast<size_t>(mq) * (cap + 1) * 4 + static_cast<size_t>(mq) * 4 * 3 +
         static_cast<size_t>(mq) * (m + 8) * 2 + 16;
}

template <int KS, int QB>
void scan_bf16_inst(StoreView s, QueryView q, RoundBufs b, int kprime, int cap, uint64_t *cand, int grid,
                    hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  constexpr int MQ = 16 * QB;
  const size_t lds = scan_bf16_lds(MQ, cap, 32 * KS);
  auto kern = k_scan_bf16<KS, QB>;
  allow_lds(reinterpret_cast<const void *>(kern), lds);
  grid = resident_grid(kern, lds, grid);
  if (e0 || e1)  // start / stop timestamps of this dispatch itself
    hipExtLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, st, e0, e1, 0, s, q, b, kprime, cap, cand);
  else
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, st, s, q, b, kprime, cap, cand);
  LAUNCH_OK("scan_bf16");
}

template <int QB>
void scan_bf16_ks(int ks, StoreView s, QueryView q, RoundBufs b, int kprime, int cap, uint64_t *cand, int grid,
                  hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  switch (ks) {
    case 1: scan_bf16_inst<1, QB>(s, q, b, kprime, cap, cand, grid, st, e0, e1); break;
    case 2: scan_bf16_inst<2, QB>(s, q, b, kprime, cap, cand, grid, st, e0, e1); break;
    case 3: scan_bf16_inst<3, QB>(s, q, b, kprime, cap, cand, grid, st, e0, e1); break;
    case 4: scan_bf16_inst<4, QB>(s, q, b, kprime, cap, cand, grid, st, e0, e1); break;
    case 5: scan_bf16_inst<5, QB>(s, q, b, kprime, cap, cand, grid, st, e0, e1); break;
    case 6: scan_bf16_inst<6, QB>(s, q, b, kprime, cap, cand, grid, st, e0, e1); break;
    case 7: scan_bf16_inst<7, QB>(s, q, b, kprime, cap, cand, grid, st, e0, e1); break;
    case 8: scan_bf16_inst<8, QB>(s, q, b, kprime, cap, cand, grid, st, e0, e1); break;
    default: fail(LEAFI_EINVAL, "bf16 scan supports m <= 256");
  }
}

template <int EPL>
void scan_fp32_inst(StoreView s, QueryView q, RoundBufs b, int mq, int kprime, int cap, uint64_t *cand, int grid,
                    hipStream_t st) {
  size_t lds = static_cast<size_t>(mq) * (cap + 1) * 8 + mq * 8 + mq * 4 * 2 + static_cast<size_t>(mq) * s.m * 4 + 16;
  auto kern = k_scan_fp32<EPL>;
  allow_lds(reinterpret_cast<const void *>(kern), lds);
  grid = resident_grid(kern, lds, grid);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, st, s, q, b, mq, kprime, cap, cand);
  LAUNCH_OK("scan_fp32");
}

}  // namespace

// Candidate-list geometry for a given kprime: (queries per tile, list
// capacity).  A list is cut back to its kprime best whenever the next 64 (or
// 128) rows could overflow it, so the capacity is at least kprime + 64.
// BF16 (32-bit keys): above that, as large as the LDS allows at the
// work-groups per CU a tile of mq queries is meant to run with (4, 3 and 2
// for 16, 32 and 48 queries, fewer when even the minimum does not fit), up
// to 3 kprime + 64 (128 for kprime <= 16, whose lists are cut by
// selection): fewer cuts where many rows enter the lists (a first round,
// with no tau yet).  FP32: 64-bit keys, power-of-two capacities.
void scan_geometry(bool bf16, int kprime, int mq_pref, int m, int *mq, int *cap) {
  if (bf16) {
    const int q = (mq_pref == 16 || mq_pref == 32 || mq_pref == 48 || mq_pref == 64) ? mq_pref : 32;
    const int kp = std::max(kprime, 4);
    const int lo = (kp + 15) / 16 * 16 + 64;
    const int hi = kp <= kListSelectMax ? 128 : (3 * kp + 15) / 16 * 16 + 64;
    const int want = q <= 16 ? 4 : q <= 32 ? 3 : 2;
    int fit = 0;
    for (int wgs = want; wgs >= 1; --wgs) {
      const int64_t room = static_cast<int64_t>(kLdsPerCu) / wgs - static_cast<int64_t>(scan_bf16_lds(q, 0, m)) + 4 * q;
      fit = static_cast<int>(room / (4 * q)) - 1;
      if (fit >= lo) break;
    }
    *mq = q;
    *cap = std::max(lo, std::min(hi, fit));
    return;
  }
  int kc = pow2_at_least(kprime < 4 ? 4 : kprime);
  if (kc <= 32) { *mq = mq_pref == 16 ? 16 : 32; *cap = 128; }
  else if (kc <= 128) { *mq = 16; *cap = 256; }
  else { *mq = 16; *cap = 512; }
}

void launch_scan_bf16(StoreView s, QueryView q, RoundBufs b, int mq, int kprime, uint64_t *cand, int grid,
                      hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  int mq2, cap;
  scan_geometry(true, kprime, mq, s.m, &mq2, &cap);
  if (mq != mq2) fail(LEAFI_EINTERNAL, "scan_bf16: tile geometry mismatch");
  if (b.chunk > (1 << kLocalBits)) fail(LEAFI_EINTERNAL, "scan_bf16: tiles of at most 4096 rows");
  int ks = s.m / 32;
  switch (mq) {
    case 16: scan_bf16_ks<1>(ks, s, q, b, kprime, cap, cand, grid, st, e0, e1); break;
    case 32: scan_bf16_ks<2>(ks, s, q, b, kprime, cap, cand, grid, st, e0, e1); break;
    case 48: scan_bf16_ks<3>(ks, s, q, b, kprime, cap, cand, grid, st, e0, e1); break;
    default: scan_bf16_ks<4>(ks, s, q, b, kprime, cap, cand, grid, st, e0, e1); break;
  }
}

void launch_scan_fp32(StoreView s, QueryView q, RoundBufs b, int mq, int kprime, uint64_t *cand, int grid,
                      hipStream_t st) {
  int mq2, cap;
  scan_geometry(false, kprime, 32, s.m, &mq2, &cap);
  if (mq > mq2) fail(LEAFI_EINTERNAL, "scan_fp32: tile geometry mismatch");
  switch (s.m / 16) {
    case 2: scan_fp32_inst<2>(s, q, b, mq, kprime, cap, cand, grid, st); break;
    case 4: scan_fp32_inst<4>(s, q, b, mq, kprime, cap, cand, grid, st); break;
    case 6: scan_fp32_inst<6>(s, q, b, mq, kprime, cap, cand, grid, st); break;
    case 8: scan_fp32_inst<8>(s, q, b, mq, kprime, cap, cand, grid, st); break;
    case 10: scan_fp32_inst<10>(s, q, b, mq, kprime, cap, cand, grid, st); break;
    case 12: scan_fp32_inst<12>(s, q, b, mq, kprime, cap, cand, grid, st); break;
    case 14: scan_fp32_inst<14>(s, q, b, mq, kprime, cap, cand, grid, st); break;
    case 16: scan_fp32_inst<16>(s, q, b, mq, kprime, cap, cand, grid, st); break;
    case 24: scan_fp32_inst<24>(s, q, b, mq, kprime, cap, cand, grid, st); break;
    case 32: scan_fp32_inst<32>(s, q, b, mq, kprime, cap, cand, grid, st); break;
    default: fail(LEAFI_EINVAL, "fp32 scan supports m in {32,64,...,256,384,512}");
  }
}

}  // namespace leafi
