// Leaf-scan kernels (SearchNode of Algorithm 2 for many (query, leaf) items at
// once) and the per-item candidate rerank.
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

namespace leafi {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// 32-bit scan keys (BF16 form): row index within the tile in the low
// kLocalBits bits (tiles of at most 4096 rows), above it the float bits of
// the squared distance without its sign bit and its kDropBits lowest bits.
constexpr int kLocalBits = 12;
constexpr int kDropBits = kLocalBits - 1;
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

// Error bound of the BF16 scan's squared distance for a query with bf16
// norm^2 qn (rows have norm^2 <= 1.02 m): the computed value is within
// delta16 of the exact squared distance of the bf16 vectors.
__device__ __forceinline__ double bf16_delta(double qn, int m) {
  const double u = 1.0 / 16777216.0;  // 2^-24
  const double x2 = 1.02 * m;
  return (m + 3) * 2.0 * u * (qn + x2 + 2.0 * sqrt(qn * x2));
}

// A query's scan threshold from its best-so-far tau: rows whose computed
// squared distance reaches it are provably farther than tau (1 + 2^-12), so
// they can neither enter the query's top k nor need a place in its candidate
// list.  With rounding moving q and x by at most qeps and leps, a row is at
// least sqrt(d2 - delta16) - qeps - leps away.  +inf while tau is +inf.
__device__ __forceinline__ float tau_threshold(float tau, double qn, float qeps, float leps, int m) {
  if (!(tau < __builtin_inff())) return __builtin_inff();
  const double t = static_cast<double>(tau) * (1.0 + 1.0 / 4096.0) + qeps + leps;
  const double v = t * t + bf16_delta(qn, m);
  float T = static_cast<float>(v);
  if (static_cast<double>(T) < v) T = nextafterf(T, __builtin_inff());
  return T;
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
                                           bf16x8 (&nxt)[KS], bool more, const uint16_t *qs, int qstride,
                                           const float (&qn)[QB], uint32_t *keys, int *cnt, uint32_t *thr, int cap,
                                           const int *kpl, bool check, int room, int wave, int lane) {
  constexpr int kWaves = 4;
  const int64_t rowc = base + 16 * wave + 4 * (lane >> 4);
  const float4 xn = *reinterpret_cast<const float4 *>(s.xn16 + rowc);
  // unconditional (the last block of a tile re-reads its own rows, which are
  // cached): a branch here would leave the in-flight load count ambiguous and
  // make the compiler drain every load before the MFMAs
  load_rows<KS>(s.x16, more ? base + 64 : base, wave, lane, s.m, nxt);
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
    bf16x8 a0[KS], a1[KS];
    load_rows<KS>(s.x16, ti.r0, wave, lane, m, a0);
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
    for (int64_t base = ti.r0; base < ti.r1; base += 128) {
      scan_block<KS, QB>(s, ti, base, a0, a1, true, qs, qstride, qn, keys, cnt, thr, cap, kpl, !pair, room, wave,
                         lane);
      scan_block<KS, QB>(s, ti, base + 64, a1, a0, base + 128 < ti.r1, qs, qstride, qn, keys, cnt, thr, cap, kpl,
                         true, room, wave, lane);
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

// Selection instead of a full sort when at most kSelectMax of at most
// 64 * kSelectPerLane chunk candidates are wanted.
constexpr int kSelectMax = 16;
constexpr int kSelectPerLane = 16;

// One wavefront per item.  LDS: merged keys [P], then per candidate the fp32
// key, FP64 distance and row.
// The kp smallest of an item's n chunk-list keys (kprime slots per chunk)
// into buf (ascending, kKeyMax past the last real key): kp rounds of a
// the keys above the previous one (keys are unique), U per lane in registers
// (unconditional loads of clamped entries, so all of a lane's loads are in
// flight together; n >= kprime >= kp >= 1, so entry 0 exists; n <= 64 U).
template <int U>
__device__ inline void select_keys(const uint64_t *__restrict__ cand, int64_t t0, int G, int g, int mq, int j,
                                   int kprime, int kp, int n, int lane, uint64_t *buf) {
  uint64_t mine[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = lane + u * kWave;
    const int ec = e < n ? e : 0;
    const int c = ec / kprime;
    const uint64_t v = cand[((t0 + static_cast<int64_t>(c) * G + g) * mq + j) * kprime + (ec - c * kprime)];
    mine[u] = e < n ? v : kKeyMax;
  }
  uint64_t prev = 0;
  bool first = true;
  for (int r = 0; r < kp; ++r) {
    uint64_t lo = kKeyMax;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if ((first || mine[u] > prev) && mine[u] < lo) lo = mine[u];
    lo = wave_min_u64(lo);
    if (lane == 0) buf[r] = lo;
    prev = lo;
    first = false;
    if (lo == kKeyMax) {  // no keys left: the rest stay empty
      for (int e = r + 1 + lane; e < kp; e += kWave) buf[e] = kKeyMax;
      break;
    }
  }
}

// ---- a query's bound for the rerank --------------------------------------------
//
// After a search round's BF16 scan, every candidate list of a query is sorted
// by key (bf16 squared distance, row).  The k smallest keys over all of them
// belong to k distinct rows, each no farther than sqrt(key + delta16) + eps_q
// + eps_L, so the query's k-th exact distance after this round's merge is at
// most U = sqrt(kth key + delta16) + eps_q + max_L eps_L (and at most its tau
// before the round).  A candidate whose lower bound sqrt(key - delta16) -
// eps_q - eps_L exceeds U can never enter the query's top k, so the rerank
// skips its FP32 and FP64 distances.  The k-th smallest key is found by a
// tournament over the list heads (k rounds of a wavefront minimum), 64 x
// kBoundSlots lists per pass; a pass keeps the k smallest so far in LDS for
// the next.
constexpr int kBoundSlots = 4;

__device__ inline int bound_pass(int64_t q, int N, int k, int kprime, int mq, int chunk, int cmax, const RoundBufs &b,
                                 const StoreView &s, const uint64_t *__restrict__ cand, int l0, int nl,
                                 const uint64_t *in, int n_in, uint64_t *out, int lane) {
  uint64_t hd[kBoundSlots], n1[kBoundSlots], n2[kBoundSlots];
  int64_t base[kBoundSlots];
  int pos[kBoundSlots], cnt[kBoundSlots];
  const int kp = item_kprime(b.kp_query, kprime, k, true);
#pragma unroll
  for (int i = 0; i < kBoundSlots; ++i) {
    const int lam = l0 + lane + kWave * i;
    cnt[i] = 0;
    base[i] = 0;
    if (lam < l0 + nl) {
      const int r = lam / cmax, c = lam - r * cmax;
      const int idx = b.qitem_idx[q * N + r];
      const int L = b.item_leaf[idx];
      const int ist0 = b.leaf_istart[L], ist1 = b.leaf_istart[L + 1];
      const int C = static_cast<int>((s.leaf_off[L + 1] - s.leaf_off[L] + chunk - 1) / chunk);
      if (c < C) {
        const int p = idx - ist0, g = p / mq, j = p - g * mq, G = (ist1 - ist0 + mq - 1) / mq;
        base[i] = (tile_of(b.tile_start, L, g, c, G) * mq + j) * kprime;
        cnt[i] = kp;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kBoundSlots; ++i) {
    hd[i] = cnt[i] > 0 ? cand[base[i]] : kKeyMax;
    n1[i] = cnt[i] > 1 ? cand[base[i] + 1] : kKeyMax;
    n2[i] = cnt[i] > 2 ? cand[base[i] + 2] : kKeyMax;
    pos[i] = 3;
  }
  int o = 0, rp = 0;
  while (o < k) {
    uint64_t lo = kKeyMax;
#pragma unroll
    for (int i = 0; i < kBoundSlots; ++i) lo = hd[i] < lo ? hd[i] : lo;
    uint64_t g = wave_min_u64(lo);
    const uint64_t rv = rp < n_in ? in[rp] : kKeyMax;
    g = rv < g ? rv : g;
    if (g == kKeyMax) break;  // every list is exhausted
    if (lane == 0) out[o] = g;
    ++o;
    if (rv == g) ++rp;
#pragma unroll
    for (int i = 0; i < kBoundSlots; ++i) {
      if (hd[i] == g) {  // the row may sit in two lists (a leaf rescanned): every copy advances
        hd[i] = n1[i];
        n1[i] = n2[i];
        n2[i] = pos[i] < cnt[i] ? cand[base[i] + pos[i]] : kKeyMax;
        ++pos[i];
      }
    }
  }
  wave_lds_sync();
  return o;
}

// One work-group per query: its four wavefronts take every fourth pass of
// 64 x kBoundSlots lists each and keep their k smallest keys; wavefront 0
// then merges the four sorted results (a key held by two of them is one row,
// counted once) up to the k-th.
__global__ void __launch_bounds__(256) k_query_bound(StoreView s, QueryView qv, RoundBufs b, int64_t nq, int mq,
                                                     int kprime, int kmax, int cmax, float eps_max,
                                                     const uint64_t *__restrict__ cand, float *qbound) {
  extern __shared__ uint64_t bsm[];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  uint64_t *buf0 = bsm + static_cast<size_t>(wave) * 2 * kmax, *buf1 = buf0 + kmax;
  int *s_n = reinterpret_cast<int *>(bsm + 8 * static_cast<size_t>(kmax));  // [4] result sizes
  int *s_res = s_n + 4;                                                     // [4] result offsets
  // after a capacity overflow the item lists were never placed
  if (b.ctl[kCtlOverflow] != 0) return;
  const int N = s.N, m = s.m;
  constexpr int kPass = kWave * kBoundSlots;
  for (int64_t q = blockIdx.x; q < nq; q += gridDim.x) {
    const int n_it = b.qitem_cnt[q];
    const int k = b.kq[q];
    float U = b.tau[q];
    if (n_it > 0) {
      const int nlists = n_it * cmax;
      uint64_t *in = buf0, *out = buf1;
      int n_in = 0;
      for (int l0 = wave * kPass; l0 < nlists; l0 += 4 * kPass) {
        const int nl = nlists - l0 < kPass ? nlists - l0 : kPass;
        n_in = bound_pass(q, N, k, kprime, mq, b.chunk, cmax, b, s, cand, l0, nl, in, n_in, out, lane);
        uint64_t *t = in;
        in = out;
        out = t;
      }
      if (lane == 0) {
        s_n[wave] = n_in;
        s_res[wave] = static_cast<int>(in - bsm);  // offset of this wavefront's result
      }
      __syncthreads();
      if (wave == 0) {
        // lanes 0..3 walk the four sorted results
        const int w = lane < 4 ? lane : 0;
        const uint64_t *res = bsm + s_res[w];
        const int cnt = lane < 4 ? s_n[w] : 0;
        int pos = 0;
        uint64_t hd = cnt > 0 ? res[0] : kKeyMax;
        uint64_t g = kKeyMax;
        int o = 0;
        while (o < k) {
          g = wave_min_u64(hd);
          if (g == kKeyMax) break;  // fewer than k keys in all
          ++o;
          if (hd == g) {
            ++pos;
            hd = pos < cnt ? res[pos] : kKeyMax;
          }
        }
        if (o == k) {
          // the key's distance was rounded down to its truncation step: the
          // computed value is at most the step's largest float
          const float kt = key_d2(g);
          const double kd = static_cast<double>(kt < __builtin_inff() ? u2f(f2u(kt) | ((1u << kDropBits) - 1)) : kt);
          const double v = sqrt(kd + bf16_delta(static_cast<double>(qv.qn16[q]), m)) + qv.qeps[q] + eps_max;
          float u = static_cast<float>(v);
          if (static_cast<double>(u) < v) u = nextafterf(u, __builtin_inff());
          U = u < U ? u : U;
        }
      }
    }
    if (threadIdx.x == 0) qbound[q] = U;
    __syncthreads();  // LDS is reused by the next query
  }
}

// Per item of a search round, one lane each: each chunk list is sorted, so
// its first key is its smallest, and every row of the item has a key at least
// the smallest of them (or was never a candidate: key >= the tau threshold).
// When even that bound exceeds the query's bound U, no row of the item can
// enter the query's top k: the item contributes nothing and is certified by
// that bound (no sort, no rerank).  The others are appended to item_live.
__global__ void __launch_bounds__(256) k_rerank_skip(StoreView s, QueryView qv, RoundBufs b, int mq, int kprime,
                                                     const uint64_t *__restrict__ cand,
                                                     const float *__restrict__ qbound) {
  const int n_items = static_cast<int>(b.ctl[kCtlItems]);
  const int lane = threadIdx.x & (kWave - 1);
  const int m = s.m;
  // whole wavefronts step together (the append below is wavefront-wide)
  for (int base = blockIdx.x * blockDim.x + (threadIdx.x - lane); base < n_items; base += gridDim.x * blockDim.x) {
    const int item = base + lane;
    bool live = false;
    if (item < n_items) {
      const int L = b.item_leaf[item];
      const int64_t q = b.item_q[item];
      const int ist0 = b.leaf_istart[L], ist1 = b.leaf_istart[L + 1];
      const int64_t off0 = s.leaf_off[L], off1 = s.leaf_off[L + 1];
      const float tau_q = b.tau[q], qn_q = qv.qn16[q], qe_q = qv.qeps[q], le_L = s.leaf_eps[L];
      const float U = qbound[q];
      const int64_t t0 = b.tile_start[L];
      const int pos = item - ist0;
      const int g = pos / mq, j = pos - g * mq;
      const int C = static_cast<int>((off1 - off0 + b.chunk - 1) / b.chunk);
      const int G = (ist1 - ist0 + mq - 1) / mq;
      uint64_t h = kKeyMax;
      for (int c = 0; c < C; ++c) {
        const uint64_t v = cand[((t0 + static_cast<int64_t>(c) * G + g) * mq + j) * kprime];
        h = v < h ? v : h;
      }
      float kd = h != kKeyMax ? key_d2(h) : __builtin_inff();
      kd = fminf(kd, tau_threshold(tau_q, qn_q, qe_q, le_L, m));
      double lower = -1.0;
      if (kd < __builtin_inff()) {
        const double v = static_cast<double>(kd) - bf16_delta(qn_q, m);
        lower = (v > 0.0 ? sqrt(v) : 0.0) - qe_q - le_L;
      }
      if (lower > static_cast<double>(U)) {
        float lb = static_cast<float>(lower);
        if (static_cast<double>(lb) > lower) lb = nextafterf(lb, -__builtin_inff());
        b.item_cnt[item] = 0;
        b.item_bound[item] = lb;
      } else {
        live = true;
      }
    }
    const uint64_t mask = __ballot(live);
    if (mask != 0) {
      const int lead = __ffsll(static_cast<unsigned long long>(mask)) - 1;
      int at = 0;
      if (lane == lead)
        at = static_cast<int>(atomicAdd(reinterpret_cast<unsigned long long *>(b.ctl + kCtlLive),
                                        static_cast<unsigned long long>(__popcll(mask))));
      at = __shfl(at, lead, kWave);
      if (live) b.item_live[at + __popcll(mask & ((1ull << lane) - 1))] = item;
    }
  }
}

__global__ void __launch_bounds__(256, 3) k_item_rerank(StoreView s, QueryView qv, RoundBufs b, int mq, int kprime,
                                                     int kmax, int bf16, int PB, int slice_u64,
                                                     const uint64_t *__restrict__ cand,
                                                     const float *__restrict__ qbound) {
  extern __shared__ uint64_t smem[];
  // blockDim / 64 wavefronts per work-group, one item each, own LDS slice
  const int wave = threadIdx.x / kWave, wpb = blockDim.x / kWave;
  uint64_t *buf = smem + static_cast<size_t>(wave) * slice_u64;        // [PB]
  uint64_t *k32 = buf + PB;                                             // [PK]
  const int PK = pow2_at_least(kprime < 2 ? 2 : kprime);
  double *d64 = reinterpret_cast<double *>(buf + PB + PK);             // [PK]
  uint32_t *r64 = reinterpret_cast<uint32_t *>(d64 + PK);              // [PK]
  const int lane = threadIdx.x & (kWave - 1);
  const int m = s.m;
  const int n_items = static_cast<int>(b.ctl[kCtlItems]);
  // the round's per-leaf item counts were consumed by its layout: zero them
  // for the merge, which counts rescan items into them
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < s.N;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    b.leaf_cnt[i] = 0;
  // error constants (see the certificate below)
  const double u = 1.0 / 16777216.0;  // 2^-24
  const float delta32 = static_cast<float>(2.0 * (m + 4) * u);
  // a search round reranks only the items k_rerank_skip listed
  const int n_work = qbound ? static_cast<int>(b.ctl[kCtlLive]) : n_items;
  for (int w_i = blockIdx.x * wpb + wave; w_i < n_work; w_i += gridDim.x * wpb) {
    const int item = qbound ? b.item_live[w_i] : w_i;
    const int L = b.item_leaf[item];
    const int64_t q = b.item_q[item];
    // everything else the item needs from memory, requested together
    const int k = b.kq[q];
    const int ist0 = b.leaf_istart[L], ist1 = b.leaf_istart[L + 1];
    const int64_t off0 = s.leaf_off[L], off1 = s.leaf_off[L + 1];
    const float tau_q = b.tau[q], qn_q = qv.qn16[q], qe_q = qv.qeps[q], le_L = s.leaf_eps[L];
    const int pos = item - ist0;
    const int g = pos / mq, j = pos - (pos / mq) * mq;
    const int C = static_cast<int>((off1 - off0 + b.chunk - 1) / b.chunk);
    const int G = (ist1 - ist0 + mq - 1) / mq;
    // the query's own candidate count (its lists hold kp keys in kprime slots)
    const int kp = item_kprime(b.kp_query, kprime, k, bf16 != 0);
    const int PKi = pow2_at_least(kp < 2 ? 2 : kp);
    int n = C * kprime;
    if (kp <= kSelectMax && n <= kWave * kSelectPerLane) {
      // few keys wanted from many: kp rounds of a wavefront minimum, each
      // lane holding as few registers as n needs
      const int64_t t0 = b.tile_start[L];
      if (n <= kWave) select_keys<1>(cand, t0, G, g, mq, j, kprime, kp, n, lane, buf);
      else if (n <= 4 * kWave) select_keys<4>(cand, t0, G, g, mq, j, kprime, kp, n, lane, buf);
      else select_keys<kSelectPerLane>(cand, t0, G, g, mq, j, kprime, kp, n, lane, buf);
      wave_lds_sync();
    } else {
      int P = pow2_at_least(n < 2 ? 2 : n);
      for (int e = lane; e < P; e += kWave) {
        uint64_t v = kKeyMax;
        if (e < n) {
          int c = e / kprime;
          v = cand[(tile_of(b.tile_start, L, g, c, G) * mq + j) * kprime + (e - c * kprime)];
        }
        buf[e] = v;
      }
      wave_lds_sync();
      wave_sort_u64(buf, P, lane);
    }
    uint64_t kth = buf[kp - 1];
    // number of real candidates among the first kp
    int nc = 0;
    for (int e = 0; e < kp; ++e) nc += buf[e] != kKeyMax ? 1 : 0;
    if (qbound) {
      // search rounds: only candidates that can still enter the query's top k
      // (lower bound not above the query's bound) are reranked; the keys are
      // ascending, so they are a prefix
      const float U = qbound[q];
      const double dq = bf16_delta(static_cast<double>(qn_q), m);
      int use = 0;
      for (int e = 0; e < nc; ++e) {
        const double v = static_cast<double>(key_d2(buf[e])) - dq;
        const double lower = (v > 0.0 ? sqrt(v) : 0.0) - qe_q - le_L;
        if (lower > static_cast<double>(U)) break;
        ++use;
      }
      nc = use;
    }
    // FP32 direct-difference rerank: CB candidates at a time, G lanes each
    // (all their rows are in flight together), 4 consecutive elements per lane
    const float *qp = qv.q32 + q * m;
    const int CB = PKi < 8 ? PKi : 8, GL = kWave / CB;
    const int sub = lane & (GL - 1), cb = lane / GL;
    // FP64 for every candidate within the FP32 error band of the k-th
    float band = __builtin_inff();
    int nb = 0;
    if (PKi <= 8 && m <= 16 * GL) {
      // Few candidates (CB == PK): each lane group holds its candidate's row
      // and the query's matching elements in registers for both passes, so
      // the rows are read once.  Same sums in the same order as below.
      constexpr int kHold = 4;
      const int e = cb;
      uint32_t row = 0;
      float4 qa[kHold], xa[kHold];
      float p = 0.0f;
      if (e < nc) {
        row = key_row(buf[e]);
        const float *xp = s.x32 + static_cast<int64_t>(row) * m;
#pragma unroll
        for (int i = 0; i < kHold; ++i) {
          const int t = 4 * sub + i * 4 * GL;
          if (t < m) {
            qa[i] = *reinterpret_cast<const float4 *>(qp + t);
            xa[i] = *reinterpret_cast<const float4 *>(xp + t);
          }
        }
#pragma unroll
        for (int i = 0; i < kHold; ++i) {
          if (4 * sub + i * 4 * GL < m) {
            float d = qa[i].x - xa[i].x;
            p = fmaf(d, d, p);
            d = qa[i].y - xa[i].y;
            p = fmaf(d, d, p);
            d = qa[i].z - xa[i].z;
            p = fmaf(d, d, p);
            d = qa[i].w - xa[i].w;
            p = fmaf(d, d, p);
          }
        }
      }
      for (int o = GL >> 1; o > 0; o >>= 1) p += __shfl_xor(p, o, kWave);
      if (sub == 0) k32[e] = e < nc ? make_key(p, row) : kKeyMax;
      wave_lds_sync();
      wave_sort_u64(k32, PKi, lane);
      if (nc >= k) band = key_d2(k32[k - 1]) * (1.0f + 2.0f * delta32);
      for (int i = 0; i < nc; ++i) nb += key_d2(k32[i]) <= band ? 1 : 0;
      // the band's members are exactly the candidates whose FP32 value is
      // within it (every lane of a group holds its candidate's value)
      const bool inb = e < nc && p <= band;
      double pd = 0.0;
      if (inb) {
#pragma unroll
        for (int i = 0; i < kHold; ++i) {
          if (4 * sub + i * 4 * GL < m) {
            double d = static_cast<double>(qa[i].x) - static_cast<double>(xa[i].x);
            pd = fma(d, d, pd);
            d = static_cast<double>(qa[i].y) - static_cast<double>(xa[i].y);
            pd = fma(d, d, pd);
            d = static_cast<double>(qa[i].z) - static_cast<double>(xa[i].z);
            pd = fma(d, d, pd);
            d = static_cast<double>(qa[i].w) - static_cast<double>(xa[i].w);
            pd = fma(d, d, pd);
          }
        }
      }
      for (int o = GL >> 1; o > 0; o >>= 1) pd += __shfl_xor(pd, o, kWave);
      if (sub == 0) {
        d64[e] = inb ? pd : __builtin_inf();
        r64[e] = inb ? row : 0xffffffffu;
      }
    } else if (!bf16) {
      // FP32 scan items: the candidates' keys already hold FP32
      // direct-difference values (same error bound), ascending
      for (int e = lane; e < PKi; e += kWave) k32[e] = e < nc ? buf[e] : kKeyMax;
      wave_lds_sync();
    } else {
      for (int e0 = 0; e0 < PKi; e0 += CB) {
        const int e = e0 + cb;
        float p = 0.0f;
        uint32_t row = 0;
        if (e < nc) {
          row = key_row(buf[e]);
          const float *xp = s.x32 + static_cast<int64_t>(row) * m;
          // unrolled so a lane's loads of the row are in flight together (at
          // most 8 per lane for m <= 256: GL >= 8)
#pragma unroll 8
          for (int t = 4 * sub; t < m; t += 4 * GL) {
            const float4 a = *reinterpret_cast<const float4 *>(qp + t);
            const float4 x = *reinterpret_cast<const float4 *>(xp + t);
            float d = a.x - x.x;
            p = fmaf(d, d, p);
            d = a.y - x.y;
            p = fmaf(d, d, p);
            d = a.z - x.z;
            p = fmaf(d, d, p);
            d = a.w - x.w;
            p = fmaf(d, d, p);
          }
        }
        for (int o = GL >> 1; o > 0; o >>= 1) p += __shfl_xor(p, o, kWave);
        if (sub == 0) k32[e] = e < nc ? make_key(p, row) : kKeyMax;
      }
      wave_lds_sync();
      wave_sort_u64(k32, PKi, lane);
    }
    if (!(PKi <= 8 && m <= 16 * GL)) {
      if (nc >= k) band = key_d2(k32[k - 1]) * (1.0f + 2.0f * delta32);
      for (int e = 0; e < nc; ++e) nb += key_d2(k32[e]) <= band ? 1 : 0;
      for (int e0 = 0; e0 < PKi; e0 += CB) {
        const int e = e0 + cb;
        double p = 0.0;
        uint32_t row = 0xffffffffu;
        if (e < nb) {
          row = key_row(k32[e]);
          const float *xp = s.x32 + static_cast<int64_t>(row) * m;
#pragma unroll 8
          for (int t = 4 * sub; t < m; t += 4 * GL) {
            const float4 a = *reinterpret_cast<const float4 *>(qp + t);
            const float4 x = *reinterpret_cast<const float4 *>(xp + t);
            double d = static_cast<double>(a.x) - static_cast<double>(x.x);
            p = fma(d, d, p);
            d = static_cast<double>(a.y) - static_cast<double>(x.y);
            p = fma(d, d, p);
            d = static_cast<double>(a.z) - static_cast<double>(x.z);
            p = fma(d, d, p);
            d = static_cast<double>(a.w) - static_cast<double>(x.w);
            p = fma(d, d, p);
          }
        }
        for (int o = GL >> 1; o > 0; o >>= 1) p += __shfl_xor(p, o, kWave);
        if (sub == 0) {
          d64[e] = e < nb ? p : __builtin_inf();
          r64[e] = row;
        }
      }
    }
    wave_lds_sync();
    wave_sort_dbl_tag(d64, r64, PKi, lane);
    int keep = nb < k ? nb : k;
    for (int i = lane; i < keep; i += kWave) {
      b.item_d2[static_cast<int64_t>(item) * kmax + i] = d64[i];
      b.item_row[static_cast<int64_t>(item) * kmax + i] = static_cast<int32_t>(r64[i]);
    }
    // Certificate: every row of the item outside the candidate list has a
    // scan key >= kth.  BF16: the computed value is within delta16 of the
    // exact squared distance of the bf16 vectors, and rounding moved q and x
    // by at most qeps and leaf_eps, so d(q, x) >= sqrt(kth - delta16) - eps.
    // FP32: the direct-difference value is within a relative delta32.
    // With a tau threshold T (search rounds), rows at or above T were never
    // candidates, so the list's own bound is capped by T's.
    if (lane == 0) {
      float bound = __builtin_inff();
      float kd = kth != kKeyMax ? key_d2(kth) : __builtin_inff();
      if (bf16 && b.use_tau) kd = fminf(kd, tau_threshold(tau_q, qn_q, qe_q, le_L, m));
      if (kd < __builtin_inff()) {
        if (bf16) {
          double v = static_cast<double>(kd) - bf16_delta(qn_q, m);
          bound = static_cast<float>((v > 0.0 ? sqrt(v) : 0.0) - qe_q - le_L);
        } else {
          bound = static_cast<float>(sqrt(static_cast<double>(kd) * (1.0 - delta32)));
        }
      }
      b.item_cnt[item] = keep;
      b.item_bound[item] = bound;
    }
    wave_lds_sync();
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

int rerank_lds_bytes(int max_chunks, int kprime, int *PB) {
  int n = max_chunks * kprime;
  *PB = pow2_at_least(n < 2 ? 2 : n);
  int PK = pow2_at_least(kprime < 2 ? 2 : kprime);
  return (*PB + PK) * 8 + PK * 8 + PK * 4;
}

void launch_query_bound(StoreView s, QueryView q, RoundBufs b, int64_t nq, int mq, int kprime, int kmax, int cmax,
                        float eps_max, const uint64_t *cand, float *qbound, hipStream_t st) {
  if (nq <= 0) return;
  const size_t lds = 4 * 2 * static_cast<size_t>(kmax) * sizeof(uint64_t) + 8 * sizeof(int);
  const int64_t blocks = nq;  // one work-group per query
  hipLaunchKernelGGL(k_query_bound, dim3(static_cast<unsigned>(blocks < 65536 ? blocks : 65536)), dim3(256), lds, st, s,
                     q, b, nq, mq, kprime, kmax, cmax, eps_max, cand, qbound);
  LAUNCH_OK("query_bound");
}

void launch_item_rerank(StoreView s, QueryView q, RoundBufs b, int mq, int kprime, int kmax, bool bf16,
                        const uint64_t *cand, int grid, int max_chunks, hipStream_t st, const float *qbound) {
  int PB;
  const size_t slice = round_up(rerank_lds_bytes(max_chunks, kprime, &PB), 16);
  const int wpb = slice * 4 <= 65536 ? 4 : 1;
  const size_t lds = slice * wpb;
  allow_lds(reinterpret_cast<const void *>(k_item_rerank), lds);
  const int blocks = (grid + wpb - 1) / wpb;
  hipLaunchKernelGGL(k_item_rerank, dim3(blocks), dim3(64 * wpb), lds, st, s, q, b, mq, kprime, kmax, bf16 ? 1 : 0, PB,
                     static_cast<int>(slice / 8), cand, qbound);
  LAUNCH_OK("item_rerank");
}

void launch_rerank_skip(StoreView s, QueryView q, RoundBufs b, int mq, int kprime, const uint64_t *cand,
                        const float *qbound, int64_t items_bound, int num_cus, hipStream_t st) {
  const int64_t want = ceil_div(std::max<int64_t>(items_bound, 1), 256);
  const int blocks = static_cast<int>(std::min<int64_t>(want, static_cast<int64_t>(num_cus) * 8));
  hipLaunchKernelGGL(k_rerank_skip, dim3(blocks), dim3(256), 0, st, s, q, b, mq, kprime, cand, qbound);
  LAUNCH_OK("rerank_skip");
}

}  // namespace leafi
