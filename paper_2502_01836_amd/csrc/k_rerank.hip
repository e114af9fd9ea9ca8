// Per-item rerank of a round's candidate lists and the per-query bound that
// lets a search round skip items and candidates (SearchNode of Algorithm 2:
// the result update after a leaf's scan).
//
// After a pass's scan every (query, tile) list holds its kprime best keys
// (truncated BF16 or FP32 squared distances with rows).  k_query_bound finds
// per query an upper bound U of its k-th distance after the round, then
// certifies the query's items whose every candidate is provably beyond U and
// lists the rest; k_item_rerank merges each listed item's chunk lists
// and reranks its candidates in FP32 (FP64 within the error band of the k-th),
// writing the item's exact top-k and the bound that certifies the rest.
#include <algorithm>

#include "device_util.h"
#include "kernels.h"
#include "scan_bounds.h"

namespace leafi {

namespace {

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
// tournament over the list heads, 64 x kBoundSlots lists per pass; a pass
// keeps the k smallest so far in LDS for the next, and each round emits the
// run of those below the lists' smallest head (up to 64 at once) or that
// head.
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
    const uint64_t g = wave_min_u64(lo);
    // the running list's keys below the lists' smallest head come next, as
    // one run (lane j checks entry rp + j)
    const bool below = rp + lane < n_in && o + lane < k && in[rp + lane] < g;
    const uint64_t bm = __ballot(below);
    const int run = ~bm == 0 ? kWave : __builtin_ctzll(~bm);
    if (run > 0) {
      if (lane < run) out[o + lane] = in[rp + lane];
      o += run;
      rp += run;
      continue;
    }
    if (g == kKeyMax) break;  // every list is exhausted
    if (lane == 0) out[o] = g;
    ++o;
    if (rp < n_in && in[rp] == g) ++rp;
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

// One item of a search round: each chunk list is sorted, so its first key is
// its smallest, and every row of the item has a key at least the smallest of
// them (or was never a candidate: key >= the tau threshold).  When even that
// bound exceeds the query's bound U, no row of the item can enter the query's
// top k: the item contributes nothing and is certified by that bound (no
// sort, no rerank).  Returns whether the item still needs its rerank.
__device__ inline bool item_live_after_bound(const StoreView &s, const QueryView &qv, const RoundBufs &b, int mq,
                                             int kprime, const uint64_t *__restrict__ cand, int item, int64_t q,
                                             float U) {
  const int m = s.m;
  const int L = b.item_leaf[item];
  const int ist0 = b.leaf_istart[L], ist1 = b.leaf_istart[L + 1];
  const int64_t off0 = s.leaf_off[L], off1 = s.leaf_off[L + 1];
  const float tau_q = b.tau[q], qn_q = qv.qn16[q], qe_q = qv.qeps[q], le_L = s.leaf_eps[L];
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
    return false;
  }
  return true;
}

// One work-group per query: its four wavefronts take every fourth pass of
// 64 x kBoundSlots lists each and keep their k smallest keys; wavefront 0
// then merges the four sorted results (a key held by two of them is one row,
// counted once) up to the k-th.  With U known, the work-group certifies the
// query's items by it and lists the others for the rerank.
__global__ void __launch_bounds__(256) k_query_bound(StoreView s, QueryView qv, RoundBufs b, int64_t nq, int mq,
                                                     int kprime, int kmax, int cmax, float eps_max,
                                                     const uint64_t *__restrict__ cand, float *qbound) {
  extern __shared__ uint64_t bsm[];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  uint64_t *buf0 = bsm + static_cast<size_t>(wave) * 2 * kmax, *buf1 = buf0 + kmax;
  int *s_n = reinterpret_cast<int *>(bsm + 8 * static_cast<size_t>(kmax));  // [4] result sizes
  int *s_res = s_n + 4;                                                     // [4] result offsets
  float *s_u = reinterpret_cast<float *>(s_res + 4);                         // the query's bound
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
        if (lane == 0) *s_u = U;
      }
      __syncthreads();
      U = *s_u;
      // the query's items: certify by U what can be, list the rest in item_live
      for (int r0 = wave * kWave; r0 < n_it; r0 += 4 * kWave) {
        const int r = r0 + lane;
        const bool live = r < n_it && item_live_after_bound(s, qv, b, mq, kprime, cand, b.qitem_idx[q * N + r], q, U);
        const uint64_t mask = __ballot(live);
        if (mask != 0) {
          const int lead = __ffsll(static_cast<unsigned long long>(mask)) - 1;
          int at = 0;
          if (lane == lead)
            at = static_cast<int>(atomicAdd(reinterpret_cast<unsigned long long *>(b.ctl + kCtlLive),
                                            static_cast<unsigned long long>(__popcll(mask))));
          at = __shfl(at, lead, kWave);
          if (live) b.item_live[at + __popcll(mask & ((1ull << lane) - 1))] = b.qitem_idx[q * N + r];
        }
      }
    }
    if (threadIdx.x == 0) qbound[q] = U;
    __syncthreads();  // LDS is reused by the next query
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
  // a search round reranks only the items k_query_bound listed
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
    uint64_t kth_override = 0;  // nonzero: the certificate's key (see below)
    if (kp <= kSelectMax && n <= kWave * kSelectPerLane) {
      // few keys wanted from many: kp rounds of a wavefront minimum, each
      // lane holding as few registers as n needs
      const int64_t t0 = b.tile_start[L];
      if (n <= kWave) select_keys<1>(cand, t0, G, g, mq, j, kprime, kp, n, lane, buf);
      else if (n <= 4 * kWave) select_keys<4>(cand, t0, G, g, mq, j, kprime, kp, n, lane, buf);
      else select_keys<kSelectPerLane>(cand, t0, G, g, mq, j, kprime, kp, n, lane, buf);
      wave_lds_sync();
    } else if (qbound) {
      // Search rounds: only keys whose lower bound does not exceed the
      // query's bound U can enter its top k.  They are a prefix of the sorted
      // keys (the bound grows with the key), so they are gathered and sorted
      // alone and the item's results do not change.  With fewer than kp of
      // them the kp-th key is among the dropped ones: the smallest dropped
      // key, whose bound exceeds U, certifies every row left out.
      const double Ud = static_cast<double>(qbound[q]);
      const double dq = bf16_delta(static_cast<double>(qn_q), m);
      const uint64_t lanes_below = (1ull << lane) - 1ull;
      int nf = 0;
      uint64_t dropped = kKeyMax;
      for (int e0 = 0; e0 < n; e0 += kWave) {
        const int e = e0 + lane;
        uint64_t v = kKeyMax;
        if (e < n) {
          const int c = e / kprime;
          v = cand[(tile_of(b.tile_start, L, g, c, G) * mq + j) * kprime + (e - c * kprime)];
        }
        bool keep = false;
        if (v != kKeyMax) {
          const double x = static_cast<double>(key_d2(v)) - dq;
          const double lower = (x > 0.0 ? sqrt(x) : 0.0) - qe_q - le_L;
          keep = !(lower > Ud);
          if (!keep) dropped = v < dropped ? v : dropped;
        }
        const uint64_t km = __ballot(keep);
        if (keep) buf[nf + __popcll(km & lanes_below)] = v;
        nf += __popcll(km);
      }
      dropped = wave_min_u64(dropped);
      const int want = nf > kp ? nf : kp;
      const int P = pow2_at_least(want < 2 ? 2 : want);
      for (int e = nf + lane; e < P; e += kWave) buf[e] = kKeyMax;
      wave_lds_sync();
      wave_sort_u64(buf, P, lane);
      if (nf < kp) kth_override = dropped;
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
    uint64_t kth = kth_override != 0 ? kth_override : buf[kp - 1];
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

}  // namespace

int rerank_lds_bytes(int max_chunks, int kprime, int *PB) {
  int n = max_chunks * kprime;
  *PB = pow2_at_least(n < 2 ? 2 : n);
  int PK = pow2_at_least(kprime < 2 ? 2 : kprime);
  return (*PB + PK) * 8 + PK * 8 + PK * 4;
}

void launch_query_bound(StoreView s, QueryView q, RoundBufs b, int64_t nq, int mq, int kprime, int kmax, int cmax,
                        float eps_max, const uint64_t *cand, float *qbound, hipStream_t st) {
  if (nq <= 0) return;
  const size_t lds = 4 * 2 * static_cast<size_t>(kmax) * sizeof(uint64_t) + 12 * sizeof(int);
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

}  // namespace leafi
