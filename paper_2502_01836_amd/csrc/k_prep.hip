// Ingest and query-preparation kernels: z-normalisation with FP64 statistics,
// segment summaries, the leaf-store pack, summary lower bounds and visit order.
//
// Layouts: series/queries are row-major [rows, m]; one wavefront handles one
// row (lanes stride over t), four rows per 256-thread work-group.
#include "device_util.h"
#include "kernels.h"

namespace leafi {

namespace {

constexpr int kRowsPerBlock = 4;  // wavefronts (rows) per work-group
constexpr int kMaxM = 1024;

// FP64 mean and population std of one row (wave-cooperative).
__device__ inline void row_moments(const float *r, int m, int lane, double &mu, double &sd) {
  double s = 0.0;
  for (int t = lane; t < m; t += kWave) s += static_cast<double>(r[t]);
  s = wave_sum(s);
  mu = s / m;
  double v = 0.0;
  for (int t = lane; t < m; t += kWave) {
    double d = static_cast<double>(r[t]) - mu;
    v += d * d;
  }
  v = wave_sum(v);
  sd = sqrt(v / m);
}

__device__ __forceinline__ float normalise(float x, double mu, double sd) {
  return sd < 1e-8 ? 0.0f : static_cast<float>((static_cast<double>(x) - mu) / sd);
}

// Per-segment mean and population std of the normalised values held in
// LDS (seg s covers [floor(s m / S), floor((s+1) m / S))), lane s does segment s.
__device__ inline void segment_moments(const float *z, int m, int S, int s, float &smu, float &ssd) {
  int a = (s * m) / S, b = ((s + 1) * m) / S;
  double acc = 0.0;
  for (int t = a; t < b; ++t) acc += static_cast<double>(z[t]);
  double mu = acc / (b - a);
  double v = 0.0;
  for (int t = a; t < b; ++t) {
    double d = static_cast<double>(z[t]) - mu;
    v += d * d;
  }
  smu = static_cast<float>(mu);
  ssd = static_cast<float>(sqrt(v / (b - a)));
}

__global__ void __launch_bounds__(256) k_series_stats(const float *__restrict__ raw, int64_t n, int m, int S,
                                                      double *mean, double *sdv, float *seg_mu, float *seg_sd) {
  __shared__ float zs[kRowsPerBlock][kMaxM];
  int lane = threadIdx.x & (kWave - 1);
  int w = threadIdx.x / kWave;
  int64_t row = static_cast<int64_t>(blockIdx.x) * kRowsPerBlock + w;
  if (row >= n) return;  // whole wavefront leaves together (no block barrier below)
  const float *r = raw + row * m;
  double mu, sd;
  row_moments(r, m, lane, mu, sd);
  for (int t = lane; t < m; t += kWave) zs[w][t] = normalise(r[t], mu, sd);
  wave_lds_sync();
  if (lane == 0) {
    mean[row] = mu;
    sdv[row] = sd;
  }
  for (int s = lane; s < S; s += kWave) {
    float a, b;
    segment_moments(zs[w], m, S, s, a, b);
    seg_mu[row * S + s] = a;
    seg_sd[row * S + s] = b;
  }
}

__global__ void __launch_bounds__(256) k_pack(const float *__restrict__ raw, const int64_t *__restrict__ src_of_row,
                                              const int32_t *__restrict__ leaf_of_row, int64_t rows, int m,
                                              const double *__restrict__ mean, const double *__restrict__ sdv,
                                              float *x32, uint16_t *x16, float *xn16, int64_t *rowid,
                                              float *leaf_eps) {
  int lane = threadIdx.x & (kWave - 1);
  int64_t row = static_cast<int64_t>(blockIdx.x) * kRowsPerBlock + threadIdx.x / kWave;
  if (row >= rows) return;
  int64_t src = src_of_row[row];
  float *o32 = x32 + row * m;
  // bf16 copy in 16-row panels (see panel_index)
  uint16_t *o16 = x16 + (row >> 4) * 16 * m;
  const int rr = static_cast<int>(row & 15);
  if (src < 0) {
    for (int t = lane; t < m; t += kWave) {
      o32[t] = 0.0f;
      o16[panel_index(rr, t)] = 0;
    }
    if (lane == 0) {
      xn16[row] = __builtin_inff();
      rowid[row] = -1;
    }
    return;
  }
  const float *r = raw + src * m;
  double mu = mean[src], sd = sdv[src];
  float nrm = 0.0f, err = 0.0f;
  for (int t = lane; t < m; t += kWave) {
    float z = normalise(r[t], mu, sd);
    uint16_t b = f32_to_bf16(z);
    float zb = bf16_to_f32(b);
    o32[t] = z;
    o16[panel_index(rr, t)] = b;
    nrm = fmaf(zb, zb, nrm);
    float e = z - zb;
    err = fmaf(e, e, err);
  }
  nrm = wave_sum(nrm);
  err = wave_sum(err);
  if (lane == 0) {
    xn16[row] = nrm;
    rowid[row] = src;
    // non-negative floats order like their bit patterns
    float e = sqrtf(err) * (1.0f + 1e-5f);
    atomicMax(reinterpret_cast<unsigned int *>(leaf_eps + leaf_of_row[row]), f2u(e));
  }
}

__global__ void __launch_bounds__(256) k_znorm(const float *x, int64_t n, int m, float *out) {
  int lane = threadIdx.x & (kWave - 1);
  int64_t row = static_cast<int64_t>(blockIdx.x) * kRowsPerBlock + threadIdx.x / kWave;
  if (row >= n) return;
  const float *r = x + row * m;
  double mu, sd;
  row_moments(r, m, lane, mu, sd);
  // every lane has read its elements before any lane writes (out may alias x)
  float vals[kMaxM / kWave];
  int c = 0;
  for (int t = lane; t < m; t += kWave) vals[c++] = normalise(r[t], mu, sd);
  c = 0;
  for (int t = lane; t < m; t += kWave) out[row * m + t] = vals[c++];
}

// Raw row i is written to output row slots[i] (i when slots is null).
__global__ void __launch_bounds__(256) k_qprep(const float *__restrict__ raw, int64_t nq, int m, int S, float *q32,
                                               uint16_t *q16, float *qn16, float *qeps, float *qstat,
                                               const int32_t *__restrict__ slots) {
  __shared__ float zs[kRowsPerBlock][kMaxM];
  int lane = threadIdx.x & (kWave - 1);
  int w = threadIdx.x / kWave;
  int64_t i = static_cast<int64_t>(blockIdx.x) * kRowsPerBlock + w;
  if (i >= nq) return;
  const float *r = raw + i * m;
  const int64_t row = slots ? slots[i] : i;
  double mu, sd;
  row_moments(r, m, lane, mu, sd);
  float nrm = 0.0f, err = 0.0f;
  for (int t = lane; t < m; t += kWave) {
    float z = normalise(r[t], mu, sd);
    uint16_t b = f32_to_bf16(z);
    float zb = bf16_to_f32(b);
    zs[w][t] = z;
    q32[row * m + t] = z;
    q16[row * m + t] = b;
    nrm = fmaf(zb, zb, nrm);
    float e = z - zb;
    err = fmaf(e, e, err);
  }
  nrm = wave_sum(nrm);
  err = wave_sum(err);
  if (lane == 0) {
    qn16[row] = nrm;
    qeps[row] = sqrtf(err) * (1.0f + 1e-5f);
  }
  wave_lds_sync();
  for (int s = lane; s < S; s += kWave) {
    float a, b;
    segment_moments(zs[w], m, S, s, a, b);
    qstat[(row * S + s) * 2 + 0] = a;
    qstat[(row * S + s) * 2 + 1] = b;
  }
}

// d^lb(q, L)^2 = sum_s l_s [gap(mu_q, [mu_lo, mu_hi])^2 + gap(sd_q, [sd_lo, sd_hi])^2].
__global__ void __launch_bounds__(256) k_lb(const float *__restrict__ qstat, int64_t nq,
                                            const float *__restrict__ boxes, int N, int S, int m, float *lb,
                                            const int32_t *__restrict__ slots) {
  int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= nq * N) return;
  int64_t i = idx / N;
  int L = static_cast<int>(idx - i * N);
  const int64_t q = slots ? slots[i] : i;
  lb[q * N + L] = summary_lb(qstat + q * S * 2, boxes + static_cast<int64_t>(L) * S * 4, S, m);
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
  const uint32_t lo = __shfl_xor(static_cast<uint32_t>(v), mask, kWave);
  const uint32_t hi = __shfl_xor(static_cast<uint32_t>(v >> 32), mask, kWave);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Bitonic stage `size`, strides smax .. 1, on a wavefront's chunk of 128 keys
// at `base` held in registers (x: element lane, y: element 64 + lane): the
// same compare-exchanges as the work-group passes below, without LDS or
// barriers.  A pair (lo, lo + stride) ascends when (base + lo) & size is 0.
__device__ inline void chunk_stages(uint64_t &x, uint64_t &y, int base, int size, int smax, int lane) {
  for (int stride = smax; stride >= 1; stride >>= 1) {
    if (stride == kWave) {
      const bool up = ((base + lane) & size) == 0;
      const uint64_t a = x < y ? x : y, b = x < y ? y : x;
      x = up ? a : b;
      y = up ? b : a;
    } else {
      const uint64_t px = shfl_xor_u64(x, stride), py = shfl_xor_u64(y, stride);
      const int lo = lane & ~stride;
      const bool am_lo = (lane & stride) == 0;
      const bool upx = ((base + lo) & size) == 0, upy = ((base + kWave + lo) & size) == 0;
      x = (am_lo == upx) ? (x < px ? x : px) : (x < px ? px : x);
      y = (am_lo == upy) ? (y < py ? y : py) : (y < py ? py : y);
    }
  }
}

// Work-group bitonic sort of P keys in LDS (P a power of two; the
// work-group a multiple of 64 threads).  Stages of stride below 128 run in
// registers on chunks of 128 keys, one wavefront per chunk; only the larger
// strides go through LDS with a barrier each.
__device__ inline void block_sort_u64(uint64_t *keys, int P) {
  if (P < 2 * kWave) {
    for (int size = 2; size <= P; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = threadIdx.x; i < (P >> 1); i += blockDim.x) {
          int lo = 2 * i - (i & (stride - 1));
          int hi = lo + stride;
          bool up = (lo & size) == 0;
          uint64_t x = keys[lo], y = keys[hi];
          if ((x > y) == up) {
            keys[lo] = y;
            keys[hi] = x;
          }
        }
        __syncthreads();
      }
    }
    return;
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
  constexpr int kChunk = 2 * kWave;
  for (int c = wave; c < P / kChunk; c += nw) {
    const int base = c * kChunk;
    uint64_t x = keys[base + lane], y = keys[base + kWave + lane];
    for (int size = 2; size <= kChunk; size <<= 1) chunk_stages(x, y, base, size, size >> 1, lane);
    keys[base + lane] = x;
    keys[base + kWave + lane] = y;
  }
  __syncthreads();
  for (int size = 2 * kChunk; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride >= kChunk; stride >>= 1) {
      for (int i = threadIdx.x; i < (P >> 1); i += blockDim.x) {
        int lo = 2 * i - (i & (stride - 1));
        int hi = lo + stride;
        bool up = (lo & size) == 0;
        uint64_t x = keys[lo], y = keys[hi];
        if ((x > y) == up) {
          keys[lo] = y;
          keys[hi] = x;
        }
      }
      __syncthreads();
    }
    for (int c = wave; c < P / kChunk; c += nw) {
      const int base = c * kChunk;
      uint64_t x = keys[base + lane], y = keys[base + kWave + lane];
      chunk_stages(x, y, base, size, kWave, lane);
      keys[base + lane] = x;
      keys[base + kWave + lane] = y;
    }
    __syncthreads();
  }
}

// Everything a query needs before its first round, one work-group per query:
// z-normalisation (fp32 and bf16 copies, norms, rounding error), segment
// statistics, the summary bound of every leaf, the visit order (bitonic sort
// of (bound, leaf id)), the calibrated (k, target) row and the search state.
// The same arithmetic as the separate kernels (k_qprep, k_lb, k_order,
// select_pair_of).  Work-group 0 also zeroes the batch's control words, leaf
// counts and filter-pair counts.
// summary_lb of leaf L from the boxes laid out as [S][4][N] (consecutive
// leaves read consecutive words): the same operations in the same order, so
// the same value.
__device__ __forceinline__ float summary_lb_cols(const float *qs, const float *__restrict__ bt, int N, int L, int S,
                                                 int m) {
  float acc = 0.0f;
  for (int s = 0; s < S; ++s) {
    const float *b = bt + static_cast<int64_t>(4 * s) * N + L;
    float len = static_cast<float>(((s + 1) * m) / S - (s * m) / S);
    float mq = qs[2 * s], sq = qs[2 * s + 1];
    float gm = fmaxf(fmaxf(b[0] - mq, mq - b[N]), 0.0f);
    float gs = fmaxf(fmaxf(b[2 * N] - sq, sq - b[3 * N]), 0.0f);
    acc += len * (gm * gm + gs * gs);
  }
  return sqrtf(acc);
}

__global__ void __launch_bounds__(512) k_query_setup(const float *__restrict__ raw, int m, int S,
                                                     const float *__restrict__ boxes_t, int N, int P, float *q32,
                                                     uint16_t *q16, float *qn16, float *qeps, float *qstat, float *lb, int32_t *order, float *lbs,
                                                     const int32_t *__restrict__ k_dev, const float *__restrict__ t_dev,
                                                     int n_pairs, const int32_t *__restrict__ pair_k,
                                                     const float *__restrict__ pair_t, int kmax, RoundBufs b,
                                                     int F, int32_t *pcnt) {
  extern __shared__ uint64_t keys[];                    // [P]
  float *zs = reinterpret_cast<float *>(keys + P);       // [m]
  float *st = zs + m;                                    // [S][2]
  const int64_t q = blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < kCtlCount; i += blockDim.x) b.ctl[i] = 0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) b.leaf_cnt[i] = 0;
    if (pcnt)
      for (int i = threadIdx.x; i < F; i += blockDim.x) pcnt[i] = 0;
  }
  if (w == 0) {
    const float *r = raw + q * m;
    double mu, sd;
    row_moments(r, m, lane, mu, sd);
    float nrm = 0.0f, err = 0.0f;
    for (int t = lane; t < m; t += kWave) {
      float z = normalise(r[t], mu, sd);
      uint16_t bb = f32_to_bf16(z);
      float zb = bf16_to_f32(bb);
      zs[t] = z;
      q32[q * m + t] = z;
      q16[q * m + t] = bb;
      nrm = fmaf(zb, zb, nrm);
      float e = z - zb;
      err = fmaf(e, e, err);
    }
    nrm = wave_sum(nrm);
    err = wave_sum(err);
    if (lane == 0) {
      qn16[q] = nrm;
      qeps[q] = sqrtf(err) * (1.0f + 1e-5f);
      const int k = min(max(k_dev[q], 1), kmax);
      b.pair[q] = select_pair_of(k, t_dev[q], n_pairs, pair_k, pair_t);
      b.kq[q] = k;
      b.cursor[q] = 0;
      b.tau[q] = __builtin_inff();
      b.res_cnt[q] = 0;
      b.qitem_cnt[q] = 0;
    }
    wave_lds_sync();
    for (int s = lane; s < S; s += kWave) {
      float a, c;
      segment_moments(zs, m, S, s, a, c);
      st[2 * s] = a;
      st[2 * s + 1] = c;
      qstat[(q * S + s) * 2 + 0] = a;
      qstat[(q * S + s) * 2 + 1] = c;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    uint64_t key = kKeyMax;
    if (i < N) {
      const float v = summary_lb_cols(st, boxes_t, N, i, S, m);
      lb[q * N + i] = v;
      key = make_key(v, static_cast<uint32_t>(i));
    }
    keys[i] = key;
  }
  __syncthreads();
  block_sort_u64(keys, P);
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    order[q * N + i] = static_cast<int32_t>(key_row(keys[i]));
    lbs[q * N + i] = key_d2(keys[i]);
  }
}

// k_query_setup with one wavefront per query (four per work-group) for up to
// kSetupWaveMaxN leaves: the same arithmetic in the same order (so the same
// values), with no work-group barrier on a query's path.  The row is read
// once into registers; the visit order comes from each key's rank among the
// query's N keys (distinct, since the leaf id breaks ties), written straight
// to its sorted position.
constexpr int kSetupWaveMaxN = 256;
constexpr int kSetupMaxPerLane = 1024 / kWave;  // row values per lane (m <= 1024)

// summary_lb of leaf L from the boxes laid out as [S][4][N] (a wavefront's
// lanes, one leaf each, read consecutive words), with the segment count
// fixed at compile time: the same operations in the same order, so the same
// value.
template <int kS>
__device__ __forceinline__ float summary_lb_t(const float *qs, const float *__restrict__ bt, int N, int L, int m) {
  float acc = 0.0f;
#pragma unroll
  for (int s = 0; s < kS; ++s) {
    const float *b = bt + static_cast<int64_t>(4 * s) * N + L;
    float len = static_cast<float>(((s + 1) * m) / kS - (s * m) / kS);
    float mq = qs[2 * s], sq = qs[2 * s + 1];
    float gm = fmaxf(fmaxf(b[0] - mq, mq - b[N]), 0.0f);
    float gs = fmaxf(fmaxf(b[2 * N] - sq, sq - b[3 * N]), 0.0f);
    acc += len * (gm * gm + gs * gs);
  }
  return sqrtf(acc);
}

template <int J>  // keys per lane: N <= 64 J
__device__ inline void rank_and_write(const uint64_t *keys, int N, int lane, int32_t *order_q, float *lbs_q) {
  uint64_t mk[J];
  int rk[J];
#pragma unroll
  for (int c = 0; c < J; ++c) {
    const int i = lane + kWave * c;
    mk[c] = i < N ? keys[i] : kKeyMax;
    rk[c] = 0;
  }
#pragma unroll 8
  for (int j = 0; j < N; ++j) {
    const uint64_t kj = keys[j];
#pragma unroll
    for (int c = 0; c < J; ++c) rk[c] += kj < mk[c] ? 1 : 0;
  }
#pragma unroll
  for (int c = 0; c < J; ++c)
    if (lane + kWave * c < N) {
      order_q[rk[c]] = static_cast<int32_t>(key_row(mk[c]));
      lbs_q[rk[c]] = key_d2(mk[c]);
    }
}

// The calibrated (k, target) row of a query, found by its whole wavefront
// (k and t are uniform across it): the first pair that matches, as
// select_pair_of, with 64 pairs tested per step instead of one.
__device__ inline int select_pair_wave(int k, float t, int n_pairs, const int32_t *__restrict__ pair_k,
                                       const float *__restrict__ pair_t, int lane) {
  if (!(t < 1.0f)) return -1;
  for (int base = 0; base < n_pairs; base += kWave) {
    const int i = base + lane;
    const uint64_t hit = __ballot(i < n_pairs && pair_k[i] == k && pair_t[i] == t);
    if (hit) return base + __builtin_ctzll(hit);
  }
  return -1;
}

__global__ void __launch_bounds__(256) k_query_setup_wave(const float *__restrict__ raw, int64_t nq, int m, int S,
                                                          const float *__restrict__ boxes,
                                                          const float *__restrict__ boxes_t, int N, int slice64,
                                                          float *q32, uint16_t *q16, float *qn16, float *qeps,
                                                          float *qstat, float *lb, int32_t *order, float *lbs,
                                                          const int32_t *__restrict__ k_dev,
                                                          const float *__restrict__ t_dev, int n_pairs,
                                                          const int32_t *__restrict__ pair_k,
                                                          const float *__restrict__ pair_t, int kmax, RoundBufs b,
                                                          int F, int32_t *pcnt) {
  extern __shared__ uint64_t smem[];  // per wavefront: keys [N], zs [m], st [S][2] (floats)
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  uint64_t *keys = smem + static_cast<size_t>(w) * slice64;
  float *zs = reinterpret_cast<float *>(keys + N);
  float *st = zs + m;
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < kCtlCount; i += blockDim.x) b.ctl[i] = 0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) b.leaf_cnt[i] = 0;
    if (pcnt)
      for (int i = threadIdx.x; i < F; i += blockDim.x) pcnt[i] = 0;
  }
  const int64_t q = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + w;
  if (q >= nq) return;  // no work-group barrier below
  const float *r = raw + q * m;
  float rv[kSetupMaxPerLane];
#pragma unroll
  for (int c = 0; c < kSetupMaxPerLane; ++c) {
    const int t = lane + kWave * c;
    rv[c] = t < m ? r[t] : 0.0f;
  }
  // FP64 mean and population std (row_moments' order of operations)
  double sum = 0.0;
#pragma unroll
  for (int c = 0; c < kSetupMaxPerLane; ++c)
    if (lane + kWave * c < m) sum += static_cast<double>(rv[c]);
  sum = wave_sum(sum);
  const double mu = sum / m;
  double var = 0.0;
#pragma unroll
  for (int c = 0; c < kSetupMaxPerLane; ++c)
    if (lane + kWave * c < m) {
      const double d = static_cast<double>(rv[c]) - mu;
      var += d * d;
    }
  var = wave_sum(var);
  const double sd = sqrt(var / m);
  float nrm = 0.0f, err = 0.0f;
#pragma unroll
  for (int c = 0; c < kSetupMaxPerLane; ++c) {
    const int t = lane + kWave * c;
    if (t < m) {
      const float z = normalise(rv[c], mu, sd);
      const uint16_t bb = f32_to_bf16(z);
      const float zb = bf16_to_f32(bb);
      zs[t] = z;
      q32[q * m + t] = z;
      q16[q * m + t] = bb;
      nrm = fmaf(zb, zb, nrm);
      const float e = z - zb;
      err = fmaf(e, e, err);
    }
  }
  nrm = wave_sum(nrm);
  err = wave_sum(err);
  if (lane == 0) {
    qn16[q] = nrm;
    qeps[q] = sqrtf(err) * (1.0f + 1e-5f);
    b.cursor[q] = 0;
    b.tau[q] = __builtin_inff();
    b.res_cnt[q] = 0;
    b.qitem_cnt[q] = 0;
  }
  {
    const int k = min(max(k_dev[q], 1), kmax);
    const int pr = select_pair_wave(k, t_dev[q], n_pairs, pair_k, pair_t, lane);
    if (lane == 0) {
      b.pair[q] = pr;
      b.kq[q] = k;
    }
  }
  wave_lds_sync();
  for (int s = lane; s < S; s += kWave) {
    float a, c;
    segment_moments(zs, m, S, s, a, c);
    st[2 * s] = a;
    st[2 * s + 1] = c;
    qstat[(q * S + s) * 2 + 0] = a;
    qstat[(q * S + s) * 2 + 1] = c;
  }
  wave_lds_sync();
  for (int i = lane; i < N; i += kWave) {
    const float v = S == 16 ? summary_lb_t<16>(st, boxes_t, N, i, m)
                            : summary_lb(st, boxes + static_cast<int64_t>(i) * S * 4, S, m);
    lb[q * N + i] = v;
    keys[i] = make_key(v, static_cast<uint32_t>(i));
  }
  wave_lds_sync();
  int32_t *oq = order + q * N;
  float *lq = lbs + q * N;
  if (N <= kWave) rank_and_write<1>(keys, N, lane, oq, lq);
  else if (N <= 2 * kWave) rank_and_write<2>(keys, N, lane, oq, lq);
  else rank_and_write<4>(keys, N, lane, oq, lq);
}

// One work-group per query: bitonic sort of (lb bits, leaf id) keys in LDS.
__global__ void __launch_bounds__(256) k_order(const float *__restrict__ lb, int N, int P, int32_t *order,
                                               float *lbs, const int32_t *__restrict__ slots) {
  extern __shared__ uint64_t keys[];
  const int64_t q = slots ? slots[blockIdx.x] : static_cast<int64_t>(blockIdx.x);
  for (int i = threadIdx.x; i < P; i += blockDim.x)
    keys[i] = i < N ? make_key(lb[q * N + i], static_cast<uint32_t>(i)) : kKeyMax;
  __syncthreads();
  block_sort_u64(keys, P);
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    order[q * N + i] = static_cast<int32_t>(key_row(keys[i]));
    lbs[q * N + i] = key_d2(keys[i]);  // the bound itself, in visit order
  }
}

__global__ void __launch_bounds__(256) k_make_queries(const float *__restrict__ x32, const int64_t *__restrict__ rows,
                                                      const float *__restrict__ sigma, int64_t nq, int m,
                                                      uint64_t seed, float *out) {
  int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= nq * m) return;
  int64_t j = idx / m;
  int t = static_cast<int>(idx - j * m);
  uint64_t base = mix64(seed ^ mix64(static_cast<uint64_t>(j) * 0x100000001b3ull + t));
  double u1 = u01(mix64(base + 1)), u2 = u01(mix64(base + 2));
  double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);  // Box-Muller
  out[idx] = static_cast<float>(x32[rows[j] * m + t] + sigma[j] * g);
}

}  // namespace

void launch_series_stats(const float *raw, int64_t n, int m, int S, double *mean, double *sd, float *seg_mu,
                         float *seg_sd, hipStream_t st) {
  int64_t blocks = ceil_div(n, kRowsPerBlock);
  hipLaunchKernelGGL(k_series_stats, dim3(blocks), dim3(256), 0, st, raw, n, m, S, mean, sd, seg_mu, seg_sd);
  LAUNCH_OK("series_stats");
}

void launch_pack(const float *raw, const int64_t *src_of_row, const int32_t *leaf_of_row, int64_t rows, int m,
                 const double *mean, const double *sd, float *x32, uint16_t *x16, float *xn16, int64_t *rowid,
                 float *leaf_eps, hipStream_t st) {
  int64_t blocks = ceil_div(rows, kRowsPerBlock);
  hipLaunchKernelGGL(k_pack, dim3(blocks), dim3(256), 0, st, raw, src_of_row, leaf_of_row, rows, m, mean, sd, x32,
                     x16, xn16, rowid, leaf_eps);
  LAUNCH_OK("pack");
}

void launch_znorm(const float *x, int64_t n, int m, float *out, hipStream_t st) {
  int64_t blocks = ceil_div(n, kRowsPerBlock);
  hipLaunchKernelGGL(k_znorm, dim3(blocks), dim3(256), 0, st, x, n, m, out);
  LAUNCH_OK("znorm");
}

void launch_qprep(const float *raw, int64_t nq, int m, int S, float *q32, uint16_t *q16, float *qn16, float *qeps,
                  float *qstat, hipStream_t st, const int32_t *slots) {
  int64_t blocks = ceil_div(nq, kRowsPerBlock);
  hipLaunchKernelGGL(k_qprep, dim3(blocks), dim3(256), 0, st, raw, nq, m, S, q32, q16, qn16, qeps, qstat, slots);
  LAUNCH_OK("qprep");
}

void launch_lb(const float *qstat, int64_t nq, const float *boxes, int N, int S, int m, float *lb, hipStream_t st,
               const int32_t *slots) {
  int64_t total = nq * N;
  hipLaunchKernelGGL(k_lb, dim3(ceil_div(total, 256)), dim3(256), 0, st, qstat, nq, boxes, N, S, m, lb, slots);
  LAUNCH_OK("lb");
}

void launch_order(const float *lb, int64_t nq, int N, int32_t *order, float *lbs, hipStream_t st,
                  const int32_t *slots) {
  int P = pow2_at_least(N < 2 ? 2 : N);
  size_t lds = static_cast<size_t>(P) * sizeof(uint64_t);  // <= 128 KiB for N <= 16384
  allow_lds(reinterpret_cast<const void *>(k_order), lds);
  hipLaunchKernelGGL(k_order, dim3(nq), dim3(256), lds, st, lb, N, P, order, lbs, slots);
  LAUNCH_OK("order");
}

void launch_query_setup(const float *raw, int64_t nq, int m, int S, const float *boxes, const float *boxes_t, int N,
                        float *q32,
                        uint16_t *q16, float *qn16, float *qeps, float *qstat, float *lb, int32_t *order, float *lbs, const int32_t *k_dev, const float *t_dev,
                        int n_pairs, const int32_t *pair_k, const float *pair_t, int kmax, RoundBufs b, int F,
                        int32_t *pcnt, hipStream_t st) {
  if (nq <= 0) return;
  if (N <= kSetupWaveMaxN && m <= kSetupMaxPerLane * kWave) {
    const int slice64 = N + (m + 2 * S + 1) / 2;  // keys, then zs and st in 8-byte units
    const size_t lds_w = 4 * static_cast<size_t>(slice64) * sizeof(uint64_t);
    allow_lds(reinterpret_cast<const void *>(k_query_setup_wave), lds_w);
    hipLaunchKernelGGL(k_query_setup_wave, dim3(static_cast<unsigned>(ceil_div(nq, 4))), dim3(256), lds_w, st, raw, nq,
                       m, S, boxes, boxes_t, N, slice64, q32, q16, qn16, qeps, qstat, lb, order, lbs, k_dev, t_dev, n_pairs,
                       pair_k, pair_t, kmax, b, F, pcnt);
    LAUNCH_OK("query_setup");
    return;
  }
  const int P = pow2_at_least(N < 2 ? 2 : N);
  const size_t lds = static_cast<size_t>(P) * sizeof(uint64_t) + (static_cast<size_t>(m) + 2 * S) * sizeof(float);
  allow_lds(reinterpret_cast<const void *>(k_query_setup), lds);
  hipLaunchKernelGGL(k_query_setup, dim3(static_cast<unsigned>(nq)), dim3(512), lds, st, raw, m, S, boxes_t, N, P, q32,
                     q16, qn16, qeps, qstat, lb, order, lbs, k_dev, t_dev, n_pairs, pair_k, pair_t, kmax, b, F, pcnt);
  LAUNCH_OK("query_setup");
}

void launch_make_queries(const float *x32, const int64_t *rows, const float *sigma, int64_t nq, int m,
                         uint64_t seed, float *out, hipStream_t st) {
  int64_t total = nq * m;
  hipLaunchKernelGGL(k_make_queries, dim3(ceil_div(total, 256)), dim3(256), 0, st, x32, rows, sigma, nq, m, seed,
                     out);
  LAUNCH_OK("make_queries");
}

}  // namespace leafi
