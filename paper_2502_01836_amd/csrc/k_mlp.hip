// Learned-filter kernels: batched MLP inference d^f = w2 . ReLU(W1 q + b1) + b2
// for every (query, filter) pair, and plain SGD training of every filter
// (one work-group per filter, the whole epoch loop on the device).
//
// Packed filter layout (P = h*m + 2h + 1 floats): W1 input-major (element
// (i, j) = input i, hidden unit j at i*h + j), b1 [h], w2 [h], b2.
#include <algorithm>

#include "device_util.h"
#include "kernels.h"

namespace leafi {

namespace {

// Inference tile: 16 queries x all hidden units per work-group, on FP32
// matrix cores (v_mfma_f32_16x16x4_f32: A = W1^T, 16 hidden units x 4 inputs;
// B = 4 inputs x the 16 queries; FP32 accumulation).  Each of the 4
// wavefronts owns 64 hidden units of every 256-unit chunk (four 16 x 16
// accumulator tiles).  The queries are staged in LDS (row stride m + 4, so
// the B reads of one instruction hit distinct banks).  The output layer is
// summed per lane over its hidden units, then across the 4 lanes sharing a
// query and across the wavefronts in a fixed order, so the result of a
// (query, filter) pair does not depend on which tile or batch holds it.
constexpr int kMlpQ = 32;             // queries per tile
constexpr int kMlpQBig = 64;          // queries per tile of a large pair batch (W1 read half as often)
constexpr int kMlpXcds = 8;           // XCDs (separate L2 caches) per device

// LDS for tiles of up to Q queries: the query tile [Q][m + 4], the
// per-wavefront output sums [4][Q], the tile's query rows [Q] (int64) and
// 8 ints for the tile search and the tile-prefix scan.  (All carved from the
// dynamic block: a static __shared__ variable would move it off its 16-byte
// alignment.)
__host__ __device__ constexpr size_t mlp_tile_floats(int m, int Q) { return static_cast<size_t>(Q) * (m + 4) + 6 * Q; }
size_t mlp_infer_lds(int m, int Q = kMlpQ) { return (mlp_tile_floats(m, Q) + 8) * sizeof(float); }

template <int Q, typename RowIdx, typename Out>
__device__ inline void mlp_tile(const float *__restrict__ w, int f, int m, int h, const float *__restrict__ x,
                                int64_t r0, int64_t nrows, RowIdx qidx, Out out, float *xs) {
  constexpr int kMlpQ = Q;              // queries per tile
  constexpr int kMlpQB = Q / 16;        // 16-query column blocks per tile
  typedef float floatx4 __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int S = m + 4;
  float *red = xs + kMlpQ * S;
  int64_t *qrow = reinterpret_cast<int64_t *>(red + 4 * kMlpQ);
  const int64_t P = static_cast<int64_t>(h) * m + 2 * h + 1;
  const float *W1 = w + f * P;
  const float *b1 = W1 + static_cast<int64_t>(h) * m;
  const float *w2 = b1 + h;
  const float b2 = w2[h];
  const int c = lane & 15, kq = lane >> 4;
  float part[kMlpQB];
#pragma unroll
  for (int qb = 0; qb < kMlpQB; ++qb) part[qb] = 0.0f;
  // The tile's query rows into LDS (every thread, once: called after the
  // first block's weights are requested, so the two latencies overlap).
  // Wavefront w stages rows w, w + 4, ... with 16-byte loads (m is a
  // multiple of 4 and x 16-byte aligned, so every row, in x and in the
  // padded tile, starts 16-byte aligned); all of a lane's loads are in
  // flight before the first store.
  auto stage = [&]() {
    __syncthreads();  // the previous tile's readers of xs / red / qrow are done
    if (tid < kMlpQ) qrow[tid] = r0 + tid < nrows ? qidx(r0 + tid) : -1;
    __syncthreads();
    constexpr int kRowsPerWave = kMlpQ / 4;
    for (int i4 = lane; 4 * i4 < m; i4 += kWave) {
      float4 v[kRowsPerWave];
#pragma unroll
      for (int rr = 0; rr < kRowsPerWave; ++rr) {
        const int64_t rq = qrow[wave + 4 * rr];
        v[rr] = reinterpret_cast<const float4 *>(x + (rq < 0 ? 0 : rq) * m)[i4];
      }
#pragma unroll
      for (int rr = 0; rr < kRowsPerWave; ++rr) {
        const bool live = qrow[wave + 4 * rr] >= 0;
        reinterpret_cast<float4 *>(xs + (wave + 4 * rr) * S)[i4] = live ? v[rr] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
    }
    __syncthreads();
  };
  for (int jb = 0; jb < h; jb += 256) {
    const int jw = jb + 64 * wave;  // this wavefront's first hidden unit
    // (a wavefront past h still takes part in the staging below; its loads
    // are clamped into the weights and its products are skipped)
    const bool live = jw < h;  // uniform across the wavefront
    floatx4 acc[4][kMlpQB];
    int col[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int qb = 0; qb < kMlpQB; ++qb) acc[t][qb] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
      col[t] = jw + 16 * t + c;
      if (col[t] >= h) col[t] = 0;
    }
    // output-layer weights of this lane's hidden units, loaded now so their
    // latency hides under the products (a unit past h reads unit 0; its
    // term is skipped below)
    float w2v[4][4], b1v[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jw + 16 * t + 4 * kq + r;
        w2v[t][r] = w2[j < h ? j : 0];
        b1v[t][r] = b1[j < h ? j : 0];
      }
    const float *xq = xs + c * S + kq;
    const float *wk = W1 + static_cast<int64_t>(kq) * h;
    int i0 = 0;
    // 16 inputs per step; the W1 operands of the next step are loaded while
    // the current step's products run (two register buffers, unconditional
    // loads: the last prefetch re-reads the current step).  Each A value (a
    // W1 element) serves both 16-query column blocks.
    const int steps = m / 16;
    // four register buffers in rotation: the W1 operands of step s + 3 are
    // loaded while step s computes (about four steps of products cover the
    // load latency; the tile's single wavefront per SIMD has no other work
    // to hide it behind)
    float av0[4][4], av1[4][4], av2[4][4], av3[4][4];
    auto load_a = [&](float (&av)[4][4], int sidx) {
      const int base = 16 * (sidx < steps ? sidx : steps - 1);  // past the end: re-read the last step
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float *wr = wk + static_cast<int64_t>(base + 4 * u) * h;
#pragma unroll
        // unconditional load: a hidden unit past h reads column 0 instead, and
        // its output row is skipped in the output layer below
        for (int t = 0; t < 4; ++t) av[u][t] = wr[col[t]];
      }
    };
    auto step = [&](const float (&av)[4][4], int sidx) {
      const int base = 16 * sidx;
      float bv[4][kMlpQB];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int qb = 0; qb < kMlpQB; ++qb) bv[u][qb] = xq[16 * qb * S + base + 4 * u];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int qb = 0; qb < kMlpQB; ++qb)
            acc[t][qb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u][t], bv[u][qb], acc[t][qb], 0, 0, 0);
    };
    if (steps > 0) {
      load_a(av0, 0);
      load_a(av1, 1);
      load_a(av2, 2);
    }
    if (jb == 0) stage();
    if (!live) continue;  // no work-group barrier below in this iteration
    if (steps > 0) {
      int sidx = 0;
      // scheduling barriers keep the prefetches ahead of the products (the
      // compiler would otherwise sink the loads to where they are used)
      for (; sidx + 4 <= steps; sidx += 4) {
        load_a(av3, sidx + 3);
        __builtin_amdgcn_sched_barrier(0);
        step(av0, sidx);
        __builtin_amdgcn_sched_barrier(0);
        load_a(av0, sidx + 4);
        __builtin_amdgcn_sched_barrier(0);
        step(av1, sidx + 1);
        __builtin_amdgcn_sched_barrier(0);
        load_a(av1, sidx + 5);
        __builtin_amdgcn_sched_barrier(0);
        step(av2, sidx + 2);
        __builtin_amdgcn_sched_barrier(0);
        load_a(av2, sidx + 6);
        __builtin_amdgcn_sched_barrier(0);
        step(av3, sidx + 3);
        __builtin_amdgcn_sched_barrier(0);
      }
      // at most three steps left, already in av0, av1, av2
      if (sidx < steps) step(av0, sidx);
      if (sidx + 1 < steps) step(av1, sidx + 1);
      if (sidx + 2 < steps) step(av2, sidx + 2);
      i0 = 16 * steps;
    }
    for (; i0 < m; i0 += 4) {
      const float *wr = wk + static_cast<int64_t>(i0) * h;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float av = wr[col[t]];
#pragma unroll
        for (int qb = 0; qb < kMlpQB; ++qb)
          acc[t][qb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, xq[16 * qb * S + i0], acc[t][qb], 0, 0, 0);
      }
    }
    // lane holds hidden units jw + 16 t + 4 kq + r of queries c + 16 qb
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jw + 16 * t + 4 * kq + r;
        if (j < h) {
#pragma unroll
          for (int qb = 0; qb < kMlpQB; ++qb)
            part[qb] = fmaf(w2v[t][r], fmaxf(acc[t][qb][r] + b1v[t][r], 0.0f), part[qb]);
        }
      }
  }
#pragma unroll
  for (int qb = 0; qb < kMlpQB; ++qb) {
    part[qb] += __shfl_xor(part[qb], 16);
    part[qb] += __shfl_xor(part[qb], 32);
    if (lane < 16) red[wave * kMlpQ + 16 * qb + lane] = part[qb];
  }
  __syncthreads();
  if (tid < kMlpQ) {
    const int64_t r = r0 + tid;
    if (r < nrows)
      out(r, qrow[tid], ((red[tid] + red[kMlpQ + tid]) + (red[2 * kMlpQ + tid] + red[3 * kMlpQ + tid])) + b2);
  }
}

// d^f for every (query, filter): grid (F, tiles), 16 queries per tile.
__global__ void __launch_bounds__(256, 2) k_mlp_infer(const float *__restrict__ w, int F, int m, int h,
                                                   const float *__restrict__ x, int64_t nq, float *out) {
  extern __shared__ float xs[];
  const int f = blockIdx.x;
  for (int64_t r0 = static_cast<int64_t>(blockIdx.y) * kMlpQ; r0 < nq; r0 += static_cast<int64_t>(gridDim.y) * kMlpQ)
    mlp_tile<kMlpQ>(w, f, m, h, x, r0, nq, [](int64_t r) { return r; },
                    [=](int64_t r, int64_t, float v) { out[r * F + f] = v; }, xs);
}

// Exclusive prefix of the filters' tile counts ceil(pcnt[f] / 16) (one
// work-group; tile_prefix[F] = total).
__global__ void __launch_bounds__(1024) k_mlp_tiles(int F, const int32_t *__restrict__ pcnt, int32_t *tile_prefix,
                                                    int Q) {
  __shared__ int32_t sh[16];
  const int tid = threadIdx.x;
  const int per = (F + 1023) / 1024;
  const int f0 = min(F, tid * per), f1 = min(F, f0 + per);
  int sum = 0;
  for (int f = f0; f < f1; ++f) sum += (pcnt[f] + Q - 1) / Q;
  int total;
  int run = block_scan_excl<1024>(sum, sh, total);
  for (int f = f0; f < f1; ++f) {
    tile_prefix[f] = run;
    run += (pcnt[f] + Q - 1) / Q;
  }
  if (tid == 0) tile_prefix[F] = total;
}

// The persistent walk over the non-empty tiles of Q queries: tile t belongs
// to the filter f with tile_prefix[f] <= t < tile_prefix[f + 1].  Work-groups
// are dispatched to the 8 XCDs round-robin (blockIdx % 8), and each XCD has
// its own L2.  Tiles are numbered filter by filter, so the work-groups of XCD
// x take the contiguous eighth [x T / 8, (x + 1) T / 8) of the T tiles: a
// filter's W1 is fetched into one or two L2s instead of all eight.  (Any grid
// not a multiple of 8 walks the tiles in plain stride; either way every tile
// is taken exactly once.)
template <int Q>
__device__ inline void infer_pair_tiles(const float *__restrict__ w, int F, int m, int h, const float *__restrict__ x,
                                        const int64_t *__restrict__ plist, const int32_t *__restrict__ pcnt,
                                        int64_t stride, int N, const int32_t *__restrict__ pair,
                                        const float *__restrict__ offsets, const int32_t *tile_prefix, float *dfo,
                                        float *xs, int *ints) {
  int &s_lo = ints[0];
  int &s_f = ints[1];
  const int total = tile_prefix[F];
  // filters per bucket of the two-level search (at most 64 for F <= 16384)
  const int B = (F + blockDim.x - 1) / blockDim.x;
  const bool by_xcd = gridDim.x % kMlpXcds == 0;
  const int xcd = blockIdx.x % kMlpXcds;
  const int t_lo = by_xcd ? static_cast<int>(static_cast<int64_t>(total) * xcd / kMlpXcds) : 0;
  const int t_hi = by_xcd ? static_cast<int>(static_cast<int64_t>(total) * (xcd + 1) / kMlpXcds) : total;
  const int t_step = by_xcd ? gridDim.x / kMlpXcds : gridDim.x;
  for (int t = t_lo + (by_xcd ? blockIdx.x / kMlpXcds : blockIdx.x); t < t_hi; t += t_step) {
    // filter of tile t (tile_prefix is non-decreasing, so exactly one f
    // qualifies): one thread per bucket of B filters finds the bucket, then
    // one thread per filter of that bucket the filter: two dependent loads,
    // not log2 F
    __syncthreads();  // the previous tile's readers of s_lo / s_f are done
    {
      const int lo = threadIdx.x * B;
      if (lo < F && tile_prefix[lo] <= t && t < tile_prefix[min(lo + B, F)]) s_lo = lo;
    }
    __syncthreads();
    {
      const int f = s_lo + static_cast<int>(threadIdx.x);
      if (static_cast<int>(threadIdx.x) < B && f < F && tile_prefix[f] <= t && t < tile_prefix[f + 1]) s_f = f;
    }
    __syncthreads();
    const int f = __builtin_amdgcn_readfirstlane(s_f);  // uniform: kept in scalar registers
    const int64_t r0 = static_cast<int64_t>(t - tile_prefix[f]) * Q;
    const int64_t *pl = plist + f * stride;
    mlp_tile<Q>(
        w, f, m, h, x, r0, static_cast<int64_t>(pcnt[f]), [=](int64_t r) { return pl[r] / N; },
        [=](int64_t r, int64_t q, float v) { dfo[pl[r]] = v - offsets[static_cast<int64_t>(pair[q]) * F + f]; },
        xs);
  }
}

// Pruning values for listed pairs: filter f evaluates the entries
// plist[f * stride + 0 .. pcnt[f]) (q * N + visit position) and writes
// d^f - o for the query's calibrated (k, target) row.  A persistent grid
// walks the non-empty tiles of all filters.  With local_prefix every
// work-group computes the filters' tile prefix itself (into LDS, F + 1
// entries after 4 scan words: no separate launch for it) and, when big_fixed
// is -1 and the batch has at least big_min tiles of kMlpQ queries, uses tiles
// of kMlpQBig queries instead (W1 is then read half as often; a small batch
// keeps the smaller tiles, which spread over more CUs).  big_fixed 0 / 1
// forces the small / large tiles (without local_prefix, tile_prefix must be
// the prefix at that size).  lds_q is the tile size the LDS block is sized
// for.  The tile size changes no value: every (query, filter) pair is summed
// in the same order either way.
__global__ void __launch_bounds__(256, 2) k_mlp_infer_pairs(const float *__restrict__ w, int F, int m, int h,
                                                         const float *__restrict__ x,
                                                         const int64_t *__restrict__ plist,
                                                         const int32_t *__restrict__ pcnt, int64_t stride, int N,
                                                         const int32_t *__restrict__ pair,
                                                         const float *__restrict__ offsets,
                                                         const int32_t *__restrict__ tile_prefix, float *dfo,
                                                         int local_prefix, int big_min, int big_fixed, int lds_q) {
  extern __shared__ float xs[];
  // the tile area is sized for the largest tile this launch may use
  int *ints = reinterpret_cast<int *>(xs + mlp_tile_floats(m, lds_q));
  bool big = big_fixed == 1;
  if (local_prefix) {
    // tile counts at both sizes in one scan (each total < 2^31: packed as
    // small + big * 2^32, the low half never carries)
    int32_t *tp = ints + 12;  // after s_lo, s_f, 2 spare ints and the scan's 4 int64 words
    const int per = (F + blockDim.x - 1) / blockDim.x;
    const int f0 = min(F, static_cast<int>(threadIdx.x) * per), f1 = min(F, f0 + per);
    int64_t sum = 0;
    for (int f = f0; f < f1; ++f)
      sum += (pcnt[f] + kMlpQ - 1) / kMlpQ + (static_cast<int64_t>((pcnt[f] + kMlpQBig - 1) / kMlpQBig) << 32);
    int64_t tot;
    const int64_t run2 = block_scan_excl<256>(sum, reinterpret_cast<int64_t *>(ints + 4), tot);
    if (big_fixed < 0) big = big_min > 0 && (tot & 0xffffffffll) >= big_min;  // uniform
    const int Q = big ? kMlpQBig : kMlpQ;
    int run = static_cast<int>(big ? run2 >> 32 : run2 & 0xffffffffll);
    for (int f = f0; f < f1; ++f) {
      tp[f] = run;
      run += (pcnt[f] + Q - 1) / Q;
    }
    if (threadIdx.x == 0) tp[F] = static_cast<int>(big ? tot >> 32 : tot & 0xffffffffll);
    __syncthreads();
    tile_prefix = tp;
  }
  if (big)
    infer_pair_tiles<kMlpQBig>(w, F, m, h, x, plist, pcnt, stride, N, pair, offsets, tile_prefix, dfo, xs, ints);
  else
    infer_pair_tiles<kMlpQ>(w, F, m, h, x, plist, pcnt, stride, N, pair, offsets, tile_prefix, dfo, xs, ints);
}

constexpr int kTB = 64;  // training mini-batch capacity (columns of the LDS batch)

struct StepLds {
  float *xb;    // [m][kTB] batch, transposed
  float *red;   // [4][kTB] per-wave partial sums
  float *yh;    // [kTB] predictions
  float *gy;    // [kTB] dLoss/dyhat
  float *yt;    // [kTB] targets
};

// Forward pass of one batch (columns 0..nb-1 of the LDS batch): z for hidden
// unit j = threadIdx.x, predictions into s.yh.  Returns nothing; z stays in
// the caller's registers.
__device__ inline void batch_forward(const float *W1, const float *b1, const float *w2, float b2, int m, int h,
                                     int nb, const StepLds &s, float (&z)[kTB]) {
  const int j = threadIdx.x;
  const int lane = j & (kWave - 1), wv = j / kWave;
#pragma unroll
  for (int c = 0; c < kTB; ++c) z[c] = 0.0f;
  if (j < h) {
    float bj = b1[j];
#pragma unroll
    for (int c = 0; c < kTB; ++c) z[c] = bj;
    for (int i = 0; i < m; ++i) {
      float wij = W1[static_cast<int64_t>(i) * h + j];
      const float4 *xr = reinterpret_cast<const float4 *>(s.xb + i * kTB);
#pragma unroll
      for (int c4 = 0; c4 < kTB / 4; ++c4) {
        float4 xv = xr[c4];
        z[4 * c4 + 0] = fmaf(wij, xv.x, z[4 * c4 + 0]);
        z[4 * c4 + 1] = fmaf(wij, xv.y, z[4 * c4 + 1]);
        z[4 * c4 + 2] = fmaf(wij, xv.z, z[4 * c4 + 2]);
        z[4 * c4 + 3] = fmaf(wij, xv.w, z[4 * c4 + 3]);
      }
    }
  }
  float w2j = j < h ? w2[j] : 0.0f;
#pragma unroll
  for (int c = 0; c < kTB; ++c) {
    float p = wave_sum(w2j * fmaxf(z[c], 0.0f));
    if (lane == 0) s.red[wv * kTB + c] = p;
  }
  __syncthreads();
  if (j < kTB) {
    float acc = b2;
    for (int w = 0; w < static_cast<int>(blockDim.x / kWave); ++w) acc += s.red[w * kTB + j];
    s.yh[j] = j < nb ? acc : 0.0f;
  }
  __syncthreads();
}

// Gradient step on the batch whose forward pass left z in registers and
// predictions in s.yh; targets in s.yt.  Returns the batch loss (thread 0).
__device__ inline float batch_sgd(float *W1, float *b1, float *w2, float *b2p, int m, int h, int nb, float lr,
                                  const StepLds &s, const float (&z)[kTB]) {
  const int j = threadIdx.x;
  if (j < kTB) s.gy[j] = j < nb ? 2.0f * (s.yh[j] - s.yt[j]) / nb : 0.0f;
  __syncthreads();
  float loss = 0.0f;
  if (j == 0) {
    float gs = 0.0f;
    for (int c = 0; c < nb; ++c) {
      float r = s.yh[c] - s.yt[c];
      loss += r * r;
      gs += s.gy[c];
    }
    loss /= nb;
    *b2p -= lr * gs;
  }
  if (j < h) {
    float w2j = w2[j];
    float gw2 = 0.0f, gb1 = 0.0f;
    float delta[kTB];
#pragma unroll
    for (int c = 0; c < kTB; ++c) {
      float g = s.gy[c];
      gw2 = fmaf(g, fmaxf(z[c], 0.0f), gw2);
      delta[c] = z[c] > 0.0f ? g * w2j : 0.0f;
      gb1 += delta[c];
    }
    for (int i = 0; i < m; ++i) {
      const float4 *xr = reinterpret_cast<const float4 *>(s.xb + i * kTB);
      float gw = 0.0f;
#pragma unroll
      for (int c4 = 0; c4 < kTB / 4; ++c4) {
        float4 xv = xr[c4];
        gw = fmaf(delta[4 * c4 + 0], xv.x, gw);
        gw = fmaf(delta[4 * c4 + 1], xv.y, gw);
        gw = fmaf(delta[4 * c4 + 2], xv.z, gw);
        gw = fmaf(delta[4 * c4 + 3], xv.w, gw);
      }
      W1[static_cast<int64_t>(i) * h + j] -= lr * gw;
    }
    w2[j] = w2j - lr * gw2;
    b1[j] -= lr * gb1;
  }
  __syncthreads();
  return loss;
}

__device__ inline StepLds carve(float *base, int m) {
  StepLds s;
  s.xb = base;
  s.red = s.xb + m * kTB;
  s.yh = s.red + 4 * kTB;
  s.gy = s.yh + kTB;
  s.yt = s.gy + kTB;
  return s;
}

// Load examples ex[0..nb) (query indices into xq) into the LDS batch.
__device__ inline void load_batch(const float *xq, int m, const int32_t *qidx, const float *y, int nb,
                                  const StepLds &s) {
  for (int e = threadIdx.x; e < kTB * m; e += blockDim.x) {
    int c = e / m, i = e - (e / m) * m;
    s.xb[i * kTB + c] = c < nb ? xq[static_cast<int64_t>(qidx[c]) * m + i] : 0.0f;
  }
  for (int c = threadIdx.x; c < kTB; c += blockDim.x) s.yt[c] = c < nb ? y[c] : 0.0f;
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_mlp_sgd_step(float *w, int F, int m, int h, const float *x, const float *y,
                                                      int batch, float lr, float *loss_out) {
  extern __shared__ float lds[];
  StepLds s = carve(lds, m);
  const int f = blockIdx.x;
  const int64_t P = static_cast<int64_t>(h) * m + 2 * h + 1;
  float *W1 = w + f * P;
  float *b1 = W1 + static_cast<int64_t>(h) * m;
  float *w2 = b1 + h;
  for (int e = threadIdx.x; e < kTB * m; e += blockDim.x) {
    int c = e / m, i = e - (e / m) * m;
    s.xb[i * kTB + c] = c < batch ? x[(static_cast<int64_t>(f) * batch + c) * m + i] : 0.0f;
  }
  for (int c = threadIdx.x; c < kTB; c += blockDim.x) s.yt[c] = c < batch ? y[static_cast<int64_t>(f) * batch + c] : 0.0f;
  __syncthreads();
  float z[kTB];
  batch_forward(W1, b1, w2, w2[h], m, h, batch, s, z);
  float loss = batch_sgd(W1, b1, w2, w2 + h, m, h, batch, lr, s, z);
  if (threadIdx.x == 0 && loss_out) loss_out[f] = loss;
}

__global__ void __launch_bounds__(256) k_mlp_train(TrainArgs a) {
  // 16-byte aligned after the static variables below (float4 reads)
  extern __shared__ __align__(16) float lds[];
  StepLds s = carve(lds, a.m);
  int32_t *perm = reinterpret_cast<int32_t *>(s.yt + kTB);
  int32_t *bq = perm + a.n_train;   // [kTB] query indices of the current batch
  float *by = reinterpret_cast<float *>(bq + kTB);  // [kTB]
  __shared__ float vsum;
  __shared__ int stop;
  __shared__ float b2s;  // output bias, kept in LDS while training
  const int f = blockIdx.x;
  const int m = a.m, h = a.h;
  const int64_t P = static_cast<int64_t>(h) * m + 2 * h + 1;
  float *W1 = a.w + f * P;
  float *b1 = W1 + static_cast<int64_t>(h) * m;
  float *w2 = b1 + h;
  float *b2 = w2 + h;
  float *wb = a.w_best + f * P;
  const int32_t *exq = a.ex_q + static_cast<int64_t>(f) * a.n_ex;
  const float *exy = a.ex_y + static_cast<int64_t>(f) * a.n_ex;
  const int n_val = a.n_ex - a.n_train;
  // output bias starts at the mean training target
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int e = 0; e < a.n_train; ++e) acc += exy[e];
    b2s = static_cast<float>(acc / (a.n_train > 0 ? a.n_train : 1));
    wb[P - 1] = b2s;
  }
  for (int e = threadIdx.x; e < a.n_train; e += blockDim.x) perm[e] = e;
  for (int64_t e = threadIdx.x; e < P - 1; e += blockDim.x) wb[e] = W1[e];
  __syncthreads();
  float best = __builtin_inff();
  float lr = a.lr0;
  int bad = 0, epoch = 0;
  float z[kTB];
  for (; epoch < a.max_epochs; ++epoch) {
    if (threadIdx.x == 0) {  // Fisher-Yates shuffle with a counter-based generator
      for (int e = a.n_train - 1; e > 0; --e) {
        uint64_t r = mix64(a.seed ^ mix64((static_cast<uint64_t>(f) << 40) ^ (static_cast<uint64_t>(epoch) << 20) ^ e));
        int o = static_cast<int>(r % static_cast<uint64_t>(e + 1));
        int tmp = perm[e];
        perm[e] = perm[o];
        perm[o] = tmp;
      }
    }
    __syncthreads();
    for (int s0 = 0; s0 < a.n_train; s0 += a.batch) {
      int nb = a.n_train - s0 < a.batch ? a.n_train - s0 : a.batch;
      for (int c = threadIdx.x; c < nb; c += blockDim.x) {
        bq[c] = exq[perm[s0 + c]];
        by[c] = exy[perm[s0 + c]];
      }
      __syncthreads();
      load_batch(a.xq, m, bq, by, nb, s);
      batch_forward(W1, b1, w2, b2s, m, h, nb, s, z);
      batch_sgd(W1, b1, w2, &b2s, m, h, nb, lr, s, z);
    }
    // validation error
    if (threadIdx.x == 0) vsum = 0.0f;
    __syncthreads();
    for (int s0 = 0; s0 < n_val; s0 += kTB) {
      int nb = n_val - s0 < kTB ? n_val - s0 : kTB;
      load_batch(a.xq, m, exq + a.n_train + s0, exy + a.n_train + s0, nb, s);
      batch_forward(W1, b1, w2, b2s, m, h, nb, s, z);
      if (threadIdx.x == 0)
        for (int c = 0; c < nb; ++c) {
          float r = s.yh[c] - s.yt[c];
          vsum += r * r;
        }
      __syncthreads();
    }
    float vm = n_val > 0 ? vsum / n_val : 0.0f;
    bool improved = vm < best * (1.0f - 1e-4f);
    if (improved) {
      best = vm;
      bad = 0;
      for (int64_t e = threadIdx.x; e < P - 1; e += blockDim.x) wb[e] = W1[e];
      if (threadIdx.x == 0) wb[P - 1] = b2s;
    } else if (++bad >= a.patience) {
      lr *= 0.1f;
      bad = 0;
    }
    if (threadIdx.x == 0) stop = (lr < a.lr_min * (1.0f - 1e-3f)) || !(vm == vm);
    __syncthreads();
    if (stop) {
      ++epoch;
      break;
    }
    __syncthreads();
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < P - 1; e += blockDim.x) W1[e] = wb[e];
  if (threadIdx.x == 0) {
    *b2 = wb[P - 1];
    a.val_mse[f] = best;
    a.epochs_run[f] = epoch;
  }
}

// ---- SGD on FP32 matrix cores ------------------------------------------------
//
// One work-group of kTrainWaves wavefronts per filter; wavefront w owns the
// kTrainHT 16-unit hidden tiles kTrainHT w .. (32 hidden units) and holds
// that slice of W1 in registers for the whole run (per hidden tile, m / 16
// input tiles x 4 values per lane), so the weights never travel to memory
// between steps.  Both products of a step run on v_mfma_f32_16x16x4_f32
// (16 x 16 output tile, 4 inputs per instruction; A: lane l holds
// A[l mod 16][l / 16]; B: B[l / 16][l mod 16]; D: lane l, register r holds
// D[4 (l / 16) + r][l mod 16]):
//   forward   Z = X W1 (batch x hidden): K step s of input tile ti takes the
//             inputs 16 ti + 4 q + s (q = lane / 16), so register s of the
//             wavefront's W1 tile is the B operand; the batch rows come from
//             LDS as the A operand;
//   backward  dW1 = X^T Delta (inputs x hidden): Delta = dL/dZ is the forward
//             output tile itself, so its register s is the B operand of K
//             step s (batch row 4 q + s of the tile), and the output tile
//             lands in exactly the layout of the W1 registers, which are
//             updated in place.
// The output layer, its gradient and the loss are summed in a fixed order
// (per lane over its hidden units, then a fixed butterfly over the 16 lanes
// of a quarter, then the wavefronts in turn), so a run is deterministic.
constexpr int kTrainWaves = 8;            // wavefronts per filter
constexpr int kTrainHT = 2;               // 16-unit hidden tiles per wavefront: hidden units <= 256
constexpr int kTrainThreads = 64 * kTrainWaves;
constexpr int kTrainB = 64;               // mini-batch capacity: four 16-row tiles
typedef float floatx4_t __attribute__((ext_vector_type(4)));

struct TrainLds {
  float *xb;     // [kTrainB][m + 1] the batch rows (odd row stride: the A reads of 16 rows hit 16 banks)
  float *yt;     // [kTrainB] targets
  float *gy;     // [kTrainB] dLoss / dyhat
  float *sq;     // [kTrainB] squared errors
  float *red;    // [kTrainWaves][kTrainB] per-wavefront output-layer sums
  float *scal;   // [4]: b2, validation error
  int ldx;
};

__device__ inline TrainLds train_lds(float *base, int m) {
  TrainLds t;
  t.ldx = m + 1;
  t.xb = base;
  t.yt = t.xb + kTrainB * t.ldx;
  t.gy = t.yt + kTrainB;
  t.sq = t.gy + kTrainB;
  t.red = t.sq + kTrainB;
  t.scal = t.red + kTrainWaves * kTrainB;
  return t;
}
size_t train_lds_floats(int m) { return static_cast<size_t>(kTrainB) * (m + 1) + 3 * kTrainB + kTrainWaves * kTrainB + 4; }

// Hidden unit of this lane in hidden tile i of its wavefront.
__device__ __forceinline__ int train_unit(int i) {
  return 16 * (kTrainHT * (threadIdx.x / kWave) + i) + (threadIdx.x & 15);
}

// The wavefront's W1 slice, b1 and w2 from the packed weights (units >= h: zero).
template <int MT>
__device__ inline void train_load(const float *wf, int m, int h, float (&W)[kTrainHT][MT][4], float (&b1r)[kTrainHT],
                                  float (&w2r)[kTrainHT]) {
  const int q = (threadIdx.x & (kWave - 1)) >> 4;
#pragma unroll
  for (int i = 0; i < kTrainHT; ++i) {
    const int j = train_unit(i);
    const bool act = j < h;
#pragma unroll
    for (int ti = 0; ti < MT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) W[i][ti][r] = act ? wf[static_cast<int64_t>(16 * ti + 4 * q + r) * h + j] : 0.0f;
    b1r[i] = act ? wf[static_cast<int64_t>(h) * m + j] : 0.0f;
    w2r[i] = act ? wf[static_cast<int64_t>(h) * m + h + j] : 0.0f;
  }
}

// Write the wavefront's W1 slice, b1 and w2 into packed weights (the four
// quarters of the wavefront hold the same b1 and w2; the first writes them).
template <int MT>
__device__ inline void train_store(float *wf, int m, int h, const float (&W)[kTrainHT][MT][4],
                                   const float (&b1r)[kTrainHT], const float (&w2r)[kTrainHT]) {
  const int q = (threadIdx.x & (kWave - 1)) >> 4;
#pragma unroll
  for (int i = 0; i < kTrainHT; ++i) {
    const int j = train_unit(i);
    if (j >= h) continue;
    // one running address, made opaque after every step: the compiler would
    // otherwise compute all MT x 4 addresses once and keep them live across
    // the whole training loop that calls this
    float *p = wf + static_cast<int64_t>(4 * q) * h + j;
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        *p = W[i][ti][r];
        p += h;
        asm volatile("" : "+v"(p));
      }
      p += static_cast<int64_t>(12) * h;
    }
    if (q == 0) {
      wf[static_cast<int64_t>(h) * m + j] = b1r[i];
      wf[static_cast<int64_t>(h) * m + h + j] = w2r[i];
    }
  }
}

// One step on the nb (<= 64) rows staged in LDS (rows nb .. 63 are zero):
// forward pass and squared errors, and with `update` the plain SGD step of
// the mean squared error with learning rate lr.  Returns the sum of squared
// errors (valid in thread 0).  Every thread of the work-group calls it.
// Hidden units >= h have zero weights, b1 and w2 and are never updated
// (their Delta is zero), so they add nothing.
template <int MT, bool update>
__device__ inline float train_step(float (&W)[kTrainHT][MT][4], float (&b1r)[kTrainHT], float (&w2r)[kTrainHT], int h,
                                   int nb, float lr, const TrainLds &t) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int q = lane >> 4, col = lane & 15;
  const bool act = 16 * kTrainHT * wave < h;  // any hidden unit of this wavefront in use
  constexpr int ldx = 16 * MT + 1;            // t.ldx as a constant: LDS offsets become immediates
  floatx4_t Z[kTrainHT][4];
#pragma unroll
  for (int i = 0; i < kTrainHT; ++i)
#pragma unroll
    for (int tb = 0; tb < 4; ++tb) Z[i][tb] = floatx4_t{0.0f, 0.0f, 0.0f, 0.0f};
  if (act) {
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) {
      __builtin_amdgcn_sched_barrier(0);  // one input tile's operands in flight at a time
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int tb = 0; tb < 4; ++tb) {
          const float a = t.xb[(16 * tb + col) * ldx + 16 * ti + 4 * q + s];
#pragma unroll
          for (int i = 0; i < kTrainHT; ++i) Z[i][tb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, W[i][ti][s], Z[i][tb], 0, 0, 0);
        }
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  // output layer: per lane over its hidden units, then over the quarter's 16 lanes
#pragma unroll
  for (int tb = 0; tb < 4; ++tb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float p = 0.0f;
#pragma unroll
      for (int i = 0; i < kTrainHT; ++i) p = fmaf(w2r[i], fmaxf(Z[i][tb][r] + b1r[i], 0.0f), p);
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) p += __shfl_xor(p, o, kWave);
      if (col == 0) t.red[wave * kTrainB + 16 * tb + 4 * q + r] = p;
    }
  __syncthreads();
  if (threadIdx.x < kTrainB) {
    const int c = threadIdx.x;
    float yh = t.scal[0];
    for (int w = 0; w < kTrainWaves; ++w) yh += t.red[w * kTrainB + c];
    const float e = c < nb ? yh - t.yt[c] : 0.0f;
    t.gy[c] = 2.0f * e / static_cast<float>(nb);
    t.sq[c] = e * e;
  }
  __syncthreads();
  float loss = 0.0f;
  if (threadIdx.x == 0)
    for (int c = 0; c < nb; ++c) loss += t.sq[c];
  if (!update) return loss;
  // Delta = dL/dZ into the forward tiles; gradients of w2 and b1
  float gw2[kTrainHT], gb1[kTrainHT];
#pragma unroll
  for (int i = 0; i < kTrainHT; ++i) gw2[i] = gb1[i] = 0.0f;
#pragma unroll
  for (int tb = 0; tb < 4; ++tb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float g = t.gy[16 * tb + 4 * q + r];
#pragma unroll
      for (int i = 0; i < kTrainHT; ++i) {
        const float z = Z[i][tb][r] + b1r[i];
        gw2[i] = fmaf(g, fmaxf(z, 0.0f), gw2[i]);
        const float d = z > 0.0f ? g * w2r[i] : 0.0f;
        Z[i][tb][r] = d;
        gb1[i] += d;
      }
    }
#pragma unroll
  for (int i = 0; i < kTrainHT; ++i) {
    gw2[i] += __shfl_xor(gw2[i], 16, kWave);
    gb1[i] += __shfl_xor(gb1[i], 16, kWave);
    gw2[i] += __shfl_xor(gw2[i], 32, kWave);
    gb1[i] += __shfl_xor(gb1[i], 32, kWave);
  }
  // dW1 = X^T Delta, one 16-input tile at a time, applied at once
  if (act) {
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) {
      __builtin_amdgcn_sched_barrier(0);
      floatx4_t G[kTrainHT];
#pragma unroll
      for (int i = 0; i < kTrainHT; ++i) G[i] = floatx4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int tb = 0; tb < 4; ++tb)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const float a = t.xb[(16 * tb + 4 * q + s) * ldx + 16 * ti + col];
#pragma unroll
          for (int i = 0; i < kTrainHT; ++i) G[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, Z[i][tb][s], G[i], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < kTrainHT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) W[i][ti][r] = fmaf(-lr, G[i][r], W[i][ti][r]);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = 0; i < kTrainHT; ++i) {
    b1r[i] = fmaf(-lr, gb1[i], b1r[i]);
    w2r[i] = fmaf(-lr, gw2[i], w2r[i]);
  }
  __syncthreads();  // every thread has read b2 and gy
  if (threadIdx.x == 0) {
    float gs = 0.0f;
    for (int c = 0; c < nb; ++c) gs += t.gy[c];
    t.scal[0] = fmaf(-lr, gs, t.scal[0]);
  }
  return loss;
}

// Stage nb rows into the batch: row c is xq[qidx[c]] (or x + c m without an
// index), rows nb .. 63 zero; targets likewise.
__device__ inline void train_stage(const float *xq, const int32_t *qidx, const float *y, int nb, int m,
                                   const TrainLds &t) {
  for (int e = threadIdx.x; e < kTrainB * m; e += blockDim.x) {
    const int c = e / m, i = e - c * m;
    float v = 0.0f;
    if (c < nb) v = xq[static_cast<int64_t>(qidx ? qidx[c] : c) * m + i];
    t.xb[c * t.ldx + i] = v;
  }
  for (int c = threadIdx.x; c < kTrainB; c += blockDim.x) t.yt[c] = c < nb ? y[c] : 0.0f;
  __syncthreads();
}

template <int MT>
__global__ void __launch_bounds__(kTrainThreads, 1) k_mlp_sgd_step_mfma(float *w, int m, int h, const float *x,
                                                                        const float *y, int batch, float lr,
                                                                        float *loss_out) {
  extern __shared__ __align__(16) float lds[];
  const TrainLds t = train_lds(lds, m);
  const int f = blockIdx.x;
  const int64_t P = static_cast<int64_t>(h) * m + 2 * h + 1;
  float *wf = w + f * P;
  float W[kTrainHT][MT][4], b1r[kTrainHT], w2r[kTrainHT];
  train_load<MT>(wf, m, h, W, b1r, w2r);
  if (threadIdx.x == 0) t.scal[0] = wf[P - 1];
  train_stage(x + static_cast<int64_t>(f) * batch * m, nullptr, y + static_cast<int64_t>(f) * batch, batch, m, t);
  const float sse = train_step<MT, true>(W, b1r, w2r, h, batch, lr, t);
  __syncthreads();
  train_store<MT>(wf, m, h, W, b1r, w2r);
  if (threadIdx.x == 0) {
    wf[P - 1] = t.scal[0];
    if (loss_out) loss_out[f] = sse / static_cast<float>(batch);
  }
}

// The whole SGD run of one filter per work-group (same schedule as
// k_mlp_train: per-epoch shuffle, validation after each epoch, the learning
// rate divided by 10 after `patience` epochs without a 1e-4 relative
// improvement, stop below lr_min, best-validation weights kept).
template <int MT>
__global__ void __launch_bounds__(kTrainThreads, 1) k_mlp_train_mfma(TrainArgs a) {
  extern __shared__ __align__(16) float lds[];
  const int m = a.m, h = a.h;
  const TrainLds t = train_lds(lds, m);
  int32_t *perm = reinterpret_cast<int32_t *>(t.scal + 4);  // [n_train]
  int32_t *bq = perm + a.n_train;                            // [kTrainB]
  float *by = reinterpret_cast<float *>(bq + kTrainB);       // [kTrainB]
  __shared__ int stop;
  const int f = blockIdx.x;
  const int64_t P = static_cast<int64_t>(h) * m + 2 * h + 1;
  float *wf = a.w + f * P;
  float *wb = a.w_best + f * P;
  const int32_t *exq = a.ex_q + static_cast<int64_t>(f) * a.n_ex;
  const float *exy = a.ex_y + static_cast<int64_t>(f) * a.n_ex;
  const int n_val = a.n_ex - a.n_train;
  float W[kTrainHT][MT][4], b1r[kTrainHT], w2r[kTrainHT];
  train_load<MT>(wf, m, h, W, b1r, w2r);
  // output bias starts at the mean training target
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int e = 0; e < a.n_train; ++e) acc += exy[e];
    t.scal[0] = static_cast<float>(acc / (a.n_train > 0 ? a.n_train : 1));
    wb[P - 1] = t.scal[0];
  }
  for (int e = threadIdx.x; e < a.n_train; e += blockDim.x) perm[e] = e;
  train_store<MT>(wb, m, h, W, b1r, w2r);
  __syncthreads();
  float best = __builtin_inff();
  float lr = a.lr0;
  int bad = 0, epoch = 0;
  for (; epoch < a.max_epochs; ++epoch) {
    if (threadIdx.x == 0) {  // Fisher-Yates shuffle with a counter-based generator
      for (int e = a.n_train - 1; e > 0; --e) {
        uint64_t r = mix64(a.seed ^ mix64((static_cast<uint64_t>(f) << 40) ^ (static_cast<uint64_t>(epoch) << 20) ^ e));
        int o = static_cast<int>(r % static_cast<uint64_t>(e + 1));
        int tmp = perm[e];
        perm[e] = perm[o];
        perm[o] = tmp;
      }
    }
    __syncthreads();
    for (int s0 = 0; s0 < a.n_train; s0 += a.batch) {
      const int nb = a.n_train - s0 < a.batch ? a.n_train - s0 : a.batch;
      for (int c = threadIdx.x; c < nb; c += blockDim.x) {
        bq[c] = exq[perm[s0 + c]];
        by[c] = exy[perm[s0 + c]];
      }
      __syncthreads();
      train_stage(a.xq, bq, by, nb, m, t);
      train_step<MT, true>(W, b1r, w2r, h, nb, lr, t);
      __syncthreads();
    }
    // validation error (forward passes only)
    float vsum = 0.0f;
    for (int s0 = 0; s0 < n_val; s0 += kTrainB) {
      const int nb = n_val - s0 < kTrainB ? n_val - s0 : kTrainB;
      train_stage(a.xq, exq + a.n_train + s0, exy + a.n_train + s0, nb, m, t);
      vsum += train_step<MT, false>(W, b1r, w2r, h, nb, 0.0f, t);
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const float vm = n_val > 0 ? vsum / n_val : 0.0f;
      if (a.val_trace) a.val_trace[static_cast<int64_t>(f) * a.max_epochs + epoch] = vm;
      t.scal[1] = vm;
    }
    __syncthreads();
    const float vm = t.scal[1];
    const bool improved = vm < best * (1.0f - 1e-4f);
    if (improved) {
      best = vm;
      bad = 0;
      train_store<MT>(wb, m, h, W, b1r, w2r);
      if (threadIdx.x == 0) wb[P - 1] = t.scal[0];
    } else if (++bad >= a.patience) {
      lr *= 0.1f;
      bad = 0;
    }
    if (threadIdx.x == 0) stop = (lr < a.lr_min * (1.0f - 1e-3f)) || !(vm == vm);
    __syncthreads();
    if (stop) {
      ++epoch;
      break;
    }
    __syncthreads();
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < P; e += blockDim.x) wf[e] = wb[e];
  if (threadIdx.x == 0) {
    a.val_mse[f] = best;
    a.epochs_run[f] = epoch;
  }
}

// ---- inference with the weights held in registers ---------------------------
//
// For the shapes the matrix-core training serves: a persistent grid of
// work-groups of kTrainWaves wavefronts, each taking whole filters.  A
// filter's W1 slice is read once into registers in the training layout
// (train_load), then its rows -- every query, or the filter's listed (query,
// leaf) pairs -- pass through LDS up to 64 at a time: the forward product on
// v_mfma_f32_16x16x4_f32 exactly as in training (16-row blocks past the
// batch's rows skipped), ReLU and the output layer summed per lane over its
// hidden units, over the 16 lanes of a quarter, then b2 plus the wavefronts
// in turn.  Every row's value is computed the same way whichever rows share
// its batch, so the dense and the listed forms give the same d^f.
template <int MT>
__device__ inline void infer_batch(const float (&W)[kTrainHT][MT][4], const float (&b1r)[kTrainHT],
                                   const float (&w2r)[kTrainHT], int h, int nrb, const TrainLds &t) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int q = lane >> 4, col = lane & 15;
  const bool act = 16 * kTrainHT * wave < h;
  constexpr int ldx = 16 * MT + 1;
  floatx4_t Z[kTrainHT][4];
#pragma unroll
  for (int i = 0; i < kTrainHT; ++i)
#pragma unroll
    for (int tb = 0; tb < 4; ++tb) Z[i][tb] = floatx4_t{0.0f, 0.0f, 0.0f, 0.0f};
  if (act) {
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int tb = 0; tb < 4; ++tb) {
          if (tb < nrb) {  // uniform
            const float a = t.xb[(16 * tb + col) * ldx + 16 * ti + 4 * q + s];
#pragma unroll
            for (int i = 0; i < kTrainHT; ++i)
              Z[i][tb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, W[i][ti][s], Z[i][tb], 0, 0, 0);
          }
        }
    }
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int tb = 0; tb < 4; ++tb) {
    if (tb >= nrb) break;  // uniform
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float p = 0.0f;
#pragma unroll
      for (int i = 0; i < kTrainHT; ++i) p = fmaf(w2r[i], fmaxf(Z[i][tb][r] + b1r[i], 0.0f), p);
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) p += __shfl_xor(p, o, kWave);
      if (col == 0) t.red[wave * kTrainB + 16 * tb + 4 * q + r] = p;
    }
  }
}

// The wavefront's W1 slice, b1 and w2 as train_load reads them, through one
// running address made opaque after every step (the compiler would otherwise
// compute all MT x 4 x kTrainHT 64-bit addresses before the first load).
template <int MT>
__device__ inline void infer_load(const float *wf, int m, int h, float (&W)[kTrainHT][MT][4], float (&b1r)[kTrainHT],
                                  float (&w2r)[kTrainHT]) {
  const int q = (threadIdx.x & (kWave - 1)) >> 4;
#pragma unroll
  for (int i = 0; i < kTrainHT; ++i) {
    const int j = train_unit(i);
    const bool act = j < h;
    const float *p = wf + static_cast<int64_t>(4 * q) * h + (act ? j : 0);
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float v = *p;
        W[i][ti][r] = act ? v : 0.0f;
        p += h;
        asm volatile("" : "+v"(p));
      }
      p += static_cast<int64_t>(12) * h;
    }
    b1r[i] = act ? wf[static_cast<int64_t>(h) * m + j] : 0.0f;
    w2r[i] = act ? wf[static_cast<int64_t>(h) * m + h + j] : 0.0f;
  }
}

// Dense form (plist NULL): out[r F + f] = d^f of query r for r < nq.  Listed
// form: for the pcnt[f] entries e = plist[f stride + i] (e = q N + visit
// position), dfo[e] = d^f - offsets[pair[q] F + f].  rows_cap (32 or 64)
// rows per batch.
template <int MT>
__global__ void __launch_bounds__(kTrainThreads, 1) k_mlp_infer_ws(const float *__restrict__ w, int F, int m, int h,
                                                                   const float *__restrict__ x, int64_t nq, float *out,
                                                                   const int64_t *__restrict__ plist,
                                                                   const int32_t *__restrict__ pcnt, int64_t stride,
                                                                   int N, const int32_t *__restrict__ pair,
                                                                   const float *__restrict__ offsets, float *dfo,
                                                                   int rows_cap) {
  extern __shared__ __align__(16) float lds[];
  const TrainLds t = train_lds(lds, m);
  int64_t *rowq = reinterpret_cast<int64_t *>(t.scal + 4);  // [kTrainB] query row of each batch row
  int64_t *rent = rowq + kTrainB;                           // [kTrainB] its list entry
  const int64_t P = static_cast<int64_t>(h) * m + 2 * h + 1;
  const int m4 = m / 4;
  for (int f = blockIdx.x; f < F; f += gridDim.x) {
    const int64_t n = plist ? static_cast<int64_t>(pcnt[f]) : nq;
    if (n <= 0) continue;  // uniform
    const float *wf = w + f * P;
    float W[kTrainHT][MT][4], b1r[kTrainHT], w2r[kTrainHT];
    infer_load<MT>(wf, m, h, W, b1r, w2r);
    const float b2 = wf[P - 1];
    for (int64_t r0 = 0; r0 < n; r0 += rows_cap) {
      const int nr = static_cast<int>(n - r0 < rows_cap ? n - r0 : rows_cap);
      if (threadIdx.x < kTrainB) {
        const int c = threadIdx.x;
        int64_t qr = -1, e = -1;
        if (c < nr) {
          if (plist) {
            e = plist[f * stride + r0 + c];
            qr = e / N;
          } else {
            qr = r0 + c;
          }
        }
        rowq[c] = qr;
        rent[c] = e;
      }
      __syncthreads();
      // the batch's rows (16-byte loads; rows past nr in the last 16-row block are zero)
      const int rows16 = (nr + 15) / 16 * 16;
      for (int e4 = threadIdx.x; e4 < rows16 * m4; e4 += blockDim.x) {
        const int c = e4 / m4, i4 = e4 - c * m4;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (c < nr) v = reinterpret_cast<const float4 *>(x + rowq[c] * m)[i4];
        float *d = t.xb + c * t.ldx + 4 * i4;
        d[0] = v.x;
        d[1] = v.y;
        d[2] = v.z;
        d[3] = v.w;
      }
      __syncthreads();
      infer_batch<MT>(W, b1r, w2r, h, rows16 / 16, t);
      __syncthreads();
      if (threadIdx.x < nr) {
        const int c = threadIdx.x;
        float yh = b2;
        for (int wv = 0; wv < kTrainWaves; ++wv) yh += t.red[wv * kTrainB + c];
        if (plist) {
          const int64_t e = rent[c];
          dfo[e] = yh - offsets[static_cast<int64_t>(pair[rowq[c]]) * F + f];
        } else {
          out[(r0 + c) * F + f] = yh;
        }
      }
      __syncthreads();  // the next batch overwrites the rows, the batch and the sums
    }
  }
}

// Shapes the matrix-core training serves: inputs and hidden units multiples
// of 16, at most 256 each.
bool train_mfma_ok(int m, int h) { return m % 16 == 0 && h % 16 == 0 && m <= 256 && h <= 16 * kTrainHT * kTrainWaves; }

template <int MT>
void launch_train_mfma_mt(const TrainArgs &a, hipStream_t st) {
  const size_t lds = train_lds_floats(a.m) * 4 + static_cast<size_t>(a.n_train) * 4 + kTrainB * 8;
  auto kern = k_mlp_train_mfma<MT>;
  allow_lds(reinterpret_cast<const void *>(kern), lds);
  hipLaunchKernelGGL(kern, dim3(a.F), dim3(kTrainThreads), lds, st, a);
  LAUNCH_OK("mlp_train_mfma");
}

template <int MT>
void launch_sgd_mfma_mt(float *w, int F, int m, int h, const float *x, const float *y, int batch, float lr,
                        float *loss, hipStream_t st) {
  const size_t lds = train_lds_floats(m) * 4;
  auto kern = k_mlp_sgd_step_mfma<MT>;
  allow_lds(reinterpret_cast<const void *>(kern), lds);
  hipLaunchKernelGGL(kern, dim3(F), dim3(kTrainThreads), lds, st, w, m, h, x, y, batch, lr, loss);
  LAUNCH_OK("mlp_sgd_step_mfma");
}

template <int MT>
void infer_ws_mt(const float *w, int F, int m, int h, const float *x, int64_t nq, float *out, const int64_t *plist,
                 const int32_t *pcnt, int64_t stride, int N, const int32_t *pair, const float *offsets, float *dfo,
                 int rows_cap, hipStream_t st) {
  const size_t lds = train_lds_floats(m) * 4 + 2 * kTrainB * sizeof(int64_t) + 16;
  auto kern = k_mlp_infer_ws<MT>;
  allow_lds(reinterpret_cast<const void *>(kern), lds);
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  const int grid = F < cus ? F : cus;  // one resident work-group per CU (registers), each taking whole filters
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kTrainThreads), lds, st, w, F, m, h, x, nq, out, plist, pcnt, stride, N,
                     pair, offsets, dfo, rows_cap);
  LAUNCH_OK("mlp_infer_ws");
}

// The weights-in-registers inference for the shapes the matrix-core training
// serves and at least one filter per CU; false (nothing launched) otherwise.
bool infer_ws(const float *w, int F, int m, int h, const float *x, int64_t nq, float *out, const int64_t *plist,
              const int32_t *pcnt, int64_t stride, int N, const int32_t *pair, const float *offsets, float *dfo,
              int rows_cap, hipStream_t st) {
  if (!train_mfma_ok(m, h)) return false;
  // one work-group per filter: with fewer filters than CUs the query-tile
  // kernels, which spread a filter's rows over several work-groups, finish first
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  if (F < cus) return false;
  switch (m / 16) {
#define LEAFI_WS(k) \
  case k: infer_ws_mt<k>(w, F, m, h, x, nq, out, plist, pcnt, stride, N, pair, offsets, dfo, rows_cap, st); return true;
    LEAFI_WS(1) LEAFI_WS(2) LEAFI_WS(3) LEAFI_WS(4) LEAFI_WS(5) LEAFI_WS(6) LEAFI_WS(7) LEAFI_WS(8)
    LEAFI_WS(9) LEAFI_WS(10) LEAFI_WS(11) LEAFI_WS(12) LEAFI_WS(13) LEAFI_WS(14) LEAFI_WS(15) LEAFI_WS(16)
#undef LEAFI_WS
  }
  return false;
}

}  // namespace

void launch_mlp_infer(const float *w, int F, int m, int h, const float *x, int64_t nq, float *out, hipStream_t st) {
  if (nq <= 0 || F <= 0) return;
  if (infer_ws(w, F, m, h, x, nq, out, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr, kTrainB, st)) return;
  const int64_t tiles = ceil_div(nq, kMlpQ);
  dim3 grid(F, static_cast<unsigned>(tiles < 65535 ? tiles : 65535));
  const size_t lds = mlp_infer_lds(m);
  allow_lds(reinterpret_cast<const void *>(k_mlp_infer), lds);
  hipLaunchKernelGGL(k_mlp_infer, grid, dim3(256), lds, st, w, F, m, h, x, nq, out);
  LAUNCH_OK("mlp_infer");
}

void launch_mlp_infer_pairs(const float *w, int F, int m, int h, const float *x, const int64_t *plist,
                            const int32_t *pcnt, int64_t stride, int N, const int32_t *pair, const float *offsets,
                            int32_t *tile_prefix, float *dfo, hipStream_t st, int tile_mode) {
  if (F <= 0 || stride <= 0) return;
  // weights in registers: tile_mode 1 takes 32 rows per batch, else 64 (the values do not depend on it)
  if (infer_ws(w, F, m, h, x, 0, nullptr, plist, pcnt, stride, N, pair, offsets, dfo, tile_mode == 1 ? 32 : kTrainB,
               st))
    return;
  // up to kLocalPrefixMax filters the inference kernel computes the tile
  // prefix itself (one launch instead of two)
  constexpr int kLocalPrefixMax = 4096;
  const bool local = F <= kLocalPrefixMax;
  // tile_mode 0: large tiles for a large batch (decided on the device, with
  // the local prefix only); 1: always small; 2: always large
  const int big_fixed = tile_mode == 1 ? 0 : tile_mode == 2 ? 1 : (local ? -1 : 0);
  if (!local) {
    hipLaunchKernelGGL(k_mlp_tiles, dim3(1), dim3(1024), 0, st, F, pcnt, tile_prefix,
                       big_fixed == 1 ? kMlpQBig : kMlpQ);
    LAUNCH_OK("mlp_tiles");
  }
  // persistent grid: a few work-groups per CU, never more than the tiles can be
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  const int64_t tiles_bound = static_cast<int64_t>(F) * ceil_div(stride, kMlpQ);
  // (a multiple of 8 for the per-XCD tile ranges; spare work-groups exit)
  const int grid = static_cast<int>(
      ceil_div(std::min<int64_t>(tiles_bound, static_cast<int64_t>(cus) * 4), kMlpXcds) * kMlpXcds);
  // with the prefix computed locally, a batch of at least one small tile per
  // CU runs on the large tiles
  const int big_min = local && big_fixed < 0 ? cus : 0;
  const int lds_q = big_fixed == 0 ? kMlpQ : kMlpQBig;
  const size_t lds = mlp_infer_lds(m, lds_q) + (local ? (static_cast<size_t>(F) + 1 + 4) * sizeof(int32_t) : 0);
  allow_lds(reinterpret_cast<const void *>(k_mlp_infer_pairs), lds);
  hipLaunchKernelGGL(k_mlp_infer_pairs, dim3(grid), dim3(256), lds, st, w, F, m, h, x, plist, pcnt, stride, N, pair,
                     offsets, tile_prefix, dfo, local ? 1 : 0, big_min, big_fixed, lds_q);
  LAUNCH_OK("mlp_infer_pairs");
}

static size_t step_lds(int m) { return static_cast<size_t>(m) * kTB * 4 + (4 + 3) * kTB * 4; }

void launch_mlp_sgd_step(float *w, int F, int m, int h, const float *x, const float *y, int batch, float lr,
                         float *loss, hipStream_t st) {
  if (train_mfma_ok(m, h)) {
    switch (m / 16) {
      case 1: launch_sgd_mfma_mt<1>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 2: launch_sgd_mfma_mt<2>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 3: launch_sgd_mfma_mt<3>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 4: launch_sgd_mfma_mt<4>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 5: launch_sgd_mfma_mt<5>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 6: launch_sgd_mfma_mt<6>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 7: launch_sgd_mfma_mt<7>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 8: launch_sgd_mfma_mt<8>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 9: launch_sgd_mfma_mt<9>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 10: launch_sgd_mfma_mt<10>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 11: launch_sgd_mfma_mt<11>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 12: launch_sgd_mfma_mt<12>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 13: launch_sgd_mfma_mt<13>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 14: launch_sgd_mfma_mt<14>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 15: launch_sgd_mfma_mt<15>(w, F, m, h, x, y, batch, lr, loss, st); return;
      case 16: launch_sgd_mfma_mt<16>(w, F, m, h, x, y, batch, lr, loss, st); return;
    }
  }
  size_t lds = step_lds(m);
  allow_lds(reinterpret_cast<const void *>(k_mlp_sgd_step), lds);
  hipLaunchKernelGGL(k_mlp_sgd_step, dim3(F), dim3(256), lds, st, w, F, m, h, x, y, batch, lr, loss);
  LAUNCH_OK("mlp_sgd_step");
}

void launch_mlp_train(const TrainArgs &a, hipStream_t st) {
  if (train_mfma_ok(a.m, a.h)) {
    switch (a.m / 16) {
      case 1: launch_train_mfma_mt<1>(a, st); return;
      case 2: launch_train_mfma_mt<2>(a, st); return;
      case 3: launch_train_mfma_mt<3>(a, st); return;
      case 4: launch_train_mfma_mt<4>(a, st); return;
      case 5: launch_train_mfma_mt<5>(a, st); return;
      case 6: launch_train_mfma_mt<6>(a, st); return;
      case 7: launch_train_mfma_mt<7>(a, st); return;
      case 8: launch_train_mfma_mt<8>(a, st); return;
      case 9: launch_train_mfma_mt<9>(a, st); return;
      case 10: launch_train_mfma_mt<10>(a, st); return;
      case 11: launch_train_mfma_mt<11>(a, st); return;
      case 12: launch_train_mfma_mt<12>(a, st); return;
      case 13: launch_train_mfma_mt<13>(a, st); return;
      case 14: launch_train_mfma_mt<14>(a, st); return;
      case 15: launch_train_mfma_mt<15>(a, st); return;
      case 16: launch_train_mfma_mt<16>(a, st); return;
    }
  }
  size_t lds = step_lds(a.m) + static_cast<size_t>(a.n_train) * 4 + kTB * 8;
  allow_lds(reinterpret_cast<const void *>(k_mlp_train), lds);
  hipLaunchKernelGGL(k_mlp_train, dim3(a.F), dim3(256), lds, st, a);
  LAUNCH_OK("mlp_train");
}

}  // namespace leafi
