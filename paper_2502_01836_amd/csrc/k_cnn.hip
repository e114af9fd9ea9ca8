// CNN learned filters: two zero-padded cross-correlations of kernel 3 over
// the series positions (1 -> C channels, C -> C channels), ReLU after each,
// the second layer's channels averaged over the positions and read out
// linearly (paper: Section "Varying Model Type"; the padding, activations and
// readout are this library's reading of the two-layer CNN it names).
//
// Packed weights per filter (P = 3C^2 + 6C + 1 floats):
//   [W1 (C, 3) | b1 (C) | W2 (C_out, C_in, 3) | b2 (C) | w3 (C) | b3]
// Tap t of a layer reads position p + t - 1 of its input (zero outside).
//
// Inference: one work-group per filter at a time (persistent over filters),
// the filter's weights staged in LDS once (W2 transposed to [c][t][o] so
// four output channels are one 16-byte read) and its queries (all of them,
// or the (query, leaf) pairs listed for it) passed through one by one: the
// first layer into LDS, then the second as 4 x 4 blocks of (channel,
// position) outputs per thread in FP32 FMAs, ReLU and per-block position
// sums, reduced in a fixed order.  The conv2 weights must fit in LDS, which
// bounds the channel count (96 channels of length 96 fit).
//
// Training: one work-group per filter, mini-batch SGD on the mean squared
// error with the MLP filters' schedule (shuffled epochs, validation after
// each, learning rate divided by 10 after `patience` epochs without a
// relative improvement of 1e-4, stop below lr_min, best weights kept).  The
// weights stay in global memory; per example the activations live in LDS
// and the gradient is accumulated in a per-filter buffer each thread owns
// entries of.
#include "device_util.h"
#include "kernels.h"

namespace leafi {

namespace {

constexpr int kCnnThreads = 256;

__host__ __device__ inline int64_t cnn_params(int C) { return 3LL * C * C + 6LL * C + 1; }

// Offsets inside a packed filter.
struct CnnOff {
  int64_t W1, b1, W2, b2, w3, b3;
  __host__ __device__ explicit CnnOff(int C)
      : W1(0), b1(3LL * C), W2(4LL * C), b2(4LL * C + 3LL * C * C), w3(5LL * C + 3LL * C * C),
        b3(6LL * C + 3LL * C * C) {}
};

// Row stride of the padded first-layer activations (16-byte aligned rows;
// element 0 and elements m + 1 .. m + 3 are zero).
__host__ __device__ inline int cnn_row(int m) { return m + 4; }

// LDS floats of the inference kernel: W2T, W1 | b1 | b2 | w3 | b3 (rounded
// up to 4), the padded query, the padded first layer, per-block sums.
__host__ __device__ inline int64_t cnn_infer_lds_floats(int m, int C) {
  return 3LL * C * C + ((6LL * C + 1 + 3) / 4) * 4 + cnn_row(m) + static_cast<int64_t>(C) * cnn_row(m) +
         static_cast<int64_t>(m / 4) * C + 4;
}

struct CnnLds {
  float *W2T;  // [C][3][C]: (c, t, o)
  float *w1;   // [C][3]
  float *b1, *b2, *w3, *b3;
  float *xp;   // [m + 4]
  float *h1p;  // [C][m + 4]
  float *red;  // [m / 4][C]
  float *bcast;  // [4]: the prediction, for every thread
};

__device__ inline CnnLds cnn_carve(float *lds, int m, int C) {
  CnnLds s;
  s.W2T = lds;
  s.w1 = s.W2T + 3 * C * C;
  s.b1 = s.w1 + 3 * C;
  s.b2 = s.b1 + C;
  s.w3 = s.b2 + C;
  s.b3 = s.w3 + C;
  s.xp = s.w1 + ((6 * C + 1 + 3) / 4) * 4;
  s.h1p = s.xp + cnn_row(m);
  s.red = s.h1p + C * cnn_row(m);
  s.bcast = s.red + (m / 4) * C;
  return s;
}

// Stage filter wf's weights (and the zero borders) in LDS.
__device__ inline void cnn_stage(const float *__restrict__ wf, int m, int C, const CnnLds &s) {
  const CnnOff o(C);
  for (int e = threadIdx.x; e < 3 * C * C; e += blockDim.x) {
    // e walks the packed W2 (o, c, t); its LDS place is (c, t, o)
    const int oc = e / (3 * C), rest = e - oc * 3 * C;
    const int c = rest / 3, t = rest - c * 3;
    s.W2T[(c * 3 + t) * C + oc] = wf[o.W2 + e];
  }
  for (int e = threadIdx.x; e < 3 * C; e += blockDim.x) s.w1[e] = wf[o.W1 + e];
  for (int e = threadIdx.x; e < C; e += blockDim.x) {
    s.b1[e] = wf[o.b1 + e];
    s.b2[e] = wf[o.b2 + e];
    s.w3[e] = wf[o.w3 + e];
  }
  if (threadIdx.x == 0) s.b3[0] = wf[o.b3];
  const int R = cnn_row(m);
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    s.h1p[c * R] = 0.0f;
    for (int p = m + 1; p < R; ++p) s.h1p[c * R + p] = 0.0f;
  }
  if (threadIdx.x == 0) {
    s.xp[0] = 0.0f;
    for (int p = m + 1; p < R; ++p) s.xp[p] = 0.0f;
  }
}

// d^f of query row xq (global, m floats) with the staged filter.  Every
// thread of the work-group calls it; the result is returned to all.
__device__ inline float cnn_eval(const float *__restrict__ xq, int m, int C, const CnnLds &s) {
  const int R = cnn_row(m);
  for (int p = threadIdx.x; p < m; p += blockDim.x) s.xp[p + 1] = xq[p];
  __syncthreads();
  // first layer: h1[c][p] = ReLU(b1 + w1[c][0] x[p-1] + w1[c][1] x[p] + w1[c][2] x[p+1])
  for (int e = threadIdx.x; e < C * m; e += blockDim.x) {
    const int c = e / m, p = e - c * m;
    float z = s.b1[c];
    z = fmaf(s.w1[3 * c + 0], s.xp[p], z);
    z = fmaf(s.w1[3 * c + 1], s.xp[p + 1], z);
    z = fmaf(s.w1[3 * c + 2], s.xp[p + 2], z);
    s.h1p[c * R + p + 1] = fmaxf(z, 0.0f);
  }
  __syncthreads();
  // second layer in 4 (channels) x 4 (positions) blocks; each block's
  // ReLU outputs summed over its positions into red[pb][o]
  const int PBn = m / 4, tiles = (C / 4) * PBn;
  for (int tile = threadIdx.x; tile < tiles; tile += blockDim.x) {
    const int ob = tile / PBn, pb = tile - ob * PBn;
    const int o0 = 4 * ob, p0 = 4 * pb;
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
    for (int c = 0; c < C; ++c) {
      const float *hr = s.h1p + c * R + p0;
      const float4 ha = *reinterpret_cast<const float4 *>(hr);
      const float2 hb = *reinterpret_cast<const float2 *>(hr + 4);
      const float hv[6] = {ha.x, ha.y, ha.z, ha.w, hb.x, hb.y};
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const float4 wv4 = *reinterpret_cast<const float4 *>(s.W2T + (c * 3 + t) * C + o0);
        const float wv[4] = {wv4.x, wv4.y, wv4.z, wv4.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(wv[i], hv[j + t], acc[i][j]);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float b = s.b2[o0 + i];
      float r = 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) r += fmaxf(acc[i][j] + b, 0.0f);
      s.red[pb * C + o0 + i] = r;
    }
  }
  __syncthreads();
  // readout by wavefront 0: channel o (lanes o, o + 64) sums its blocks in
  // order, weighted by w3[o] / m; a fixed butterfly adds the lanes
  if (threadIdx.x < kWave) {
    float v = 0.0f;
    for (int o = threadIdx.x; o < C; o += kWave) {
      float sum = 0.0f;
      for (int pb = 0; pb < PBn; ++pb) sum += s.red[pb * C + o];
      v = fmaf(s.w3[o], sum / static_cast<float>(m), v);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if (threadIdx.x == 0) s.bcast[0] = v + s.b3[0];
  }
  __syncthreads();
  return s.bcast[0];
}

// mode 0: dense, out[q * F + f] = d^f for every query; mode 1: listed pairs,
// dfo[e] = d^f - offsets[pair[q] * F + f] for e = plist[f * stride + i].
__global__ void __launch_bounds__(kCnnThreads) k_cnn_infer(const float *__restrict__ w, int F, int m, int C,
                                                           const float *__restrict__ x, int64_t nq, float *out,
                                                           int mode, const int64_t *__restrict__ plist,
                                                           const int32_t *__restrict__ pcnt, int64_t stride, int N,
                                                           const int32_t *__restrict__ pair,
                                                           const float *__restrict__ offsets, float *dfo) {
  extern __shared__ __align__(16) float lds[];
  const CnnLds s = cnn_carve(lds, m, C);
  const int64_t P = cnn_params(C);
  for (int f = blockIdx.x; f < F; f += gridDim.x) {
    const int64_t n = mode == 0 ? nq : pcnt[f];
    if (n == 0) continue;  // uniform
    __syncthreads();       // the previous filter's LDS is no longer read
    cnn_stage(w + f * P, m, C, s);
    for (int64_t i = 0; i < n; ++i) {
      int64_t q = i, e = 0;
      if (mode == 1) {
        e = plist[f * stride + i];
        q = e / N;
      }
      const float v = cnn_eval(x + q * m, m, C, s);
      if (threadIdx.x == 0) {
        if (mode == 0) out[q * F + f] = v;
        else dfo[e] = v - offsets[static_cast<int64_t>(pair[q]) * F + f];
      }
    }
  }
}

// ---- training ---------------------------------------------------------------

// LDS floats of the training kernel: padded query, padded first layer, the
// second layer's pre-activations then their gradient [C][m], the first
// layer's gradient [C][m], pooled [C], then the shuffle and batch tables.
__host__ __device__ inline int64_t cnn_train_lds_floats(int m, int C) {
  return cnn_row(m) + static_cast<int64_t>(C) * cnn_row(m) + 2LL * C * m + C + 4;
}

struct TrainLds {
  float *xp, *h1p, *z2, *d1, *pooled, *scal;
};

__device__ inline TrainLds train_carve(float *lds, int m, int C) {
  TrainLds s;
  s.xp = lds;
  s.h1p = s.xp + cnn_row(m);
  s.z2 = s.h1p + C * cnn_row(m);
  s.d1 = s.z2 + C * m;
  s.pooled = s.d1 + C * m;
  s.scal = s.pooled + C;
  return s;
}

// Forward pass of example row xq through filter wf (global): leaves the
// padded query, the first layer, the second layer's pre-activations and the
// pooled activations in LDS; returns the prediction to all threads.
__device__ inline float cnn_forward_train(const float *__restrict__ wf, const float *__restrict__ xq, int m, int C,
                                          const TrainLds &s) {
  const CnnOff o(C);
  const int R = cnn_row(m);
  for (int p = threadIdx.x; p < R; p += blockDim.x) s.xp[p] = (p >= 1 && p <= m) ? xq[p - 1] : 0.0f;
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    s.h1p[c * R] = 0.0f;
    for (int p = m + 1; p < R; ++p) s.h1p[c * R + p] = 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < C * m; e += blockDim.x) {
    const int c = e / m, p = e - c * m;
    float z = wf[o.b1 + c];
    z = fmaf(wf[o.W1 + 3 * c + 0], s.xp[p], z);
    z = fmaf(wf[o.W1 + 3 * c + 1], s.xp[p + 1], z);
    z = fmaf(wf[o.W1 + 3 * c + 2], s.xp[p + 2], z);
    s.h1p[c * R + p + 1] = fmaxf(z, 0.0f);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < C * m; e += blockDim.x) {
    const int oc = e / m, p = e - oc * m;
    const float *w2 = wf + o.W2 + static_cast<int64_t>(oc) * 3 * C;
    float z = 0.0f;
    for (int c = 0; c < C; ++c) {
      const float *hr = s.h1p + c * R + p;
      z = fmaf(w2[3 * c + 0], hr[0], z);
      z = fmaf(w2[3 * c + 1], hr[1], z);
      z = fmaf(w2[3 * c + 2], hr[2], z);
    }
    s.z2[e] = z + wf[o.b2 + oc];
  }
  __syncthreads();
  for (int oc = threadIdx.x; oc < C; oc += blockDim.x) {
    float sum = 0.0f;
    for (int p = 0; p < m; ++p) sum += fmaxf(s.z2[oc * m + p], 0.0f);
    s.pooled[oc] = sum / static_cast<float>(m);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float v = wf[o.b3];
    for (int oc = 0; oc < C; ++oc) v = fmaf(wf[o.w3 + oc], s.pooled[oc], v);
    s.scal[0] = v;
  }
  __syncthreads();
  return s.scal[0];
}

// Add g * dL/dw of the last forward pass (g = dL/dprediction) to grad.
__device__ inline void cnn_backward(const float *__restrict__ wf, int m, int C, float g, const TrainLds &s,
                                    float *grad) {
  const CnnOff o(C);
  const int R = cnn_row(m);
  // readout
  for (int oc = threadIdx.x; oc < C; oc += blockDim.x) grad[o.w3 + oc] += g * s.pooled[oc];
  if (threadIdx.x == 0) grad[o.b3] += g;
  // dL/dz2 = g w3[o] / m where z2 > 0 (in place of z2)
  __syncthreads();
  for (int e = threadIdx.x; e < C * m; e += blockDim.x) {
    const int oc = e / m;
    s.z2[e] = s.z2[e] > 0.0f ? g * wf[o.w3 + oc] / static_cast<float>(m) : 0.0f;
  }
  __syncthreads();
  const float *d2 = s.z2;
  for (int oc = threadIdx.x; oc < C; oc += blockDim.x) {
    float sum = 0.0f;
    for (int p = 0; p < m; ++p) sum += d2[oc * m + p];
    grad[o.b2 + oc] += sum;
  }
  // dW2[o][c][t] = sum_p d2[o][p] h1p[c][p + t]
  for (int e = threadIdx.x; e < 3 * C * C; e += blockDim.x) {
    const int oc = e / (3 * C), rest = e - oc * 3 * C;
    const int c = rest / 3, t = rest - c * 3;
    float sum = 0.0f;
    for (int p = 0; p < m; ++p) sum = fmaf(d2[oc * m + p], s.h1p[c * R + p + t], sum);
    grad[o.W2 + e] += sum;
  }
  // dL/dz1[c][q] = [h1 > 0] sum_o sum_t W2[o][c][t] d2[o][q - t + 1]
  for (int e = threadIdx.x; e < C * m; e += blockDim.x) {
    const int c = e / m, q = e - c * m;
    float sum = 0.0f;
    if (s.h1p[c * R + q + 1] > 0.0f) {
      for (int oc = 0; oc < C; ++oc) {
        const float *w2 = wf + o.W2 + (static_cast<int64_t>(oc) * C + c) * 3;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const int p = q - t + 1;
          if (p >= 0 && p < m) sum = fmaf(w2[t], d2[oc * m + p], sum);
        }
      }
    }
    s.d1[e] = sum;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 3 * C; e += blockDim.x) {
    const int c = e / 3, t = e - c * 3;
    float sum = 0.0f;
    for (int p = 0; p < m; ++p) sum = fmaf(s.d1[c * m + p], s.xp[p + t], sum);
    grad[o.W1 + e] += sum;
  }
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    float sum = 0.0f;
    for (int p = 0; p < m; ++p) sum += s.d1[c * m + p];
    grad[o.b1 + c] += sum;
  }
  __syncthreads();
}

// One SGD step per filter on an explicit batch: x [F, batch, m], y [F, batch];
// loss[f] = the batch's mean squared error before the step.
__global__ void __launch_bounds__(kCnnThreads) k_cnn_sgd_step(float *w, int m, int C, const float *x, const float *y,
                                                              int batch, float lr, float *loss, float *gbuf) {
  extern __shared__ __align__(16) float lds[];
  const TrainLds s = train_carve(lds, m, C);
  const int f = blockIdx.x;
  const int64_t P = cnn_params(C);
  float *wf = w + f * P;
  float *grad = gbuf + f * P;
  for (int64_t e = threadIdx.x; e < P; e += blockDim.x) grad[e] = 0.0f;
  __syncthreads();  // other threads own the entries they accumulate into
  float se = 0.0f;
  for (int b = 0; b < batch; ++b) {
    const int64_t row = static_cast<int64_t>(f) * batch + b;
    const float yh = cnn_forward_train(wf, x + row * m, m, C, s);
    const float r = yh - y[row];
    se += r * r;
    cnn_backward(wf, m, C, 2.0f * r / static_cast<float>(batch), s, grad);
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < P; e += blockDim.x) wf[e] -= lr * grad[e];
  if (threadIdx.x == 0) loss[f] = se / static_cast<float>(batch);
}

__global__ void __launch_bounds__(kCnnThreads) k_cnn_train(TrainArgs a, float *gbuf) {
  extern __shared__ __align__(16) float lds[];
  const int m = a.m, C = a.h;
  const TrainLds s = train_carve(lds, m, C);
  int32_t *perm = reinterpret_cast<int32_t *>(s.scal + 4);
  float *vsum = s.scal + 1;  // validation error sum
  float *stop = s.scal + 2;  // nonzero: training ends
  const int f = blockIdx.x;
  const int64_t P = cnn_params(C);
  const CnnOff off(C);
  float *wf = a.w + f * P;
  float *wb = a.w_best + f * P;
  float *grad = gbuf + f * P;
  const int32_t *exq = a.ex_q + static_cast<int64_t>(f) * a.n_ex;
  const float *exy = a.ex_y + static_cast<int64_t>(f) * a.n_ex;
  const int n_val = a.n_ex - a.n_train;
  // output bias starts at the mean training target
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int e = 0; e < a.n_train; ++e) acc += exy[e];
    wf[off.b3] = static_cast<float>(acc / (a.n_train > 0 ? a.n_train : 1));
  }
  for (int e = threadIdx.x; e < a.n_train; e += blockDim.x) perm[e] = e;
  __syncthreads();
  for (int64_t e = threadIdx.x; e < P; e += blockDim.x) wb[e] = wf[e];
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
      for (int64_t e = threadIdx.x; e < P; e += blockDim.x) grad[e] = 0.0f;
      __syncthreads();  // other threads own the entries they accumulate into
      for (int b = 0; b < nb; ++b) {
        const int ex = perm[s0 + b];
        const float yh = cnn_forward_train(wf, a.xq + static_cast<int64_t>(exq[ex]) * m, m, C, s);
        cnn_backward(wf, m, C, 2.0f * (yh - exy[ex]) / static_cast<float>(nb), s, grad);
      }
      __syncthreads();
      for (int64_t e = threadIdx.x; e < P; e += blockDim.x) wf[e] -= lr * grad[e];
      __syncthreads();
    }
    // validation error
    if (threadIdx.x == 0) *vsum = 0.0f;
    __syncthreads();
    for (int v = 0; v < n_val; ++v) {
      const int ex = a.n_train + v;
      const float yh = cnn_forward_train(wf, a.xq + static_cast<int64_t>(exq[ex]) * m, m, C, s);
      if (threadIdx.x == 0) {
        const float r = yh - exy[ex];
        *vsum += r * r;
      }
    }
    __syncthreads();
    const float vm = n_val > 0 ? *vsum / n_val : 0.0f;
    if (a.val_trace && threadIdx.x == 0) a.val_trace[static_cast<int64_t>(f) * a.max_epochs + epoch] = vm;
    const bool improved = vm < best * (1.0f - 1e-4f);
    if (improved) {
      best = vm;
      bad = 0;
      for (int64_t e = threadIdx.x; e < P; e += blockDim.x) wb[e] = wf[e];
    } else if (++bad >= a.patience) {
      lr *= 0.1f;
      bad = 0;
    }
    if (threadIdx.x == 0) *stop = (lr < a.lr_min * (1.0f - 1e-3f)) || !(vm == vm) ? 1.0f : 0.0f;
    __syncthreads();
    if (*stop != 0.0f) {
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

void check_cnn_shape(int m, int C) {
  if (m < 4 || m % 4 != 0 || C < 4 || C % 4 != 0)
    fail(LEAFI_EINVAL, "CNN filters need the series length and the channel count to be multiples of 4");
  if (cnn_infer_lds_floats(m, C) * 4 > 160 * 1024)
    fail(LEAFI_EINVAL, "CNN filter too large: its second-layer weights and activations must fit in 160 KiB of LDS "
                       "(e.g. 96 channels for length 96)");
}

}  // namespace

int64_t cnn_param_count(int C) { return cnn_params(C); }

void cnn_check(int m, int C) { check_cnn_shape(m, C); }

void launch_cnn_infer(const float *w, int F, int m, int C, const float *x, int64_t nq, float *out, hipStream_t st) {
  check_cnn_shape(m, C);
  if (F <= 0 || nq <= 0) return;
  const size_t lds = static_cast<size_t>(cnn_infer_lds_floats(m, C)) * sizeof(float);
  allow_lds(reinterpret_cast<const void *>(k_cnn_infer), lds);
  hipLaunchKernelGGL(k_cnn_infer, dim3(F), dim3(kCnnThreads), lds, st, w, F, m, C, x, nq, out, 0, nullptr, nullptr,
                     int64_t(0), 0, nullptr, nullptr, nullptr);
  LAUNCH_OK("cnn_infer");
}

void launch_cnn_infer_pairs(const float *w, int F, int m, int C, const float *x, const int64_t *plist,
                            const int32_t *pcnt, int64_t stride, int N, const int32_t *pair, const float *offsets,
                            float *dfo, hipStream_t st) {
  check_cnn_shape(m, C);
  if (F <= 0 || stride <= 0) return;
  const size_t lds = static_cast<size_t>(cnn_infer_lds_floats(m, C)) * sizeof(float);
  allow_lds(reinterpret_cast<const void *>(k_cnn_infer), lds);
  hipLaunchKernelGGL(k_cnn_infer, dim3(F), dim3(kCnnThreads), lds, st, w, F, m, C, x, int64_t(0), nullptr, 1, plist,
                     pcnt, stride, N, pair, offsets, dfo);
  LAUNCH_OK("cnn_infer_pairs");
}

void launch_cnn_train(const TrainArgs &a, float *gbuf, hipStream_t st) {
  check_cnn_shape(a.m, a.h);
  if (a.F <= 0) return;
  const size_t lds = static_cast<size_t>(cnn_train_lds_floats(a.m, a.h)) * sizeof(float) +
                     static_cast<size_t>(a.n_train) * sizeof(int32_t);
  if (lds > 160 * 1024) fail(LEAFI_EINVAL, "CNN training: activations and shuffle table exceed the LDS");
  allow_lds(reinterpret_cast<const void *>(k_cnn_train), lds);
  hipLaunchKernelGGL(k_cnn_train, dim3(a.F), dim3(kCnnThreads), lds, st, a, gbuf);
  LAUNCH_OK("cnn_train");
}

void launch_cnn_sgd_step(float *w, int F, int m, int C, const float *x, const float *y, int batch, float lr,
                         float *loss, float *gbuf, hipStream_t st) {
  check_cnn_shape(m, C);
  if (F <= 0) return;
  const size_t lds = static_cast<size_t>(cnn_train_lds_floats(m, C)) * sizeof(float);
  allow_lds(reinterpret_cast<const void *>(k_cnn_sgd_step), lds);
  hipLaunchKernelGGL(k_cnn_sgd_step, dim3(F), dim3(kCnnThreads), lds, st, w, m, C, x, y, batch, lr, loss, gbuf);
  LAUNCH_OK("cnn_sgd_step");
}

}  // namespace leafi
