// Device-side helpers for the gfx950 kernels (64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace leafi {

constexpr int kWave = 64;
constexpr uint64_t kKeyMax = ~0ull;

__device__ __forceinline__ uint32_t f2u(float f) { return __float_as_uint(f); }
__device__ __forceinline__ float u2f(uint32_t u) { return __uint_as_float(u); }

// fp32 -> bf16 bits, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = f2u(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return u2f(static_cast<uint32_t>(b) << 16); }

// Sort key of a non-negative squared distance and a row: orders by
// (distance, row) as an unsigned integer.
__device__ __forceinline__ uint64_t make_key(float d2, uint32_t row) {
  return (static_cast<uint64_t>(f2u(d2)) << 32) | row;
}
__device__ __forceinline__ float key_d2(uint64_t k) { return u2f(static_cast<uint32_t>(k >> 32)); }
__device__ __forceinline__ uint32_t key_row(uint64_t k) { return static_cast<uint32_t>(k); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, kWave);
    v = w > v ? w : v;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, kWave);
    v = w < v ? w : v;
  }
  return v;
}

// DPP move of a 64-bit value (two 32-bit halves); lanes whose source is out
// of their row or whose row is masked off keep their own value.
template <int Ctrl, int RowMask>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(v), static_cast<int>(v), Ctrl, RowMask, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(v >> 32), static_cast<int>(v >> 32), Ctrl, RowMask, 0xf,
                                             false);
  return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

// Minimum of a 64-bit key over the wavefront, returned to every lane, on
// DPP lane moves (no LDS round trips, unlike shuffles): row_shr 1, 2, 4, 8
// leave each 16-lane row's minimum in its lane 15, row_bcast 15 and 31 carry
// it across the rows to lane 63, which is read back.
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  uint64_t t;
  t = dpp_u64<0x111, 0xf>(v);  // row_shr:1
  v = t < v ? t : v;
  t = dpp_u64<0x112, 0xf>(v);  // row_shr:2
  v = t < v ? t : v;
  t = dpp_u64<0x114, 0xf>(v);  // row_shr:4
  v = t < v ? t : v;
  t = dpp_u64<0x118, 0xf>(v);  // row_shr:8
  v = t < v ? t : v;
  t = dpp_u64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = t < v ? t : v;
  t = dpp_u64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  v = t < v ? t : v;
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(v), 63);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(v >> 32), 63);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Minimum of a 32-bit key over the wavefront, returned to every lane (the
// same DPP steps as wave_min_u64 on one half).
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  uint32_t t;
#define LEAFI_DPP32(ctrl, rmask) \
  static_cast<uint32_t>(__builtin_amdgcn_update_dpp(static_cast<int>(v), static_cast<int>(v), ctrl, rmask, 0xf, false))
  t = LEAFI_DPP32(0x111, 0xf);  // row_shr:1
  v = t < v ? t : v;
  t = LEAFI_DPP32(0x112, 0xf);  // row_shr:2
  v = t < v ? t : v;
  t = LEAFI_DPP32(0x114, 0xf);  // row_shr:4
  v = t < v ? t : v;
  t = LEAFI_DPP32(0x118, 0xf);  // row_shr:8
  v = t < v ? t : v;
  t = LEAFI_DPP32(0x142, 0xa);  // row_bcast:15 into rows 1 and 3
  v = t < v ? t : v;
  t = LEAFI_DPP32(0x143, 0xc);  // row_bcast:31 into rows 2 and 3
  v = t < v ? t : v;
#undef LEAFI_DPP32
  return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 63));
}
__device__ __forceinline__ uint64_t wave_min_key(uint64_t v) { return wave_min_u64(v); }
__device__ __forceinline__ uint32_t wave_min_key(uint32_t v) { return wave_min_u32(v); }

// Exclusive prefix sum over a work-group of NT threads (NT / 64 <= 64
// wavefronts): wavefront scans by shuffles, then one scan of the wavefront
// totals.  `sh` holds NT / 64 values of LDS; `total` receives the sum.  Every
// thread of the work-group must call it.
template <int NT, typename T>
__device__ inline T block_scan_excl(T v, T *sh, T &total) {
  static_assert(NT % 64 == 0 && NT / 64 <= 64, "work-group size");
  constexpr int kW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();  // sh may still be read by a previous call
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  if (wave == 0) {
    T t = lane < kW ? sh[lane] : T(0);
#pragma unroll
    for (int o = 1; o < kW; o <<= 1) {
      const T y = __shfl_up(t, o, 64);
      if (lane >= o) t += y;
    }
    if (lane < kW) sh[lane] = t;
  }
  __syncthreads();
  total = sh[kW - 1];
  return (wave > 0 ? sh[wave - 1] : T(0)) + x - v;
}

// Leaf store bf16 layout: 16-row panels (row r of the store is row r % 16 of
// panel r / 16, whose 16 x m block starts at element 16 m (r / 16)).  Within a
// panel, column t of row rr sits in the 32-column block t / 32 (16 x 32
// elements, 1 KiB), at ((t % 32) / 8 * 16 + rr) * 8 + t % 8: exactly the
// order in which a wavefront's 64 lanes take the 16-row x 32-column A operand
// of one v_mfma_f32_16x16x32_bf16 (lane = 16 g + rr, eight elements each), so
// one load instruction reads 1 KiB of consecutive memory.
__host__ __device__ __forceinline__ int panel_index(int rr, int t) {
  return (t >> 5) * 512 + (((t & 31) >> 3) * 16 + rr) * 8 + (t & 7);
}

// Summary lower bound of one (query, leaf): per segment s of length l_s,
// l_s [gap(mu_q, [mu_lo, mu_hi])^2 + gap(sd_q, [sd_lo, sd_hi])^2], summed in
// segment order; qs = (mu, sd) per segment, bx = (mu lo, mu hi, sd lo, sd hi).
__device__ __forceinline__ float summary_lb(const float *qs, const float *bx, int S, int m) {
  float acc = 0.0f;
  for (int s = 0; s < S; ++s) {
    float len = static_cast<float>(((s + 1) * m) / S - (s * m) / S);
    float mq = qs[2 * s], sq = qs[2 * s + 1];
    float gm = fmaxf(fmaxf(bx[4 * s] - mq, mq - bx[4 * s + 1]), 0.0f);
    float gs = fmaxf(fmaxf(bx[4 * s + 2] - sq, sq - bx[4 * s + 3]), 0.0f);
    acc += len * (gm * gm + gs * gs);
  }
  return sqrtf(acc);
}

// Calibrated (k, target) row of a query: -1 (filters off) for a target >= 1
// or a pair that was not calibrated.  k is clamped to [1, kmax].
__device__ __forceinline__ int select_pair_of(int k, float t, int n_pairs, const int32_t *pair_k, const float *pair_t) {
  int p = -1;
  if (t < 1.0f)
    for (int i = 0; i < n_pairs; ++i)
      if (pair_k[i] == k && pair_t[i] == t) {
        p = i;
        break;
      }
  return p;
}

// Orders LDS traffic of one wavefront between stages of a cooperative
// algorithm (lanes read what other lanes wrote in the previous stage).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ __forceinline__ int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Bitonic sort of P (power of two) 32- or 64-bit keys in LDS by one
// wavefront, ascending.
template <typename K>
__device__ inline void wave_sort_keys(K *a, int P, int lane) {
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = lane; i < (P >> 1); i += kWave) {
        int lo = 2 * i - (i & (stride - 1));
        int hi = lo + stride;
        bool up = (lo & size) == 0;
        const K x = a[lo], y = a[hi];
        if ((x > y) == up) {
          a[lo] = y;
          a[hi] = x;
        }
      }
      wave_lds_sync();
    }
  }
}
__device__ inline void wave_sort_u64(uint64_t *a, int P, int lane) { wave_sort_keys(a, P, lane); }

// Sort of the first n keys of a (any n >= 0), ascending, by one wavefront,
// touching no entry at or past n.  Bitonic network in the form whose every
// comparator puts the smaller key at the lower index (each merge starts by
// comparing i with its mirror in the block, then halves): entries past n act
// as +infinity and such a comparator never moves them, so they are neither
// read nor written.
template <typename K>
__device__ inline void wave_sort_keys_n(K *a, int n, int lane) {
  const int P = pow2_at_least(n < 2 ? 2 : n);
  for (int size = 2; size <= P; size <<= 1) {
    const int half = size >> 1;
    for (int p = lane; p < (P >> 1); p += kWave) {
      const int blk = p / half, off = p - blk * half;
      const int lo = blk * size + off, hi = blk * size + size - 1 - off;
      if (hi < n) {
        const K x = a[lo], y = a[hi];
        if (x > y) {
          a[lo] = y;
          a[hi] = x;
        }
      }
    }
    wave_lds_sync();
    for (int stride = size >> 2; stride > 0; stride >>= 1) {
      for (int p = lane; p < (P >> 1); p += kWave) {
        const int lo = 2 * p - (p & (stride - 1)), hi = lo + stride;
        if (hi < n) {
          const K x = a[lo], y = a[hi];
          if (x > y) {
            a[lo] = y;
            a[hi] = x;
          }
        }
      }
      wave_lds_sync();
    }
  }
}

// Bitonic sort of P (power of two) (double, uint32) pairs, ascending by
// (value, tag), by one wavefront.
__device__ inline void wave_sort_dbl_tag(double *v, uint32_t *t, int P, int lane) {
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = lane; i < (P >> 1); i += kWave) {
        int lo = 2 * i - (i & (stride - 1));
        int hi = lo + stride;
        bool up = (lo & size) == 0;
        double x = v[lo], y = v[hi];
        uint32_t tx = t[lo], ty = t[hi];
        bool gt = (x > y) || (x == y && tx > ty);
        if (gt == up) {
          v[lo] = y;
          v[hi] = x;
          t[lo] = ty;
          t[hi] = tx;
        }
      }
      wave_lds_sync();
    }
  }
}

// Counter-based generator: SplitMix64 finaliser of a mixed counter.
__device__ __host__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
__device__ __host__ __forceinline__ double u01(uint64_t z) {  // (0, 1)
  return (static_cast<double>(z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

}  // namespace leafi
