// Error bounds shared by the BF16 leaf scan and the kernels that read its
// candidate lists (query bound, rerank).
#pragma once

#include "device_util.h"

namespace leafi {

// 32-bit scan keys (BF16 form): row index within the tile in the low
// kLocalBits bits (tiles of at most 4096 rows), above it the float bits of
// the squared distance without its sign bit and its kDropBits lowest bits.
constexpr int kLocalBits = 12;
constexpr int kDropBits = kLocalBits - 1;

// Error bound of the BF16 scan's squared distance for a query with bf16
// norm^2 qn (rows have norm^2 <= 1.02 m): the computed value is within
// delta16 of the exact squared distance of the bf16 vectors.
__device__ inline double bf16_delta(double qn, int m) {
  const double u = 1.0 / 16777216.0;  // 2^-24
  const double x2 = 1.02 * m;
  return (m + 3) * 2.0 * u * (qn + x2 + 2.0 * sqrt(qn * x2));
}

// A query's scan threshold from its best-so-far tau: rows whose computed
// squared distance reaches it are provably farther than tau (1 + 2^-12), so
// they can neither enter the query's top k nor need a place in its candidate
// list.  With rounding moving q and x by at most qeps and leps, a row is at
// least sqrt(d2 - delta16) - qeps - leps away.  +inf while tau is +inf.
__device__ inline float tau_threshold(float tau, double qn, float qeps, float leps, int m) {
  if (!(tau < __builtin_inff())) return __builtin_inff();
  const double t = static_cast<double>(tau) * (1.0 + 1.0 / 4096.0) + qeps + leps;
  const double v = t * t + bf16_delta(qn, m);
  float T = static_cast<float>(v);
  if (static_cast<double>(T) < v) T = nextafterf(T, __builtin_inff());
  return T;
}

}  // namespace leafi
