// Conformal auto-tuning on the host (paper: Section "Filter Conformal
// Auto-tuning", Algorithm 4).
//
// Inputs come from the device: per calibration query the visit order, the
// exact per-leaf top-k distances (the leaf scan in all-pairs mode) and the
// filter predictions d^f.  For one k:
//   - d^bsf(c, i): the k-th smallest distance over the leaves that precede
//     leaf i in c's visit order (the exact search's best-so-far when it
//     reaches i; +inf while fewer than k series precede);
//   - the non-conformity scores alpha = |d^f - d^L| per filter, sorted;
//   - for sorted position j, offsets o_i = alpha_{i,(j)}; a true neighbour of
//     c in a filtered leaf i survives iff d^f(c, i) - o_i <= d^bsf(c, i); the
//     recall q_j is the surviving share of all (query, neighbour) pairs.  The
//     predicate is monotone in j, so each pair contributes from the first j
//     at which it survives and q_j is a prefix sum;
//   - a target maps to the first j whose recall reaches it (optionally after
//     the finite-sample correction ceil((n_c + 1) t) / n_c), or, in the
//     Steffen variant, to the monotone interpolant of offset against recall.
#include <algorithm>
#include <cmath>
#include <limits>
#include <thread>

#include "index.h"

namespace leafi {

namespace {

struct Steffen {
  std::vector<double> x, y, yp;
  void fit() {
    size_t n = x.size();
    yp.assign(n, 0.0);
    if (n < 2) return;
    std::vector<double> h(n - 1), s(n - 1);
    for (size_t i = 0; i + 1 < n; ++i) {
      h[i] = x[i + 1] - x[i];
      s[i] = (y[i + 1] - y[i]) / h[i];
    }
    if (n == 2) {
      yp[0] = yp[1] = s[0];
      return;
    }
    auto sgn = [](double v) { return v > 0 ? 1.0 : (v < 0 ? -1.0 : 0.0); };
    for (size_t i = 1; i + 1 < n; ++i) {
      double p = (s[i - 1] * h[i] + s[i] * h[i - 1]) / (h[i - 1] + h[i]);
      yp[i] = (sgn(s[i - 1]) + sgn(s[i])) * std::min(std::min(std::fabs(s[i - 1]), std::fabs(s[i])), 0.5 * std::fabs(p));
    }
    // one-sided parabolic end slopes, limited to keep monotonicity
    auto end_slope = [](double s0, double s1, double h0, double h1) {
      double p = s0 * (1.0 + h0 / (h0 + h1)) - s1 * h0 / (h0 + h1);
      if (p * s0 <= 0.0) return 0.0;
      if (std::fabs(p) > 2.0 * std::fabs(s0)) return 2.0 * s0;
      return p;
    };
    yp[0] = end_slope(s[0], s[1], h[0], h[1]);
    yp[n - 1] = end_slope(s[n - 2], s[n - 3], h[n - 2], h[n - 3]);
  }
  double eval(double t) const {
    size_t n = x.size();
    if (t <= x[0]) return y[0];
    if (t >= x[n - 1]) return y[n - 1];
    size_t i = static_cast<size_t>(std::upper_bound(x.begin(), x.end(), t) - x.begin()) - 1;
    double hh = x[i + 1] - x[i];
    double s = (y[i + 1] - y[i]) / hh;
    double a = (yp[i] + yp[i + 1] - 2.0 * s) / (hh * hh);
    double b = (3.0 * s - 2.0 * yp[i] - yp[i + 1]) / hh;
    double dx = t - x[i];
    return ((a * dx + b) * dx + yp[i]) * dx + y[i];
  }
};

}  // namespace

double steffen_eval(const std::vector<double> &x, const std::vector<double> &y, double t) {
  Steffen sf{x, y, {}};
  sf.fit();
  return sf.eval(t);
}

std::vector<float> calibrate_k(const CalibInput &in, int k, const std::vector<float> &targets, int mapping,
                               bool corrected) {
  const int nc = in.nc, N = in.N, F = in.F, K = in.kmax;
  const double inf = std::numeric_limits<double>::infinity();
  std::vector<int32_t> filt_of_leaf(N, -1);
  for (int f = 0; f < F; ++f) filt_of_leaf[in.leaf_of_filter[f]] = f;

  // true top-k leaves and d^bsf along each query's visit order: the k best
  // (distance, id) so far, merged with each leaf's sorted list in turn
  // (queries split over host threads; each query's result is its own)
  std::vector<int32_t> nbr_leaf(static_cast<size_t>(nc) * k, -1);
  std::vector<double> dbsf(static_cast<size_t>(nc) * N, inf);
  struct Entry {
    double d;
    int64_t id;
    int32_t leaf;
    bool operator<(const Entry &o) const { return d < o.d || (d == o.d && id < o.id); }
  };
  const unsigned hc = std::thread::hardware_concurrency();
  const int nthreads = static_cast<int>(std::max(1u, std::min({hc == 0 ? 1u : hc, 16u, static_cast<unsigned>(nc)})));
  auto per_query = [&](int c0, int c1) {
    std::vector<Entry> pool, lst, merged;
    pool.reserve(k);
    lst.reserve(k);
    merged.reserve(k);
    for (int c = c0; c < c1; ++c) {
      pool.clear();
      for (int pos = 0; pos < N; ++pos) {
        const int L = in.order[static_cast<size_t>(c) * N + pos];
        dbsf[static_cast<size_t>(c) * N + L] = static_cast<int>(pool.size()) >= k ? pool[k - 1].d : inf;
        const double *ld = &in.leaf_d[(static_cast<size_t>(c) * N + L) * K];
        const int64_t *li = &in.leaf_ids[(static_cast<size_t>(c) * N + L) * K];
        lst.clear();
        for (int e = 0; e < k && e < K; ++e) {
          if (li[e] < 0) break;
          lst.push_back({ld[e], li[e], L});
        }
        if (!std::is_sorted(lst.begin(), lst.end())) std::sort(lst.begin(), lst.end());
        merged.clear();
        size_t a = 0, b = 0;
        while (static_cast<int>(merged.size()) < k && (a < pool.size() || b < lst.size())) {
          if (b >= lst.size() || (a < pool.size() && pool[a] < lst[b])) merged.push_back(pool[a++]);
          else merged.push_back(lst[b++]);
        }
        pool.swap(merged);
      }
      for (size_t e = 0; e < pool.size(); ++e) nbr_leaf[static_cast<size_t>(c) * k + e] = pool[e].leaf;
    }
  };
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t)
      th.emplace_back(per_query, static_cast<int>(static_cast<int64_t>(nc) * t / nthreads),
                      static_cast<int>(static_cast<int64_t>(nc) * (t + 1) / nthreads));
    for (auto &x : th) x.join();
  }

  // sorted non-conformity scores per filter
  std::vector<std::vector<double>> alpha(F, std::vector<double>(nc));
  for (int f = 0; f < F; ++f) {
    int L = in.leaf_of_filter[f];
    for (int c = 0; c < nc; ++c) {
      double dl = in.leaf_d[(static_cast<size_t>(c) * N + L) * K];
      alpha[f][c] = std::fabs(static_cast<double>(in.dfilt[static_cast<size_t>(c) * F + f]) - dl);
    }
    std::sort(alpha[f].begin(), alpha[f].end());
  }

  // first sorted position at which each (query, neighbour) pair survives
  std::vector<int64_t> hist(nc + 1, 0);
  int64_t pairs = 0;
  for (int c = 0; c < nc; ++c) {
    for (int e = 0; e < k; ++e) {
      int L = nbr_leaf[static_cast<size_t>(c) * k + e];
      if (L < 0) continue;
      ++pairs;
      int f = filt_of_leaf[L];
      if (f < 0) {
        ++hist[0];
        continue;
      }
      double df = in.dfilt[static_cast<size_t>(c) * F + f];
      double db = dbsf[static_cast<size_t>(c) * N + L];
      // survives at j iff !(df - alpha_j > db); alpha ascending -> monotone
      int lo = 0, hi = nc;  // answer in [0, nc]; nc = only with offsets +inf
      while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (!(df - alpha[f][mid] > db)) hi = mid; else lo = mid + 1;
      }
      ++hist[lo];
    }
  }
  std::vector<int64_t> kept(nc + 1);
  int64_t run = 0;
  for (int j = 0; j <= nc; ++j) {
    run += hist[j];
    kept[j] = run;
  }
  const double denom = static_cast<double>(nc) * k;

  std::vector<float> out(targets.size() * F, INFINITY);
  for (size_t ti = 0; ti < targets.size(); ++ti) {
    double t = targets[ti];
    int jstar = nc;
    if (corrected) {
      int64_t T = static_cast<int64_t>(std::ceil((nc + 1) * t - 1e-9));
      if (T > nc) T = nc;
      for (int j = 0; j <= nc; ++j)
        if (kept[j] >= T * k) { jstar = j; break; }
    } else {
      for (int j = 0; j <= nc; ++j)
        if (static_cast<double>(kept[j]) / denom >= t - 1e-12) { jstar = j; break; }
    }
    (void)pairs;
    double tq = corrected ? std::min(1.0, std::ceil((nc + 1) * t - 1e-9) / nc) : t;
    for (int f = 0; f < F; ++f) {
      float o;
      if (mapping == 0) {
        o = jstar < nc ? static_cast<float>(alpha[f][jstar]) : INFINITY;
      } else {
        // points (q_j, alpha_(j)), equal recalls keep the largest offset
        std::vector<double> xs, ys;
        for (int j = 0; j < nc; ++j) {
          double q = static_cast<double>(kept[j]) / denom;
          if (!xs.empty() && q == xs.back()) {
            ys.back() = std::max(ys.back(), alpha[f][j]);
          } else {
            xs.push_back(q);
            ys.push_back(alpha[f][j]);
          }
        }
        if (xs.empty() || tq > xs.back()) o = INFINITY;
        else if (tq <= xs.front()) o = static_cast<float>(ys.front());
        else o = static_cast<float>(steffen_eval(xs, ys, tq));
      }
      out[ti * F + f] = o;
    }
  }
  return out;
}

}  // namespace leafi
