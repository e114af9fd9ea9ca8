// Host tree build over the per-segment summaries (the DSTree-style backbone of
// the paper's Section "Preliminaries": internal nodes route, leaves hold the
// series, every node keeps a summary of its members).
//
// A node holding more than `capacity` series splits on the (segment,
// statistic) pair whose member range has the largest seg_len * range^2
// (ties: lowest 2 * segment + statistic, mean before std).  Median rule: the
// first ceil(n/2) members in (value, id) order go left.  Midpoint rule:
// members with value <= lo + (hi - lo) / 2 go left, with the median rule as
// fallback when one side would be empty.  Leaves are numbered depth-first,
// left child first; members stay in ascending id order.
#include <algorithm>
#include <cmath>

#include "index.h"

namespace leafi {

namespace {

struct Builder {
  const std::vector<float> &mu, &sd;
  int S;
  int capacity;
  int rule;
  std::vector<double> seglen;
  TreeResult out;

  float stat(int64_t id, int s, int st) const { return st == 0 ? mu[id * S + s] : sd[id * S + s]; }

  void split(std::vector<int64_t> &&ids) {
    if (static_cast<int64_t>(ids.size()) <= capacity) {
      out.leaves.push_back(std::move(ids));
      return;
    }
    double best = -1.0;
    int bs = 0, bst = 0;
    for (int s = 0; s < S; ++s) {
      for (int st = 0; st < 2; ++st) {
        float lo = stat(ids[0], s, st), hi = lo;
        for (int64_t id : ids) {
          float v = stat(id, s, st);
          lo = v < lo ? v : lo;
          hi = v > hi ? v : hi;
        }
        double d = static_cast<double>(hi) - static_cast<double>(lo);
        double score = seglen[s] * (d * d);
        if (score > best) {
          best = score;
          bs = s;
          bst = st;
        }
      }
    }
    std::vector<char> go_left(ids.size(), 0);
    bool done = false;
    if (rule == 1) {
      double lo = stat(ids[0], bs, bst), hi = lo;
      for (int64_t id : ids) {
        double v = stat(id, bs, bst);
        lo = std::min(lo, v);
        hi = std::max(hi, v);
      }
      double mid = lo + (hi - lo) / 2.0;
      size_t nl = 0;
      for (size_t i = 0; i < ids.size(); ++i) {
        go_left[i] = static_cast<double>(stat(ids[i], bs, bst)) <= mid;
        nl += go_left[i];
      }
      done = nl > 0 && nl < ids.size();
    }
    if (!done) {
      // the ceil(n/2) smallest members by (value, id)
      std::vector<size_t> idx(ids.size());
      for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
      size_t nl = (ids.size() + 1) / 2;
      auto less = [&](size_t a, size_t b) {
        float va = stat(ids[a], bs, bst), vb = stat(ids[b], bs, bst);
        return va < vb || (va == vb && ids[a] < ids[b]);
      };
      std::nth_element(idx.begin(), idx.begin() + (nl - 1), idx.end(), less);
      size_t pivot = idx[nl - 1];
      for (size_t i = 0; i < ids.size(); ++i) go_left[i] = !less(pivot, i);
    }
    std::vector<int64_t> left, right;
    left.reserve(ids.size() / 2 + 1);
    right.reserve(ids.size() / 2 + 1);
    for (size_t i = 0; i < ids.size(); ++i) (go_left[i] ? left : right).push_back(ids[i]);
    std::vector<int64_t>().swap(ids);
    split(std::move(left));
    split(std::move(right));
  }
};

}  // namespace

TreeResult build_tree(const std::vector<float> &seg_mu, const std::vector<float> &seg_sd, int64_t n, int S, int m,
                      int capacity, int rule) {
  Builder b{seg_mu, seg_sd, S, capacity, rule, {}, {}};
  b.seglen.resize(S);
  for (int s = 0; s < S; ++s) b.seglen[s] = static_cast<double>(((s + 1) * m) / S - (s * m) / S);
  std::vector<int64_t> all(n);
  for (int64_t i = 0; i < n; ++i) all[i] = i;
  b.split(std::move(all));
  return std::move(b.out);
}

std::vector<float> leaf_boxes(const std::vector<float> &seg_mu, const std::vector<float> &seg_sd, int S,
                              const TreeResult &t) {
  size_t N = t.leaves.size();
  std::vector<float> box(N * S * 4);
  for (size_t L = 0; L < N; ++L) {
    const auto &mem = t.leaves[L];
    for (int s = 0; s < S; ++s) {
      float mlo = seg_mu[mem[0] * S + s], mhi = mlo, slo = seg_sd[mem[0] * S + s], shi = slo;
      for (int64_t id : mem) {
        float a = seg_mu[id * S + s], b = seg_sd[id * S + s];
        mlo = std::min(mlo, a);
        mhi = std::max(mhi, a);
        slo = std::min(slo, b);
        shi = std::max(shi, b);
      }
      float *o = &box[(L * S + s) * 4];
      o[0] = std::nextafter(mlo, -INFINITY);
      o[1] = std::nextafter(mhi, INFINITY);
      o[2] = std::nextafter(slo, -INFINITY);
      o[3] = std::nextafter(shi, INFINITY);
    }
  }
  return box;
}

std::vector<int32_t> select_leaves(const std::vector<int64_t> &sizes, double th, double w, double cM) {
  std::vector<int32_t> idx(sizes.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = static_cast<int32_t>(i);
  std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return sizes[a] > sizes[b]; });
  std::vector<int32_t> sel;
  double used = 0.0;
  for (int32_t L : idx) {
    if (static_cast<double>(sizes[L]) >= th && used + w <= cM) {
      sel.push_back(L);
      used += w;
    }
  }
  return sel;
}

}  // namespace leafi
