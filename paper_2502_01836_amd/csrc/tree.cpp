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
//
// Large nodes are processed with several host threads: the member ranges in
// one pass over each member's contiguous summary row (per-thread partial
// ranges, combined in thread order), the split column gathered once, and the
// two children built concurrently.  Every decision is the same as a
// sequential build: min / max and the selection by (value, id) do not depend
// on the order of evaluation.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <future>
#include <thread>

#include "index.h"

namespace leafi {

namespace {

// Host threads for the tree build (the machine's, at most 16).
int build_threads() {
  const unsigned hc = std::thread::hardware_concurrency();
  return static_cast<int>(std::max(1u, std::min(hc == 0 ? 1u : hc, 16u)));
}

// Run fn(t, lo, hi) over [0, n) split into `parts` contiguous ranges.
template <typename Fn>
void parallel_ranges(int64_t n, int parts, Fn fn) {
  if (parts <= 1 || n < 2) {
    fn(0, int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < parts; ++t) {
    const int64_t lo = n * t / parts, hi = n * (t + 1) / parts;
    th.emplace_back([=] { fn(t, lo, hi); });
  }
  for (auto &x : th) x.join();
}

constexpr int64_t kParallelMin = 1 << 18;  // members below which a node is handled by one thread

struct Builder {
  const std::vector<float> &mu, &sd;
  int S;
  int capacity;
  int rule;
  std::vector<double> seglen;
  int threads;

  // Leaves of the subtree rooted at the node holding `ids` (ascending), depth-first.
  std::vector<std::vector<int64_t>> split(std::vector<int64_t> &&ids, int budget) {
    std::vector<std::vector<int64_t>> leaves;
    if (static_cast<int64_t>(ids.size()) <= capacity) {
      leaves.push_back(std::move(ids));
      return leaves;
    }
    const int64_t n = static_cast<int64_t>(ids.size());
    const int parts = n >= kParallelMin ? std::max(1, budget) : 1;
    // member ranges of every (segment, statistic): per-thread partials
    std::vector<float> lo(static_cast<size_t>(parts) * 2 * S, INFINITY), hi(static_cast<size_t>(parts) * 2 * S, -INFINITY);
    parallel_ranges(n, parts, [&](int t, int64_t a, int64_t b) {
      float *l = &lo[static_cast<size_t>(t) * 2 * S], *h = &hi[static_cast<size_t>(t) * 2 * S];
      for (int64_t i = a; i < b; ++i) {
        const float *rm = &mu[ids[i] * S], *rs = &sd[ids[i] * S];
        for (int s = 0; s < S; ++s) {
          l[2 * s] = std::min(l[2 * s], rm[s]);
          h[2 * s] = std::max(h[2 * s], rm[s]);
          l[2 * s + 1] = std::min(l[2 * s + 1], rs[s]);
          h[2 * s + 1] = std::max(h[2 * s + 1], rs[s]);
        }
      }
    });
    double best = -1.0;
    int bs = 0, bst = 0;
    float blo = 0.0f, bhi = 0.0f;
    for (int s = 0; s < S; ++s) {
      for (int st = 0; st < 2; ++st) {
        float l = INFINITY, h = -INFINITY;
        for (int t = 0; t < parts; ++t) {
          l = std::min(l, lo[static_cast<size_t>(t) * 2 * S + 2 * s + st]);
          h = std::max(h, hi[static_cast<size_t>(t) * 2 * S + 2 * s + st]);
        }
        const double d = static_cast<double>(h) - static_cast<double>(l);
        const double score = seglen[s] * (d * d);
        if (score > best) {
          best = score;
          bs = s;
          bst = st;
          blo = l;
          bhi = h;
        }
      }
    }
    // the split column, gathered once
    const std::vector<float> &src = bst == 0 ? mu : sd;
    std::vector<float> col(n);
    parallel_ranges(n, parts, [&](int, int64_t a, int64_t b) {
      for (int64_t i = a; i < b; ++i) col[i] = src[ids[i] * S + bs];
    });
    std::vector<char> go_left(n, 0);
    bool done = false;
    if (rule == 1) {
      const double mid = static_cast<double>(blo) + (static_cast<double>(bhi) - static_cast<double>(blo)) / 2.0;
      int64_t nl = 0;
      for (int64_t i = 0; i < n; ++i) {
        go_left[i] = static_cast<double>(col[i]) <= mid;
        nl += go_left[i];
      }
      done = nl > 0 && nl < n;
    }
    if (!done) {
      // the ceil(n/2) smallest members by (value, id); ids ascending, so the
      // position breaks value ties exactly as the id does
      std::vector<int64_t> idx(n);
      for (int64_t i = 0; i < n; ++i) idx[i] = i;
      const int64_t nl = (n + 1) / 2;
      auto less = [&](int64_t a, int64_t b) { return col[a] < col[b] || (col[a] == col[b] && a < b); };
      std::nth_element(idx.begin(), idx.begin() + (nl - 1), idx.end(), less);
      const int64_t pivot = idx[nl - 1];
      for (int64_t i = 0; i < n; ++i) go_left[i] = !less(pivot, i);
    }
    std::vector<int64_t> left, right;
    left.reserve(n / 2 + 1);
    right.reserve(n / 2 + 1);
    for (int64_t i = 0; i < n; ++i) (go_left[i] ? left : right).push_back(ids[i]);
    std::vector<int64_t>().swap(ids);
    std::vector<float>().swap(col);
    std::vector<char>().swap(go_left);
    if (budget > 1 && n >= kParallelMin) {
      // the two children concurrently, each with half of the threads
      const int bl = budget / 2, br = budget - bl;
      auto fut = std::async(std::launch::async, [&, bl] { return split(std::move(left), bl); });
      std::vector<std::vector<int64_t>> r = split(std::move(right), br);
      leaves = fut.get();
      for (auto &v : r) leaves.push_back(std::move(v));
    } else {
      leaves = split(std::move(left), budget);
      std::vector<std::vector<int64_t>> r = split(std::move(right), budget);
      for (auto &v : r) leaves.push_back(std::move(v));
    }
    return leaves;
  }
};

}  // namespace

TreeResult build_tree(const std::vector<float> &seg_mu, const std::vector<float> &seg_sd, int64_t n, int S, int m,
                      int capacity, int rule) {
  if (rule == 2) return build_isax_tree(seg_mu, n, S, capacity);
  Builder b{seg_mu, seg_sd, S, capacity, rule, {}, build_threads()};
  b.seglen.resize(S);
  for (int s = 0; s < S; ++s) b.seglen[s] = static_cast<double>(((s + 1) * m) / S - (s * m) / S);
  std::vector<int64_t> all(n);
  for (int64_t i = 0; i < n; ++i) all[i] = i;
  TreeResult out;
  out.leaves = b.split(std::move(all), b.threads);
  return out;
}

// ---- iSAX backbone -------------------------------------------------------------
//
// The MESSI backbone (Section "Evaluation Setup"; SAX and iSAX as Section
// "Preliminaries" describes them): each segment mean (PAA value) becomes a
// symbol, the number of N(0, 1) quantile breakpoints at or below it; a
// symbol of b bits is the 8-bit one shifted right by 8 - b, because the
// breakpoints of cardinality 2^b are every 2^(8-b)-th of cardinality 256.
// The root's children are the words of one bit per segment, in ascending
// order with segment 0 as the highest bit; a node over capacity takes the
// next bit of the segment whose bit divides its members most evenly (ties:
// lowest segment), and splits in two when both halves are non-empty (else it
// keeps its members with the refined symbol and tries again); leaves are
// numbered depth-first, the 0 half first.

namespace {

// Standard normal CDF from the complementary error function.
double norm_cdf(double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); }

// Phi^-1(p) for 0 < p < 1: bisection on the CDF over [-40, 40] (80 halvings
// leave an interval below the spacing of doubles there), then two Newton
// steps on Phi(x) - p.
double norm_quantile(double p) {
  double lo = -40.0, hi = 40.0;
  for (int i = 0; i < 80; ++i) {
    const double mid = 0.5 * (lo + hi);
    (norm_cdf(mid) < p ? lo : hi) = mid;
  }
  double x = 0.5 * (lo + hi);
  for (int i = 0; i < 2; ++i) {
    const double dens = std::exp(-0.5 * x * x) / 2.5066282746310002;  // sqrt(2 pi)
    if (dens > 0.0) x -= (norm_cdf(x) - p) / dens;
  }
  return x;
}

}  // namespace

std::vector<float> isax_breakpoints(int bits) {
  const int c = 1 << bits;
  std::vector<float> bp(c - 1);
  for (int j = 1; j < c; ++j) {
    // the middle one is exactly 0 (p = 1/2); the rest from the lower tail,
    // where the CDF keeps its relative accuracy, mirrored for the upper half
    const int jj = j > c / 2 ? c - j : j;
    const double x = jj * 2 == c ? 0.0 : norm_quantile(static_cast<double>(jj) / c);
    bp[j - 1] = static_cast<float>(j > c / 2 ? -x : x);
  }
  return bp;
}

TreeResult build_isax_tree(const std::vector<float> &seg_mu, int64_t n, int S, int capacity) {
  const std::vector<float> bp = isax_breakpoints(kIsaxMaxBits);
  // 8-bit symbols of every (series, segment)
  std::vector<uint8_t> sym8(static_cast<size_t>(n) * S);
  parallel_ranges(n, n >= kParallelMin ? build_threads() : 1, [&](int, int64_t a, int64_t b) {
    for (int64_t i = a * S; i < b * S; ++i)
      sym8[i] = static_cast<uint8_t>(std::upper_bound(bp.begin(), bp.end(), seg_mu[i]) - bp.begin());
  });
  // root children: ids grouped by their one-bit word, ascending words, ids ascending within
  std::vector<uint64_t> word(n);
  for (int64_t i = 0; i < n; ++i) {
    uint64_t w = 0;
    for (int s = 0; s < S; ++s) w = (w << 1) | (sym8[i * S + s] >> (kIsaxMaxBits - 1));
    word[i] = w;
  }
  std::vector<int64_t> idx(n);
  if (S <= 20) {
    // counting sort over the 2^S words (ids stay ascending within a word)
    std::vector<int64_t> start((size_t(1) << S) + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++start[word[i] + 1];
    for (size_t w = 1; w < start.size(); ++w) start[w] += start[w - 1];
    for (int64_t i = 0; i < n; ++i) idx[start[word[i]]++] = i;
  } else {
    for (int64_t i = 0; i < n; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return word[a] < word[b]; });
  }
  // depth-first, 0 half first: an explicit stack of (members, bits, symbols)
  struct Task {
    std::vector<int64_t> ids;
    std::vector<uint8_t> bits, sym;
  };
  auto run = [&](Task root, TreeResult &out) {
    std::vector<Task> stack;
    stack.push_back(std::move(root));
    while (!stack.empty()) {
      Task t = std::move(stack.back());
      stack.pop_back();
      bool split = false;
      while (static_cast<int64_t>(t.ids.size()) > capacity) {
        int best_s = -1;
        int64_t best = -1, best_n1 = 0;
        const int64_t nn = static_cast<int64_t>(t.ids.size());
        for (int s = 0; s < S; ++s) {
          if (t.bits[s] >= kIsaxMaxBits) continue;
          const int shift = kIsaxMaxBits - 1 - t.bits[s];
          int64_t n1 = 0;
          for (int64_t id : t.ids) n1 += (sym8[id * S + s] >> shift) & 1;
          const int64_t d = nn > 2 * n1 ? nn - 2 * n1 : 2 * n1 - nn;
          if (best < 0 || d < best) {
            best = d;
            best_s = s;
            best_n1 = n1;
          }
        }
        if (best_s < 0) break;  // identical at 8 bits in every segment: an oversized leaf
        const int s = best_s, shift = kIsaxMaxBits - 1 - t.bits[s];
        t.bits[s] = static_cast<uint8_t>(t.bits[s] + 1);
        if (best_n1 > 0 && best_n1 < nn) {
          Task zero{{}, t.bits, t.sym}, one{{}, t.bits, t.sym};
          zero.sym[s] = static_cast<uint8_t>(2 * t.sym[s]);
          one.sym[s] = static_cast<uint8_t>(2 * t.sym[s] + 1);
          zero.ids.reserve(nn - best_n1);
          one.ids.reserve(best_n1);
          for (int64_t id : t.ids) (((sym8[id * S + s] >> shift) & 1) ? one : zero).ids.push_back(id);
          stack.push_back(std::move(one));   // popped after the zero half
          stack.push_back(std::move(zero));
          split = true;
          break;
        }
        t.sym[s] = static_cast<uint8_t>(2 * t.sym[s] + (best_n1 > 0 ? 1 : 0));
      }
      if (split) continue;
      out.leaves.push_back(std::move(t.ids));
      out.isax_bits.insert(out.isax_bits.end(), t.bits.begin(), t.bits.end());
      out.isax_sym.insert(out.isax_sym.end(), t.sym.begin(), t.sym.end());
    }
  };
  // the root's children, each built on its own by the host threads, then
  // their leaves concatenated in word order
  std::vector<std::pair<int64_t, int64_t>> groups;
  for (int64_t a = 0; a < n;) {
    int64_t b = a;
    while (b < n && word[idx[b]] == word[idx[a]]) ++b;
    groups.emplace_back(a, b);
    a = b;
  }
  std::vector<TreeResult> part(groups.size());
  std::atomic<size_t> next{0};
  const int threads = n >= kParallelMin ? build_threads() : 1;
  parallel_ranges(threads, threads, [&](int, int64_t, int64_t) {
    for (size_t g = next++; g < groups.size(); g = next++) {
      Task t;
      t.ids.assign(idx.begin() + groups[g].first, idx.begin() + groups[g].second);
      t.bits.assign(S, 1);
      t.sym.resize(S);
      for (int s = 0; s < S; ++s) t.sym[s] = static_cast<uint8_t>(sym8[t.ids[0] * S + s] >> (kIsaxMaxBits - 1));
      run(std::move(t), part[g]);
    }
  });
  TreeResult out;
  for (auto &p : part) {
    for (auto &l : p.leaves) out.leaves.push_back(std::move(l));
    out.isax_bits.insert(out.isax_bits.end(), p.isax_bits.begin(), p.isax_bits.end());
    out.isax_sym.insert(out.isax_sym.end(), p.isax_sym.begin(), p.isax_sym.end());
  }
  return out;
}

std::vector<float> leaf_boxes(const std::vector<float> &seg_mu, const std::vector<float> &seg_sd, int S,
                              const TreeResult &t) {
  const int64_t N = static_cast<int64_t>(t.leaves.size());
  std::vector<float> box(static_cast<size_t>(N) * S * 4);
  if (!t.isax_bits.empty()) {
    // each leaf's SAX interval per segment, widened by one ulp; any deviation
    const std::vector<float> bp = isax_breakpoints(kIsaxMaxBits);
    for (int64_t L = 0; L < N; ++L)
      for (int s = 0; s < S; ++s) {
        const int b = t.isax_bits[L * S + s], c = t.isax_sym[L * S + s];
        const int step = 1 << (kIsaxMaxBits - b);
        const float lo = c > 0 ? bp[c * step - 1] : -INFINITY;
        const float hi = c + 1 < (1 << b) ? bp[(c + 1) * step - 1] : INFINITY;
        float *o = &box[(static_cast<size_t>(L) * S + s) * 4];
        o[0] = std::nextafter(lo, -INFINITY);
        o[1] = std::nextafter(hi, INFINITY);
        o[2] = 0.0f;
        o[3] = INFINITY;
      }
    return box;
  }
  parallel_ranges(N, N >= 64 ? build_threads() : 1, [&](int, int64_t a, int64_t b) {
    for (int64_t L = a; L < b; ++L) {
      const auto &mem = t.leaves[L];
      float *o = &box[static_cast<size_t>(L) * S * 4];
      for (int s = 0; s < S; ++s) {
        o[4 * s + 0] = o[4 * s + 2] = INFINITY;
        o[4 * s + 1] = o[4 * s + 3] = -INFINITY;
      }
      for (int64_t id : mem) {
        const float *rm = &seg_mu[id * S], *rs = &seg_sd[id * S];
        for (int s = 0; s < S; ++s) {
          o[4 * s + 0] = std::min(o[4 * s + 0], rm[s]);
          o[4 * s + 1] = std::max(o[4 * s + 1], rm[s]);
          o[4 * s + 2] = std::min(o[4 * s + 2], rs[s]);
          o[4 * s + 3] = std::max(o[4 * s + 3], rs[s]);
        }
      }
      for (int s = 0; s < S; ++s) {
        o[4 * s + 0] = std::nextafter(o[4 * s + 0], -INFINITY);
        o[4 * s + 1] = std::nextafter(o[4 * s + 1], INFINITY);
        o[4 * s + 2] = std::nextafter(o[4 * s + 2], -INFINITY);
        o[4 * s + 3] = std::nextafter(o[4 * s + 3], INFINITY);
      }
    }
  });
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

std::vector<int32_t> select_knapsack(const std::vector<int64_t> &sizes, const std::vector<double> &p_lb,
                                     const std::vector<double> &p_f, double a, double tS, double tF, double w,
                                     double cM, std::vector<double> *benefit) {
  const size_t N = sizes.size();
  std::vector<double> b(N);
  std::vector<int32_t> cand;
  for (size_t i = 0; i < N; ++i) {
    b[i] = (1.0 - p_lb[i]) * (p_f[i] / a * tS * static_cast<double>(sizes[i]) - tF);
    if (b[i] > 0.0) cand.push_back(static_cast<int32_t>(i));
  }
  // Every filter weighs w bytes, so the knapsack holds floor(c^M / w) of
  // them and its optimum is that many of the largest positive benefits.
  std::stable_sort(cand.begin(), cand.end(), [&](int32_t x, int32_t y) { return b[x] > b[y]; });
  const double room = w > 0.0 ? std::floor(cM / w) : static_cast<double>(cand.size());
  if (room < static_cast<double>(cand.size())) cand.resize(room > 0.0 ? static_cast<size_t>(room) : 0);
  if (benefit) *benefit = std::move(b);
  return cand;
}

}  // namespace leafi
