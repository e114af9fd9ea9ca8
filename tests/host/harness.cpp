// Command-line harness over the library's host algorithms (tree build, leaf
// boxes, Algorithm 3 selection, Algorithm 4 calibration), built without any
// GPU code so the CPU tests can run them under AddressSanitizer and
// UndefinedBehaviorSanitizer and compare them with the oracle.
//
// Usage: harness <mode> <input file> <output file>.  Inputs and outputs are
// raw little-endian arrays in the order each mode reads or writes them.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "index.h"

using namespace leafi;

namespace {

struct In {
  FILE *f;
  template <typename T>
  T one() {
    T v{};
    if (fread(&v, sizeof(T), 1, f) != 1) throw std::runtime_error("short input");
    return v;
  }
  template <typename T>
  std::vector<T> many(size_t n) {
    std::vector<T> v(n);
    if (n && fread(v.data(), sizeof(T), n, f) != n) throw std::runtime_error("short input");
    return v;
  }
};

template <typename T>
void put(FILE *f, const T *p, size_t n) {
  if (n && fwrite(p, sizeof(T), n, f) != n) throw std::runtime_error("short write");
}

}  // namespace

int main(int argc, char **argv) {
  if (argc != 4) {
    fprintf(stderr, "usage: harness tree|select|calib <in> <out>\n");
    return 2;
  }
  try {
    const std::string mode = argv[1];
    In in{fopen(argv[2], "rb")};
    FILE *out = fopen(argv[3], "wb");
    if (!in.f || !out) throw std::runtime_error("cannot open files");
    if (mode == "tree") {
      // n, S, m, capacity, rule, mu [n, S], sd [n, S] -> N, leaf offsets [N + 1], members [n], boxes [N, S, 4]
      const int64_t n = in.one<int64_t>();
      const int S = in.one<int32_t>(), m = in.one<int32_t>(), cap = in.one<int32_t>(), rule = in.one<int32_t>();
      std::vector<float> mu = in.many<float>(n * S), sd = in.many<float>(n * S);
      TreeResult t = build_tree(mu, sd, n, S, m, cap, rule);
      std::vector<float> boxes = leaf_boxes(mu, sd, S, t);
      const int64_t N = static_cast<int64_t>(t.leaves.size());
      std::vector<int64_t> off(N + 1, 0), mem;
      for (int64_t L = 0; L < N; ++L) {
        off[L + 1] = off[L] + static_cast<int64_t>(t.leaves[L].size());
        mem.insert(mem.end(), t.leaves[L].begin(), t.leaves[L].end());
      }
      put(out, &N, 1);
      put(out, off.data(), off.size());
      put(out, mem.data(), mem.size());
      put(out, boxes.data(), boxes.size());
    } else if (mode == "select") {
      // N, th, w, cM, sizes [N] -> count, leaves [count]
      const int64_t N = in.one<int64_t>();
      const double th = in.one<double>(), w = in.one<double>(), cM = in.one<double>();
      std::vector<int64_t> sizes = in.many<int64_t>(N);
      std::vector<int32_t> sel = select_leaves(sizes, th, w, cM);
      const int64_t c = static_cast<int64_t>(sel.size());
      put(out, &c, 1);
      put(out, sel.data(), sel.size());
    } else if (mode == "calib") {
      // nc, N, F, kmax, k, n_targets, mapping, corrected, order [nc, N] int32,
      // leaf_d [nc, N, kmax] f64, leaf_ids [nc, N, kmax] i64, dfilt [nc, F] f32,
      // leaf_of_filter [F] int32, targets [n_targets] f32 -> offsets [n_targets, F] f32
      CalibInput c;
      c.nc = in.one<int32_t>();
      c.N = in.one<int32_t>();
      c.F = in.one<int32_t>();
      c.kmax = in.one<int32_t>();
      const int k = in.one<int32_t>(), nt = in.one<int32_t>(), mapping = in.one<int32_t>(),
                corrected = in.one<int32_t>();
      c.order = in.many<int32_t>(static_cast<size_t>(c.nc) * c.N);
      c.leaf_d = in.many<double>(static_cast<size_t>(c.nc) * c.N * c.kmax);
      c.leaf_ids = in.many<int64_t>(static_cast<size_t>(c.nc) * c.N * c.kmax);
      c.dfilt = in.many<float>(static_cast<size_t>(c.nc) * c.F);
      c.leaf_of_filter = in.many<int32_t>(c.F);
      std::vector<float> targets = in.many<float>(nt);
      std::vector<float> o = calibrate_k(c, k, targets, mapping, corrected != 0);
      put(out, o.data(), o.size());
    } else {
      throw std::runtime_error("unknown mode " + mode);
    }
    fclose(in.f);
    fclose(out);
  } catch (const std::exception &e) {
    fprintf(stderr, "harness: %s\n", e.what());
    return 1;
  }
  return 0;
}
