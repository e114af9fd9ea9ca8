/*
 * Oracle brute force: plain FP64 exact k-nearest-neighbour search.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference the GPU library is checked against.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code
 * with the GPU library.
 *
 * What it computes (paper, Section "Preliminaries", similarity search and the
 * node-wise nearest-neighbour distance d^L):
 *   - z-normalisation of each series, with mean and population standard
 *     deviation in FP64; the normalised values are stored as fp32, which is the
 *     form the index keeps (a series with std < 1e-8 becomes all zeros);
 *   - Euclidean distance d(q, x) = sqrt(sum_t (q_t - x_t)^2), FP64 direct
 *     difference, summed in t order;
 *   - the k nearest series ordered by (distance, id) ascending (equal
 *     distances: smaller id first);
 *   - the same restricted to each leaf of a partition (d^L and its top-k).
 *
 * Parallelism is plain OpenMP over queries; each thread walks the collection
 * in blocks so that a block is reused across the thread's queries.  Several
 * series are accumulated side by side, but each distance is still one
 * sequential FP64 sum over t.  Built with -O2 and no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* z-normalise n rows of length m; out may alias x. */
void or_znorm(const float *x, int64_t n, int32_t m, float *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const float *r = x + i * (int64_t)m;
    double s = 0.0;
    for (int32_t t = 0; t < m; ++t) s += (double)r[t];
    double mu = s / (double)m;
    double v = 0.0;
    for (int32_t t = 0; t < m; ++t) {
      double d = (double)r[t] - mu;
      v += d * d;
    }
    double sd = sqrt(v / (double)m);
    float *o = out + i * (int64_t)m;
    if (sd < 1e-8) {
      for (int32_t t = 0; t < m; ++t) o[t] = 0.0f;
    } else {
      for (int32_t t = 0; t < m; ++t) o[t] = (float)(((double)r[t] - mu) / sd);
    }
  }
}

/* Insert (d, id) into a list sorted by (d, id) holding at most k entries. */
static void topk_insert(double *kd, int64_t *ki, int32_t *cnt, int32_t k, double d, int64_t id) {
  int32_t c = *cnt;
  if (c == k) {
    double wd = kd[k - 1];
    int64_t wi = ki[k - 1];
    if (d > wd || (d == wd && id > wi)) return;
    c = k - 1; /* drop the current worst */
  }
  int32_t p = c;
  while (p > 0 && (kd[p - 1] > d || (kd[p - 1] == d && ki[p - 1] > id))) {
    kd[p] = kd[p - 1];
    ki[p] = ki[p - 1];
    --p;
  }
  kd[p] = d;
  ki[p] = id;
  *cnt = c + 1;
}

static double dist2(const float *q, const float *x, int32_t m) {
  double s = 0.0;
  for (int32_t t = 0; t < m; ++t) {
    double d = (double)q[t] - (double)x[t];
    s += d * d;
  }
  return s;
}

#define OR_BLOCK 512

/*
 * Exact k-NN over the whole collection.
 * data [n, m] and q [nq, m] are the stored (already z-normalised) fp32 series.
 * Outputs ids [nq, k] and d [nq, k] (Euclidean, not squared), sorted by
 * (d, id).  Slots beyond n stay id = -1, d = +inf.
 */
void or_knn(const float *data, int64_t n, int32_t m, const float *q, int64_t nq, int32_t k,
            int64_t *ids, double *dist) {
#pragma omp parallel
  {
    int nt = 1, tid = 0;
#ifdef _OPENMP
    nt = omp_get_num_threads();
    tid = omp_get_thread_num();
#endif
    int64_t q0 = nq * tid / nt, q1 = nq * (tid + 1) / nt;
    int64_t nql = q1 - q0;
    double *kd = (double *)malloc(sizeof(double) * (size_t)(nql > 0 ? nql : 1) * (size_t)k);
    int64_t *ki = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nql > 0 ? nql : 1) * (size_t)k);
    int32_t *cnt = (int32_t *)calloc((size_t)(nql > 0 ? nql : 1), sizeof(int32_t));
    for (int64_t b0 = 0; b0 < n && nql > 0; b0 += OR_BLOCK) {
      int64_t b1 = b0 + OR_BLOCK < n ? b0 + OR_BLOCK : n;
      for (int64_t j = 0; j < nql; ++j) {
        const float *qq = q + (q0 + j) * (int64_t)m;
        double *jd = kd + j * k;
        int64_t *ji = ki + j * k;
        int64_t i = b0;
        for (; i + 4 <= b1; i += 4) {
          const float *x0 = data + i * (int64_t)m;
          double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
          for (int32_t t = 0; t < m; ++t) {
            double a = (double)qq[t];
            double d0 = a - (double)x0[t];
            double d1 = a - (double)x0[t + m];
            double d2 = a - (double)x0[t + 2 * m];
            double d3 = a - (double)x0[t + 3 * m];
            s0 += d0 * d0;
            s1 += d1 * d1;
            s2 += d2 * d2;
            s3 += d3 * d3;
          }
          topk_insert(jd, ji, &cnt[j], k, s0, i);
          topk_insert(jd, ji, &cnt[j], k, s1, i + 1);
          topk_insert(jd, ji, &cnt[j], k, s2, i + 2);
          topk_insert(jd, ji, &cnt[j], k, s3, i + 3);
        }
        for (; i < b1; ++i) topk_insert(jd, ji, &cnt[j], k, dist2(qq, data + i * (int64_t)m, m), i);
      }
    }
    for (int64_t j = 0; j < nql; ++j) {
      for (int32_t r = 0; r < k; ++r) {
        int64_t o = (q0 + j) * k + r;
        if (r < cnt[j]) {
          ids[o] = ki[j * k + r];
          dist[o] = sqrt(kd[j * k + r]);
        } else {
          ids[o] = -1;
          dist[o] = INFINITY;
        }
      }
    }
    free(kd);
    free(ki);
    free(cnt);
  }
}

/*
 * Per-leaf exact k-NN: for every query and every leaf, the k nearest members
 * of that leaf.  The collection is given leaf by leaf: members of leaf L are
 * rows leaf_off[L] .. leaf_off[L+1]-1 of `data`, and member_id gives each
 * row's id.  Outputs d [nq, N, k] (Euclidean) and ids [nq, N, k], sorted by
 * (d, id); empty slots are id = -1, d = +inf.  Entry [., L, 0] is d^L.
 *
 * Work is split into (leaf, block of 64 queries) tasks; within a task the
 * leaf is walked in row blocks so each block is reused by the 64 queries.
 */
#define OR_QCHUNK 64
void or_leaf_knn(const float *data, const int64_t *member_id, const int64_t *leaf_off, int32_t n_leaves,
                 int32_t m, const float *q, int64_t nq, int32_t k, int64_t *ids, double *dist) {
  int64_t nqc = (nq + OR_QCHUNK - 1) / OR_QCHUNK;
  int64_t ntask = nqc * (int64_t)n_leaves;
#pragma omp parallel
  {
    double *kd = (double *)malloc(sizeof(double) * (size_t)OR_QCHUNK * (size_t)k);
    int64_t *ki = (int64_t *)malloc(sizeof(int64_t) * (size_t)OR_QCHUNK * (size_t)k);
    int32_t cnt[OR_QCHUNK];
#pragma omp for schedule(dynamic, 1)
    for (int64_t task = 0; task < ntask; ++task) {
      int32_t L = (int32_t)(task / nqc);
      int64_t j0 = (task % nqc) * OR_QCHUNK;
      int64_t j1 = j0 + OR_QCHUNK < nq ? j0 + OR_QCHUNK : nq;
      for (int64_t j = j0; j < j1; ++j) cnt[j - j0] = 0;
      for (int64_t b0 = leaf_off[L]; b0 < leaf_off[L + 1]; b0 += OR_BLOCK) {
        int64_t b1 = b0 + OR_BLOCK < leaf_off[L + 1] ? b0 + OR_BLOCK : leaf_off[L + 1];
        for (int64_t j = j0; j < j1; ++j) {
          const float *qq = q + j * (int64_t)m;
          for (int64_t r = b0; r < b1; ++r)
            topk_insert(kd + (j - j0) * k, ki + (j - j0) * k, &cnt[j - j0], k,
                        dist2(qq, data + r * (int64_t)m, m), member_id[r]);
        }
      }
      for (int64_t j = j0; j < j1; ++j) {
        for (int32_t s = 0; s < k; ++s) {
          int64_t o = (j * n_leaves + L) * (int64_t)k + s;
          if (s < cnt[j - j0]) {
            ids[o] = ki[(j - j0) * k + s];
            dist[o] = sqrt(kd[(j - j0) * k + s]);
          } else {
            ids[o] = -1;
            dist[o] = INFINITY;
          }
        }
      }
    }
    free(kd);
    free(ki);
  }
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the parallel loops above from now on (n >= 1). */
void or_set_num_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}
