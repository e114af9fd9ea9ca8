// Serving engine: continuous batching of k-NN requests over a resident index.
//
// Every admitted request owns a slot: per-query device state (normalised
// query, bounds, visit order, filter predictions, cursor, tau, running top-k,
// round count).  A worker thread runs engine rounds back to back.  Each round
// first prepares the requests admitted since the previous round into free
// slots, then advances every active slot by one round of its own schedule
// (prune cascade, leaf scan grouped by leaf across all slots, rerank, merge,
// exact rescan of uncertified items), then retires the slots whose search
// has ended.  A request arriving while others are on the GPU joins at the
// next round; a finished one frees its slot at once.  Each query's decisions
// depend only on its own state and its own schedule, and every kernel's
// arithmetic for one query is independent of the other queries in the round,
// so a result is the same whether the request ran alone or in a mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "engine.h"

using namespace leafi;

namespace {

using Clock = std::chrono::steady_clock;

double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

__global__ void k_slot_init(const int32_t *slots, int64_t n, RoundBufs b, int32_t *state, int32_t *qround) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int s = slots[i];
  b.cursor[s] = 0;
  b.tau[s] = __builtin_inff();
  b.res_cnt[s] = 0;
  qround[s] = 0;
  state[s] = 1;
}

__global__ void k_slot_reset_all(int64_t n, int N, RoundBufs b, int32_t *state, int32_t *qround) {
  int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n) return;
  b.cursor[s] = N;  // an idle slot has no leaf left: the rounds skip it
  b.res_cnt[s] = 0;
  b.qitem_cnt[s] = 0;
  qround[s] = 0;
  state[s] = 0;
}

struct Request {
  std::vector<float> q;
  int k = 1;
  float target = 1.0f;
  double t_arrive = 0.0;
  double t_done = 0.0;
  int state = 0;  // 0 queued, 1 active, 2 done
  std::vector<int64_t> ids;
  std::vector<float> d;
};

template <typename T>
struct Pinned {
  T *p = nullptr;
  T *dev = nullptr;  // device address of a mapped allocation
  size_t n = 0;
  void alloc(size_t c, bool mapped = false) {
    release();
    if (c) {
      HIP_OK(hipHostMalloc(reinterpret_cast<void **>(&p), c * sizeof(T),
                           mapped ? hipHostMallocMapped : hipHostMallocDefault));
      if (mapped) HIP_OK(hipHostGetDevicePointer(reinterpret_cast<void **>(&dev), p, 0));
    }
    n = c;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    dev = nullptr;
    n = 0;
  }
  ~Pinned() { release(); }
};

}  // namespace

struct leafi_server {
  leafi_index *ix = nullptr;
  leafi_server_opts o{};
  hipStream_t st = nullptr;
  int slots = 0;
  int kprime = 4;
  Schedule sched{};
  bool use_f = false;
  // requests
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::unordered_map<uint64_t, Request> reqs;
  std::deque<uint64_t> queue;
  uint64_t next_ticket = 1;
  std::vector<int> free_slots;
  std::vector<uint64_t> slot_ticket;
  bool stop = false;
  std::thread worker;
  std::string worker_error;
  // device state beyond the index workspace
  DevBuf<int32_t> state, qround, new_slots, new_k, n_done;
  DevBuf<float> new_t, new_raw;
  Pinned<float> h_raw, h_t;
  Pinned<int32_t> h_slots, h_k;
  // finished requests, written by the GPU straight into mapped host memory
  Pinned<float> h_done_d;
  Pinned<int32_t> h_done_slot, h_ndone;
  Pinned<int64_t> h_done_ids;
  bool device_rounds = false;  // the rescan pass runs unconditionally, sized by the round bound
  // statistics
  int64_t rounds = 0, completed = 0;
  double active_sum = 0.0;
  int max_active = 0;

  void run();
  void engine_round(int n_new, int &n_active);
  // items one round can hold: every slot's largest schedule step
  int64_t round_bound() const {
    int maxwant = 0;
    for (int i = 0; i < sched.n; ++i) maxwant = sched.r[i] == 0 ? ix->N : std::max(maxwant, sched.r[i]);
    return static_cast<int64_t>(slots) * std::min(maxwant, ix->N);
  }
  ~leafi_server();
};

void leafi_server::engine_round(int n_new, int &n_active) {
  Workspace &w = ix->ws;
  const int N = ix->N, m = ix->m, kmax = o.k_max;
  const bool bf16 = o.scan == LEAFI_SCAN_BF16;
  if (n_new > 0) {
    h2d(new_raw.get(), h_raw.p, static_cast<size_t>(n_new) * m, st);
    h2d(new_slots.get(), h_slots.p, n_new, st);
    h2d(new_k.get(), h_k.p, n_new, st);
    h2d(new_t.get(), h_t.p, n_new, st);
    launch_qprep(new_raw.get(), n_new, m, ix->S, w.q32.get(), w.q16.get(), w.qn16.get(), w.qeps.get(), w.qstat.get(),
                 st, new_slots.get());
    launch_lb(w.qstat.get(), n_new, ix->boxes.get(), N, ix->S, m, w.lb.get(), st, new_slots.get());
    launch_order(w.lb.get(), n_new, N, w.order.get(), w.lbs.get(), st, new_slots.get());
    launch_select_pairs(n_new, new_k.get(), new_t.get(), use_f ? ix->cal.pairs() : 0,
                        use_f ? ix->cal.pair_k.get() : nullptr, use_f ? ix->cal.pair_t.get() : nullptr, kmax,
                        w.pair.get(), w.kq.get(), st, new_slots.get());
    hipLaunchKernelGGL(k_slot_init, dim3(ceil_div(n_new, 256)), dim3(256), 0, st, new_slots.get(), n_new, views(w),
                       state.get(), qround.get());
    LAUNCH_OK("slot_init");
    n_active += n_new;
  }
  const int F = ix->filt.F;
  if (use_f) {
    // slots that finished their first round get the filter pairs a later round can test
    fill_i32(w.pcnt.get(), F, 0, st);
    launch_filter_pairs(slots, N, w.lbs.get(), w.order.get(), ix->filt.filt_of_leaf.get(), views(w), w.plist.get(),
                        w.pcnt.get(), w.dfo.get(), st, qround.get());
    infer_filter_pairs(ix, slots, 0, st);
  }
  reset_round(ix, st);
  launch_worklist(slots, N, w.lbs.get(), w.order.get(), use_f ? w.dfo.get() : nullptr, ix->leaf_n.get(), 0, views(w),
                  st, &sched, qround.get());
  const int64_t bound = round_bound();
  RoundOpts ro;
  ro.may_read = !device_rounds;
  ro.use_tau = true;
  ro.kp_query = true;
  if (scan_round(ix, slots, bf16, kprime, kmax, st, nullptr, bound, &ro) != 0)
    launch_query_merge(slots, N, kmax, true, false, views(w), st);
  if (device_rounds) {
    // exact rescan of the uncertified items, sized on the device (an empty
    // pass exits at once): no read-back inside the round
    RoundOpts rf = ro;
    rf.small = true;
    rf.use_tau = false;
    scan_round(ix, slots, false, default_kprime(kmax, false), kmax, st, nullptr, bound, &rf);
    launch_query_merge(slots, N, kmax, false, true, views(w), st);
  } else {
    read_ctl(ix, st);
    const int64_t n_fb = w.h_ctl[kCtlFallback];
    if (n_fb > 0) {
      RoundOpts rf;
      rf.kp_query = true;
      if (scan_round(ix, slots, false, default_kprime(kmax, false), kmax, st, nullptr, n_fb, &rf) != 0)
        launch_query_merge(slots, N, kmax, false, true, views(w), st);
    }
  }
  // finished requests go straight to mapped host memory (plain stores; the
  // count is a device atomic, copied back): one synchronisation per round
  fill_i32(n_done.get(), 1, 0, st);
  launch_collect_done(slots, N, kmax, ix->rowid.get(), views(w), state.get(), h_done_slot.dev, h_done_ids.dev,
                      h_done_d.dev, n_done.get(), st);
  d2h(h_ndone.p, n_done.get(), 1, st);
  HIP_OK(hipStreamSynchronize(st));
  const int nd = h_ndone.p[0];
  const double t = now_s();
  {
    std::lock_guard<std::mutex> lk(mu);
    ++rounds;
    active_sum += n_active;
    max_active = std::max(max_active, n_active);
    for (int j = 0; j < nd; ++j) {
      const int s = h_done_slot.p[j];
      auto it = reqs.find(slot_ticket[s]);
      if (it != reqs.end()) {
        Request &r = it->second;
        r.ids.assign(h_done_ids.p + static_cast<size_t>(j) * kmax, h_done_ids.p + static_cast<size_t>(j + 1) * kmax);
        r.d.assign(h_done_d.p + static_cast<size_t>(j) * kmax, h_done_d.p + static_cast<size_t>(j + 1) * kmax);
        r.t_done = t;
        r.state = 2;
        ++completed;
      }
      slot_ticket[s] = 0;
      free_slots.push_back(s);
    }
  }
  n_active -= nd;
  if (nd > 0) cv_done.notify_all();
}

void leafi_server::run() {
  int rc = guarded([&] {
    INDEX_ALLOC_SCOPE(ix);
    HIP_OK(hipSetDevice(ix->device));
    int n_active = 0;
    const int m = ix->m;
    for (;;) {
      int n_new = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        if (n_active == 0 && queue.empty() && !stop)
          cv_work.wait_for(lk, std::chrono::milliseconds(50), [&] { return stop || !queue.empty(); });
        if (stop && n_active == 0 && queue.empty()) break;
        while (!queue.empty() && !free_slots.empty()) {
          uint64_t tk = queue.front();
          queue.pop_front();
          auto it = reqs.find(tk);
          if (it == reqs.end()) continue;
          const int s = free_slots.back();
          free_slots.pop_back();
          slot_ticket[s] = tk;
          Request &r = it->second;
          r.state = 1;
          std::memcpy(h_raw.p + static_cast<size_t>(n_new) * m, r.q.data(), m * sizeof(float));
          h_slots.p[n_new] = s;
          h_k.p[n_new] = r.k;
          h_t.p[n_new] = r.target;
          ++n_new;
        }
      }
      if (n_new == 0 && n_active == 0) continue;
      engine_round(n_new, n_active);
    }
  });
  if (rc != LEAFI_OK) {
    std::lock_guard<std::mutex> lk(mu);
    worker_error = g_last_error;
    stop = true;
    cv_done.notify_all();
  }
}

leafi_server::~leafi_server() {
  {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;
  }
  cv_work.notify_all();
  if (worker.joinable()) worker.join();
  if (st) (void)hipStreamDestroy(st);
}

namespace {

int submit_at(leafi_server *sv, const float *q, int32_t k, float target, double t_arrive, uint64_t *ticket) {
  return guarded([&] {
    LEAFI_CHECK_ARG(sv && q && ticket, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!sv->worker_error.empty()) fail(LEAFI_EINTERNAL, "serving engine stopped: " + sv->worker_error);
    if (static_cast<int>(sv->queue.size()) >= sv->o.queue_capacity)
      fail(LEAFI_EAGAIN, "request queue full; retry later");
    Request r;
    r.q.assign(q, q + sv->ix->m);
    r.k = std::min(std::max(k, 1), sv->o.k_max);
    r.target = target;
    r.t_arrive = t_arrive;
    const uint64_t tk = sv->next_ticket++;
    sv->reqs.emplace(tk, std::move(r));
    sv->queue.push_back(tk);
    *ticket = tk;
  });
}

}  // namespace

extern "C" {

void leafi_default_server_opts(leafi_server_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_slots = 1024;
  o->k_max = 1;
  o->scan = LEAFI_SCAN_BF16;
  o->use_filters = 1;
  o->n_schedule = 2;
  o->schedule[0] = 1;
  o->schedule[1] = 0;
  o->queue_capacity = 1 << 20;
  o->mem_budget = int64_t(4) << 30;
}

int leafi_server_create(leafi_index *ix, const leafi_server_opts *o, leafi_server **out) {
  return guarded([&] {
    INDEX_ALLOC_SCOPE(ix);
    require_built(ix);
    LEAFI_CHECK_ARG(o != nullptr && out != nullptr, "NULL argument");
    LEAFI_CHECK_ARG(o->k_max >= 1 && o->k_max <= 256, "k_max must be in [1, 256]");
    LEAFI_CHECK_ARG(o->scan == LEAFI_SCAN_BF16 || o->scan == LEAFI_SCAN_FP32, "unknown scan kind");
    LEAFI_CHECK_ARG(o->scan != LEAFI_SCAN_BF16 || ix->m <= 256, "the bf16 scan supports m <= 256");
    LEAFI_CHECK_ARG(o->n_schedule >= 1 && o->n_schedule <= 8, "n_schedule must be in [1, 8]");
    for (int i = 0; i < o->n_schedule; ++i) LEAFI_CHECK_ARG(o->schedule[i] >= 0, "schedule entries must be >= 0");
    LEAFI_CHECK_ARG(o->max_slots >= 0 && o->queue_capacity >= 1 && o->mem_budget >= 0, "bad capacities");
    auto sv = std::make_unique<leafi_server>();
    sv->ix = ix;
    sv->o = *o;
    sv->use_f = o->use_filters != 0 && ix->filt.F > 0 && ix->cal.pairs() > 0;
    sv->kprime = default_kprime(o->k_max, o->scan == LEAFI_SCAN_BF16);
    sv->sched.n = o->n_schedule;
    for (int i = 0; i < 8; ++i) sv->sched.r[i] = i < o->n_schedule ? o->schedule[i] : 0;
    // admission by memory: per-slot device state (query copies, bounds, visit
    // order, item lists, filter predictions and pairs, results) and its share
    // of a round's item and candidate buffers
    const double N = ix->N, m = ix->m, F = std::max(ix->filt.F, 1), k = o->k_max;
    const double per_slot = m * 10.0 + ix->S * 8.0 + N * 16.0 + F * 8.0 + k * 12.0 + 64.0 +
                            N * (k * 12.0 + 32.0) + N * ix->max_chunks_for(kChunkRows) * 4.0 * sv->kprime * 8.0 / 16.0;
    int by_mem = o->mem_budget > 0 ? static_cast<int>(static_cast<double>(o->mem_budget) / per_slot) : (1 << 30);
    int slots = o->max_slots > 0 ? std::min(o->max_slots, by_mem) : by_mem;
    LEAFI_CHECK_ARG(slots >= 1, "memory budget admits no query");
    slots = std::min(slots, 1 << 20);
    sv->slots = slots;
    ensure_queries(ix, slots, o->k_max);
    Workspace &w = ix->ws;
    if (sv->use_f) {
      w.plist.reserve(static_cast<size_t>(ix->filt.F) * slots);
      w.pcnt.reserve(ix->filt.F);
      w.ptile.reserve(ix->filt.F + 1);
    }
    sv->state.alloc(slots);
    sv->qround.alloc(slots);
    sv->new_slots.alloc(slots);
    sv->new_k.alloc(slots);
    sv->new_t.alloc(slots);
    sv->new_raw.alloc(static_cast<size_t>(slots) * ix->m);
    {
      // the rescan pass can run without read-back if both passes' buffers fit
      const int64_t bnd = sv->round_bound();
      const bool bf = o->scan == LEAFI_SCAN_BF16;
      sv->device_rounds =
          round_bytes_bound(ix, slots, bnd, bf, sv->kprime, o->k_max) <= kPlannedLimit &&
          round_bytes_bound(ix, slots, bnd, false, default_kprime(o->k_max, false), o->k_max) <= kPlannedLimit;
    }
    sv->h_raw.alloc(static_cast<size_t>(slots) * ix->m);
    sv->h_slots.alloc(slots);
    sv->h_k.alloc(slots);
    sv->h_t.alloc(slots);
    sv->h_done_slot.alloc(slots, true);
    sv->h_ndone.alloc(1);
    sv->n_done.alloc(1);
    sv->h_done_ids.alloc(static_cast<size_t>(slots) * o->k_max, true);
    sv->h_done_d.alloc(static_cast<size_t>(slots) * o->k_max, true);
    HIP_OK(hipStreamCreate(&sv->st));
    hipLaunchKernelGGL(k_slot_reset_all, dim3(ceil_div(slots, 256)), dim3(256), 0, sv->st, static_cast<int64_t>(slots),
                       ix->N, views(w), sv->state.get(), sv->qround.get());
    LAUNCH_OK("slot_reset_all");
    HIP_OK(hipStreamSynchronize(sv->st));
    sv->slot_ticket.assign(slots, 0);
    sv->free_slots.reserve(slots);
    for (int s = slots - 1; s >= 0; --s) sv->free_slots.push_back(s);
    leafi_server *p = sv.release();
    p->worker = std::thread([p] { p->run(); });
    *out = p;
  });
}

void leafi_server_destroy(leafi_server *sv) { delete sv; }

int leafi_server_info(const leafi_server *sv, int32_t *max_slots) {
  return guarded([&] {
    LEAFI_CHECK_ARG(sv && max_slots, "NULL argument");
    *max_slots = sv->slots;
  });
}

int leafi_server_submit(leafi_server *sv, const float *query, int32_t k, float target, uint64_t *ticket) {
  int rc = submit_at(sv, query, k, target, now_s(), ticket);
  if (rc == LEAFI_OK) sv->cv_work.notify_one();
  return rc;
}

int leafi_server_poll(leafi_server *sv, uint64_t ticket, int64_t *ids, float *dists, double *latency_ms,
                      int32_t *done) {
  return guarded([&] {
    LEAFI_CHECK_ARG(sv && done, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    LEAFI_CHECK_ARG(it != sv->reqs.end(), "unknown ticket");
    if (!sv->worker_error.empty()) fail(LEAFI_EINTERNAL, "serving engine stopped: " + sv->worker_error);
    Request &r = it->second;
    *done = r.state == 2 ? 1 : 0;
    if (r.state == 2) {
      if (ids) std::copy(r.ids.begin(), r.ids.end(), ids);
      if (dists) std::copy(r.d.begin(), r.d.end(), dists);
      if (latency_ms) *latency_ms = 1e3 * (r.t_done - r.t_arrive);
      sv->reqs.erase(it);
    }
  });
}

int leafi_server_replay(leafi_server *sv, const float *queries, int64_t n, const double *arrival_s, const int32_t *ks,
                        const float *targets, int64_t *ids, float *dists, double *latency_ms,
                        leafi_server_report *rep) {
  return guarded([&] {
    LEAFI_CHECK_ARG(sv && (n == 0 || (queries && arrival_s && ks && targets && ids && dists && latency_ms)),
                    "NULL argument");
    const int m = sv->ix->m, kmax = sv->o.k_max;
    std::vector<uint64_t> tickets(n);
    int64_t r0, c0;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      r0 = sv->rounds;
      c0 = sv->completed;
      sv->active_sum = 0.0;
      sv->max_active = 0;
    }
    const double t0 = now_s();
    for (int64_t i = 0; i < n; ++i) {
      const double ta = t0 + arrival_s[i];
      for (;;) {
        const double dt = ta - now_s();
        if (dt <= 0) break;
        if (dt > 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(dt - 1e-4));
      }
      int rc;
      while ((rc = submit_at(sv, queries + i * m, ks[i], targets[i], ta, &tickets[i])) == LEAFI_EAGAIN)
        std::this_thread::sleep_for(std::chrono::microseconds(50));
      if (rc != LEAFI_OK) fail(rc, g_last_error);
      sv->cv_work.notify_one();
    }
    for (int64_t i = 0; i < n; ++i) {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_done.wait(lk, [&] {
        auto it = sv->reqs.find(tickets[i]);
        return !sv->worker_error.empty() || (it != sv->reqs.end() && it->second.state == 2);
      });
      if (!sv->worker_error.empty()) fail(LEAFI_EINTERNAL, "serving engine stopped: " + sv->worker_error);
      auto it = sv->reqs.find(tickets[i]);
      Request &r = it->second;
      std::copy(r.ids.begin(), r.ids.end(), ids + i * kmax);
      std::copy(r.d.begin(), r.d.end(), dists + i * kmax);
      latency_ms[i] = 1e3 * (r.t_done - r.t_arrive);
      sv->reqs.erase(it);
    }
    const double t1 = now_s();
    if (rep) {
      std::lock_guard<std::mutex> lk(sv->mu);
      std::memset(rep, 0, sizeof(*rep));
      rep->completed = sv->completed - c0;
      rep->rounds = sv->rounds - r0;
      rep->wall_s = t1 - t0;
      rep->mean_active = rep->rounds > 0 ? sv->active_sum / static_cast<double>(rep->rounds) : 0.0;
      rep->max_active = sv->max_active;
    }
  });
}

}  // extern "C"
