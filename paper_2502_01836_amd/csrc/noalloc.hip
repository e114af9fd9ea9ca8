// The batch search for callers that cannot allocate device memory: every
// per-batch buffer is carved out of one fixed device array per GPU instead of
// being allocated.  The launch sequence is the planned one of
// leafi_search_knn, so results are identical to it.
#include <mutex>
#include <utility>

#include "engine.h"

// Scratch area of the no-allocation search, one per GPU, held until the
// process ends.  Host code never takes this name as an address: the address
// on each device comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[LEAFI_NOALLOC_SCRATCH_BYTES];

namespace leafi {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch[kMaxDevices] = {};

// This device's scratch address (looked up once per device, with the device current).
char *scratch_ptr(int dev) {
  LEAFI_CHECK_ARG(dev >= 0 && dev < kMaxDevices, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) fail(LEAFI_EHIP, "hipGetSymbolAddress returned no address for the scratch area");
    g_scratch[dev] = static_cast<char *>(p);
  }
  return g_scratch[dev];
}

// Puts the handle's own workspace back when the call ends (also on error).
struct WorkspaceSwap {
  leafi_index *ix;
  Workspace own;
  explicit WorkspaceSwap(leafi_index *i) : ix(i) { std::swap(own, ix->ws); }
  ~WorkspaceSwap() { std::swap(own, ix->ws); }
};

}  // namespace
}  // namespace leafi

using namespace leafi;

extern "C" int leafi_search_knn_noalloc(leafi_index *ix, const float *queries, int64_t nq, const int32_t *k_dev,
                                        const float *t_dev, const leafi_search_opts *o, int64_t *ids, float *dists,
                                        void *stream) {
  return guarded([&] {
    require_built(ix);
    check_queries(ix, queries, nq);
    SearchPlan p = make_plan(ix, o);
    LEAFI_CHECK_ARG(p.bf16, "the no-allocation search runs the BF16 scan");
    LEAFI_CHECK_ARG((o->flags & LEAFI_SEARCH_HOST_ROUNDS) == 0, "the no-allocation search has no host-driven rounds");
    if (nq == 0) return;
    LEAFI_CHECK_ARG(k_dev && t_dev && ids && dists, "NULL k, target or output pointer");
    LEAFI_CHECK_ARG(can_plan(ix, nq, p),
                    "the batch does not run as a planned launch sequence (its schedule needs a 0 within 8 rounds)");
    LEAFI_CHECK_ARG(!plan_checked(ix, nq, p),
                    "the batch's worst case exceeds the planned buffer limit (a capacity-checked plan may have to "
                    "run again with host rounds, which allocate); pass fewer queries per call");
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    LEAFI_CHECK_ARG(dev == ix->device, "the current device is not the index's device");
    char *base = scratch_ptr(dev);
    const bool use_f = p.filters && ix->filt.F > 0 && ix->cal.pairs() > 0;
    WorkspaceSwap swap(ix);  // the call works in a workspace of its own
    // size every buffer of the batch first (stand-in addresses, nothing touched) ...
    Arena measure;
    measure.cap = static_cast<size_t>(1) << 62;
    {
      ArenaScope a(&measure);
      prepare_planned(ix, nq, p, use_f);
    }
    ix->ws = Workspace();
    if (measure.used > LEAFI_NOALLOC_SCRATCH_BYTES)
      fail(LEAFI_EINVAL, "the batch needs " + std::to_string(measure.used) + " bytes of scratch, more than the " +
                             std::to_string(static_cast<size_t>(LEAFI_NOALLOC_SCRATCH_BYTES)) +
                             " bytes of the no-allocation search; pass fewer queries per call");
    // ... then carve them from the scratch area and enqueue the planned sequence
    // (query preparation zeroes the control words and counters a batch starts from)
    Arena area;
    area.base = base;
    area.cap = LEAFI_NOALLOC_SCRATCH_BYTES;
    ArenaScope a(&area);
    prepare_planned(ix, nq, p, use_f);
    enqueue_planned(ix, queries, nq, k_dev, t_dev, p, use_f, ids, dists, false, as_stream(stream));
  });
}
