// Internal helpers shared by the host runtime and the kernels of libleafi.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/leafi.h"

namespace leafi {

// Error carried to the C boundary, where it becomes a LEAFI_E* code.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &msg) : std::runtime_error(msg), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string &msg) { throw Error(code, msg); }

#define LEAFI_CHECK_ARG(cond, msg)                                              \
  do {                                                                          \
    if (!(cond)) ::leafi::fail(LEAFI_EINVAL, std::string(__func__) + ": " + (msg)); \
  } while (0)

#define HIP_OK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) {                                                                \
      if (e_ == hipErrorOutOfMemory)                                                       \
        ::leafi::fail(LEAFI_ENOMEM, std::string("out of device memory: ") + #expr);       \
      ::leafi::fail(LEAFI_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    }                                                                                      \
  } while (0)

// Check the launch just enqueued.
#define LAUNCH_OK(name) HIP_OK(hipGetLastError())

// A kernel that may be launched with more than 64 KiB of dynamic LDS: its
// limit is raised to `lds` when a launch needs more than any before it, and
// otherwise left alone (so a sequence being captured into a graph, which
// repeats launches made eagerly before, makes no such call).
void allow_lds(const void *kernel, size_t lds);

// Where device memory comes from.  Allocations of an index handle go through
// the caller's allocator when leafi_create was given one (else hipMalloc);
// the no-allocation search carves its buffers out of a fixed device array
// instead (an arena: nothing is freed, the arena is rewound per call).
struct AllocFns {
  leafi_alloc_fn alloc = nullptr;
  leafi_free_fn free = nullptr;
  void *ctx = nullptr;
};
struct Arena {
  char *base = nullptr;
  size_t cap = 0;
  size_t used = 0;
};
// In effect on the calling thread (set by the entry points, see AllocScope).
extern thread_local const AllocFns *t_alloc;
extern thread_local Arena *t_arena;

// Allocate bytes of device memory from the thread's arena, the handle's
// allocator or hipMalloc; `how` records which (for the matching free).
void *dev_alloc(size_t bytes, AllocFns *how, bool *from_arena);
// Release memory from dev_alloc (arena memory is never released one by one).
void dev_free(void *p, const AllocFns &how, bool from_arena) noexcept;

// Makes `fns` the calling thread's allocator until the scope ends.
struct AllocScope {
  const AllocFns *prev;
  explicit AllocScope(const AllocFns *fns) : prev(t_alloc) { t_alloc = fns; }
  ~AllocScope() { t_alloc = prev; }
  AllocScope(const AllocScope &) = delete;
  AllocScope &operator=(const AllocScope &) = delete;
};

// Makes `a` the calling thread's arena until the scope ends.
struct ArenaScope {
  Arena *prev;
  explicit ArenaScope(Arena *a) : prev(t_arena) { t_arena = a; }
  ~ArenaScope() { t_arena = prev; }
  ArenaScope(const ArenaScope &) = delete;
  ArenaScope &operator=(const ArenaScope &) = delete;
};

// Owning device allocation (see dev_alloc for where the bytes come from).
template <typename T>
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p_(o.p_), n_(o.n_), how_(o.how_), arena_(o.arena_) { o.p_ = nullptr; o.n_ = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p_ = o.p_;
      n_ = o.n_;
      how_ = o.how_;
      arena_ = o.arena_;
      o.p_ = nullptr;
      o.n_ = 0;
    }
    return *this;
  }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    p_ = static_cast<T *>(dev_alloc(n * sizeof(T), &how_, &arena_));
    n_ = n;
  }
  // Grow-only reallocation (contents not kept).
  void reserve(size_t n) { if (n > n_) alloc(n); }
  void release() {
    if (p_) dev_free(p_, how_, arena_);
    p_ = nullptr;
    n_ = 0;
  }
  T *get() const { return p_; }
  size_t size() const { return n_; }
  size_t bytes() const { return n_ * sizeof(T); }

 private:
  T *p_ = nullptr;
  size_t n_ = 0;
  AllocFns how_;
  bool arena_ = false;
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Rows of each leaf are padded to a multiple of this in the leaf store (an
// even number of the scan's 64-row blocks, so its unrolled loop has no tail).
constexpr int kRowAlign = 128;
// Rows of one scan tile of the BF16 scan (multiple of kRowAlign); passes may
// use any of the kChunkSizes sizes kRowAlign << j.
constexpr int kChunkRows = 1024;
constexpr int kChunkSizes = 6;  // 128 .. 4096 rows
inline int chunk_log(int chunk) {
  int j = 0;
  while ((kRowAlign << j) < chunk && j < kChunkSizes - 1) ++j;
  return j;
}
// Relative slack applied to tau before a summary bound may prune (covers the
// fp32 evaluation of the bound).
constexpr float kLbSlack = 1e-5f;

}  // namespace leafi
