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

// Owning device allocation (hipMalloc / hipFree).
template <typename T>
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) { release(); p_ = o.p_; n_ = o.n_; o.p_ = nullptr; o.n_ = 0; }
    return *this;
  }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    HIP_OK(hipMalloc(reinterpret_cast<void **>(&p_), n * sizeof(T)));
    n_ = n;
  }
  // Grow-only reallocation (contents not kept).
  void reserve(size_t n) { if (n > n_) alloc(n); }
  void release() {
    if (p_) (void)hipFree(p_);
    p_ = nullptr;
    n_ = 0;
  }
  T *get() const { return p_; }
  size_t size() const { return n_; }
  size_t bytes() const { return n_ * sizeof(T); }

 private:
  T *p_ = nullptr;
  size_t n_ = 0;
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
