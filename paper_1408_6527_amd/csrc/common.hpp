// Shared host/device helpers of the pfmm library: error handling, device buffers, small math.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/pfmm.h"

namespace pfmm {

// Internal exception carrying a status code; converted to a return value at the C boundary.
struct Error : public std::runtime_error {
  pfmm_status status;
  Error(pfmm_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define PFMM_HIP(call)                                                                      \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw ::pfmm::Error(e_ == hipErrorOutOfMemory ? PFMM_ERR_OOM : PFMM_ERR_HIP,          \
                          std::string(#call) + ": " + hipGetErrorString(e_));               \
  } while (0)

#define PFMM_LAUNCH_CHECK() PFMM_HIP(hipGetLastError())

// A device allocation that only grows.  Contents are not preserved across growth.
// `ptr` is the storage in use: normally the buffer's own allocation; borrow() points it at memory
// the buffer does not own (a region of the library's static scratch array) without releasing its
// own, and the next reserve() returns to the own allocation.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  void* own = nullptr;
  size_t own_bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (own) (void)hipFree(own);
    own = ptr = nullptr;
    own_bytes = bytes = 0;
  }
  void* reserve(size_t want) {
    ptr = own;
    bytes = own_bytes;
    if (want == 0) want = 256;
    if (want > bytes) {
      release();
      size_t b = want + want / 4;
      hipError_t e = hipMalloc(&own, b);
      if (e != hipSuccess) {
        own = nullptr;
        throw Error(PFMM_ERR_OOM, "device allocation of " + std::to_string(b) + " bytes failed");
      }
      ptr = own;
      own_bytes = bytes = b;
    }
    return ptr;
  }
  void borrow(void* p, size_t b) {
    ptr = p;
    bytes = b;
  }
  template <class T>
  T* as() const { return static_cast<T*>(ptr); }
};

// Carves consecutive 256-byte-aligned regions out of a fixed device range (the static scratch
// array); never allocates.  Asking for more than is left throws before anything uses the memory.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  void* take(size_t want, const char* what) {
    const size_t b = (want == 0 ? 256 : want + 255) / 256 * 256;
    if (used + b > cap)
      throw Error(PFMM_ERR_INVALID_ARG, std::string("workspace for this evaluation exceeds the scratch maximum of ") +
                                            std::to_string(cap) + " bytes (" + what + ": " + std::to_string(used) +
                                            " used, " + std::to_string(b) + " more needed)");
    void* p = base + used;
    used += b;
    return p;
  }
};

inline int ncoef(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
inline int round_up(int x, int m) { return (x + m - 1) / m * m; }
inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace pfmm
