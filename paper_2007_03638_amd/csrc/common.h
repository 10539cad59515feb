// Internal shared definitions: error handling, device buffers, the context object.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "mera.h"  // include/mera.h (on the include path)

namespace mera {

// Errors inside the library are C++ exceptions carrying a status; the C ABI converts them.
struct Error : std::runtime_error {
  mera_status status;
  Error(mera_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define MERA_HIP(call)                                                                               \
  do {                                                                                               \
    hipError_t e_ = (call);                                                                          \
    if (e_ != hipSuccess)                                                                            \
      throw ::mera::Error(MERA_EHIP, std::string(#call) + ": " + hipGetErrorString(e_) + " at " +   \
                                         __FILE__ + ":" + std::to_string(__LINE__));                 \
  } while (0)

#define MERA_CHECK(cond, status, msg)                            \
  do {                                                           \
    if (!(cond)) throw ::mera::Error((status), std::string(msg)); \
  } while (0)

// Owning device allocation.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : ptr(o.ptr), bytes(o.bytes) { o.ptr = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); ptr = o.ptr; bytes = o.bytes; o.ptr = nullptr; o.bytes = 0; }
    return *this;
  }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
      ptr = nullptr;
      (void)hipGetLastError();
      throw Error(MERA_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
  }
  // Grow-only reallocation; contents are not preserved.
  void ensure(size_t n) { if (n > bytes) alloc(n); }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  template <typename T> T* as() const { return static_cast<T*>(ptr); }
};

enum class Prec { F64 = 0, F32 = 1, BF16X3 = 2 };
inline size_t elem_bytes(Prec p) { return p == Prec::F64 ? 8 : 4; }

struct PlanCache;  // network.h
struct Batcher;    // network.h

// Per-launch timing of contraction kernels with HIP events on the context stream (profiling mode).
struct LaunchRecord {
  std::string kernel;
  hipEvent_t start, stop;
  double flops;
  double bytes;  // algorithmic: each operand and the result read or written once
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  double macs = 0.0;
  // Named grow-only scratch buffers (intermediates, partial sums), reused across calls.
  std::map<std::string, DevBuf> scratch;
  std::shared_ptr<PlanCache> plans;  // may be shared by the contexts of one server
  Batcher* batcher = nullptr;        // non-null: contraction programs go through the server's batcher
  DevBuf red;        // reduction partials (doubles)
  size_t inter_limit = (size_t)32 << 30;  // largest 7-leg intermediate built in one piece (bytes)
  bool profiling = false;
  int verbose = 0;  // > 0: Krylov solves report each restart on stderr
  std::vector<LaunchRecord> records;
  std::vector<hipEvent_t> event_pool;
  hipEvent_t take_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e;
    MERA_HIP(hipEventCreate(&e));
    return e;
  }

  Ctx();
  ~Ctx();
  void* buf(const std::string& name, size_t bytes) {
    DevBuf& b = scratch[name];
    b.ensure(bytes);
    return b.ptr;
  }
  void sync() { MERA_HIP(hipStreamSynchronize(stream)); }
};

// Scoped device selection.
struct DeviceGuard {
  int prev = 0;
  explicit DeviceGuard(int dev) {
    MERA_HIP(hipGetDevice(&prev));
    if (prev != dev) MERA_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

}  // namespace mera
