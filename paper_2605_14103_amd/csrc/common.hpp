// Host-side plumbing shared by the library's translation units: status and
// error text, HIP error checks, RAII device buffers and the context.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <stdexcept>
#include <string>
#include <vector>

#include "pfx.h"

namespace pfx {

// Every failure inside the library is raised as PfError and converted to a
// pf_status (plus the thread's last-error text) at the C ABI.
struct PfError : std::runtime_error {
  pf_status status;
  PfError(pf_status s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

[[noreturn]] inline void fail(pf_status s, const std::string& msg) { throw PfError(s, msg); }

inline void require(bool ok, const std::string& msg) {
  if (!ok) fail(PF_INVALID_ARG, msg);
}

#define PFX_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      ::pfx::fail(PF_HIP_ERROR, std::string(#call) + ": " + hipGetErrorString(e_));        \
  } while (0)

void set_last_error(const std::string& msg);

struct Context;

// Device allocation charged against the owning context's budget.
class DeviceBuffer {
 public:
  DeviceBuffer() = default;
  DeviceBuffer(Context* ctx, size_t bytes) { allocate(ctx, bytes); }
  ~DeviceBuffer() { release(); }
  DeviceBuffer(const DeviceBuffer&) = delete;
  DeviceBuffer& operator=(const DeviceBuffer&) = delete;
  DeviceBuffer(DeviceBuffer&& o) noexcept { *this = std::move(o); }
  DeviceBuffer& operator=(DeviceBuffer&& o) noexcept {
    if (this != &o) {
      release();
      ctx_ = o.ctx_;
      ptr_ = o.ptr_;
      bytes_ = o.bytes_;
      o.ctx_ = nullptr;
      o.ptr_ = nullptr;
      o.bytes_ = 0;
    }
    return *this;
  }
  void allocate(Context* ctx, size_t bytes);
  // Grow-only: keeps the current allocation when it is already large enough.
  void ensure(Context* ctx, size_t bytes) {
    if (bytes > bytes_) {
      release();
      allocate(ctx, bytes);
    }
  }
  void release();
  template <typename T>
  T* as() const { return static_cast<T*>(ptr_); }
  size_t bytes() const { return bytes_; }

 private:
  Context* ctx_ = nullptr;
  void* ptr_ = nullptr;
  size_t bytes_ = 0;
};

// Upload a host vector into a fresh device buffer.
template <typename T>
DeviceBuffer upload(Context* ctx, const std::vector<T>& v) {
  DeviceBuffer b(ctx, std::max<size_t>(v.size(), 1) * sizeof(T));
  if (!v.empty()) PFX_HIP(hipMemcpy(b.as<void>(), v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return b;
}

// Orders the calls that share one network's workspace.  A call holds `mu` on
// the host for as long as it enqueues work; on the device its stream first
// waits for the previous call's work, which may sit on another stream, and
// then records its own completion, so two calls enqueued on different streams
// never run over the same workspace at once.  A workspace is reallocated only
// after the host has waited for the previous call's work.
struct CallOrder {
  std::mutex mu;
  hipEvent_t ev = nullptr;
  bool pending = false;
  CallOrder() = default;
  CallOrder(const CallOrder&) = delete;
  CallOrder& operator=(const CallOrder&) = delete;
  ~CallOrder() {
    if (ev) (void)hipEventDestroy(ev);
  }
  void begin(hipStream_t s) {
    if (!ev) PFX_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    if (pending) PFX_HIP(hipStreamWaitEvent(s, ev, 0));
  }
  void end(hipStream_t s) {
    PFX_HIP(hipEventRecord(ev, s));
    pending = true;
  }
  void drain() {
    if (pending) PFX_HIP(hipEventSynchronize(ev));
  }
  void grow(DeviceBuffer& b, Context* ctx, size_t bytes) {
    if (bytes > b.bytes()) {
      drain();
      b.ensure(ctx, bytes);
    }
  }
};

struct Context {
  int device = 0;
  uint64_t budget = 0;       // 0 = unbounded
  uint64_t held = 0;         // bytes currently allocated through this context
  std::mutex mu;
  int cu_count = 0;
  std::set<void*> tx_nets, dist_nets, engines;   // owned objects, destroyed with the context
};

// Take the device address of the no-allocation entry point's fixed scratch
// array on `device` (current), once per device (noalloc.hip).
void scratch_init(int device);

// Make the context's device current for the calling thread.
inline void activate(Context* ctx) { PFX_HIP(hipSetDevice(ctx->device)); }

pf_opts resolve_opts(const pf_opts* o);

// Live-handle registry: handles are checked before use so a null or destroyed
// handle yields PF_BAD_HANDLE instead of a crash.
struct Registry {
  std::mutex mu;
  std::set<const void*> live;
  void add(const void* p) {
    std::lock_guard<std::mutex> lk(mu);
    live.insert(p);
  }
  void remove(const void* p) {
    std::lock_guard<std::mutex> lk(mu);
    live.erase(p);
  }
  bool has(const void* p) {
    std::lock_guard<std::mutex> lk(mu);
    return p && live.count(p);
  }
};
Registry& registry();

inline void check_handle(const void* p, const char* what) {
  if (!registry().has(p)) fail(PF_BAD_HANDLE, std::string("invalid or destroyed ") + what + " handle");
}

// Run f, converting exceptions into a pf_status and the thread's last error.
template <typename F>
pf_status guarded(F&& f) {
  try {
    f();
    return PF_OK;
  } catch (const PfError& e) {
    set_last_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return PF_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return PF_INVALID_ARG;
  }
}

// CSR output of the admittance builders (columns sorted, duplicates summed).
void emit_csr(int n, const std::vector<std::map<int, std::complex<double>>>& rows, int cap,
              int32_t* row_ptr, int32_t* col_idx, double* y_re, double* y_im, int32_t* nnz_out);

}  // namespace pfx
