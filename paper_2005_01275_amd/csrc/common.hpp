// Shared infrastructure of the spfas library: error propagation, device
// buffers, launch helpers.  Every HIP call is checked; failures become
// spfas::Error exceptions that the C ABI layer turns into status codes.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdlib>
#include <type_traits>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/spfas.h"
#include "amg_host.hpp"

namespace spfas {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

inline void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e != hipSuccess) {
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s failed at %s:%d: %s", what, file, line, hipGetErrorString(e));
    fail(e == hipErrorOutOfMemory ? SPFAS_ERR_OOM : SPFAS_ERR_DEVICE, buf);
  }
}
#define HIPCHECK(x) ::spfas::hip_check((x), #x, __FILE__, __LINE__)
#define LAUNCHCHECK() ::spfas::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

// Where a hierarchy's device memory comes from: the caller's allocator
// callbacks (spfas_allocator), or hipMalloc / hipFree when none was given.
// Bytes are counted either way.
struct AllocCtx {
  spfas_allocator user{};              // user.alloc == nullptr: hipMalloc / hipFree
  hipStream_t stream = nullptr;        // stream handed to the callbacks
  std::atomic<int64_t> bytes{0};       // allocated now
  std::atomic<int64_t> peak{0};
};

// Allocation context of the calling thread: device buffers allocated while
// an AllocScope is active come from (and return to) its context.
inline thread_local AllocCtx* tl_alloc = nullptr;
struct AllocScope {
  AllocCtx* prev;
  explicit AllocScope(AllocCtx* c) : prev(tl_alloc) { tl_alloc = c; }
  ~AllocScope() { tl_alloc = prev; }
  AllocScope(const AllocScope&) = delete;
  AllocScope& operator=(const AllocScope&) = delete;
};

inline void* dev_alloc(AllocCtx* c, size_t bytes) {
  void* p = nullptr;
  if (c && c->user.alloc) {
    p = c->user.alloc(bytes, (void*)c->stream, c->user.ctx);
    if (!p) fail(SPFAS_ERR_OOM, "the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes");
  } else {
    HIPCHECK(hipMalloc(&p, bytes));
  }
  if (c) {
    const int64_t now = c->bytes.fetch_add((int64_t)bytes) + (int64_t)bytes;
    int64_t pk = c->peak.load();
    while (now > pk && !c->peak.compare_exchange_weak(pk, now)) {
    }
  }
  return p;
}

inline void dev_free(AllocCtx* c, void* p, size_t bytes) noexcept {
  if (!p) return;
  if (c && c->user.alloc) {
    if (c->user.free) c->user.free(p, bytes, (void*)c->stream, c->user.ctx);
  } else {
    (void)hipFree(p);
  }
  if (c) c->bytes.fetch_sub((int64_t)bytes);
}

// SPFAS_TRACE=1 prints setup timings and solver events to stderr; 2 also
// times the AMG levels with events.
inline int trace_level() {
  static const int lv = [] {
    const char* e = std::getenv("SPFAS_TRACE");
    return (e && e[0] && e[0] != '0') ? std::max(1, std::atoi(e)) : 0;
  }();
  return lv;
}

// f(lo, hi) on contiguous, ordered ranges of [0, n), one host thread each
// (at most host_thread_limit(), and at most one per kParGrain units of `work`, which defaults
// to n: small inputs run inline, without thread start-up); every range
// writes only its own part of the output.
constexpr int64_t kParGrain = 16384;
template <class F>
void parallel_ranges(int64_t n, F&& f, int64_t work = -1) {
  const int64_t w = work < 0 ? n : work;
  const int64_t nth = std::max<int64_t>(1, std::min<int64_t>({(int64_t)host_thread_limit(), n, w / kParGrain}));
  if (nth <= 1) {
    f((int64_t)0, n);
    return;
  }
  const int64_t per = (n + nth - 1) / nth;
  std::vector<std::thread> th;
  for (int64_t t = 0; t < nth; ++t) {
    const int64_t lo = std::min(n, t * per), hi = std::min(n, lo + per);
    th.emplace_back([&f, lo, hi] { f(lo, hi); });
  }
  for (auto& x : th) x.join();
}

inline double wall_ms() {
  return 1e3 * std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

inline bool poison_on() {
  static const bool on = [] {
    const char* e = std::getenv("SPFAS_POISON");
    return e && e[0] == '1';
  }();
  return on;
}

// Typed device buffer; freed with the owning object, through the allocation
// context that was active when it was allocated.
template <class T>
struct DVec {
  T* p = nullptr;
  size_t n = 0;
  AllocCtx* ctx = nullptr;
  DVec() = default;
  DVec(const DVec&) = delete;
  DVec& operator=(const DVec&) = delete;
  DVec(DVec&& o) noexcept : p(o.p), n(o.n), ctx(o.ctx) { o.p = nullptr; o.n = 0; }
  DVec& operator=(DVec&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; ctx = o.ctx; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DVec() { release(); }
  void release() {
    if (p) dev_free(ctx, p, n * sizeof(T));
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    release();
    ctx = tl_alloc;
    if (count) p = static_cast<T*>(dev_alloc(ctx, count * sizeof(T)));
    n = count;
    // SPFAS_POISON=1 (diagnostics): floating-point buffers start as NaN, so
    // a read before the first write shows up in the results
    if constexpr (std::is_floating_point<T>::value || std::is_same<T, _Float16>::value)
      if (count && poison_on()) HIPCHECK(hipMemset(p, 0xFF, count * sizeof(T)));
  }
  void zero(hipStream_t s) {
    if (n) HIPCHECK(hipMemsetAsync(p, 0, n * sizeof(T), s));
  }
  // Uploads complete before returning: sources are often short-lived host
  // temporaries in pageable memory.
  void upload(const std::vector<T>& v, hipStream_t s) {
    alloc(v.size());
    if (n) {
      HIPCHECK(hipMemcpyAsync(p, v.data(), n * sizeof(T), hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));
    }
  }
  void upload(const T* src, size_t count, hipStream_t s) {
    alloc(count);
    if (n) {
      HIPCHECK(hipMemcpyAsync(p, src, n * sizeof(T), hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));
    }
  }
  std::vector<T> download(hipStream_t s) const {
    std::vector<T> v(n);
    if (n) {
      HIPCHECK(hipMemcpyAsync(v.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
    }
    return v;
  }
};

inline unsigned grid_for(size_t n, unsigned block) {
  size_t g = (n + block - 1) / block;
  if (g == 0) g = 1;
  return (unsigned)g;
}

// Host-side bounds assertions used before launches.
inline void require(bool ok, const char* msg) {
  if (!ok) fail(SPFAS_ERR_INVALID, msg);
}

}  // namespace spfas
