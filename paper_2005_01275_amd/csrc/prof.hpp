// Kernel timing with HIP events recorded on the launching stream, for the
// measurement entry points (spfas_profile_*).  Disabled by default; when
// enabled, every instrumented launch is bracketed by two events taken from a
// pool, and the elapsed times are summed when the counters are read.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "common.hpp"

namespace spfas {

struct KernelProf {
  bool on = false;
  struct Rec {
    int id;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::vector<long long> launches;
  std::vector<double> ms, bytes;

  explicit KernelProf(int n_ids = SPFAS_PROF_COUNT) : launches(n_ids, 0), ms(n_ids, 0.0), bytes(n_ids, 0.0) {}
  ~KernelProf() {
    for (auto& r : pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    return e;
  }
  // brackets fn() (one kernel launch) when profiling is on
  template <class F>
  void run(int id, double algo_bytes, hipStream_t s, F&& fn) {
    if (!on) {
      fn();
      return;
    }
    Rec r{id, take(), take(), algo_bytes};
    HIPCHECK(hipEventRecord(r.a, s));
    fn();
    HIPCHECK(hipEventRecord(r.b, s));
    pending.push_back(r);
    if (pending.size() > 4096) collect();
  }
  void collect() {
    for (auto& r : pending) {
      HIPCHECK(hipEventSynchronize(r.b));
      float t = 0.f;
      HIPCHECK(hipEventElapsedTime(&t, r.a, r.b));
      launches[r.id]++;
      ms[r.id] += t;
      bytes[r.id] += r.bytes;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  void reset() {
    collect();
    std::fill(launches.begin(), launches.end(), 0);
    std::fill(ms.begin(), ms.end(), 0.0);
    std::fill(bytes.begin(), bytes.end(), 0.0);
  }
};

}  // namespace spfas
