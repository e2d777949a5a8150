// Optional per-kernel-class timing with HIP events on the launch stream.
// When a plan has profiling enabled, every launch of a timed class records an
// event pair around it and its algorithmic flop count; the totals are read
// back by nudft2_get_info.
#pragma once

#include "common.h"

namespace nd {

enum KClass { KC_APPLY = 0, KC_GEMM32 = 1, KC_GEMM64 = 2, KC_QRPANEL = 3, KC_COUNT = 4 };

struct Profiler {
  struct Rec {
    hipEvent_t a, b;
    int cls;
    double flops;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double ms[KC_COUNT] = {0, 0, 0, 0};
  double flops[KC_COUNT] = {0, 0, 0, 0};
  int64_t launches[KC_COUNT] = {0, 0, 0, 0};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    ND_HIP(hipEventCreate(&e));
    return e;
  }
  void begin(hipStream_t s, int cls, double fl, hipEvent_t& a) {
    a = get();
    ND_HIP(hipEventRecord(a, s));
    (void)cls;
    (void)fl;
  }
  void end(hipStream_t s, int cls, double fl, hipEvent_t a) {
    hipEvent_t b = get();
    ND_HIP(hipEventRecord(b, s));
    recs.push_back({a, b, cls, fl});
  }
  // fold recorded pairs into the totals (synchronises on the last event)
  void collect() {
    for (auto& r : recs) {
      ND_HIP(hipEventSynchronize(r.b));
      float t = 0;
      ND_HIP(hipEventElapsedTime(&t, r.a, r.b));
      ms[r.cls] += t;
      flops[r.cls] += r.flops;
      launches[r.cls] += 1;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
  }
  void reset() {
    collect();
    for (int i = 0; i < KC_COUNT; ++i) {
      ms[i] = flops[i] = 0;
      launches[i] = 0;
    }
  }
  ~Profiler() {
    for (auto& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// Profiler of the plan whose entry point is running on this thread (or null).
extern thread_local Profiler* g_prof;

struct ProfScope {
  hipStream_t s;
  int cls;
  double fl;
  hipEvent_t a = nullptr;
  ProfScope(hipStream_t st, int c, double f) : s(st), cls(c), fl(f) {
    if (g_prof) g_prof->begin(s, cls, fl, a);
  }
  ~ProfScope() {
    if (g_prof && a) g_prof->end(s, cls, fl, a);
  }
};

}  // namespace nd
