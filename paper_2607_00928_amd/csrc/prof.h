// Optional per-kernel-class timing with HIP events on the launch stream.
// When a plan has profiling enabled, every launch of a timed class records an
// event pair around it and its algorithmic flop count; the totals are read
// back by nudft2_get_info.
#pragma once

#include <cstdlib>

#include "common.h"

namespace nd {

// Timed kernel classes: the exact FP64 apply, the matrix-core GEMMs (tile,
// small-output and reduction kernels) in FP32 / FP64, the Householder panels,
// and the memory-bound skinny products (at most 8 columns) in FP32 / FP64.
enum KClass {
  KC_APPLY = 0, KC_GEMM32 = 1, KC_GEMM64 = 2, KC_QRPANEL = 3, KC_GEMV32 = 4, KC_GEMV64 = 5,
  KC_COUNT = 6
};

// Timing events are reused across plans through a process-wide cache with one
// list per device (an event belongs to the device current at its creation):
// a profiler takes its events from the cache and returns them once read, so
// profiled runs after the first create no events (creating one per launch had
// cost about 2% of an n512 factor + solve).
hipEvent_t event_cache_get(int dev);
void event_cache_put(int dev, hipEvent_t e);

// Step of the factorization or solve that issues the current launches
// (ProfSite below); written as the last column of the optional launch log.
enum PSite {
  PS_NONE = 0, PS_1D = 1, PS_FACESPLIT = 2, PS_S1_QR = 3, PS_S1_PROJ = 4, PS_S2_GRAM = 5,
  PS_S2_PCHOL = 6, PS_S2_ORTH = 7, PS_S2_UPDATE = 8, PS_URV_SIZERED = 9, PS_URV_VQR = 10,
  PS_URV_DQ = 11, PS_URV_PARTIAL = 12, PS_URV_MERGE = 13, PS_URV_ROOT = 14, PS_URV_INV = 15,
  PS_SOLVE = 16, PS_APPLY = 17
};
extern thread_local int g_prof_site;
struct ProfSite {
  int old;
  explicit ProfSite(int s) : old(g_prof_site) { g_prof_site = s; }
  ~ProfSite() { g_prof_site = old; }
};

struct Profiler {
  struct Rec {
    hipEvent_t a, b;
    int cls;
    double flops;
    int info[5];   // launch shape for the optional log: descriptors, max m, n, k, variant
    int site;      // PSite of the launch
  };
  std::vector<Rec> recs;
  int dev = -1;   // the plan's device, taken at the first event
  double ms[KC_COUNT] = {};
  double flops[KC_COUNT] = {};
  int64_t launches[KC_COUNT] = {};
  unsigned mask = (1u << KC_COUNT) - 1;   // classes that record events
  hipEvent_t get() {
    if (dev < 0) ND_HIP(hipGetDevice(&dev));
    return event_cache_get(dev);
  }
  void begin(hipStream_t s, int cls, double fl, hipEvent_t& a) {
    a = get();
    ND_HIP(hipEventRecord(a, s));
    (void)cls;
    (void)fl;
  }
  // a pair whose timestamps the dispatches record themselves
  void push(hipEvent_t a, hipEvent_t b, int cls, double fl, const int* info) {
    Rec r{a, b, cls, fl, {0, 0, 0, 0, 0}, g_prof_site};
    for (int i = 0; i < 5; ++i) r.info[i] = info[i];
    recs.push_back(r);
  }
  void end(hipStream_t s, int cls, double fl, hipEvent_t a, const int* info) {
    hipEvent_t b = get();
    ND_HIP(hipEventRecord(b, s));
    Rec r{a, b, cls, fl, {0, 0, 0, 0, 0}, g_prof_site};
    for (int i = 0; i < 5; ++i) r.info[i] = info[i];
    recs.push_back(r);
  }
  // fold recorded pairs into the totals (synchronises on the last event)
  void collect() {
    // NUDFT2_PROF_LOG=<file>: one line per timed launch (class, ms, flops,
    // shape, step)
    static const char* logname = std::getenv("NUDFT2_PROF_LOG");
    FILE* log = logname ? std::fopen(logname, "a") : nullptr;
    for (auto& r : recs) {
      ND_HIP(hipEventSynchronize(r.b));
      float t = 0;
      ND_HIP(hipEventElapsedTime(&t, r.a, r.b));
      if (log)
        std::fprintf(log, "%d %.6f %.6e %d %d %d %d %d %d\n", r.cls, t, r.flops, r.info[0],
                     r.info[1], r.info[2], r.info[3], r.info[4], r.site);
      ms[r.cls] += t;
      flops[r.cls] += r.flops;
      launches[r.cls] += 1;
      event_cache_put(dev, r.a);
      event_cache_put(dev, r.b);
    }
    if (log) std::fclose(log);
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
      event_cache_put(dev, r.a);
      event_cache_put(dev, r.b);
    }
  }
};

// Profiler of the plan whose entry point is running on this thread (or null).
extern thread_local Profiler* g_prof;

// Timing of the launches inside a scope.  ext = false: an event pair is
// recorded on the stream around them.  ext = true: nothing is queued for the
// timing; the scope's first kernel takes start() and its last kernel takes
// stop() at dispatch (hipExtLaunchKernelGGL), so the timestamps come with the
// dispatches themselves and the stream carries no extra packets.  Every ext
// scope must launch at least one kernel with each event.
struct ProfScope {
  hipStream_t s;
  int cls;
  double fl;
  bool ext;
  hipEvent_t a = nullptr, b = nullptr;
  int info[5] = {0, 0, 0, 0, 0};
  ProfScope(hipStream_t st, int c, double f, int nd = 0, int m = 0, int n = 0, int k = 0,
            int var = 0, bool ext_ = false)
      : s(st), cls(c), fl(f), ext(ext_), info{nd, m, n, k, var} {
    if (!g_prof || !(g_prof->mask >> cls & 1u)) return;
    if (ext) {
      a = g_prof->get();
      b = g_prof->get();
    } else {
      g_prof->begin(s, cls, fl, a);
    }
  }
  hipEvent_t start() const { return a; }
  hipEvent_t stop() const { return b; }
  ~ProfScope() {
    if (!g_prof || !a) return;
    if (ext) g_prof->push(a, b, cls, fl, info);
    else g_prof->end(s, cls, fl, a, info);
  }
};

}  // namespace nd
