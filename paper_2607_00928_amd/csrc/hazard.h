// Debug check for batched launches: no element written by one descriptor of a
// launch may be read or written by another descriptor (or read by the same
// descriptor) of that launch, because all tiles of a launch run concurrently.
// Enabled by the environment variable NUDFT2_CHECK_HAZARDS=1; a violation
// raises E_INTERNAL naming the launch and the two descriptors.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <string>
#include <vector>

#include "common.h"

namespace nd {

inline bool hazards_enabled() {
  static int on = [] {
    const char* e = std::getenv("NUDFT2_CHECK_HAZARDS");
    return (e && e[0] == '1') ? 1 : 0;
  }();
  return on != 0;
}

struct Region {
  uintptr_t p = 0;        // byte address of element (0, 0)
  int64_t esz = 0;        // element bytes
  int64_t ld = 0, r = 0, c = 0;
  bool write = false;
  int desc = 0;
  uintptr_t end() const { return p + (uintptr_t)(((c - 1) * ld + r) * esz); }
};

inline Region region(const void* p, int64_t esz, int64_t r, int64_t c, int64_t ld, bool w,
                     int desc) {
  Region g;
  g.p = (uintptr_t)p;
  g.esz = esz;
  g.r = r;
  g.c = c;
  g.ld = std::max<int64_t>(ld, 1);
  g.write = w;
  g.desc = desc;
  return g;
}

inline bool iv(int64_t a0, int64_t a1, int64_t b0, int64_t b1) { return a0 < b1 && b0 < a1; }

// Exact element overlap for equal leading dimensions and element sizes,
// conservative (span overlap) otherwise.
inline bool regions_overlap(const Region& x0, const Region& y0) {
  if (x0.r <= 0 || x0.c <= 0 || y0.r <= 0 || y0.c <= 0) return false;
  if (!(x0.p < y0.end() && y0.p < x0.end())) return false;
  if (x0.ld != y0.ld || x0.esz != y0.esz) return true;
  const Region& x = x0.p <= y0.p ? x0 : y0;
  const Region& y = x0.p <= y0.p ? y0 : x0;
  uintptr_t db = y.p - x.p;
  if (db % (uintptr_t)x.esz) return true;
  int64_t d = (int64_t)(db / (uintptr_t)x.esz);
  int64_t co = d / x.ld, ro = d % x.ld;
  if (ro + y.r <= x.ld) return iv(0, x.r, ro, ro + y.r) && iv(0, x.c, co, co + y.c);
  return (iv(0, x.r, ro, x.ld) && iv(0, x.c, co, co + y.c)) ||
         (iv(0, x.r, 0, ro + y.r - x.ld) && iv(0, x.c, co + 1, co + y.c + 1));
}

inline void check_hazards(const char* what, std::vector<Region>& v) {
  std::vector<Region> g;
  g.reserve(v.size());
  for (auto& x : v)
    if (x.r > 0 && x.c > 0) g.push_back(x);
  std::sort(g.begin(), g.end(), [](const Region& a, const Region& b) { return a.p < b.p; });
  std::vector<const Region*> act;
  for (const Region& x : g) {
    act.erase(std::remove_if(act.begin(), act.end(),
                             [&](const Region* a) { return a->end() <= x.p; }),
              act.end());
    for (const Region* a : act) {
      if (!a->write && !x.write) continue;
      if (a->desc == x.desc && a->write && x.write) continue;
      if (regions_overlap(*a, x)) {
        throw Error(NUDFT2_E_INTERNAL,
                    std::string("hazard in ") + what + ": descriptor " + std::to_string(a->desc) +
                        (a->write ? " (write)" : " (read)") + " overlaps descriptor " +
                        std::to_string(x.desc) + (x.write ? " (write)" : " (read)") +
                        " [" + std::to_string(a->r) + "x" + std::to_string(a->c) + " ld " +
                        std::to_string(a->ld) + " vs " + std::to_string(x.r) + "x" +
                        std::to_string(x.c) + " ld " + std::to_string(x.ld) + "]");
      }
    }
    act.push_back(&x);
  }
}

}  // namespace nd
