// Shared host/device definitions of the nudft2 library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <set>
#include <unordered_map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/nudft2.h"

namespace nd {

// ----------------------------------------------------------------- errors
struct Error : std::runtime_error {
  nudft2_status status;
  Error(nudft2_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

void set_last_error(const std::string& msg);

#define ND_HIP(call)                                                          \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      throw ::nd::Error(e_ == hipErrorOutOfMemory ? NUDFT2_E_NOMEM            \
                                                  : NUDFT2_E_DEVICE,          \
                        std::string(#call) + ": " + hipGetErrorString(e_));   \
    }                                                                         \
  } while (0)

#define ND_CHECK(cond, status, msg)                                           \
  do {                                                                        \
    if (!(cond)) throw ::nd::Error(status, msg);                              \
  } while (0)

// ----------------------------------------------------------------- complex
template <typename T> struct cx;
template <> struct cx<float> { using type = float2; };
template <> struct cx<double> { using type = double2; };
template <typename T> using cplx = typename cx<T>::type;

template <typename T>
__host__ __device__ inline cplx<T> mk(T r, T i) { cplx<T> z; z.x = r; z.y = i; return z; }
template <typename C>
__host__ __device__ inline C cmul(C a, C b) { C z; z.x = a.x * b.x - a.y * b.y; z.y = a.x * b.y + a.y * b.x; return z; }
template <typename C>
__host__ __device__ inline C cmulc(C a, C b) { C z; z.x = a.x * b.x + a.y * b.y; z.y = a.x * b.y - a.y * b.x; return z; }  // conj(a) * b
template <typename C>
__host__ __device__ inline C cadd(C a, C b) { C z; z.x = a.x + b.x; z.y = a.y + b.y; return z; }
template <typename C>
__host__ __device__ inline C csub(C a, C b) { C z; z.x = a.x - b.x; z.y = a.y - b.y; return z; }
template <typename C>
__host__ __device__ inline C cconj(C a) { a.y = -a.y; return a; }

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ----------------------------------------------------------------- memory
// Device memory of a plan: a sub-allocator over large slabs obtained from
// hipMalloc once and returned only by release_all (plan destruction).
// Released blocks go to a free list (best fit, coalescing within a slab), so
// the many short-lived temporaries of a factorization never reach hipMalloc /
// hipFree.  mem_cap bounds the bytes reserved in slabs.
//
// Debug switches (environment): NUDFT2_POISON=1 fills new blocks with NaN;
// NUDFT2_GUARD=1 appends a patterned tail to every block that check() and
// release() verify; NUDFT2_QUARANTINE=1 never reuses released blocks
// (they are filled with NaN, and check() reports later writes into them).
struct Arena {
  std::vector<std::pair<void*, size_t>> slabs;
  std::set<uintptr_t> slab_start;
  std::map<uintptr_t, size_t> free_by_addr;
  std::multimap<size_t, uintptr_t> free_by_size;
  std::unordered_map<uintptr_t, std::pair<size_t, size_t>> live;   // block -> (size, span)
  size_t bytes = 0, peak = 0, cap = 0, reserved = 0;
  void* alloc(size_t n);
  void release(void* p);
  void release_all();
  size_t block_size(const void* p) const;
  // hand slabs that hold no live block back to the device (synchronises the
  // device first); returns the bytes freed
  size_t trim();
  void check(const char* where);
  ~Arena() { release_all(); }

 private:
  void add_free(uintptr_t a, size_t n);
  void take_free(std::map<uintptr_t, size_t>::iterator it);
};

}  // namespace nd
