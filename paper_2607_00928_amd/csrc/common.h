// Shared host/device definitions of the nudft2 library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
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
// Every device buffer of a plan is registered here so that destroy (and
// error paths) can release it; mem_cap is enforced on the running total.
struct Arena {
  std::vector<std::pair<void*, size_t>> blocks;
  size_t bytes = 0, peak = 0, cap = 0;
  void* alloc(size_t n);
  void release(void* p);
  void release_all();
  ~Arena() { release_all(); }
};

}  // namespace nd
