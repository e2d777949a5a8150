// Device helpers: MFMA wrappers, exact phase evaluation, reductions.
#pragma once

#include "common.h"

namespace nd {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core step.  Operand layout (wave64): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register v of lane l
// holds D[mrow<T>(l, v)][l % 16] (measured with the layout probe: the FP64
// instruction interleaves rows, i = l/16 + 4v; the FP32 one blocks them,
// i = 4(l/16) + v).
__device__ inline dbl4 mfma16(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline flt4 mfma16(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> __device__ inline int mrow(int lane, int v);
template <> __device__ inline int mrow<double>(int lane, int v) { return (lane >> 4) + 4 * v; }
template <> __device__ inline int mrow<float>(int lane, int v) { return 4 * (lane >> 4) + v; }

// Loads and stores through the global address space.  Pointers read out of a
// descriptor are generic, and generic (flat) accesses also count against the
// LDS wait counter: a wait for an LDS read would then wait for every global
// load in flight, serialising a register prefetch with the LDS work.
template <typename T> __device__ __forceinline__ T ldg(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T> __device__ __forceinline__ void stg(T* p, const T& v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
// complex elements go through a builtin two-vector (a struct copy would take
// its source by generic reference and turn the access back into a flat one)
typedef float gf2 __attribute__((ext_vector_type(2)));
typedef double gd2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ldc(const float2* p) {
  const gf2 v = *(const __attribute__((address_space(1))) gf2*)p;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 ldc(const double2* p) {
  const gd2 v = *(const __attribute__((address_space(1))) gd2*)p;
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void stc(float2* p, float2 c) {
  *(__attribute__((address_space(1))) gf2*)p = gf2{c.x, c.y};
}
__device__ __forceinline__ void stc(double2* p, double2 c) {
  *(__attribute__((address_space(1))) gd2*)p = gd2{c.x, c.y};
}
template <typename T> __device__ __forceinline__ void atomic_addg(T* p, T v) {
  __hip_atomic_fetch_add((__attribute__((address_space(1))) T*)p, v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T> struct acc4;
template <> struct acc4<double> { using type = dbl4; };
template <> struct acc4<float> { using type = flt4; };

// exp(-2 pi i k x) for integer k (|k| < 2^20) and x in [0, 1): the product
// k x is split into its rounded value and exact error (fma), reduced mod 1,
// so the phase carries no error proportional to |k|.  Contraction is off:
// fusing k x - rint(p) into one fma would add the error e twice.
__device__ inline double2 expi_kx(double k, double x) {
#pragma clang fp contract(off)
  double p = k * x;
  double e = fma(k, x, -p);
  double t = (p - rint(p)) + e;
  double s, c;
  sincospi(2.0 * t, &s, &c);
  double2 z;
  z.x = c;
  z.y = -s;
  return z;
}

// Lane moves through the DPP crossbar (no LDS traffic): the value of the
// lane selected by CTRL in rows enabled by RMASK, 0 elsewhere.
template <int CTRL, int RMASK>
__device__ inline float dpp_get(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, RMASK, 0xF, false));
}
template <int CTRL, int RMASK>
__device__ inline double dpp_get(double v) {
  int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, RMASK, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, RMASK, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ inline float lane_bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double lane_bcast(double v, int l) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave, returned to every lane (all lanes must be
// active): rotations within each row of 16 lanes (row_ror 1, 2, 4, 8) give
// every lane its row's sum; row_bcast 15 and 31 carry the row sums into the
// last row, whose lane 63 then holds the total.
template <typename T>
__device__ inline T warp_sum(T v) {
  v += dpp_get<0x121, 0xF>(v);
  v += dpp_get<0x122, 0xF>(v);
  v += dpp_get<0x124, 0xF>(v);
  v += dpp_get<0x128, 0xF>(v);
  v += dpp_get<0x142, 0xA>(v);
  v += dpp_get<0x143, 0xC>(v);
  return lane_bcast(v, 63);
}

}  // namespace nd
