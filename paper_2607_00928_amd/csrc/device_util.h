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

template <typename T> struct acc4;
template <> struct acc4<double> { using type = dbl4; };
template <> struct acc4<float> { using type = flt4; };

// exp(-2 pi i k x) for integer k (|k| < 2^20) and x in [0, 1): the product
// k x is split into its rounded value and exact error (fma), reduced mod 1,
// so the phase carries no error proportional to |k|.
__device__ inline double2 expi_kx(double k, double x) {
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

template <typename T>
__device__ inline T warp_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace nd
