// Batched complex GEMM / Householder QR / pivoted Cholesky / triangular solve
// for gfx950.  GEMM-shaped work runs on the matrix cores.  On the 16x16x4
// FP64 / FP32 instructions a complex product is three real products in
// Gauss's form, p1 = Ar Br, p2 = Ai Bi, p3 = (Ar + Ai)(Br + Bi), with
// Cr = p1 - p2 and Ci = p3 - p1 - p2 formed at the store.  FP32 tile
// products run by default on the bf16 instructions through an exact
// three-way split of every operand entry (gemm_tile_bf).
#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <type_traits>

#include "device_util.h"
#include <hip/hip_ext.h>

#include "la.h"
#include "hazard.h"
#include "prof.h"

namespace nd {

thread_local bool g_fp32_split = true;

// ------------------------------------------------------------ descriptor pool
void DescPool::init(size_t bytes, hipStream_t s) {
  destroy();
  cap = bytes;
  stream = s;
  valid = 0;
  tainted = false;
  ND_HIP(hipHostMalloc((void**)&host, cap, hipHostMallocDefault));
  ND_HIP(hipMalloc((void**)&dev, cap + 256));
  flag = (int*)(dev + cap);
  ND_HIP(hipMemsetAsync(flag, 0, sizeof(int), stream));
  used = 0;
}

void DescPool::check_flag() {
  int h = 0;
  ND_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, stream));
  ND_HIP(hipStreamSynchronize(stream));
  ND_CHECK(h == 0, NUDFT2_E_INTERNAL, "a cooperative QR panel timed out in its group barrier");
}

void DescPool::destroy() {
  if (host) (void)hipHostFree(host);
  if (dev) (void)hipFree(dev);
  if (sscr) (void)hipFree(sscr);
  host = dev = sscr = nullptr;
  sscr_cap = 0;
  flag = nullptr;
  cap = used = 0;
}

void DescPool::adopt(DescPool& o) {
  if (&o == this) return;
  destroy();
  host = o.host;
  dev = o.dev;
  flag = o.flag;
  cap = o.cap;
  used = o.used;
  stream = o.stream;
  deferred = o.deferred;
  sscr = o.sscr;
  sscr_cap = o.sscr_cap;
  valid = o.valid;
  tainted = o.tainted;
  o.host = o.dev = o.sscr = nullptr;
  o.flag = nullptr;
  o.cap = o.used = o.sscr_cap = o.valid = 0;
  o.tainted = false;
}

void DescPool::sync_reset() {
  if (deferred) return;
  ND_HIP(hipStreamSynchronize(stream));
  // after a plain push the device copy may differ from the staging (kernel
  // scratch): nothing is reusable until the next cycle has uploaded again
  if (!tainted) valid = std::max(valid, used);
  else valid = 0;
  tainted = false;
  used = 0;
}

void* DescPool::push_ro(const void* src, size_t n) {
  if (!deferred && !tainted && used + n <= valid && std::memcmp(host + used, src, n) == 0) {
    void* d = dev + used;
    used += (n + 255) & ~size_t(255);
    return d;
  }
  const bool t = tainted;
  void* d = push(src, n);
  tainted = t;
  return d;
}

void* DescPool::push(const void* src, size_t n) {
  tainted = true;
  size_t need = (n + 255) & ~size_t(255);
  ND_CHECK(used + need <= cap, NUDFT2_E_INTERNAL, "descriptor pool exhausted");
  std::memcpy(host + used, src, n);
  if (!deferred) ND_HIP(hipMemcpyAsync(dev + used, host + used, n, hipMemcpyHostToDevice, stream));
  void* d = dev + used;
  used += need;
  return d;
}

void* DescPool::reserve(size_t n) {
  tainted = true;
  size_t need = (n + 255) & ~size_t(255);
  ND_CHECK(used + need <= cap, NUDFT2_E_INTERNAL, "descriptor pool exhausted");
  void* d = dev + used;
  used += need;
  return d;
}

void* DescPool::stream_scratch(size_t n) {
  if (deferred) return nullptr;
  if (n > sscr_cap) {
    if (sscr) {
      ND_HIP(hipStreamSynchronize(stream));
      ND_HIP(hipFree(sscr));
      sscr = nullptr;
      sscr_cap = 0;
    }
    if (hipMalloc((void**)&sscr, n) != hipSuccess) {
      (void)hipGetLastError();   // out of memory: the caller falls back
      sscr = nullptr;
      return nullptr;
    }
    sscr_cap = n;
  }
  return sscr;
}

void DescPool::flush() {
  if (used > 0) ND_HIP(hipMemcpyAsync(dev, host, used, hipMemcpyHostToDevice, stream));
}

namespace {

// ------------------------------------------------------ descriptor lists
// A kernel reads its descriptor list through device memory (a copy into the
// pool) or, for a short list, from its own kernel arguments: then no
// host-to-device copy sits between two kernels of the stream, and the
// dispatches follow each other without the copy's gap.
constexpr size_t kArgDescBytes = 3072;
template <typename D>
struct DescMem {
  const D* p;
  __device__ const D& operator[](int i) const { return p[i]; }
};
template <typename D, int N>
struct DescArg {
  D d[N];
  __device__ const D& operator[](int i) const { return d[i]; }
};
// launch(list) with the list as DescArg (short) or DescMem (pool copy)
template <typename D, class F>
void with_descs(DescPool& pool, const D* v, size_t n, F&& launch) {
  constexpr int N = (int)(kArgDescBytes / sizeof(D));
  if (n <= (size_t)N) {
    DescArg<D, N> a{};
    std::memcpy(a.d, v, sizeof(D) * n);
    launch(a);
  } else {
    launch(DescMem<D>{(const D*)pool.push_ro(v, sizeof(D) * n)});
  }
}

// ------------------------------------------------------------------- GEMM
constexpr int GT = 64;    // output tile
constexpr int GK = 16;    // k per stage

// The next k stage is loaded into registers while the current one is
// multiplied out of LDS (double buffered, one barrier per stage).  LDS rows are padded to an odd multiple
// of 16 banks, so the 16-lane groups of an operand read hit distinct banks.
template <typename T> constexpr int gemm_ldt() { return GT + 64 / (int)sizeof(T); }

// Store of a workgroup's 64 x 64 output tile, held by its four waves as 2 x 2
// blocks of 16 x 16 matrix-core accumulators: the wave at (wr, wc) =
// (32 (wave / 2), 32 (wave % 2)) holds Re and Im of element (wr + 16 a +
// mrow(lane, v), wc + 16 b + lane % 16) in cr[a][b][v] and ci[a][b][v].
// alpha P is stored (adding beta times the old value) or, when `atomic`,
// added atomically, at cb + (i - i0) + (j - j0) cld for the tile's rows i < m
// and columns j < n.
template <typename T>
__device__ __forceinline__ void gemm_store_tile(const GemmDesc<T>& d, int i0, int j0, bool atomic,
                                                cplx<T>* cb, int64_t cld, T beta,
                                                const typename acc4<T>::type (&cr)[2][2],
                                                const typename acc4<T>::type (&ci)[2][2]) {
  using C2 = cplx<T>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  if constexpr (sizeof(T) == 4) {
    // FP32 accumulators: a lane holds rows 4 (lane / 16) .. + 3 of one column,
    // 32 contiguous bytes of column-major C, read and written as two 16-byte
    // accesses (8-byte aligned: dword alignment is all the hardware needs)
    if (!atomic) {
      typedef float f4u __attribute__((ext_vector_type(4), aligned(8)));
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int ib = i0 + wr + a * 16 + 4 * (lane >> 4);
          const int j = j0 + wc + b * 16 + (lane & 15);
          if (j >= d.n || ib >= d.m) continue;
          C2 out[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T re = cr[a][b][v], im = ci[a][b][v];
            out[v] = mk<T>(d.ar * re - d.ai * im, d.ar * im + d.ai * re);
          }
          C2* p = cb + (int64_t)(ib - i0) + (int64_t)(j - j0) * cld;
          if (ib + 3 < d.m) {
            f4u* q = (f4u*)p;
            f4u w0 = {out[0].x, out[0].y, out[1].x, out[1].y};
            f4u w1 = {out[2].x, out[2].y, out[3].x, out[3].y};
            if (beta != T(0)) {
              const f4u o0 = ldg(q), o1 = ldg(q + 1);
              w0 += beta * o0;
              w1 += beta * o1;
            }
            stg(q, w0);
            stg(q + 1, w1);
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              if (ib + v >= d.m) break;
              C2 o = out[v];
              if (beta != T(0)) {
                const C2 c = ldc(p + v);
                o.x += beta * c.x;
                o.y += beta * c.y;
              }
              stc(p + v, o);
            }
          }
        }
      return;
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = i0 + wr + a * 16 + mrow<T>(lane, v);
        int j = j0 + wc + b * 16 + (lane & 15);
        if (i < d.m && j < d.n) {
          const T re = cr[a][b][v], im = ci[a][b][v];
          C2 out = mk<T>(d.ar * re - d.ai * im, d.ar * im + d.ai * re);
          C2* p = cb + (int64_t)(i - i0) + (int64_t)(j - j0) * cld;
          if (atomic) {
            atomic_addg(&p->x, out.x);
            atomic_addg(&p->y, out.y);
            continue;
          }
          if (beta != T(0)) {
            const C2 o = ldc(p);
            out.x += beta * o.x;
            out.y += beta * o.y;
          }
          stc(p, out);
        }
      }
}

// Narrows [kbeg, kend) to the k beyond which op(A)'s rows i0.. or op(B)'s
// columns j0.. of a 64 x 64 output tile hold only stored zeros (an empty
// range leaves the accumulators at zero).
template <typename T, int OPA, int OPB>
__device__ __forceinline__ void tri_krange(const GemmDesc<T>& d, int i0, int j0, int& kbeg,
                                           int& kend) {
  const int ta = d.tri, tb = d.trib;
  // op(A)(i, l) = 0 for l > i: A unit lower (op N) or upper (op C)
  if ((OPA == OpN && ta == 1) || (OPA == OpC && ta == 2)) kend = min(kend, i0 + GT);
  // op(A)(i, l) = 0 for l < i
  if ((OPA == OpN && ta == 2) || (OPA == OpC && ta == 1)) kbeg = max(kbeg, i0);
  // op(B)(l, j) = 0 for l > j: B upper (op N) or unit lower (op C)
  if ((OPB == OpN && tb == 2) || (OPB == OpC && tb == 1)) kend = min(kend, j0 + GT);
  // op(B)(l, j) = 0 for l < j
  if ((OPB == OpN && tb == 1) || (OPB == OpC && tb == 2)) kbeg = max(kbeg, j0);
}

// The output tile at (i0, j0) over the k range [kbeg, kend): alpha P is
// stored (adding beta times the old value) or, when `atomic`, added
// atomically, at cb + (i - i0) + (j - j0) cld for the tile's rows i < m and
// columns j < n.  Called uniformly by the whole workgroup; leaves the LDS
// buffers free on return.
template <typename T, int OPA, int OPB>
__device__ __forceinline__ void gemm_tile(const GemmDesc<T>& d, int i0, int j0, int kbeg, int kend,
                                          bool atomic, cplx<T>* cb, int64_t cld, T beta,
                                          T (&As)[2][2][GK][gemm_ldt<T>()],
                                          T (&Bs)[2][2][GK][gemm_ldt<T>()]) {
  using C2 = cplx<T>;
  using A4 = typename acc4<T>::type;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  tri_krange<T, OPA, OPB>(d, i0, j0, kbeg, kend);
  // Gauss (3M) products: p1 = Ar Br, p2 = Ai Bi, p3 = (Ar + Ai)(Br + Bi);
  // Re = p1 - p2, Im = p3 - p1 - p2
  A4 acc1[2][2], acc2[2][2], acc3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc1[a][b] = A4{0, 0, 0, 0};
      acc2[a][b] = A4{0, 0, 0, 0};
      acc3[a][b] = A4{0, 0, 0, 0};
    }
  // this thread's 4 elements of each stage: (row, k) of op(A), (k, column) of op(B)
  auto a_at = [&](int u, int& i, int& l) {
    if (OPA == OpN) { i = tid & 63; l = (tid >> 6) + 4 * u; }
    else { l = tid & 15; i = (tid >> 4) + 16 * u; }
  };
  auto b_at = [&](int u, int& l, int& j) {
    if (OPB == OpN) { l = tid & 15; j = (tid >> 4) + 16 * u; }
    else { j = tid & 63; l = (tid >> 6) + 4 * u; }
  };
  C2 ra[4], rb[4];
  auto gload = [&](int l0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int i, l;
      a_at(u, i, l);
      C2 v = mk<T>(0, 0);
      if (i0 + i < d.m && l0 + l < kend)
        v = OPA == OpN ? ldc(d.A + (int64_t)(i0 + i) + (int64_t)(l0 + l) * d.lda)
                       : ldc(d.A + (int64_t)(l0 + l) + (int64_t)(i0 + i) * d.lda);
      ra[u] = v;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int l, j;
      b_at(u, l, j);
      C2 v = mk<T>(0, 0);
      if (j0 + j < d.n && l0 + l < kend)
        v = OPB == OpN ? ldc(d.B + (int64_t)(l0 + l) + (int64_t)(j0 + j) * d.ldb)
                       : ldc(d.B + (int64_t)(j0 + j) + (int64_t)(l0 + l) * d.ldb);
      rb[u] = v;
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int i, l;
      a_at(u, i, l);
      As[buf][0][l][i] = ra[u].x;
      As[buf][1][l][i] = OPA == OpN ? ra[u].y : -ra[u].y;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int l, j;
      b_at(u, l, j);
      Bs[buf][0][l][j] = rb[u].x;
      Bs[buf][1][l][j] = OPB == OpN ? rb[u].y : -rb[u].y;
    }
  };
  const int nst = (kend - kbeg + GK - 1) / GK;
  if (nst > 0) {
    gload(kbeg);
    lstore(0);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (st + 1 < nst) gload(kbeg + (st + 1) * GK);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int l = kk * 4 + (lane >> 4);
      T ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ar[a] = As[buf][0][l][wr + a * 16 + (lane & 15)];
        ai[a] = As[buf][1][l][wr + a * 16 + (lane & 15)];
        br[a] = Bs[buf][0][l][wc + a * 16 + (lane & 15)];
        bi[a] = Bs[buf][1][l][wc + a * 16 + (lane & 15)];
      }
      T as[2], bs[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        as[a] = ar[a] + ai[a];
        bs[a] = br[a] + bi[a];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc1[a][b] = mfma16(ar[a], br[b], acc1[a][b]);
          acc2[a][b] = mfma16(ai[a], bi[b], acc2[a][b]);
          acc3[a][b] = mfma16(as[a], bs[b], acc3[a][b]);
        }
    }
    if (st + 1 < nst) lstore(buf ^ 1);
    __syncthreads();
  }
  A4 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = acc1[a][b] - acc2[a][b];
      ci[a][b] = acc3[a][b] - acc1[a][b] - acc2[a][b];
    }
  gemm_store_tile<T>(d, i0, j0, atomic, cb, cld, beta, cr, ci);
}

// ------------------------------------- FP32 products on the bf16 matrix cores
// Every FP32 entry x of op(A) and op(B) is split into three bf16 values:
// x0 = bf16(x) rounded to nearest, x1 = bf16(x - x0), x2 = x - x0 - x1.  Both
// differences are exact in FP32 and x2 keeps at most 8 significant bits, so
// x = x0 + x1 + x2 exactly.  A real product a b is summed from the six bf16
// products a_p b_q with p + q <= 2, each exact in the FP32 accumulator; the
// three left out (a1 b2, a2 b1, a2 b2) are below (2^-23 + 2^-32) |a| |b|, so
// the result carries the error of an FP32 dot product (one more unit of
// 2^-24 |a| |b| a term) and keeps FP32's exponent range.  A complex product
// takes four real ones in three accumulators per block (Ar Br, Ai Bi, and
// Ar Bi + Ai Br).  The bf16 matrix instructions do 16 times the FP32 ones'
// multiply-adds per cycle, so the 24 bf16 products of a complex
// multiply-add cost 3/8 of the FP32 path's three Gauss products.  Each
// operand entry is split once, as its stage is written to LDS.
constexpr int BK = 32;   // k per stage: two 32x32x16 instructions
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
// One stage: [op(A), op(B)][plane: Re x0, x1, x2, Im x0, x1, x2][row i of
// op(A) / column j of op(B)][k] (48 KB: three workgroups a CU).  A row's
// 32 k are four 16-byte chunks; chunk c of row r sits at position
// c ^ ((r / 4) % 4), so the 8 rows of a 16-byte access phase start on
// distinct banks.
struct BfStage {
  unsigned short p[2][6][GT][BK];
};
__device__ __forceinline__ int bf_chunk(int r, int c) { return (c ^ (r >> 2)) & 3; }

__device__ __forceinline__ unsigned bf16_pair(float lo, float hi) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f2{lo, hi}, b2));
}
// the three bf16 parts of a and b, packed in pairs (a in the low half)
__device__ __forceinline__ void bf16_split3(float a, float b, unsigned& h, unsigned& m,
                                            unsigned& l) {
  h = bf16_pair(a, b);
  const float ra = a - __uint_as_float(h << 16), rb = b - __uint_as_float(h & 0xffff0000u);
  m = bf16_pair(ra, rb);
  l = bf16_pair(ra - __uint_as_float(m << 16), rb - __uint_as_float(m & 0xffff0000u));
}

// 8 consecutive k (k0 .. k0 + 7) of row r of an operand tile whose element
// (r, k) sits at p[k + r ld] (KC: k contiguous) or p[r + k ld], as loaded:
// indices are clamped into the stored matrix (kq: its k extent from p; KC:
// >= 2, pairs of entries are read) and nothing is selected, so no
// instruction waits for the loads until bf_split8 masks them.
template <bool KC>
__device__ __forceinline__ void bf_load8(const float2* p, int64_t ld, int r, int k0, int kq,
                                         float2 (&v)[8]) {
  if constexpr (KC) {
    typedef float f4u __attribute__((ext_vector_type(4), aligned(8)));
    const float2* q = p + (int64_t)r * ld;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const f4u w = ldg((const f4u*)(q + min(k0 + 2 * u, kq - 2)));
      v[2 * u] = make_float2(w.x, w.y);
      v[2 * u + 1] = make_float2(w.z, w.w);
    }
  } else {
    const float2* q = p + r;
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = ldc(q + (int64_t)min(k0 + u, kq - 1) * ld);
  }
}

// The entries bf_load8 loaded with the same k0, kq, masked (zero where `rv`
// is false or k >= kn) and conjugated when `cj`, split into the three bf16
// planes: w[plane][pair], planes Re x0, x1, x2, Im x0, x1, x2.
template <bool KC>
__device__ __forceinline__ void bf_split8(const float2 (&v)[8], bool rv, int k0, int kn, int kq,
                                          bool cj, unsigned (&w)[6][4]) {
  float2 x[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int e = k0 + u;
    float2 y = v[u];
    // KC: a pair read from kq - 2 because e = kq - 1 holds e in its upper half
    if (KC && (u & 1) == 0 && e == kq - 1) y = v[u + 1];
    x[u] = rv && e < kn ? y : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    bf16_split3(x[2 * q].x, x[2 * q + 1].x, w[0][q], w[1][q], w[2][q]);
    const float i0 = cj ? -x[2 * q].y : x[2 * q].y, i1 = cj ? -x[2 * q + 1].y : x[2 * q + 1].y;
    bf16_split3(i0, i1, w[3][q], w[4][q], w[5][q]);
  }
}

__device__ __forceinline__ void bf_store8(unsigned short (&pl)[6][GT][BK], int r, int k0,
                                          const unsigned (&w)[6][4]) {
  const int c = 8 * bf_chunk(r, k0 >> 3);
#pragma unroll
  for (int p = 0; p < 6; ++p) *(u32x4*)&pl[p][r][c] = u32x4{w[p][0], w[p][1], w[p][2], w[p][3]};
}

typedef float flt16 __attribute__((ext_vector_type(16)));
// 32x32x16 bf16 step: lane l supplies A[l % 32][8 (l / 32) .. + 7] and
// B[8 (l / 32) .. + 7][l % 32]; accumulator register v of lane l holds
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32]
__device__ __forceinline__ flt16 mfma_bf16(u32x4 a, u32x4 b, flt16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Store of the 64 x 64 tile as gemm_store_tile, held by the four waves as one
// 32 x 32 block each (wave at (32 (wave / 2), 32 (wave % 2))) in the layout
// of mfma_bf16.
__device__ __forceinline__ void gemm_store_tile32(const GemmDesc<float>& d, int i0, int j0,
                                                  bool atomic, float2* cb, int64_t cld, float beta,
                                                  const flt16& cr, const flt16& ci) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = j0 + (wave & 1) * 32 + (lane & 31);
  if (j >= d.n) return;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int ib = i0 + (wave >> 1) * 32 + 8 * g + 4 * (lane >> 5);
    if (ib >= d.m) continue;
    float2 out[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float re = cr[4 * g + v], im = ci[4 * g + v];
      out[v] = make_float2(d.ar * re - d.ai * im, d.ar * im + d.ai * re);
    }
    float2* p = cb + (int64_t)(ib - i0) + (int64_t)(j - j0) * cld;
    if (atomic) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (ib + v >= d.m) break;
        atomic_addg(&p[v].x, out[v].x);
        atomic_addg(&p[v].y, out[v].y);
      }
    } else if (ib + 3 < d.m) {
      typedef float f4u __attribute__((ext_vector_type(4), aligned(8)));
      f4u* q = (f4u*)p;
      f4u w0 = {out[0].x, out[0].y, out[1].x, out[1].y};
      f4u w1 = {out[2].x, out[2].y, out[3].x, out[3].y};
      if (beta != 0.f) {
        const f4u o0 = ldg(q), o1 = ldg(q + 1);
        w0 += beta * o0;
        w1 += beta * o1;
      }
      stg(q, w0);
      stg(q + 1, w1);
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (ib + v >= d.m) break;
        float2 o = out[v];
        if (beta != 0.f) {
          const float2 c = ldc(p + v);
          o.x += beta * c.x;
          o.y += beta * c.y;
        }
        stc(p + v, o);
      }
    }
  }
}

// gemm_tile for FP32 operands through the bf16 split (same contract).  One
// LDS stage: its entries, loaded during the previous stage, are masked, split
// and written between two barriers, then the next stage's loads are issued
// and the stage is multiplied out one k half at a time.  Register use is
// held to three workgroups a CU, whose phases overlap.
template <int OPA, int OPB>
__device__ __forceinline__ void gemm_tile_bf(const GemmDesc<float>& d, int i0, int j0, int kbeg,
                                             int kend, bool atomic, float2* cb, int64_t cld,
                                             float beta, BfStage& S) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  tri_krange<float, OPA, OPB>(d, i0, j0, kbeg, kend);
  flt16 arr, aii, ax;
#pragma unroll
  for (int v = 0; v < 16; ++v) arr[v] = aii[v] = ax[v] = 0.f;
  // op(A)(i, l): A[i + l lda] (op N: rows contiguous) or conj A[l + i lda];
  // op(B)(l, j): B[l + j ldb] (op N: k contiguous) or conj B[j + l ldb]
  constexpr bool AKC = OPA != OpN, BKC = OPB == OpN;
  const int ra = AKC ? tid >> 2 : tid & 63, ka = AKC ? 8 * (tid & 3) : 8 * (tid >> 6);
  const int rb = BKC ? tid >> 2 : tid & 63, kb = BKC ? 8 * (tid & 3) : 8 * (tid >> 6);
  const bool rva = ra < d.m - i0, rvb = rb < d.n - j0;
  const int rac = min(ra, d.m - i0 - 1), rbc = min(rb, d.n - j0 - 1);
  const int nst = (kend - kbeg + BK - 1) / BK;
  const int llast = kbeg + max(nst - 1, 0) * BK;   // stages past the end reload the last
  float2 va[8], vb[8];
  auto gload = [&](int l0) __attribute__((always_inline)) {
    l0 = min(l0, llast);
    const float2* pa = AKC ? d.A + l0 + (int64_t)i0 * d.lda : d.A + i0 + (int64_t)l0 * d.lda;
    const float2* pb = BKC ? d.B + l0 + (int64_t)j0 * d.ldb : d.B + j0 + (int64_t)l0 * d.ldb;
    bf_load8<AKC>(pa, d.lda, rac, ka, d.k - l0, va);
    bf_load8<BKC>(pb, d.ldb, rbc, kb, d.k - l0, vb);
  };
  if (nst > 0) gload(kbeg);
  const int gc = lane >> 5, rl = lane & 31;
  const int rA = wr + rl, rB = wc + rl;
  for (int st = 0; st < nst; ++st) {
    const int l0 = kbeg + st * BK;
    {
      unsigned w[6][4];
      bf_split8<AKC>(va, rva, ka, kend - l0, d.k - l0, OPA != OpN, w);
      bf_store8(S.p[0], ra, ka, w);
      bf_split8<BKC>(vb, rvb, kb, kend - l0, d.k - l0, OPB != OpN, w);
      bf_store8(S.p[1], rb, kb, w);
    }
    __syncthreads();
    gload(l0 + BK);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      u32x4 fa[6], fb[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        fa[q] = *(const u32x4*)&S.p[0][q][rA][8 * bf_chunk(rA, 2 * h + gc)];
        fb[q] = *(const u32x4*)&S.p[1][q][rB][8 * bf_chunk(rB, 2 * h + gc)];
      }
      // terms (p, q), p + q <= 2, smallest first
#pragma unroll
      for (int p = 2; p >= 0; --p)
#pragma unroll
        for (int q = 2 - p; q >= 0; --q) {
          arr = mfma_bf16(fa[p], fb[q], arr);
          aii = mfma_bf16(fa[3 + p], fb[3 + q], aii);
          ax = mfma_bf16(fa[p], fb[3 + q], ax);
          ax = mfma_bf16(fa[3 + p], fb[q], ax);
        }
    }
    __syncthreads();
  }
  gemm_store_tile32(d, i0, j0, atomic, cb, cld, beta, arr - aii, ax);
}

// The workgroup's share of a launch: tile(i0, j0, kbeg, kend, atomic, cb,
// cld, beta) for each output tile (and k range) it takes.
// splits > 1: blockIdx.z takes the k range [z kc, (z+1) kc) and the result is
// added atomically (C must already hold beta C), or, with `part`, stored as
// the 64 x 64 partial tile part[((y splits + z) gridDim.x + x) 4096] (column
// major, leading dimension 64; ranges past k store nothing) for
// gemm_reduce_kernel to sum.
// sk > 0 (stream-K): the descriptor's tiles x k stages are dealt out in equal
// contiguous shares to its sk workgroups (blockIdx.x); a share may end in
// one tile and go on in the next, and every piece is added atomically to a
// pre-scaled C.  Equal shares leave no partial last round of workgroups.
template <typename T, class F>
__device__ __forceinline__ void gemm_share(const GemmDesc<T>& d, int splits, int sk, cplx<T>* part,
                                           F&& tile) {
  const int tm = (d.m + GT - 1) / GT, tn = (d.n + GT - 1) / GT;
  if (sk > 0) {
    const int nst = (d.k + GK - 1) / GK;
    const int64_t units = (int64_t)tm * tn * nst;
    int64_t u = units * blockIdx.x / sk;
    const int64_t u1 = units * (blockIdx.x + 1) / sk;
    while (u < u1) {
      const int tl = (int)(u / nst), s0 = (int)(u % nst);
      const int s1 = (int)min((int64_t)nst, s0 + (u1 - u));
      const int i0 = (tl % tm) * GT, j0 = (tl / tm) * GT;
      tile(i0, j0, s0 * GK, min(d.k, s1 * GK), true, d.C + i0 + (int64_t)j0 * d.ldc, d.ldc, T(0));
      u += s1 - s0;
    }
    return;
  }
  if ((int)blockIdx.x >= tm * tn) return;
  int kc = (((d.k + splits - 1) / splits) + GK - 1) / GK * GK;
  const int kbeg = (int)blockIdx.z * kc;
  const int kend = min(d.k, kbeg + kc);
  if (kbeg >= kend && splits > 1) return;
  const int i0 = (blockIdx.x % tm) * GT, j0 = (blockIdx.x / tm) * GT;
  if (d.lower && j0 > i0 + GT - 1) return;   // strictly above the diagonal of a Hermitian C
  if (part) {
    cplx<T>* cb = part + (((size_t)blockIdx.y * splits + blockIdx.z) * gridDim.x + blockIdx.x) *
                             (size_t)(GT * GT);
    tile(i0, j0, kbeg, kend, false, cb, (int64_t)GT, T(0));
  } else {
    tile(i0, j0, kbeg, kend, splits > 1, d.C + i0 + (int64_t)j0 * d.ldc, (int64_t)d.ldc, d.beta);
  }
}

template <typename T, int OPA, int OPB, class DS>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 2 : 4) void gemm_kernel(DS descs, int splits,
                                                                          int sk, cplx<T>* part) {
  __shared__ T As[2][2][GK][gemm_ldt<T>()];   // [buffer][re, im][k][row]
  __shared__ T Bs[2][2][GK][gemm_ldt<T>()];
  const GemmDesc<T> d = descs[blockIdx.y];
  gemm_share<T>(d, splits, sk, part,
                [&](int i0, int j0, int kb, int ke, bool atomic, cplx<T>* cb, int64_t cld,
                    T beta) __attribute__((always_inline)) {
                  gemm_tile<T, OPA, OPB>(d, i0, j0, kb, ke, atomic, cb, cld, beta, As, Bs);
                });
}

// gemm_kernel for FP32 operands on the bf16 matrix cores (the split above)
template <int OPA, int OPB, class DS>
__global__ __launch_bounds__(256, 3) void gemm_bf_kernel(DS descs, int splits, int sk,
                                                         float2* part) {
  __shared__ BfStage S;
  const GemmDesc<float> d = descs[blockIdx.y];
  gemm_share<float>(d, splits, sk, part,
                    [&](int i0, int j0, int kb, int ke, bool atomic, float2* cb, int64_t cld,
                        float beta) __attribute__((always_inline)) {
                      gemm_tile_bf<OPA, OPB>(d, i0, j0, kb, ke, atomic, cb, cld, beta, S);
                    });
}

// C = sum over z of the partial tiles (in order z = 0, 1, ...) + beta C:
// the second pass of a k split through `part` (gemm_kernel).  Each
// descriptor's ranges are those gemm_kernel gives it: kc rounded up to a
// whole k stage, ranges starting at or past k hold nothing.
template <typename T, class DS>
__global__ __launch_bounds__(256) void gemm_reduce_kernel(DS descs, int splits, int tiles,
                                                          const cplx<T>* __restrict__ part) {
  const GemmDesc<T> d = descs[blockIdx.y];
  const int kc = (((d.k + splits - 1) / splits) + GK - 1) / GK * GK;
  const int nz = kc > 0 ? min(splits, (d.k + kc - 1) / kc) : 0;
  const int tm = (d.m + GT - 1) / GT;
  const int64_t cnt = (int64_t)d.m * d.n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % d.m), j = (int)(e / d.m);
    const size_t off = (size_t)((i / GT) + (j / GT) * tm) * (GT * GT) + (i % GT) + (j % GT) * GT;
    const cplx<T>* pz = part + (size_t)blockIdx.y * splits * tiles * (GT * GT) + off;
    T sr = 0, si = 0;
    for (int z = 0; z < nz; ++z) {
      const cplx<T> v = ldc(pz + (size_t)z * tiles * (GT * GT));
      sr += v.x;
      si += v.y;
    }
    cplx<T>* c = d.C + i + (int64_t)j * d.ldc;
    if (d.beta != T(0)) {
      const cplx<T> o = ldc(c);
      sr += d.beta * o.x;
      si += d.beta * o.y;
    }
    stc(c, mk<T>(sr, si));
  }
}

// Skinny products (n <= SK_N columns, B not transposed): memory-bound on A.
// op(A) = A: one thread per row of C, the B panel staged in LDS.
// op(A) = A^H: one wave per row of C (a dot product along a column of A).
// blockIdx.z splits the k range; with splits > 1 the results are added
// atomically to a pre-scaled C.
constexpr int SK_N = 8;
constexpr int SK_L = 64;

template <typename T>
__device__ inline void skinny_store(const GemmDesc<T>& d, int i, int j, cplx<T> v, int splits) {
  cplx<T> out = mk<T>(d.ar * v.x - d.ai * v.y, d.ar * v.y + d.ai * v.x);
  cplx<T>* p = d.C + (int64_t)i + (int64_t)j * d.ldc;
  if (splits > 1) {
    atomic_addg(&p->x, out.x);
    atomic_addg(&p->y, out.y);
    return;
  }
  if (d.beta != T(0)) {
    cplx<T> o = ldc(p);
    out.x += d.beta * o.x;
    out.y += d.beta * o.y;
  }
  stc(p, out);
}

// op(A) = A: thread i accumulates row i of C over NC columns; the k loop
// issues SK_U independent loads of A before using them (memory-level
// parallelism on a bandwidth-bound stream).
constexpr int SK_U = 8;
// rows of C per wave in gemm_skinny_c_kernel (op C, long k) and per
// workgroup in gemm_skinny_cw_kernel
constexpr int SKC_ROWS = 2;
constexpr int SKCW_ROWS = 2;

template <typename T, int NC, class DS>
__global__ __launch_bounds__(256) void gemm_skinny_n_kernel(DS descs, int splits) {
  using C2 = cplx<T>;
  const GemmDesc<T> d = descs[blockIdx.y];
  const int i0 = blockIdx.x * 256;
  if (i0 >= d.m || d.n <= 0) return;
  const int kc = (d.k + splits - 1) / splits;
  int kb = blockIdx.z * kc, ke = min(d.k, kb + kc);
  if (kb >= ke && splits > 1) return;
  // rows i0 .. i0 + 255 have no nonzeros of A outside [lo, hi)
  if (d.tri == 1) ke = min(ke, i0 + 256);
  else if (d.tri == 2) kb = max(kb, i0);
  __shared__ C2 Bs[SK_L][NC];
  const int tid = threadIdx.x, i = i0 + tid;
  const bool row = i < d.m;
  C2 acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = mk<T>(0, 0);
  for (int l0 = kb; l0 < ke; l0 += SK_L) {
    __syncthreads();
    for (int e = tid; e < SK_L * NC; e += 256) {
      int l = e % SK_L, j = e / SK_L;
      Bs[l][j] = (l0 + l < ke && j < d.n) ? ldc(d.B + (int64_t)(l0 + l) + (int64_t)j * d.ldb) : mk<T>(0, 0);
    }
    __syncthreads();
    const int lm = min(SK_L, ke - l0);
    const C2* ap = d.A + (row ? i : 0) + (int64_t)l0 * d.lda;
    int l = 0;
    for (; l + SK_U <= lm; l += SK_U) {
      C2 a[SK_U];
#pragma unroll
      for (int u = 0; u < SK_U; ++u) a[u] = row ? ldc(ap + (int64_t)(l + u) * d.lda) : mk<T>(0, 0);
#pragma unroll
      for (int u = 0; u < SK_U; ++u)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[j] = cadd(acc[j], cmul(a[u], Bs[l + u][j]));
    }
    for (; l < lm; ++l) {
      const C2 a = row ? ldc(ap + (int64_t)l * d.lda) : mk<T>(0, 0);
#pragma unroll
      for (int j = 0; j < NC; ++j) acc[j] = cadd(acc[j], cmul(a, Bs[l][j]));
    }
  }
  if (row)
#pragma unroll
    for (int j = 0; j < NC; ++j)
      if (j < d.n) skinny_store(d, i, j, acc[j], splits);
}

// op(A) = A for short, tall batches: a workgroup takes 64 rows of C and its
// four waves split the k range into quarters (lane = row, SK_U loads of A in
// flight per lane, B read by uniform loads), then the waves' partial sums
// meet in LDS.  Four times the workgroups of gemm_skinny_n_kernel for the
// same rows: the sweep's reflector updates C -= V W on a few tall nodes
// otherwise leave most CUs idle.
template <typename T, int NC, class DS>
__global__ __launch_bounds__(256) void gemm_skinny_n4_kernel(DS descs, int splits) {
  using C2 = cplx<T>;
  __shared__ C2 red[3][64][NC];
  const GemmDesc<T> d = descs[blockIdx.y];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i0 = blockIdx.x * 64;
  if (i0 >= d.m || d.n <= 0) return;
  const int kc = (d.k + splits - 1) / splits;
  int kb0 = blockIdx.z * kc, ke0 = min(d.k, kb0 + kc);
  if (kb0 >= ke0 && splits > 1) return;
  // rows i0 .. i0 + 63 have no nonzeros of A outside [lo, hi); the waves
  // still meet in LDS when that leaves nothing
  if (d.tri == 1) ke0 = min(ke0, i0 + 64);
  else if (d.tri == 2) kb0 = max(kb0, i0);
  const int kq = (max(ke0 - kb0, 0) + 3) / 4;
  const int kb = kb0 + wave * kq, ke = min(ke0, kb + kq);
  const int i = i0 + lane;
  const bool row = i < d.m;
  C2 acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = mk<T>(0, 0);
  const C2* ap = d.A + (row ? i : 0);
  int l = kb;
  for (; l + SK_U <= ke; l += SK_U) {
    C2 a[SK_U];
#pragma unroll
    for (int u = 0; u < SK_U; ++u) a[u] = row ? ldc(ap + (int64_t)(l + u) * d.lda) : mk<T>(0, 0);
#pragma unroll
    for (int u = 0; u < SK_U; ++u)
#pragma unroll
      for (int j = 0; j < NC; ++j)
        if (j < d.n) acc[j] = cadd(acc[j], cmul(a[u], ldc(d.B + (int64_t)(l + u) + (int64_t)j * d.ldb)));
  }
  for (; l < ke; ++l) {
    const C2 a = row ? ldc(ap + (int64_t)l * d.lda) : mk<T>(0, 0);
#pragma unroll
    for (int j = 0; j < NC; ++j)
      if (j < d.n) acc[j] = cadd(acc[j], cmul(a, ldc(d.B + (int64_t)l + (int64_t)j * d.ldb)));
  }
  if (wave > 0)
#pragma unroll
    for (int j = 0; j < NC; ++j) red[wave - 1][lane][j] = acc[j];
  __syncthreads();
  if (wave == 0 && row)
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (j >= d.n) break;
      const C2 v = cadd(acc[j], cadd(red[0][lane][j], cadd(red[1][lane][j], red[2][lane][j])));
      skinny_store(d, i, j, v, splits);
    }
}

// op(A) = A^H: wave w computes row i of C (a dot product along column i of
// A) over NC columns; each lane keeps SK_U / 2 independent loads in flight.
template <typename T, int NC, class DS>
__global__ __launch_bounds__(256) void gemm_skinny_c_kernel(DS descs, int splits) {
  using C2 = cplx<T>;
  constexpr int U = SK_U / 2;
  constexpr int R = SKC_ROWS;
  const GemmDesc<T> d = descs[blockIdx.y];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // R rows of C a wave: each load of B feeds all R rows' products
  const int i = R * (blockIdx.x * 4 + wave);
  if (i >= d.m || d.n <= 0) return;
  const int nr = min(R, d.m - i);
  const int kc = (d.k + splits - 1) / splits;
  int kb = blockIdx.z * kc, ke = min(d.k, kb + kc);
  if (kb >= ke && splits > 1) return;
  // columns i .. i + nr - 1 of A have no nonzeros outside the union of their
  // ranges (the entries outside a column's own range are stored zeros; the
  // result rows still get their stores, zero or not)
  if (d.tri == 1) kb = max(kb, i);
  else if (d.tri == 2) ke = min(ke, i + nr);
  C2 acc[R][NC];
  const C2* ap[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[r][j] = mk<T>(0, 0);
    ap[r] = d.A + (int64_t)(i + min(r, nr - 1)) * d.lda;   // rows past m reread the last
  }
  int l = kb + lane;
  for (; l + 64 * (U - 1) < ke; l += 64 * U) {
    C2 a[R][U], b[U][NC];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int r = 0; r < R; ++r) a[r][u] = ldc(ap[r] + l + 64 * u);
#pragma unroll
      for (int j = 0; j < NC; ++j)
        b[u][j] = j < d.n ? ldc(d.B + (int64_t)(l + 64 * u) + (int64_t)j * d.ldb) : mk<T>(0, 0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[r][j] = cadd(acc[r][j], cmulc(a[r][u], b[u][j]));
  }
  for (; l < ke; l += 64) {
    C2 a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = ldc(ap[r] + l);
#pragma unroll
    for (int j = 0; j < NC; ++j)
      if (j < d.n) {
        const C2 bb = ldc(d.B + (int64_t)l + (int64_t)j * d.ldb);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r][j] = cadd(acc[r][j], cmulc(a[r], bb));
      }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (j >= d.n) break;
      const T re = warp_sum(acc[r][j].x), im = warp_sum(acc[r][j].y);
      if (lane == 0 && r < nr) skinny_store(d, i + r, j, mk<T>(re, im), splits);
    }
}

// op(A) = A^H with a long k and too few rows of C to fill the device a wave
// per row: a workgroup per row, its four waves sharing the row's k range and
// their sums meeting in LDS in a fixed order (no k split: no atomics and no
// pre-scaling of C).
template <typename T, int NC, class DS>
__global__ __launch_bounds__(256) void gemm_skinny_cw_kernel(DS descs) {
  using C2 = cplx<T>;
  constexpr int U = SK_U / 2;
  constexpr int R = SKCW_ROWS;
  __shared__ T red[4][R][NC][2];
  const GemmDesc<T> d = descs[blockIdx.y];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = R * blockIdx.x;
  if (i >= d.m || d.n <= 0) return;   // uniform over the workgroup
  const int nr = min(R, d.m - i);
  int kb = 0, ke = d.k;
  // columns i .. i + nr - 1 of A have no nonzeros outside the union of their
  // ranges (entries outside a column's own range are stored zeros)
  if (d.tri == 1) kb = min(i, ke);
  else if (d.tri == 2) ke = min(ke, i + nr);
  C2 acc[R][NC];
  const C2* ap[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[r][j] = mk<T>(0, 0);
    ap[r] = d.A + (int64_t)(i + min(r, nr - 1)) * d.lda;   // rows past m reread the last
  }
  int l = kb + tid;
  for (; l + 256 * (U - 1) < ke; l += 256 * U) {
    C2 a[R][U], b[U][NC];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int r = 0; r < R; ++r) a[r][u] = ldc(ap[r] + l + 256 * u);
#pragma unroll
      for (int j = 0; j < NC; ++j)
        b[u][j] = j < d.n ? ldc(d.B + (int64_t)(l + 256 * u) + (int64_t)j * d.ldb) : mk<T>(0, 0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[r][j] = cadd(acc[r][j], cmulc(a[r][u], b[u][j]));
  }
  for (; l < ke; l += 256) {
    C2 a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = ldc(ap[r] + l);
#pragma unroll
    for (int j = 0; j < NC; ++j)
      if (j < d.n) {
        const C2 bb = ldc(d.B + (int64_t)l + (int64_t)j * d.ldb);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r][j] = cadd(acc[r][j], cmulc(a[r], bb));
      }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const T re = warp_sum(acc[r][j].x), im = warp_sum(acc[r][j].y);
      if (lane == 0) {
        red[wave][r][j][0] = re;
        red[wave][r][j][1] = im;
      }
    }
  __syncthreads();
  if (tid < R * NC) {
    const int r = tid / NC, j = tid % NC;
    if (r < nr && j < d.n) {
      T re = 0, im = 0;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        re += red[w][r][j][0];
        im += red[w][r][j][1];
      }
      skinny_store(d, i + r, j, mk<T>(re, im), 1);
    }
  }
}

// op(A) = A^H with a short k (at most 512): four rows of C per wave, 16 lanes
// per row (a wave per row would leave most lanes without work); the row's
// partial sums meet through row shifts within its 16 lanes.
template <typename T, int NC, class DS>
__global__ __launch_bounds__(256) void gemm_skinny_c16_kernel(DS descs, int splits) {
  using C2 = cplx<T>;
  constexpr int U = SK_U / 2;
  const GemmDesc<T> d = descs[blockIdx.y];
  if ((int)blockIdx.x * 16 >= d.m || d.n <= 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, sub = lane & 15;
  const int i = blockIdx.x * 16 + wave * 4 + (lane >> 4);
  const bool row = i < d.m;
  const int kc = (d.k + splits - 1) / splits;
  int kb = blockIdx.z * kc, ke = min(d.k, kb + kc);
  if (kb >= ke && splits > 1) return;
  if (d.tri == 1) kb = max(kb, i);
  else if (d.tri == 2) ke = min(ke, i + 1);
  C2 acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = mk<T>(0, 0);
  if (row) {
    const C2* ap = d.A + (int64_t)i * d.lda;
    int l = kb + sub;
    for (; l + 16 * (U - 1) < ke; l += 16 * U) {
      C2 a[U], b[U][NC];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        a[u] = ldc(ap + l + 16 * u);
#pragma unroll
        for (int j = 0; j < NC; ++j)
          b[u][j] = j < d.n ? ldc(d.B + (int64_t)(l + 16 * u) + (int64_t)j * d.ldb) : mk<T>(0, 0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[j] = cadd(acc[j], cmulc(a[u], b[u][j]));
    }
    for (; l < ke; l += 16) {
      const C2 a = ldc(ap + l);
#pragma unroll
      for (int j = 0; j < NC; ++j)
        if (j < d.n) acc[j] = cadd(acc[j], cmulc(a, ldc(d.B + (int64_t)l + (int64_t)j * d.ldb)));
    }
  }
  // inclusive shifts within each row of 16 lanes: lane 15 of the row holds its sum
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    T re = acc[j].x, im = acc[j].y;
    re += dpp_get<0x121, 0xF>(re);
    im += dpp_get<0x121, 0xF>(im);
    re += dpp_get<0x122, 0xF>(re);
    im += dpp_get<0x122, 0xF>(im);
    re += dpp_get<0x124, 0xF>(re);
    im += dpp_get<0x124, 0xF>(im);
    re += dpp_get<0x128, 0xF>(re);
    im += dpp_get<0x128, 0xF>(im);
    if (row && sub == 15 && j < d.n) skinny_store(d, i, j, mk<T>(re, im), splits);
  }
}

// Small products with a long k: C (m x n, m, n <= 16 MB, 16 NB) += alpha
// A^H B (the Grams of tall panels).  Memory-bound on A and B: workgroup x
// takes kc rows of k (chosen per launch for about 2048 workgroups), each wave
// a contiguous 16 U row slice per step of its loop, on 16x16x4 matrix-core
// steps (Gauss products, as in gemm_kernel).
// When A and B are the same matrix, one load feeds both operands (lane l
// supplies A(k, l % 16) for op(A) and B(k, l % 16) for B).  The four waves'
// sums meet in LDS and are added atomically to a pre-scaled C.
constexpr int SG_KMIN = 4096;   // k from which these kernels are used
constexpr int SG_U = 2;
// rows of k per workgroup: about 2048 workgroups over the batch, at least 256 rows
inline int small_out_kc(int maxk, size_t nd) {
  const int64_t want = std::max<int64_t>(1, (2048 + (int64_t)nd - 1) / (int64_t)nd);
  const int64_t chunks = std::max<int64_t>(1, std::min<int64_t>(want, maxk / 256));
  const int64_t kc = (maxk + chunks - 1) / chunks;
  return (int)((kc + 127) / 128 * 128);
}

template <typename T, int MB, int NB, class DS>
__global__ __launch_bounds__(256) void gemm_smallmn_kernel(DS descs, int kc) {
  using C2 = cplx<T>;
  using A4 = typename acc4<T>::type;
  __shared__ C2 red[16 * MB][16 * NB];
  const GemmDesc<T> d = descs[blockIdx.y];
  const int kb = (int)blockIdx.x * kc;
  if (d.m <= 0 || d.n <= 0 || kb >= d.k) return;
  const int ke = min(d.k, kb + kc);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, q = lane >> 4;
  const bool same = d.A == d.B && d.lda == d.ldb && d.m == d.n;
  A4 acc[MB][NB][3];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int t = 0; t < 3; ++t) acc[a][b][t] = A4{0, 0, 0, 0};
  bool arow[MB], bcol[NB];
#pragma unroll
  for (int a = 0; a < MB; ++a) arow[a] = 16 * a + r < d.m;
#pragma unroll
  for (int b = 0; b < NB; ++b) bcol[b] = 16 * b + r < d.n;
  constexpr int S = 4 * SG_U;   // matrix-core steps per slice
  for (int base = kb + wave * 16 * SG_U; base < ke; base += 64 * SG_U) {
    C2 av[S][MB], bv[S][NB];
#pragma unroll
    for (int st = 0; st < S; ++st) {
      const int kk = base + 4 * st + q;
#pragma unroll
      for (int a = 0; a < MB; ++a)
        av[st][a] = (kk < ke && arow[a]) ? ldc(d.A + kk + (int64_t)(16 * a + r) * d.lda)
                                         : mk<T>(0, 0);
      if (!same) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
          bv[st][b] = (kk < ke && bcol[b]) ? ldc(d.B + kk + (int64_t)(16 * b + r) * d.ldb)
                                           : mk<T>(0, 0);
      }
    }
    if (same) {
#pragma unroll
      for (int st = 0; st < S; ++st)
#pragma unroll
        for (int b = 0; b < NB; ++b) bv[st][b] = b < MB ? av[st][b] : mk<T>(0, 0);
    }
#pragma unroll
    for (int st = 0; st < S; ++st)
#pragma unroll
      for (int a = 0; a < MB; ++a) {
        // op(A) = A^H: real part A.x, imaginary part -A.y
        const T ar = av[st][a].x, ai = -av[st][a].y, as = ar + ai;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const T br = bv[st][b].x, bi = bv[st][b].y;
          acc[a][b][0] = mfma16(ar, br, acc[a][b][0]);
          acc[a][b][1] = mfma16(ai, bi, acc[a][b][1]);
          acc[a][b][2] = mfma16(as, br + bi, acc[a][b][2]);
        }
      }
  }
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T p1 = acc[a][b][0][v], p2 = acc[a][b][1][v];
            const C2 val = mk<T>(p1 - p2, acc[a][b][2][v] - p1 - p2);
            C2& o = red[16 * a + mrow<T>(lane, v)][16 * b + r];
            o = w == 0 ? val : cadd(o, val);
          }
    }
    __syncthreads();
  }
  for (int e = tid; e < d.m * d.n; e += 256) {
    const int i = e % d.m, j = e / d.m;
    const C2 v = red[i][j];
    C2* p = d.C + i + (int64_t)j * d.ldc;
    atomic_addg(&p->x, d.ar * v.x - d.ai * v.y);
    atomic_addg(&p->y, d.ar * v.y + d.ai * v.x);
  }
}

// The same products with m <= 32 and 32 < n <= 128 (a panel's reflectors
// against the columns they update): wave w owns output columns 32 w .. 32 w +
// 31 and walks the workgroup's whole k range (kc rows), adding its part of
// C atomically; the 32 x 128 output needs no cross-wave reduction.

template <typename T, class DS>
__global__ __launch_bounds__(256, 2) void gemm_smallm_wide_kernel(DS descs, int kc) {
  using C2 = cplx<T>;
  using A4 = typename acc4<T>::type;
  const GemmDesc<T> d = descs[blockIdx.y];
  const int kb = (int)blockIdx.x * kc;
  if (d.m <= 0 || d.n <= 0 || kb >= d.k) return;
  const int ke = min(d.k, kb + kc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int cb = 32 * wave;
  if (cb >= d.n) return;   // no workgroup barrier below
  A4 acc[2][2][3];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int t = 0; t < 3; ++t) acc[a][b][t] = A4{0, 0, 0, 0};
  const bool arow0 = r < d.m, arow1 = 16 + r < d.m;
  const bool bcol0 = cb + r < d.n, bcol1 = cb + 16 + r < d.n;
  constexpr int S = sizeof(T) == 8 ? 4 : 4 * SG_U;   // matrix-core steps per load batch
  for (int base = kb; base < ke; base += 4 * S) {
    C2 av[S][2], bv[S][2];
#pragma unroll
    for (int st = 0; st < S; ++st) {
      const int kk = base + 4 * st + q;
      const bool ok = kk < ke;
      av[st][0] = ok && arow0 ? ldc(d.A + kk + (int64_t)r * d.lda) : mk<T>(0, 0);
      av[st][1] = ok && arow1 ? ldc(d.A + kk + (int64_t)(16 + r) * d.lda) : mk<T>(0, 0);
      bv[st][0] = ok && bcol0 ? ldc(d.B + kk + (int64_t)(cb + r) * d.ldb) : mk<T>(0, 0);
      bv[st][1] = ok && bcol1 ? ldc(d.B + kk + (int64_t)(cb + 16 + r) * d.ldb) : mk<T>(0, 0);
    }
#pragma unroll
    for (int st = 0; st < S; ++st)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        // op(A) = A^H: real part A.x, imaginary part -A.y
        const T ar = av[st][a].x, ai = -av[st][a].y, as = ar + ai;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const T br = bv[st][b].x, bi = bv[st][b].y;
          acc[a][b][0] = mfma16(ar, br, acc[a][b][0]);
          acc[a][b][1] = mfma16(ai, bi, acc[a][b][1]);
          acc[a][b][2] = mfma16(as, br + bi, acc[a][b][2]);
        }
      }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * a + mrow<T>(lane, v), j = cb + 16 * b + r;
        if (i >= d.m || j >= d.n) continue;
        const T p1 = acc[a][b][0][v], p2 = acc[a][b][1][v];
        const T vr = p1 - p2, vi = acc[a][b][2][v] - p1 - p2;
        C2* p = d.C + i + (int64_t)j * d.ldc;
        atomic_addg(&p->x, d.ar * vr - d.ai * vi);
        atomic_addg(&p->y, d.ar * vi + d.ai * vr);
      }
}

// C <- beta C for split-k launches (beta 0 writes zeros)
template <typename T, class DS>
__global__ void gemm_prescale_kernel(DS descs) {
  const GemmDesc<T> d = descs[blockIdx.y];
  if (d.beta == T(1)) return;
  int64_t cnt = (int64_t)d.m * d.n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256) {
    int i = (int)(e % d.m), j = (int)(e / d.m);
    cplx<T>* p = d.C + (int64_t)i + (int64_t)j * d.ldc;
    if (d.beta == T(0)) stc(p, mk<T>(0, 0));
    else { cplx<T> v = ldc(p); stc(p, mk<T>(v.x * d.beta, v.y * d.beta)); }
  }
}

// -------------------------------------------------------------- QR panel
// Householder vectors follow the LAPACK larfg convention (H = I - tau v v^H,
// v_0 = 1, H^H x = beta e_1 with real beta); each panel also produces its
// compact-WY factor T (Q_panel = I - V T V^H) and the explicit V / R split
// described in la.h.
//
// Panel factorization: a group of gsize workgroups factors one problem's
// panel; workgroup w of the group holds panel rows [w 128 R, (w+1) 128 R)
// in registers.  Wave v of a workgroup owns the column group v / 2 (QP_CG
// consecutive columns) on the row half v % 2; lane l of it holds rows
// half * 64 QP_R + l + 64 k (k < QP_R) of those columns, so loads and stores
// are coalesced and the per-column sums reduce within the wave (DPP) to one
// partial per row half.  The pivot column is published to LDS with its rows
// at and above the diagonal zeroed (double-buffered), so the sums and the
// update need no row masks.  With gsize > 1 the workgroups add their sums
// atomically into a rotating scratch buffer and meet at a group barrier.
// Every thread derives the reflector (tau, beta, 1/(alpha - beta)) and the
// update u_c = A(jj, c) + conj(scal) s_c by itself.  Row jj (jj < QR_NB) is
// lane jj of the first row half of workgroup 0.  Groups loop over problems.
// Requires all workgroups to be resident (cooperative launch).
//
// Everything the workgroups of a group exchange goes through device-coherent
// operations: atomic adds of the sums, agent-scope atomic stores and loads
// of the pivot row and of the zeroed slot.  The barrier therefore needs no
// L2 writeback or invalidate (an agent-scope release or acquire costs both on
// this multi-die part); each thread waits for all its memory operations to
// complete before the workgroup arrives, which orders the exchanged stores
// before the arrival count.
//
// The wait is bounded (2^20 polls, well under a second) and gives up at once
// once err is set, by this or any other workgroup: after one timeout the
// panel's remaining barriers fall through instead of each waiting its full
// bound, and the host reports the error after the launch.
__device__ inline void group_barrier(unsigned* cnt, unsigned target, int* err) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned it = 0;
    bool failed = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    while (!failed &&
           __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if ((++it & 255) == 0 &&
          (it > (1u << 20) || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
        atomicExch(err, 1);
        failed = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
}

template <typename T>
__device__ inline void st_agent(cplx<T>* p, cplx<T> v) {
  __hip_atomic_store(&p->x, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&p->y, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline cplx<T> ld_agent(const cplx<T>* p) {
  return mk<T>(__hip_atomic_load(&p->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
               __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// FP32 exchange words: a float and the column step's tag in one 64-bit
// agent-scope atomic word, so a reader that sees the tag sees the value (no
// fence, no separate counter).
__device__ inline void st_tagged(unsigned long long* p, float v, unsigned tag) {
  const unsigned long long w = (unsigned long long)__float_as_uint(v) |
                               ((unsigned long long)tag << 32);
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long ld_tagged(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// wait until the two words at p carry tag (bounded; sets err on timeout and
// gives up at once when err is already set) and return their values
__device__ inline float2 wait_tagged2(const unsigned long long* p, unsigned tag, int* err) {
  unsigned long long a = ld_tagged(p), b = ld_tagged(p + 1);
  unsigned it = 0;
  while ((unsigned)(a >> 32) != tag || (unsigned)(b >> 32) != tag) {
    if ((++it & 255) == 0 &&
        (it > (1u << 20) || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
      atomicExch(err, 1);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
    a = ld_tagged(p);
    b = ld_tagged(p + 1);
  }
  return make_float2(__uint_as_float((unsigned)a), __uint_as_float((unsigned)b));
}
// FP32 group scratch: two sets (by column-step parity) of gsize partial-sum
// rows and one pivot row, each QR_NB complex values as tagged word pairs
__host__ __device__ inline size_t qp_tag_words(int gsize) {
  return (size_t)2 * (gsize + 1) * QR_NB * 2;
}

constexpr int QS = QR_NB + 1;          // rotating sum slots per column
constexpr int QSCR = 3 * QS + 3 * QR_NB;   // rotating sums + rotating row copies
constexpr int QP_NT = 1024;            // threads of a panel workgroup
constexpr int QP_CG = 4;               // columns per thread
// rows per lane: 4 x 4 complex FP32 or 2 x 4 complex FP64 values (32 VGPRs)
template <typename T> struct QPanel { static constexpr int R = 2; };
template <> struct QPanel<float> { static constexpr int R = 4; };

// sum over the 64 lanes of a wave, valid in lane 63 (all lanes active)
template <typename T>
__device__ inline T wave_sum63(T v) {
  v += dpp_get<0x121, 0xF>(v);
  v += dpp_get<0x122, 0xF>(v);
  v += dpp_get<0x124, 0xF>(v);
  v += dpp_get<0x128, 0xF>(v);
  v += dpp_get<0x142, 0xA>(v);
  v += dpp_get<0x143, 0xC>(v);
  return v;
}

// RM = 2 doubles the rows each lane holds, for panels taller than the
// device holds at RM = 1 (one workgroup per CU)
template <typename T, class AS, int RM = 1>
__global__ __launch_bounds__(QP_NT) void qr_panel_kernel(
    const QRDesc<T>* __restrict__ descs, AS active, int nact, int j0, int gsize,
    cplx<T>* __restrict__ scratch, unsigned* __restrict__ bar, int* __restrict__ err) {
  using C2 = cplx<T>;
  constexpr int R = QPanel<T>::R * RM;
  constexpr int HALF = 64 * R;           // rows of one row half
  constexpr int ROWS = 2 * HALF;         // rows of a workgroup
  static_assert(QP_NT / 64 == 2 * (QR_NB / QP_CG), "16 waves: 8 column groups x 2 row halves");
  __shared__ C2 X[2][ROWS];              // pivot column, double-buffered
  __shared__ C2 sp[2][QR_NB];            // per row half column sums
  __shared__ C2 tot[QR_NB];              // (gsize > 1) group column sums
  __shared__ C2 rowv[QR_NB];             // row jj
  __shared__ C2 Ts[QR_NB][QR_NB + 1];
  __shared__ C2 red[QP_NT / QR_NB][QR_NB];   // (FP32, gsize > 1) partial sums of the group
  const int ngroups = gridDim.x / gsize;
  const int g = blockIdx.x / gsize, w = blockIdx.x % gsize;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int cg = wv >> 1, hf = wv & 1;
  const int c0 = cg * QP_CG;             // first column of this thread
  const int lr = hf * HALF + lane;       // workgroup row of k = 0
  C2* sums = scratch + (size_t)g * QSCR;
  C2* rows = sums + 3 * QS;
  unsigned* cnt = bar + g;
  unsigned epoch = 0;
  int step = 0;
  for (int pi = g; pi < nact; pi += ngroups) {
    const QRDesc<T> d = descs[active[pi]];
    const int kmin = min(d.m, d.n);
    const int jb = min(QR_NB, kmin - j0);
    const int mr = d.m - j0;
    const int r0 = w * ROWS;
    C2* Ap = d.A + j0 + (int64_t)j0 * d.lda;
    C2 a[R][QP_CG];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int gi = r0 + lr + 64 * k;
#pragma unroll
      for (int l = 0; l < QP_CG; ++l)
        a[k][l] = (gi < mr && c0 + l < jb) ? ldc(Ap + gi + (int64_t)(c0 + l) * d.lda) : mk<T>(0, 0);
    }
    if (w == 0)
      for (int e = tid; e < QR_NB * QR_NB; e += QP_NT) Ts[e % QR_NB][e / QR_NB] = mk<T>(0, 0);
    if (cg == 0) {
#pragma unroll
      for (int k = 0; k < R; ++k) X[0][lr + 64 * k] = r0 + lr + 64 * k > 0 ? a[k][0] : mk<T>(0, 0);
    }
    __syncthreads();
    for (int jj = 0; jj < jb; ++jj, ++step) {
      // ---- column sums conj(x)^T A(:, c) over the rows below the diagonal
      //      (sigma^2 in the pivot's own slot), one per row half
      C2 xv[R];
#pragma unroll
      for (int k = 0; k < R; ++k) xv[k] = X[jj & 1][lr + 64 * k];
#pragma unroll
      for (int l = 0; l < QP_CG; ++l) {
        T sr = 0, si = 0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
          sr += xv[k].x * a[k][l].x + xv[k].y * a[k][l].y;
          si += xv[k].x * a[k][l].y - xv[k].y * a[k][l].x;
        }
        sr = wave_sum63(sr);
        si = wave_sum63(si);
        if (lane == 63) sp[hf][c0 + l] = mk<T>(sr, si);
      }
      const bool row_owner = r0 == 0 && hf == 0 && lane == jj;
      if (row_owner && gsize == 1) {
#pragma unroll
        for (int l = 0; l < QP_CG; ++l) rowv[c0 + l] = a[0][l];
      }
      __syncthreads();
      if constexpr (sizeof(T) == 4) {
        if (gsize > 1) {
          // publish this workgroup's sums (and, from workgroup 0, row jj) as
          // tagged words; every workgroup reads all of them: thread (j, c)
          // adds the partials of workgroups j, j + 32, ... for column c, then
          // the 32 partials per column are added in a fixed order
          unsigned long long* tg = (unsigned long long*)scratch + (size_t)g * qp_tag_words(gsize);
          unsigned long long* part = tg + (size_t)(step & 1) * (gsize + 1) * QR_NB * 2;
          unsigned long long* rowp = part + (size_t)gsize * QR_NB * 2;
          const unsigned tag = (unsigned)step + 1;
          if (tid < QR_NB) {
            unsigned long long* q = part + ((size_t)w * QR_NB + tid) * 2;
            st_tagged(q, sp[0][tid].x + sp[1][tid].x, tag);
            st_tagged(q + 1, sp[0][tid].y + sp[1][tid].y, tag);
          }
          if (row_owner) {
#pragma unroll
            for (int l = 0; l < QP_CG; ++l) {
              st_tagged(rowp + (c0 + l) * 2, (float)a[0][l].x, tag);
              st_tagged(rowp + (c0 + l) * 2 + 1, (float)a[0][l].y, tag);
            }
          }
          const int cj = tid % QR_NB, jj2 = tid / QR_NB;
          float vr = 0.f, vi = 0.f;
          for (int w2 = jj2; w2 < gsize; w2 += QP_NT / QR_NB) {
            const float2 v = wait_tagged2(part + ((size_t)w2 * QR_NB + cj) * 2, tag, err);
            vr += v.x;
            vi += v.y;
          }
          red[jj2][cj] = mk<T>(vr, vi);
          if (jj2 == 0) {
            const float2 v = wait_tagged2(rowp + cj * 2, tag, err);
            rowv[cj] = mk<T>(v.x, v.y);
          }
          __syncthreads();
          if (tid < QR_NB) {
            T tr = 0, ti = 0;
            for (int j2 = 0; j2 < QP_NT / QR_NB; ++j2) {
              tr += red[j2][tid].x;
              ti += red[j2][tid].y;
            }
            tot[tid] = mk<T>(tr, ti);
          }
          __syncthreads();
        }
      } else if (gsize > 1) {
        C2* buf = sums + (step % 3) * QS;
        C2* rbuf = rows + (step % 3) * QR_NB;
        if (tid < QR_NB) {
          const T vr = sp[0][tid].x + sp[1][tid].x, vi = sp[0][tid].y + sp[1][tid].y;
          if (vr != T(0)) atomicAdd(&buf[tid].x, vr);
          if (vi != T(0)) atomicAdd(&buf[tid].y, vi);
        }
        if (row_owner) {
#pragma unroll
          for (int l = 0; l < QP_CG; ++l) st_agent<T>(rbuf + c0 + l, a[0][l]);
        }
        if (w == 0 && tid < QS) st_agent<T>(sums + ((step + 1) % 3) * QS + tid, mk<T>(0, 0));
        group_barrier(cnt, (++epoch) * (unsigned)gsize, err);
        if (tid < QR_NB) {
          tot[tid] = ld_agent<T>(buf + tid);
          rowv[tid] = ld_agent<T>(rbuf + tid);
        }
        __syncthreads();
      }
      auto colsum = [&](int c) -> C2 {
        return gsize == 1 ? cadd(sp[0][c], sp[1][c]) : tot[c];
      };
      // ---- the reflector, derived by every thread from sigma^2 and A(jj, jj)
      C2 tau, scal;
      T beta;
      {
        const T sig = colsum(jj).x;
        const C2 alpha = rowv[jj];
        if (sig == T(0) && alpha.y == T(0)) {
          tau = mk<T>(0, 0);
          scal = mk<T>(0, 0);
          beta = alpha.x;
        } else {
          const T nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sig);
          beta = alpha.x >= T(0) ? -nrm : nrm;
          tau = mk<T>((beta - alpha.x) / beta, -alpha.y / beta);
          const T dr = alpha.x - beta, di = alpha.y;
          const T den = dr * dr + di * di;
          scal = mk<T>(dr / den, -di / den);
        }
      }
      if (w == 0) {
        // T(0:jj, jj) = -tau T(0:jj, 0:jj) z,  z_q = v_q^H v_jj = scal conj(s_q) + conj(A(jj, q)):
        // thread (q, i) = (tid % 32, tid / 32) forms T(i, q) z_q, the 32
        // lanes of row i sum them (row rotations, then row_bcast 15 into
        // lanes 16..31 of each half-wave)
        const int q = tid % QR_NB, i = tid / QR_NB;
        C2 pr = mk<T>(0, 0);
        if (i < jj && q >= i && q < jj) {
          const C2 z = cadd(cmul(scal, cconj(colsum(q))), cconj(rowv[q]));
          pr = cmul(Ts[i][q], z);
        }
        T sr = pr.x, si = pr.y;
        sr += dpp_get<0x121, 0xF>(sr);
        si += dpp_get<0x121, 0xF>(si);
        sr += dpp_get<0x122, 0xF>(sr);
        si += dpp_get<0x122, 0xF>(si);
        sr += dpp_get<0x124, 0xF>(sr);
        si += dpp_get<0x124, 0xF>(si);
        sr += dpp_get<0x128, 0xF>(sr);
        si += dpp_get<0x128, 0xF>(si);
        sr += dpp_get<0x142, 0xA>(sr);
        si += dpp_get<0x142, 0xA>(si);
        if (q == 16 && i < jj) {
          const C2 t = cmul(tau, mk<T>(sr, si));
          Ts[i][jj] = mk<T>(-t.x, -t.y);
        }
        if (tid == 0) Ts[jj][jj] = tau;
      }
      // ---- update (branches are uniform per wave): columns right of jj
      //      lose conj(tau) v u_c with v = (1, scal x); column jj becomes v
      //      below the diagonal and beta on it
#pragma unroll
      for (int l = 0; l < QP_CG; ++l) {
        const int c = c0 + l;
        if (c > jj && c < jb) {
          const C2 u = cadd(rowv[c], cmul(cconj(scal), colsum(c)));
          const C2 fu = cmul(cconj(tau), u);
          const C2 sfu = cmul(scal, fu);
#pragma unroll
          for (int k = 0; k < R; ++k) a[k][l] = csub(a[k][l], cmul(xv[k], sfu));
          if (row_owner) a[0][l] = csub(a[0][l], fu);
        } else if (c == jj) {
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const int gi = r0 + lr + 64 * k;
            if (gi == jj) a[k][l] = mk<T>(beta, 0);
            else if (gi > jj) a[k][l] = cmul(a[k][l], scal);
          }
        }
      }
      // ---- publish the next pivot column
      if (jj + 1 < jb && cg == (jj + 1) / QP_CG) {
        const int ln = (jj + 1) % QP_CG;
#pragma unroll
        for (int k = 0; k < R; ++k) {
          C2 v = a[k][0];
#pragma unroll
          for (int l = 1; l < QP_CG; ++l)
            if (l == ln) v = a[k][l];
          X[(jj + 1) & 1][lr + 64 * k] = r0 + lr + 64 * k > jj + 1 ? v : mk<T>(0, 0);
        }
      }
      __syncthreads();
    }
    // ---- write back: R block rows, explicit V, T
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int gi = r0 + lr + 64 * k;
#pragma unroll
      for (int l = 0; l < QP_CG; ++l) {
        const int c = c0 + l;
        if (gi >= mr || c >= jb) continue;
        C2* pa = Ap + gi + (int64_t)c * d.lda;
        if (gi < jb) {
          C2* pr = d.R + (j0 + gi) + (int64_t)(j0 + c) * d.ldr;
          if (gi <= c) {
            stc(pr, a[k][l]);
            stc(pa, gi == c ? mk<T>(1, 0) : mk<T>(0, 0));
          } else {
            stc(pr, mk<T>(0, 0));
            stc(pa, a[k][l]);
          }
        } else {
          stc(pa, a[k][l]);
        }
      }
    }
    if (w == 0) {
      // the rows above the panel inside its block of QR_OB columns move from
      // A to R (the block's reflectors are read from row J0 on, so these
      // must be zero before the block's later steps); the rows above the
      // block and R below the panel's diagonal block are left to
      // qr_finish_kernel, which runs with the whole device
      const int J0 = j0 - j0 % QR_OB, na = j0 - J0;
      for (int e = tid; e < jb * na; e += QP_NT) {
        const int r = J0 + e % na, c = e / na;
        C2* pa = d.A + r + (int64_t)(j0 + c) * d.lda;
        d.R[r + (int64_t)(j0 + c) * d.ldr] = *pa;
        *pa = mk<T>(0, 0);
      }
      const int blk = (j0 % QR_OB) / QR_NB;
      C2* Tb = d.Tw + (int64_t)blk * QR_NB * QR_NB;
      for (int e = tid; e < QR_NB * QR_NB; e += QP_NT) {
        const int r = e % QR_NB, c = e / QR_NB;
        Tb[r + c * QR_NB] = (r < jb && c < jb) ? Ts[r][c] : mk<T>(0, 0);
      }
    }
    __syncthreads();
  }
}

// T of one block of QR_OB reflectors from its panels' factors: with
// S = V^H V of the block's reflectors and the panels' T_j on the diagonal,
// T(0:c0, c0:c0+jb) = -T(0:c0, 0:c0) S(0:c0, c0:c0+jb) T_j for the panels in
// order (Q_A Q_B = I - [V_A V_B] [T_A, -T_A V_A^H V_B T_B; 0, T_B] [V_A V_B]^H).
template <typename T>
struct WyDesc {
  int kb, lds, ldt;    // kb <= QR_HB
  const cplx<T>* Tw;   // the panels' QR_NB x QR_NB factors
  const cplx<T>* S;    // kb x kb, lds
  cplx<T>* Tout;       // kb x kb, leading dimension ldt
};

constexpr int WY_NT = 1024;   // threads of a merge workgroup (one per problem)

template <typename T, class DS>
__global__ __launch_bounds__(WY_NT) void wy_merge_kernel(DS descs) {
  using C2 = cplx<T>;
  constexpr int NB = QR_NB, NR = QR_HB - QR_NB;   // panel width, most rows above a panel
  const WyDesc<T> d = descs[blockIdx.x];
  const int kb = d.kb, ldt = d.ldt, tid = threadIdx.x;
  const int nbi = (kb + NB - 1) / NB;
  C2* To = d.Tout;
  // X = S(0:c0, c0:c0+jb) T_j.  U holds S's block and T_j while X is formed,
  // then 32-column chunks of T(0:c0, 0:c0); rows padded by one against bank
  // conflicts.  Every operand is staged with one batch of coalesced loads.
  __shared__ C2 X[NR][NB + 1];
  __shared__ C2 U[(NR + NB) * (NB + 1)];
  C2(*Sb)[NB + 1] = reinterpret_cast<C2(*)[NB + 1]>(U);
  C2(*Tj)[NB + 1] = reinterpret_cast<C2(*)[NB + 1]>(U + NR * (NB + 1));
  C2(*Tc)[NB + 1] = reinterpret_cast<C2(*)[NB + 1]>(U);
  for (int e = tid; e < kb * kb; e += WY_NT) {
    int r = e % kb, c = e / kb;
    int bi = r / NB, bj = c / NB;
    stc(To + r + (int64_t)c * ldt,
        bi == bj ? ldc(d.Tw + (int64_t)bi * NB * NB + (r % NB) + (c % NB) * NB) : mk<T>(0, 0));
  }
  __syncthreads();
  constexpr int EPT = (NR * NB + WY_NT - 1) / WY_NT;   // output entries per thread
  for (int j = 1; j < nbi; ++j) {
    const int c0 = j * NB, jb = min(NB, kb - c0);
    for (int e = tid; e < c0 * jb; e += WY_NT) {
      const int r = e % c0, c = e / c0;
      Sb[r][c] = ldc(d.S + r + (int64_t)(c0 + c) * d.lds);
    }
    for (int e = tid; e < jb * jb; e += WY_NT) {
      const int q = e % jb, c = e / jb;
      Tj[q][c] = ldc(d.Tw + (int64_t)j * NB * NB + q + c * NB);
    }
    __syncthreads();
    for (int e = tid; e < c0 * jb; e += WY_NT) {
      const int r = e % c0, c = e / c0;
      C2 sum = mk<T>(0, 0);
      for (int q = 0; q <= c; ++q) sum = cadd(sum, cmul(Sb[r][q], Tj[q][c]));   // T_j upper
      X[r][c] = sum;
    }
    __syncthreads();
    // T(0:c0, c0:c0+jb) = -T(0:c0, 0:c0) X, T(0:c0, 0:c0) upper triangular
    C2 acc[EPT];
#pragma unroll
    for (int t = 0; t < EPT; ++t) acc[t] = mk<T>(0, 0);
    for (int qb = 0; qb < c0; qb += NB) {
      for (int e = tid; e < c0 * NB; e += WY_NT) {
        const int r = e % c0, qq = e / c0;
        Tc[r][qq] = ldc(To + r + (int64_t)(qb + qq) * ldt);
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < EPT; ++t) {
        const int e = tid + t * WY_NT;
        if (e < c0 * jb) {
          const int r = e % c0, c = e / c0;
          for (int qq = max(r - qb, 0); qq < NB; ++qq) acc[t] = cadd(acc[t], cmul(Tc[r][qq], X[qb + qq][c]));
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
      const int e = tid + t * WY_NT;
      if (e < c0 * jb) {
        const int r = e % c0, c = e / c0;
        stc(To + r + (int64_t)(c0 + c) * ldt, mk<T>(-acc[t].x, -acc[t].y));
      }
    }
    __syncthreads();
  }
}

// The end of a factorization, over all of R (kmin x n): for column c < kmin
// of the block starting at J0, the rows above J0 move from A to R (A keeps
// zeros there) and R below the diagonal block of c's panel is zero (the
// panels wrote the rows from J0 to the end of their diagonal blocks); the
// trailing columns of wide problems (n > m) are copied into R.
template <typename T>
__global__ void qr_finish_kernel(const QRDesc<T>* __restrict__ descs) {
  const QRDesc<T> d = descs[blockIdx.y];
  const int kmin = min(d.m, d.n);
  if (kmin <= 0) return;
  const int64_t cnt = (int64_t)kmin * d.n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256) {
    const int r = (int)(e % kmin), c = (int)(e / kmin);
    cplx<T>* pr = d.R + r + (int64_t)c * d.ldr;
    cplx<T>* pa = d.A + r + (int64_t)c * d.lda;
    if (c >= kmin) {
      *pr = *pa;
      continue;
    }
    const int J0 = c - c % QR_OB, pe = min(c - c % QR_NB + QR_NB, kmin);
    if (r < J0) {
      *pr = *pa;
      *pa = mk<T>(0, 0);
    } else if (r >= pe) {
      *pr = mk<T>(0, 0);
    }
  }
}

// ------------------------------------------------------------ pivoted Cholesky
constexpr int PC_NB = 128;   // pivots per panel (one Schur update of the Gram per panel)

__global__ void pchol_init_kernel(const PcholDesc* __restrict__ descs, double* trace_out) {
  const PcholDesc d = descs[blockIdx.x];
  __shared__ double red[4];
  double s = 0;
  for (int i = threadIdx.x; i < d.w; i += 256) {
    double v = d.K[i + (int64_t)i * d.ldk].x;
    d.d[i] = v;
    s += v;
  }
  s = warp_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    trace_out[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    *d.rank = 0;
  }
}

// Column-parallel pivoted Cholesky: one launch per pivot column, workgroup w
// of Gram b owning rows [256 w, 256 w + 256) (one per thread).  The
// workgroups exchange their partials of the Schur diagonal (largest entry,
// its row, positive trace) through global slots, double-buffered by column
// parity; the launch boundary orders a column's partials before their use,
// so no workgroup waits on another inside a launch.  Ties go to the lower
// row.  state[b]: 1 = still running.
constexpr int PC_ROWS = 256;

__device__ inline bool pc_better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i >= 0 && (bi < 0 || i < bi));
}

// (largest, row, sum) over the workgroup, valid in thread 0
__device__ inline void pc_reduce(double& best, int& bi, double& sum) {
  __shared__ double rv[4], rs[4];
  __shared__ int ri[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  sum = warp_sum(sum);
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (pc_better(ob, oi, best, bi)) {
      best = ob;
      bi = oi;
    }
  }
  if (lane == 0) {
    rv[wave] = best;
    ri[wave] = bi;
    rs[wave] = sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 1; v < 4; ++v) {
      rs[0] += rs[v];
      if (pc_better(rv[v], ri[v], rv[0], ri[0])) {
        rv[0] = rv[v];
        ri[0] = ri[v];
      }
    }
    best = rv[0];
    bi = ri[0];
    sum = rs[0];
  }
  __syncthreads();
}

// partial of this workgroup's rows of the diagonal workspace d
__device__ inline void pc_partial(const PcholDesc& d, int i, double di, double* slot) {
  double best = -1.0, sum = 0.0;
  int bi = -1;
  if (i < d.w && di > -1e300) {   // pivoted rows hold -inf
    sum = di > 0 ? di : 0;
    if (di > best) {
      best = di;
      bi = i;
    }
  }
  pc_reduce(best, bi, sum);
  if (threadIdx.x == 0) {
    slot[0] = best;
    slot[1] = (double)bi;
    slot[2] = sum;
  }
}

// partials of the current diagonal into slot parity `par`
__global__ __launch_bounds__(256) void pchol_part_kernel(const PcholDesc* __restrict__ descs,
                                                         int gsize, double* __restrict__ part,
                                                         int par) {
  const int b = blockIdx.x / gsize, w = blockIdx.x % gsize;
  const PcholDesc d = descs[b];
  if (w * PC_ROWS >= max(d.w, 1)) return;
  const int i = w * PC_ROWS + threadIdx.x;
  const double di = i < d.w ? d.d[i] : -1.0 / 0.0;
  pc_partial(d, i, di, part + (((size_t)b * 2 + par) * gsize + w) * 3);
}

// column k = k0 + kk of every running Gram
__global__ __launch_bounds__(256) void pchol_col_kernel(const PcholDesc* __restrict__ descs,
                                                        const double* __restrict__ trace,
                                                        int* __restrict__ state, int gsize,
                                                        double* __restrict__ part, int k0,
                                                        int kk) {
  const int b = blockIdx.x / gsize, w = blockIdx.x % gsize;
  if (!state[b]) return;
  const PcholDesc d = descs[b];
  const int gw = (max(d.w, 1) + PC_ROWS - 1) / PC_ROWS;   // workgroups holding rows
  if (w >= gw) return;
  const int tid = threadIdx.x;
  const int k = k0 + kk;
  __shared__ double2 lp[PC_NB];
  __shared__ int piv_s, stop_s;
  __shared__ double dp_s;
  // combine the workgroups' partials of this column in wave 0: lane l takes
  // partials l, l + 64, ... (all its loads in flight at once), then an xor
  // butterfly leaves every lane the same sum and the same winner (ties to
  // the lower row); the order is fixed, so every workgroup agrees
  double bb = -1.0, ss = 0.0;
  int ii = -1;
  if (tid < 64) {
    const double* sl = part + ((size_t)b * 2 + (k & 1)) * gsize * 3;
    for (int v = tid; v < gw; v += 64) {
      const double pv = sl[3 * v], pi = sl[3 * v + 1], ps = sl[3 * v + 2];
      ss += ps;
      if (pc_better(pv, (int)pi, bb, ii)) {
        bb = pv;
        ii = (int)pi;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(bb, o, 64), os = __shfl_xor(ss, o, 64);
      const int oi = __shfl_xor(ii, o, 64);
      ss += os;
      if (pc_better(ob, oi, bb, ii)) {
        bb = ob;
        ii = oi;
      }
    }
  }
  if (tid == 0) {
    const double tol = d.tol2 * trace[b];
    const int stop = (k >= d.rmax || k >= d.w || ss <= tol || ii < 0 || bb <= 0.0) ? 1 : 0;
    stop_s = stop;
    piv_s = ii;
    dp_s = bb;
    if (w == 0) {
      if (stop) {
        *d.rank = k;
        state[b] = 0;
      } else {
        d.piv[k] = ii;
      }
    }
  }
  __syncthreads();
  if (stop_s) return;
  const int p = piv_s;
  const double sdp = sqrt(dp_s);
  // conj of the pivot row's earlier entries in this panel
  if (tid < kk) lp[tid] = d.L[p + (int64_t)(k0 + tid) * d.ldl];
  __syncthreads();
  const int i = w * PC_ROWS + tid;
  double di = -1.0 / 0.0;
  if (i < d.w) {
    di = d.d[i];
    // L(i,k) = (K(i,p) - sum_q L(i,q) conj(L(p,q))) / sqrt(d_p); K holds its lower triangle
    double2 v = i >= p ? d.K[i + (int64_t)p * d.ldk] : cconj(d.K[p + (int64_t)i * d.ldk]);
    const double2* li = d.L + i + (int64_t)k0 * d.ldl;
    // the row's panel entries in batches of 16 loads in flight
    int q = 0;
    for (; q + 16 <= kk; q += 16) {
      double2 l16[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) l16[u] = li[(int64_t)(q + u) * d.ldl];
#pragma unroll
      for (int u = 0; u < 16; ++u) v = csub(v, cmulc(lp[q + u], l16[u]));
    }
    for (; q + 4 <= kk; q += 4) {
      double2 l4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) l4[u] = li[(int64_t)(q + u) * d.ldl];
#pragma unroll
      for (int u = 0; u < 4; ++u) v = csub(v, cmulc(lp[q + u], l4[u]));
    }
    for (; q < kk; ++q) v = csub(v, cmulc(lp[q], li[(int64_t)q * d.ldl]));
    if (di <= -1e300) v = mk<double>(0.0, 0.0);
    v.x /= sdp;
    v.y /= sdp;
    if (i == p) v = mk<double>(sdp, 0.0);
    d.L[i + (int64_t)k * d.ldl] = v;
    if (i == p) di = -1.0 / 0.0;
    else if (di > -1e300) di -= v.x * v.x + v.y * v.y;
    d.d[i] = di;
  }
  // partials of the next column
  pc_partial(d, i, di, part + (((size_t)b * 2 + ((k + 1) & 1)) * gsize + w) * 3);
}

__global__ void pchol_finish_kernel(const PcholDesc* __restrict__ descs, const int* state, int kend) {
  const PcholDesc d = descs[blockIdx.x];
  if (threadIdx.x == 0 && state[blockIdx.x]) *d.rank = min(kend, min(d.rmax, d.w));
}

// Schur update of the unpivoted part: K -= L_p L_p^H with the panel's columns.
// Done with the GEMM kernel (opB = C) by the host.

// ------------------------------------------------------------ triangular solve
// R X = B (CT = false, back substitution) or R^H X = B (CT = true, forward
// substitution), R upper triangular of order k <= TRS_B; one workgroup per
// (system, column of B).  The workgroup stages R's upper triangle in LDS,
// packed by columns ((r, c), r <= c, at c (c + 1) / 2 + r), with the inverted
// diagonal; one wave then substitutes with the right-hand side in registers
// (lane l holds rows l and l + 64) and broadcasts each solved entry with a
// lane read.
constexpr int TRS_B = 128;

template <typename T, bool CT, class DS>
__global__ __launch_bounds__(256) void trsv_lds_kernel(DS descs) {
  using C2 = cplx<T>;
  __shared__ C2 Rp[TRS_B * (TRS_B + 1) / 2];
  __shared__ C2 inv[TRS_B];
  const TrsDesc<T> d = descs[blockIdx.x];
  const int rhs = blockIdx.y;
  if (rhs >= d.nrhs || d.k <= 0) return;
  const int k = min(d.k, TRS_B);
  const int ne = k * (k + 1) / 2;
  const int tid = threadIdx.x;
  for (int e0 = 0; e0 < ne; e0 += 256 * 8) {
    C2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256 + tid;
      v[u] = mk<T>(0, 0);
      if (e < ne) {
        int c = (int)((sqrtf(8.f * (float)e + 1.f) - 1.f) * 0.5f);
        while ((c + 1) * (c + 2) / 2 <= e) ++c;
        while (c * (c + 1) / 2 > e) --c;
        v[u] = ldc(d.R + (e - c * (c + 1) / 2) + (int64_t)c * d.ldr);
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256 + tid;
      if (e < ne) Rp[e] = v[u];
    }
  }
  __syncthreads();
  if (tid < k) {
    C2 r = Rp[tid * (tid + 1) / 2 + tid];
    if (CT) r.y = -r.y;
    const T den = r.x * r.x + r.y * r.y;
    inv[tid] = mk<T>(r.x / den, -r.y / den);
  }
  __syncthreads();
  if (tid >= 64) return;
  const int lane = tid;
  C2* b = d.B + (int64_t)rhs * d.ldb;
  C2 x0 = lane < k ? b[lane] : mk<T>(0, 0);
  C2 x1 = lane + 64 < k ? b[lane + 64] : mk<T>(0, 0);
  for (int s = 0; s < k; ++s) {
    const int i = CT ? s : k - 1 - s;
    const int ow = i & 63;
    const C2 bi = (i >> 6) ? x1 : x0;
    C2 xi = cmul(bi, inv[i]);
    xi.x = lane_bcast(xi.x, ow);
    xi.y = lane_bcast(xi.y, ow);
    if (lane == ow) {
      if (i >> 6) x1 = xi;
      else x0 = xi;
    }
    if (!CT) {
      // rows above i: b_r -= R(r, i) x_i
      const int off = i * (i + 1) / 2;
      if (lane < i) x0 = csub(x0, cmul(Rp[off + lane], xi));
      if (lane + 64 < i) x1 = csub(x1, cmul(Rp[off + lane + 64], xi));
    } else {
      // rows below i: b_r -= conj(R(i, r)) x_i
      const int r0 = lane, r1 = lane + 64;
      if (r0 > i && r0 < k) x0 = csub(x0, cmul(cconj(Rp[r0 * (r0 + 1) / 2 + i]), xi));
      if (r1 > i && r1 < k) x1 = csub(x1, cmul(cconj(Rp[r1 * (r1 + 1) / 2 + i]), xi));
    }
  }
  if (lane < k) b[lane] = x0;
  if (lane + 64 < k) b[lane + 64] = x1;
}

// ------------------------------------------------------------ copy / fill
template <typename TD, typename TS, class DS>
__global__ void copy_kernel(DS descs) {
  const CopyDesc<TD, TS> d = descs[blockIdx.y];
  int64_t cnt = (int64_t)d.m * d.n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256) {
    int i = (int)(e % d.m), j = (int)(e / d.m);
    cplx<TS> v = d.S[i + (int64_t)j * d.lds];
    cplx<TD> o = mk<TD>((TD)v.x, (TD)v.y);
    if (d.conj_trans) {
      o.y = -o.y;
      d.D[j + (int64_t)i * d.ldd] = o;
    } else {
      d.D[i + (int64_t)j * d.ldd] = o;
    }
  }
}

// D = S^H through 32 x 32 tiles staged in LDS, so that both the reads of S
// and the writes of D run along columns (coalesced)
template <typename TD, typename TS, class DS>
__global__ __launch_bounds__(256) void copy_ct_kernel(DS descs) {
  const CopyDesc<TD, TS> d = descs[blockIdx.y];
  __shared__ cplx<TS> t[32][33];   // t[j][i] = S(i0 + i, j0 + j)
  const int tm = (d.m + 31) / 32, tn = (d.n + 31) / 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int tile = blockIdx.x; tile < tm * tn; tile += gridDim.x) {
    const int i0 = (tile % tm) * 32, j0 = (tile / tm) * 32;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + tx, j = j0 + ty + 8 * r;
      if (i < d.m && j < d.n) t[ty + 8 * r][tx] = ldc(d.S + i + (int64_t)j * d.lds);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int jd = j0 + tx, id = i0 + ty + 8 * r;   // D(jd, id) = conj(S(id, jd))
      if (id < d.m && jd < d.n) {
        const cplx<TS> v = t[tx][ty + 8 * r];
        stc(d.D + jd + (int64_t)id * d.ldd, mk<TD>((TD)v.x, -(TD)v.y));
      }
    }
  }
}

template <typename T, class DS>
__global__ void fill_kernel(DS descs) {
  const FillDesc<T> d = descs[blockIdx.y];
  int64_t cnt = (int64_t)d.m * d.n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256) {
    int i = (int)(e % d.m), j = (int)(e / d.m);
    d.D[i + (int64_t)j * d.ld] = mk<T>((d.identity && i == j) ? T(1) : T(0), T(0));
  }
}

}  // namespace

// ------------------------------------------------------------------ host API
// Autotuned tile shape and k split per launch shape class: precision (0
// FP64, 1 FP32), op(A), op(B), ceil(log2) of the largest m, n, k and of the
// descriptor count; tile 0: the 64 x 64 output tiles with `splits`; 1: the
// 32 x 128 tiles of gemm_smallm_wide_kernel; 2: the 16- or 32-square tiles of
// gemm_smallmn_kernel (both for op(A) = C, op(B) = N, m <= 32).
struct GemmTune {
  int prec, opa, opb, lm, ln, lk, lnd, splits, tile;
};
static const GemmTune kGemmTune[] = {
    {-1, 0, 0, 0, 0, 0, 0, 0},   // sentinel
#include "gemm_tuning.inc"
};

static int clog2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

template <typename T>
static const GemmTune* tuned_entry(Op opA, Op opB, int maxm, int maxn, int maxk, int nd) {
  const int prec = sizeof(T) == 4 ? 1 : 0;
  const int lm = clog2(maxm), ln = clog2(maxn), lk = clog2(maxk), lnd = clog2(nd);
  for (const GemmTune& t : kGemmTune)
    if (t.prec == prec && t.opa == (int)opA && t.opb == (int)opB && t.lm == lm && t.ln == ln &&
        t.lk == lk && t.lnd == lnd)
      return &t;
  return nullptr;
}

// Algorithmic flops of one product: 8 per complex multiply-add with a
// nonzero operand entry (entries a triangular operand stores as zeros are
// not counted), halved for a Hermitian output computed in its lower half.
template <typename T>
static double gemm_flops(const GemmDesc<T>& g, Op opA, Op opB) {
  const double m = g.m, n = g.n, k = g.k;
  if (g.m <= 0 || g.n <= 0 || g.k <= 0) return 0.0;
  // nonzeros of op(X) per row (column) index i < r over a k range: below or
  // above the diagonal
  auto lower = [](double r, double kk) {   // sum_i min(i + 1, kk)
    const double t = std::min(r, kk);
    return t * (t + 1) / 2 + (r - t) * kk;
  };
  auto upper = [](double r, double kk) {   // sum_i max(kk - i, 0)
    const double t = std::min(r, kk);
    return t * kk - t * (t - 1) / 2;
  };
  double macs = m * n * k;
  // op(A)(i, l) = 0 for l > i (A unit lower, op N; A upper, op C)
  if ((opA == OpN && g.tri == 1) || (opA == OpC && g.tri == 2)) macs = n * lower(m, k);
  else if ((opA == OpN && g.tri == 2) || (opA == OpC && g.tri == 1)) macs = n * upper(m, k);
  // op(B)(l, j) = 0 for l > j (B upper, op N; B unit lower, op C)
  else if ((opB == OpN && g.trib == 2) || (opB == OpC && g.trib == 1)) macs = m * lower(n, k);
  else if ((opB == OpN && g.trib == 1) || (opB == OpC && g.trib == 2)) macs = m * upper(n, k);
  if (g.lower) macs *= (n + 1) / (2 * n);
  return 8.0 * macs;
}

template <typename T>
static void skinny_batched(DescPool& pool, const std::vector<GemmDesc<T>>& sub, Op opA, int maxm,
                           int maxn, int maxk, int force) {
  const size_t n = sub.size();
  // op N: 256 rows per workgroup, or 64 rows with the k range split over the
  // four waves (gemm_skinny_n4_kernel) when 256-row workgroups would not
  // fill the device
  const bool n4 = opA == OpN && (int64_t)((maxm + 255) / 256) * (int64_t)n < 1024;
  // op C with a short k: 16 lanes per row of C
  const bool c16 = opA == OpC && maxk <= 512;
  const int rows_per_wg = opA == OpN ? (n4 ? 64 : 256) : (c16 ? 16 : 4);
  const int64_t bx = (maxm + rows_per_wg - 1) / rows_per_wg;
  int64_t wgs = bx * (int64_t)n;
  int splits = 1;
  const int kmin_split = opA == OpN ? 4 * SK_L : 1024;
  // op C with a long k where a wave per row leaves the device short of work:
  // a workgroup per row instead of a k split
  const bool cw = opA == OpC && !c16 && force <= 0 && wgs < 1024 && maxk >= 2 * kmin_split;
  if (cw) {
    wgs = (int64_t)maxm * (int64_t)n;
  } else if (force > 0) {
    splits = std::max(1, std::min({force, std::max(1, maxk / SK_L), 4096}));
  } else if (wgs < 1024 && maxk >= 2 * kmin_split) {
    splits = (int)std::min<int64_t>(maxk / kmin_split, (2048 + wgs - 1) / wgs);
    splits = std::max(1, std::min(splits, 256));
  }
  double fl = 0;
  for (auto& g : sub) fl += gemm_flops(g, opA, OpN);
  int64_t mx = 0;
  bool scale = false;   // some C needs beta applied before the atomic adds
  for (auto& g : sub) {
    mx = std::max<int64_t>(mx, (int64_t)g.m * g.n);
    scale = scale || (g.m > 0 && g.n > 0 && g.beta != T(1));
  }
  with_descs(pool, sub.data(), n, [&](auto dd) {
    using DS = decltype(dd);
    if (splits > 1 && scale)
      hipLaunchKernelGGL(
          (gemm_prescale_kernel<T, DS>),
          dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((mx + 255) / 256, 1024)),
               (unsigned)n),
          dim3(256), 0, pool.stream, dd);
    ProfScope ps(pool.stream, sizeof(T) == 4 ? KC_GEMV32 : KC_GEMV64, fl, (int)n, maxm, maxn,
                 maxk, (int)opA * 2 + 10 * splits + 1000, true);
    // the op C kernel takes SKC_ROWS rows a wave
    const int64_t gx =
        cw ? (maxm + SKCW_ROWS - 1) / SKCW_ROWS
           : (opA == OpC && !c16 ? (maxm + 4 * SKC_ROWS - 1) / (4 * SKC_ROWS) : bx);
    dim3 grid((unsigned)gx, (unsigned)n, (unsigned)splits);
    auto launch = [&](auto nc) {
      constexpr int NC = decltype(nc)::value;
      if (cw)
        hipExtLaunchKernelGGL((gemm_skinny_cw_kernel<T, NC, DS>), grid, dim3(256), 0, pool.stream,
                              ps.start(), ps.stop(), 0, dd);
      else if (opA == OpN && n4)
        hipExtLaunchKernelGGL((gemm_skinny_n4_kernel<T, NC, DS>), grid, dim3(256), 0, pool.stream,
                              ps.start(), ps.stop(), 0, dd, splits);
      else if (opA == OpN)
        hipExtLaunchKernelGGL((gemm_skinny_n_kernel<T, NC, DS>), grid, dim3(256), 0, pool.stream,
                              ps.start(), ps.stop(), 0, dd, splits);
      else if (c16)
        hipExtLaunchKernelGGL((gemm_skinny_c16_kernel<T, NC, DS>), grid, dim3(256), 0, pool.stream,
                              ps.start(), ps.stop(), 0, dd, splits);
      else
        hipExtLaunchKernelGGL((gemm_skinny_c_kernel<T, NC, DS>), grid, dim3(256), 0, pool.stream,
                              ps.start(), ps.stop(), 0, dd, splits);
    };
    if (maxn <= 1) launch(std::integral_constant<int, 1>{});
    else if (maxn <= 2) launch(std::integral_constant<int, 2>{});
    else if (maxn <= 4) launch(std::integral_constant<int, 4>{});
    else launch(std::integral_constant<int, 8>{});
  });
  ND_HIP(hipGetLastError());
}

template <typename T>
static void smallmn_batched(DescPool& pool, const std::vector<GemmDesc<T>>& sub, int maxm, int maxn,
                            int maxk) {
  const size_t n = sub.size();
  bool scale = false;
  for (auto& g : sub) scale = scale || (g.m > 0 && g.n > 0 && g.beta != T(1));
  double fl = 0;
  for (auto& g : sub) fl += gemm_flops(g, OpC, OpN);
  const int mb = (maxm + 15) / 16, nb = (maxn + 15) / 16;
  with_descs(pool, sub.data(), n, [&](auto dd) {
    using DS = decltype(dd);
    if (scale)
      hipLaunchKernelGGL((gemm_prescale_kernel<T, DS>), dim3(4, (unsigned)n), dim3(256), 0,
                         pool.stream, dd);
    ProfScope ps(pool.stream, sizeof(T) == 4 ? KC_GEMM32 : KC_GEMM64, fl, (int)n, maxm, maxn,
                 maxk, 2000 + 10 * mb + nb, true);
    const int kc = small_out_kc(maxk, n);
    dim3 grid((unsigned)((maxk + kc - 1) / kc), (unsigned)n);
    if (mb == 1 && nb == 1)
      hipExtLaunchKernelGGL((gemm_smallmn_kernel<T, 1, 1, DS>), grid, dim3(256), 0, pool.stream,
                            ps.start(), ps.stop(), 0, dd, kc);
    else if (mb == 1)
      hipExtLaunchKernelGGL((gemm_smallmn_kernel<T, 1, 2, DS>), grid, dim3(256), 0, pool.stream,
                            ps.start(), ps.stop(), 0, dd, kc);
    else if (nb == 1)
      hipExtLaunchKernelGGL((gemm_smallmn_kernel<T, 2, 1, DS>), grid, dim3(256), 0, pool.stream,
                            ps.start(), ps.stop(), 0, dd, kc);
    else
      hipExtLaunchKernelGGL((gemm_smallmn_kernel<T, 2, 2, DS>), grid, dim3(256), 0, pool.stream,
                            ps.start(), ps.stop(), 0, dd, kc);
  });
  ND_HIP(hipGetLastError());
}

template <typename T>
static void smallm_wide_batched(DescPool& pool, const std::vector<GemmDesc<T>>& sub, int maxm,
                                int maxn, int maxk) {
  const size_t n = sub.size();
  bool scale = false;
  for (auto& g : sub) scale = scale || (g.m > 0 && g.n > 0 && g.beta != T(1));
  double fl = 0;
  for (auto& g : sub) fl += gemm_flops(g, OpC, OpN);
  with_descs(pool, sub.data(), n, [&](auto dd) {
    using DS = decltype(dd);
    if (scale)
      hipLaunchKernelGGL((gemm_prescale_kernel<T, DS>), dim3(4, (unsigned)n), dim3(256), 0,
                         pool.stream, dd);
    ProfScope ps(pool.stream, sizeof(T) == 4 ? KC_GEMM32 : KC_GEMM64, fl, (int)n, maxm, maxn,
                 maxk, 3000, true);
    const int kc = small_out_kc(maxk, n);
    hipExtLaunchKernelGGL((gemm_smallm_wide_kernel<T, DS>),
                          dim3((unsigned)((maxk + kc - 1) / kc), (unsigned)n), dim3(256), 0,
                          pool.stream, ps.start(), ps.stop(), 0, dd, kc);
  });
  ND_HIP(hipGetLastError());
}

// stream-K for long-k products whose tiles and splits stay under two rounds
// of workgroups
constexpr bool kGemmStreamK = true;
// partial tiles plus an ordered reduction for long-k products with few tiles
constexpr bool kGemmPartials = true;

// compute units of the first device used, taken once per process
// (thread-safe initialisation; the devices of a node are alike)
static int device_cus() {
  static const int cus = [] {
    int dev = 0, n = 0;
    ND_HIP(hipGetDevice(&dev));
    ND_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
    return std::max(n, 1);
  }();
  return cus;
}

template <typename T>
void gemm_batched(DescPool& pool, const std::vector<GemmDesc<T>>& d, Op opA, Op opB,
                  int splits_force) {
  if (d.empty()) return;
  if (hazards_enabled()) {
    std::vector<Region> v;
    const int64_t es = sizeof(cplx<T>);
    for (size_t i = 0; i < d.size(); ++i) {
      const GemmDesc<T>& g = d[i];
      if (g.m <= 0 || g.n <= 0) continue;
      v.push_back(region(g.C, es, g.m, g.n, g.ldc, true, (int)i));
      if (g.k <= 0) continue;
      if (opA == OpN) v.push_back(region(g.A, es, g.m, g.k, g.lda, false, (int)i));
      else v.push_back(region(g.A, es, g.k, g.m, g.lda, false, (int)i));
      if (opB == OpN) v.push_back(region(g.B, es, g.k, g.n, g.ldb, false, (int)i));
      else v.push_back(region(g.B, es, g.n, g.k, g.ldb, false, (int)i));
    }
    check_hazards(sizeof(T) == 4 ? "gemm<float>" : "gemm<double>", v);
  }
  size_t chunk = 32768;
  for (size_t s0 = 0; s0 < d.size(); s0 += chunk) {
    size_t n = std::min(chunk, d.size() - s0);
    int maxt = 0, maxk = 0, maxn = 0, maxm = 0;
    std::vector<GemmDesc<T>> sub(d.begin() + s0, d.begin() + s0 + n);
    for (auto& g : sub) {
      if (g.m <= 0 || g.n <= 0) { g.m = 0; g.n = 0; continue; }
      if (g.k < 0) g.k = 0;
      maxt = std::max(maxt, ceil_div(g.m, GT) * ceil_div(g.n, GT));
      maxk = std::max(maxk, g.k);
      maxn = std::max(maxn, g.n);
      maxm = std::max(maxm, g.m);
    }
    if (maxt == 0) continue;
    const GemmTune* tt =
        splits_force == 0 ? tuned_entry<T>(opA, opB, maxm, maxn, maxk, (int)n) : nullptr;
    const int force =
        splits_force > 0    ? splits_force
        : splits_force == -1 ? 1
        : splits_force <= -2 ? 0
                             : (tt && tt->tile == 0 ? tt->splits : 0);
    // the small-m tiles: a tuned choice, or forced (-5: 32 x 128, -6: 16/32
    // square); a forced tile the shapes do not allow is an error
    bool lower_any = false;
    for (auto& g : sub) lower_any = lower_any || g.lower;
    const bool cn = opA == OpC && opB == OpN && maxm <= 32 && maxn > SK_N && !lower_any;
    const bool wide_ok = cn && maxn <= 128, sq_ok = cn && maxn <= 32;
    if (splits_force == -5 || splits_force == -6) {
      ND_CHECK(splits_force == -5 ? wide_ok : sq_ok, NUDFT2_E_INVAL,
               "forced small tile: needs op(A) = C, op(B) = N, m <= 32, 8 < n <= 128 (32 x "
               "128) or <= 32 (square), no Hermitian-lower output");
    }
    const int tile = splits_force == -5 ? 1
                     : splits_force == -6 ? 2
                     : tt && tt->tile == 1 && wide_ok ? 1
                     : tt && tt->tile == 2 && sq_ok ? 2
                                                    : 0;
    if (tile == 1) {
      smallm_wide_batched<T>(pool, sub, maxm, maxn, maxk);
      continue;
    }
    if (tile == 2) {
      smallmn_batched<T>(pool, sub, maxm, maxn, maxk);
      continue;
    }
    const bool auto_route = splits_force == 0 || splits_force <= -2;
    if (auto_route && opA == OpC && opB == OpN && maxm <= 32 &&
        maxn > 32 && maxn <= 128 && maxk >= SG_KMIN) {
      smallm_wide_batched<T>(pool, sub, maxm, maxn, maxk);
      continue;
    }
    if (auto_route && opA == OpC && opB == OpN && maxn > SK_N &&
        maxm <= 32 &&
        maxn <= 32 && maxk >= SG_KMIN) {
      smallmn_batched<T>(pool, sub, maxm, maxn, maxk);
      continue;
    }
    if (maxn <= SK_N && opB == OpN) {
      skinny_batched<T>(pool, sub, opA, maxm, maxn, maxk, force);
      continue;
    }
    // Splitting the k loop.  The device holds `slots` tile workgroups at once.
    // Long k (>= 4096) with at least 16 output tiles a product: about seven
    // rounds of workgroups, each split at least 2048 long; where that still
    // leaves under two rounds, stream-K instead.  Fewer than 16 tiles and
    // k >= 1024: partial-tile splits (below).  Otherwise, under one round and
    // k >= 1024: about two rounds, splits of ~1024 (up to four of 256 or more
    // for shorter k).  k < 1024 is never split (the pre-scale and the atomics
    // cost more than the extra workgroups give).  A tuned table entry for the
    // launch's class takes precedence over all of these.  Measured on the
    // factorization's shapes (FP32, TF/s): 256 x 13661 x 28495 8 splits 134
    // (3: 123); 4 x 256 x 7319 x 10595 4 splits 131 (1: 115); 4 x 256 x 2147
    // x 5704 stream-K 111 (best split 100); 128 x 128^2 x 593 unsplit 88 (2
    // splits: 36).  Four-tile outputs with k of 8K-32K (tall-panel Grams) lose
    // half their rate under stream-K, whose many short shares are bound by
    // the atomics.
    const int64_t wgs = (int64_t)maxt * (int64_t)n;
    // the split kernel reads k in pairs from a stored matrix: k = 1 stays on
    // the FP32 instructions
    bool bf = std::is_same<T, float>::value && g_fp32_split;
    for (auto& g : sub) bf = bf && g.k != 1;
    const int64_t slots = (int64_t)device_cus() * (sizeof(T) == 4 && !bf ? 4 : 2);
    int splits = 1;
    bool want_sk = splits_force == -3;
    if (force > 0) {
      splits = std::max(1, std::min({force, std::max(1, ceil_div(maxk, GK)), 4096}));
    } else if (maxk >= 4096 && maxt >= 16) {
      splits = (int)std::max<int64_t>(1, std::min<int64_t>(7 * slots / wgs, maxk / 2048));
      want_sk = want_sk || (kGemmStreamK && wgs * splits < 2 * slots && splits_force != -4);
    } else if (wgs < slots && maxk >= 1024) {
      const int64_t by_k = std::max<int64_t>(maxk / 1024, std::min<int64_t>(maxk / 256, 4));
      splits = (int)std::min<int64_t>(by_k, (2 * slots + wgs - 1) / wgs);
      splits = std::max(1, std::min(splits, 64));
    }
    // stream-K: each descriptor's tiles x k stages in equal shares over its
    // part of the workgroup slots, at least 64 stages (k = 1024) a share (not
    // for Hermitian-lower outputs; splits_force = -3 takes it wherever it
    // applies)
    int sk = 0;
    bool lower = false;
    for (auto& g : sub) lower = lower || g.lower;
    if (want_sk && !lower && splits_force != -1 && splits_force <= 0) {
      int64_t umax = 0;
      for (auto& g : sub)
        umax = std::max<int64_t>(umax, (int64_t)ceil_div(g.m, GT) * ceil_div(g.n, GT) *
                                           ceil_div(g.k, GK));
      const int64_t per = slots / (int64_t)n;
      if (per >= 2 && umax >= 128) {
        sk = (int)std::min<int64_t>(per, umax / 64);
        splits = 1;
      }
    }
    // Fewer than 16 tiles a product and k >= 1024 (tall-panel Grams): about
    // two rounds of k splits of 256 or more whose 64 x 64 partial tiles go to
    // the pool's stream scratch (plain stores) and are summed in split order
    // by gemm_reduce_kernel.  The atomics of a plain split made short splits
    // pay more than they gained, and at the split counts that kept them
    // affordable these products left one workgroup per CU (latency bound):
    // 128 x 128 x 8163 x 4 ran at 30 TF/s with the best plain split, 64 this
    // way.  splits_force = -4 takes this path wherever the scratch fits.
    cplx<T>* part = nullptr;
    if (!lower && sk == 0 &&
        (splits_force == -4 ||
         (kGemmPartials && (splits_force == 0 || splits_force == -2) && force <= 0 &&
          maxt < 16 && maxk >= 1024))) {
      const size_t tile_b = (size_t)GT * GT * sizeof(cplx<T>);
      int64_t sp = std::min<int64_t>(2 * slots / wgs, maxk / 256);
      if (splits_force == -4) sp = std::max<int64_t>(sp, 2);
      sp = std::min<int64_t>({sp, (int64_t)(kGemmPartBytes / (tile_b * (size_t)wgs)), 4096});
      if (sp >= 2) {
        part = (cplx<T>*)pool.stream_scratch(kGemmPartBytes);
        if (part) splits = (int)sp;
      }
    }
    int64_t mx = 0;
    bool scale = false;   // some C needs beta applied before the atomic adds
    for (auto& g : sub) {
      mx = std::max<int64_t>(mx, (int64_t)g.m * g.n);
      scale = scale || (g.m > 0 && g.n > 0 && g.beta != T(1));
    }
    const dim3 grid = sk > 0 ? dim3((unsigned)sk, (unsigned)n, 1) : dim3(maxt, (unsigned)n, splits);
    double fl = 0;
    int mm = 0, mn = 0;
    for (auto& g : sub) {
      fl += gemm_flops(g, opA, opB);
      mm = std::max(mm, g.m);
      mn = std::max(mn, g.n);
    }
    with_descs(pool, sub.data(), n, [&](auto dd) {
      using DS = decltype(dd);
      if (((splits > 1 && !part) || sk > 0) && scale)
        hipLaunchKernelGGL(
            (gemm_prescale_kernel<T, DS>),
            dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((mx + 255) / 256, 1024)),
                 (unsigned)n),
            dim3(256), 0, pool.stream, dd);
      ProfScope ps(pool.stream, sizeof(T) == 4 ? KC_GEMM32 : KC_GEMM64, fl, (int)n, mm, mn, maxk,
                   (int)opA * 2 + (int)opB + 10 * (sk > 0 ? 99 : part ? 98 : splits), true);
      // the reduction pass, when there is one, ends the timed span
      hipEvent_t e1 = part ? nullptr : ps.stop();
      if constexpr (std::is_same<T, float>::value) {
        if (bf) {
          if (opA == OpN && opB == OpN)
            hipExtLaunchKernelGGL((gemm_bf_kernel<OpN, OpN, DS>), grid, dim3(256), 0, pool.stream,
                                  ps.start(), e1, 0, dd, splits, sk, part);
          else if (opA == OpC && opB == OpN)
            hipExtLaunchKernelGGL((gemm_bf_kernel<OpC, OpN, DS>), grid, dim3(256), 0, pool.stream,
                                  ps.start(), e1, 0, dd, splits, sk, part);
          else if (opA == OpN && opB == OpC)
            hipExtLaunchKernelGGL((gemm_bf_kernel<OpN, OpC, DS>), grid, dim3(256), 0, pool.stream,
                                  ps.start(), e1, 0, dd, splits, sk, part);
          else
            hipExtLaunchKernelGGL((gemm_bf_kernel<OpC, OpC, DS>), grid, dim3(256), 0, pool.stream,
                                  ps.start(), e1, 0, dd, splits, sk, part);
        }
      }
      if (bf) {
      } else if (opA == OpN && opB == OpN)
        hipExtLaunchKernelGGL((gemm_kernel<T, OpN, OpN, DS>), grid, dim3(256), 0, pool.stream,
                              ps.start(), e1, 0, dd, splits, sk, part);
      else if (opA == OpC && opB == OpN)
        hipExtLaunchKernelGGL((gemm_kernel<T, OpC, OpN, DS>), grid, dim3(256), 0, pool.stream,
                              ps.start(), e1, 0, dd, splits, sk, part);
      else if (opA == OpN && opB == OpC)
        hipExtLaunchKernelGGL((gemm_kernel<T, OpN, OpC, DS>), grid, dim3(256), 0, pool.stream,
                              ps.start(), e1, 0, dd, splits, sk, part);
      else
        hipExtLaunchKernelGGL((gemm_kernel<T, OpC, OpC, DS>), grid, dim3(256), 0, pool.stream,
                              ps.start(), e1, 0, dd, splits, sk, part);
      if (part)
        hipExtLaunchKernelGGL(
            (gemm_reduce_kernel<T, DS>),
            dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((mx + 255) / 256, 1024)),
                 (unsigned)n),
            dim3(256), 0, pool.stream, nullptr, ps.stop(), 0, dd, splits, maxt,
            (const cplx<T>*)part);
    });
    ND_HIP(hipGetLastError());
  }
}

__global__ void zero_words_kernel(unsigned* p, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    p[e] = 0;
}

// Launch the cooperative panel kernel: groups of gsize workgroups, as many
// groups as fit on the device at once (they loop over the active problems).
// Their sums and barrier counters live in pool scratch zeroed by a kernel
// just before (no host copy between the two launches).
template <typename T>
void qr_panel_launch(DescPool& pool, const QRDesc<T>* dd, const std::vector<int>& act, int j0,
                     int maxmr) {
  const int nact = (int)act.size();
  const void* kern = (const void*)qr_panel_kernel<T, DescMem<int>>;
  // workgroups the device holds at once, taken once per process (per
  // precision; thread-safe initialisation) on the first device used
  static const int mres = [&] {
    int per = 0;
    ND_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, QP_NT, 0));
    // one 1024-thread workgroup per CU at most: the group barriers assume that
    // every workgroup of the grid is resident
    return std::max(1, device_cus() * std::min(std::max(per, 1), 1));
  }();
  constexpr int rows = 128 * QPanel<T>::R;
  int gsize = std::max(1, (maxmr + rows - 1) / rows);
  // Twice the rows per workgroup (RM = 2): for panels taller than the device
  // holds otherwise, and for multi-workgroup panels when the halved groups
  // still fill every CU (many problems): fewer workgroups exchange column
  // sums, which outweighs the spilled registers (1024 leaf panels of
  // 1024 x 430: 42.5 -> 32.1 ms FP32; 1024 x 500 x 300 FP64: 32.6 -> 23.7 ms);
  // with few tall problems the halved group count leaves CUs idle (16 x 5000:
  // 7.4 -> 7.9 ms), so those keep RM = 1.
  const int gsize2 = std::max(1, (maxmr + 2 * rows - 1) / (2 * rows));
  const bool tall = gsize > mres || (gsize > 1 && (int64_t)nact * gsize2 >= mres);
  if (tall) gsize = gsize2;
  ND_CHECK(gsize <= mres, NUDFT2_E_INTERNAL, "QR panel taller than the device can hold");
  int ngroups = std::max(1, std::min(nact, mres / gsize));
  const size_t per_group = sizeof(T) == 4 ? qp_tag_words(gsize) * sizeof(unsigned long long)
                                           : QSCR * sizeof(cplx<T>);
  const size_t scr_bytes = ((size_t)ngroups * per_group + 255) & ~size_t(255);
  const size_t words = (scr_bytes + (size_t)ngroups * sizeof(unsigned)) / sizeof(unsigned);
  char* z = (char*)pool.reserve(words * sizeof(unsigned));
  cplx<T>* scr = (cplx<T>*)z;
  unsigned* bar = (unsigned*)(z + scr_bytes);
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)std::min<size_t>((words + 255) / 256, 1024)),
                     dim3(256), 0, pool.stream, (unsigned*)z, (int64_t)words);
  int* err = pool.flag;
  with_descs(pool, act.data(), act.size(), [&](auto as) {
    const void* k = tall ? (const void*)qr_panel_kernel<T, decltype(as), 2>
                         : (const void*)qr_panel_kernel<T, decltype(as), 1>;
    void* args[] = {(void*)&dd, (void*)&as, (void*)&nact, (void*)&j0, (void*)&gsize,
                    (void*)&scr, (void*)&bar, (void*)&err};
    ProfScope ps(pool.stream, KC_QRPANEL, 0.0, nact, maxmr, 0, 0, gsize);
    ND_HIP(hipLaunchCooperativeKernel(k, dim3(ngroups * gsize), dim3(QP_NT), args, 0, pool.stream));
  });
}

// per problem: W and W2 (QR_OB x n), S (QR_OB x QR_OB), the panels' factors
// (QR_OB / QR_NB blocks of QR_NB x QR_NB)
template <typename T>
size_t qr_workspace(const std::vector<QRDesc<T>>& d) {
  size_t s = 0;
  for (auto& q : d)
    s += (size_t)QR_OB * std::max(q.n, 1) * 2 + (size_t)QR_OB * QR_OB + (size_t)QR_OB * QR_NB;
  return s * sizeof(cplx<T>) + 256;
}

template <typename T>
void geqrf_batched(DescPool& pool, const std::vector<QRDesc<T>>& din, void* ws) {
  if (din.empty()) return;
  if (hazards_enabled()) {
    std::vector<Region> v;
    const int64_t es = sizeof(cplx<T>);
    for (size_t i = 0; i < din.size(); ++i) {
      const QRDesc<T>& q = din[i];
      int kmin = qr_kmin(q.m, q.n);
      v.push_back(region(q.A, es, q.m, q.n, q.lda, true, (int)i));
      v.push_back(region(q.R, es, kmin, q.n, q.ldr, true, (int)i));
      v.push_back(region(q.Tb, es, qr_tsize(q.m, q.n), 1, qr_tsize(q.m, q.n), true, (int)i));
    }
    check_hazards("geqrf", v);
  }
  const int nb = (int)din.size();
  std::vector<QRDesc<T>> d(din);
  // workspace layout per problem
  std::vector<cplx<T>*> W(nb), W2(nb), S(nb);
  {
    cplx<T>* p = (cplx<T>*)ws;
    for (int i = 0; i < nb; ++i) {
      W[i] = p;
      p += (size_t)QR_OB * std::max(d[i].n, 1);
      W2[i] = p;
      p += (size_t)QR_OB * std::max(d[i].n, 1);
      S[i] = p;
      p += (size_t)QR_OB * QR_OB;
      d[i].Tw = p;
      p += (size_t)QR_OB * QR_NB;
    }
  }
  auto* dd = (QRDesc<T>*)pool.push(d.data(), sizeof(QRDesc<T>) * nb);
  int kmax = 0;
  for (auto& q : d) kmax = std::max(kmax, qr_kmin(q.m, q.n));
  std::vector<int> act;
  std::vector<GemmDesc<T>> g1, g2, g3;
  std::vector<WyDesc<T>> wy;
  std::vector<FillDesc<T>> fz;
  // Blocks of QR_OB columns, each made of two halves of QR_HB: the panels of a
  // half update the half's later columns; the left half's reflectors then
  // update the right half; the block's T joins the halves' factors; the
  // columns beyond the block get one update with the block's reflectors.
  for (int J0 = 0; J0 < kmax; J0 += QR_OB) {
    const int bidx = J0 / QR_OB;
    for (int H0 = J0; H0 < std::min(J0 + QR_OB, kmax); H0 += QR_HB) {
      for (int j0 = H0; j0 < std::min(H0 + QR_HB, kmax); j0 += QR_NB) {
        act.clear();
        g1.clear(); g2.clear(); g3.clear();
        for (int i = 0; i < nb; ++i) {
          const QRDesc<T>& q = d[i];
          int kmin = qr_kmin(q.m, q.n);
          if (kmin <= j0) continue;
          act.push_back(i);
          int jb = std::min(QR_NB, kmin - j0);
          int nt = std::min(q.n, H0 + QR_HB) - j0 - jb;
          if (nt <= 0) continue;
          int mr = q.m - j0;
          cplx<T>* V = q.A + j0 + (int64_t)j0 * q.lda;
          cplx<T>* At = q.A + j0 + (int64_t)(j0 + jb) * q.lda;
          cplx<T>* Tj = q.Tw + (int64_t)((j0 % QR_OB) / QR_NB) * QR_NB * QR_NB;
          // V unit lower trapezoidal, T upper triangular
          g1.push_back({jb, nt, mr, q.lda, q.lda, QR_NB, V, At, W[i], T(1), T(0), T(0), 0, 1});
          g2.push_back({jb, nt, jb, QR_NB, QR_NB, QR_NB, Tj, W[i], W2[i], T(1), T(0), T(0), 0, 2});
          g3.push_back({mr, nt, jb, q.lda, QR_NB, q.lda, V, W2[i], At, T(-1), T(0), T(1), 0, 1});
        }
        int maxmr = 0;
        for (int i : act) maxmr = std::max(maxmr, d[i].m - j0);
        qr_panel_launch<T>(pool, dd, act, j0, maxmr);
        gemm_batched<T>(pool, g1, OpC, OpN);
        gemm_batched<T>(pool, g2, OpC, OpN);
        gemm_batched<T>(pool, g3, OpN, OpN);
      }
      // the half's factor T_h (in its place inside the block's T) from the
      // panels' factors and S = V_h^H V_h
      g1.clear();
      wy.clear();
      for (int i = 0; i < nb; ++i) {
        const QRDesc<T>& q = d[i];
        int kmin = qr_kmin(q.m, q.n);
        if (kmin <= H0) continue;
        const int kB = std::min(QR_OB, kmin - J0), kh = std::min(QR_HB, kmin - H0);
        cplx<T>* V = q.A + H0 + (int64_t)H0 * q.lda;
        cplx<T>* Tout =
            q.Tb + (int64_t)QR_OB * QR_OB * bidx + (H0 - J0) + (int64_t)(H0 - J0) * kB;
        if (kh > QR_NB)
          g1.push_back({kh, kh, q.m - H0, q.lda, q.lda, QR_OB, V, V, S[i], T(1), T(0), T(0)});
        wy.push_back({kh, QR_OB, kB, q.Tw + (int64_t)((H0 - J0) / QR_NB) * QR_NB * QR_NB, S[i],
                      Tout});
      }
      gemm_batched<T>(pool, g1, OpC, OpN);
      if (!wy.empty()) {
        with_descs(pool, wy.data(), wy.size(), [&](auto dw) {
          hipLaunchKernelGGL((wy_merge_kernel<T, decltype(dw)>), dim3((unsigned)wy.size()),
                             dim3(WY_NT), 0, pool.stream, dw);
        });
        ND_HIP(hipGetLastError());
      }
      if (H0 != J0) continue;
      // the left half's reflectors on the right half's columns
      g1.clear(); g2.clear(); g3.clear();
      for (int i = 0; i < nb; ++i) {
        const QRDesc<T>& q = d[i];
        int kmin = qr_kmin(q.m, q.n);
        if (kmin <= H0) continue;
        const int kB = std::min(QR_OB, kmin - J0), kh = std::min(QR_HB, kmin - H0);
        const int nt = std::min(q.n, J0 + QR_OB) - (H0 + QR_HB);
        if (nt <= 0) continue;
        const int mr = q.m - H0;
        cplx<T>* V = q.A + H0 + (int64_t)H0 * q.lda;
        cplx<T>* At = q.A + H0 + (int64_t)(H0 + QR_HB) * q.lda;
        const cplx<T>* Th = q.Tb + (int64_t)QR_OB * QR_OB * bidx;
        g1.push_back({kh, nt, mr, q.lda, q.lda, QR_OB, V, At, W[i], T(1), T(0), T(0), 0, 1});
        g2.push_back({kh, nt, kh, kB, QR_OB, QR_OB, Th, W[i], W2[i], T(1), T(0), T(0), 0, 2});
        g3.push_back({mr, nt, kh, q.lda, QR_OB, q.lda, V, W2[i], At, T(-1), T(0), T(1), 0, 1});
      }
      gemm_batched<T>(pool, g1, OpC, OpN);
      gemm_batched<T>(pool, g2, OpC, OpN);
      gemm_batched<T>(pool, g3, OpN, OpN);
    }
    // blocks with two halves: T = [T_L, -T_L (V_L^H V_R) T_R; 0, T_R] (V_R is
    // zero above its first row, so V_L^H V_R runs over the rows from there)
    g1.clear(); g2.clear(); g3.clear();
    fz.clear();
    for (int i = 0; i < nb; ++i) {
      const QRDesc<T>& q = d[i];
      int kmin = qr_kmin(q.m, q.n);
      if (kmin <= J0 + QR_HB) continue;
      const int kB = std::min(QR_OB, kmin - J0), kr = kB - QR_HB;
      const int h1 = J0 + QR_HB;
      cplx<T>* Tb = q.Tb + (int64_t)QR_OB * QR_OB * bidx;
      g1.push_back({QR_HB, kr, q.m - h1, q.lda, q.lda, QR_OB, q.A + h1 + (int64_t)J0 * q.lda,
                    q.A + h1 + (int64_t)h1 * q.lda, S[i], T(1), T(0), T(0)});
      g2.push_back({QR_HB, kr, kr, QR_OB, kB, QR_OB, S[i], Tb + QR_HB + (int64_t)QR_HB * kB, W[i],
                    T(1), T(0), T(0)});
      g3.push_back({QR_HB, kr, QR_HB, kB, QR_OB, kB, Tb, W[i], Tb + (int64_t)QR_HB * kB, T(-1),
                    T(0), T(0)});
      fz.push_back({kr, QR_HB, kB, Tb + QR_HB, 0});
    }
    gemm_batched<T>(pool, g1, OpC, OpN);
    gemm_batched<T>(pool, g2, OpN, OpN);
    gemm_batched<T>(pool, g3, OpN, OpN);
    fill_batched<T>(pool, fz);
    // trailing columns beyond the block: one update with the block's reflectors
    g1.clear(); g2.clear(); g3.clear();
    for (int i = 0; i < nb; ++i) {
      const QRDesc<T>& q = d[i];
      int kmin = qr_kmin(q.m, q.n);
      if (kmin <= J0) continue;
      int kb = std::min(QR_OB, kmin - J0);
      int nt = q.n - (J0 + QR_OB);
      if (nt <= 0) continue;
      int mr = q.m - J0;
      cplx<T>* V = q.A + J0 + (int64_t)J0 * q.lda;
      cplx<T>* At = q.A + J0 + (int64_t)(J0 + QR_OB) * q.lda;
      const cplx<T>* Tb = q.Tb + (int64_t)QR_OB * QR_OB * bidx;
      g1.push_back({kb, nt, mr, q.lda, q.lda, QR_OB, V, At, W[i], T(1), T(0), T(0), 0, 1});
      g2.push_back({kb, nt, kb, kb, QR_OB, QR_OB, Tb, W[i], W2[i], T(1), T(0), T(0), 0, 2});
      g3.push_back({mr, nt, kb, q.lda, QR_OB, q.lda, V, W2[i], At, T(-1), T(0), T(1), 0, 1});
    }
    gemm_batched<T>(pool, g1, OpC, OpN);
    gemm_batched<T>(pool, g2, OpC, OpN);
    gemm_batched<T>(pool, g3, OpN, OpN);
  }
  int64_t rmax = 0;
  for (auto& q : d) rmax = std::max<int64_t>(rmax, (int64_t)qr_kmin(q.m, q.n) * std::max(q.n, 0));
  const int64_t fx = std::max<int64_t>(1, std::min<int64_t>((rmax + 2047) / 2048,
                                                          std::max(16, 16384 / nb)));
  hipLaunchKernelGGL((qr_finish_kernel<T>), dim3((unsigned)fx, nb), dim3(256), 0, pool.stream, dd);
  ND_HIP(hipGetLastError());
}

template <typename T>
size_t orm_workspace(const std::vector<OrmDesc<T>>& d) {
  size_t s = 0;
  for (auto& q : d) s += (size_t)QR_OB * std::max(q.nc, 1) * 2;
  return s * sizeof(cplx<T>) + 256;
}

// C <- Q C or Q^H C block by block (QR_OB reflectors and their T_b at a time)
template <typename T>
void ormqr_batched(DescPool& pool, const std::vector<OrmDesc<T>>& d, bool trans, void* ws,
                   bool from_identity) {
  ND_CHECK(!(from_identity && trans), NUDFT2_E_INTERNAL, "Q^H applied to an identity");
  if (d.empty()) return;
  if (hazards_enabled()) {
    std::vector<Region> v;
    const int64_t es = sizeof(cplx<T>);
    for (size_t i = 0; i < d.size(); ++i) {
      const OrmDesc<T>& q = d[i];
      if (q.nc <= 0 || q.k <= 0) continue;
      v.push_back(region(q.C, es, q.m, q.nc, q.ldc, true, (int)i));
      v.push_back(region(q.V, es, q.m, q.k, q.ldv, false, (int)i));
      v.push_back(region(q.Tb, es, qr_tsize(q.m, q.k), 1, qr_tsize(q.m, q.k), false, (int)i));
    }
    check_hazards("ormqr", v);
  }
  const int nb = (int)d.size();
  std::vector<cplx<T>*> W(nb), W2(nb);
  {
    cplx<T>* p = (cplx<T>*)ws;
    for (int i = 0; i < nb; ++i) {
      W[i] = p;
      p += (size_t)QR_OB * std::max(d[i].nc, 1);
      W2[i] = p;
      p += (size_t)QR_OB * std::max(d[i].nc, 1);
    }
  }
  int nbl = 0;
  for (auto& q : d) nbl = std::max(nbl, (q.k + QR_OB - 1) / QR_OB);
  std::vector<GemmDesc<T>> g1, g2, g3;
  for (int s = 0; s < nbl; ++s) {
    g1.clear(); g2.clear(); g3.clear();
    for (int i = 0; i < nb; ++i) {
      const OrmDesc<T>& q = d[i];
      int nblk = (q.k + QR_OB - 1) / QR_OB;
      if (s >= nblk || q.nc <= 0) continue;
      int blk = trans ? s : nblk - 1 - s;
      int j0 = blk * QR_OB;
      int kb = std::min(QR_OB, q.k - j0);
      int mr = q.m - j0;
      const int c0 = from_identity ? std::min(j0, q.nc) : 0;   // first column touched
      const int nc = q.nc - c0;
      if (nc <= 0) continue;
      const cplx<T>* V = q.V + j0 + (int64_t)j0 * q.ldv;
      const cplx<T>* Tb = q.Tb + (int64_t)QR_OB * QR_OB * blk;
      cplx<T>* Cp = q.C + j0 + (int64_t)c0 * q.ldc;
      // V unit lower trapezoidal, T upper triangular
      g1.push_back({kb, nc, mr, q.ldv, q.ldc, QR_OB, V, Cp, W[i], T(1), T(0), T(0), 0, 1});
      g2.push_back({kb, nc, kb, kb, QR_OB, QR_OB, Tb, W[i], W2[i], T(1), T(0), T(0), 0, 2});
      g3.push_back({mr, nc, kb, q.ldv, QR_OB, q.ldc, V, W2[i], Cp, T(-1), T(0), T(1), 0, 1});
    }
    gemm_batched<T>(pool, g1, OpC, OpN);
    gemm_batched<T>(pool, g2, trans ? OpC : OpN, OpN);
    gemm_batched<T>(pool, g3, OpN, OpN);
  }
}

void pchol_batched(DescPool& pool, const std::vector<PcholDesc>& d) {
  if (d.empty()) return;
  if (hazards_enabled()) {
    std::vector<Region> v;
    for (size_t i = 0; i < d.size(); ++i) {
      const PcholDesc& q = d[i];
      v.push_back(region(q.K, 16, q.w, q.w, q.ldk, true, (int)i));
      v.push_back(region(q.L, 16, q.w, q.rmax, q.ldl, true, (int)i));
      v.push_back(region(q.d, 8, q.w, 1, q.w, true, (int)i));
      v.push_back(region(q.piv, 4, q.rmax, 1, q.rmax, true, (int)i));
      v.push_back(region(q.rank, 4, 1, 1, 1, true, (int)i));
    }
    check_hazards("pchol", v);
  }
  const int nb = (int)d.size();
  auto* dd = (PcholDesc*)pool.push(d.data(), sizeof(PcholDesc) * nb);
  std::vector<int> ones(nb, 1);
  std::vector<double> zeros(nb, 0.0);
  double* trace = (double*)pool.push(zeros.data(), sizeof(double) * nb);
  int* state = (int*)pool.push(ones.data(), sizeof(int) * nb);
  hipLaunchKernelGGL(pchol_init_kernel, dim3(nb), dim3(256), 0, pool.stream, dd, trace);
  int rmax = 0;
  for (auto& q : d) rmax = std::max(rmax, std::min(q.rmax, q.w));
  std::vector<GemmDesc<double>> g;
  std::vector<int> hstate(nb);
  int maxw = 1;
  for (auto& q : d) maxw = std::max(maxw, q.w);
  const int gsize = (maxw + PC_ROWS - 1) / PC_ROWS;
  const int64_t grid = (int64_t)nb * gsize;
  ND_CHECK(grid < (int64_t(1) << 31), NUDFT2_E_INTERNAL, "too many Gram rows for one launch");
  std::vector<double> pz((size_t)nb * 2 * gsize * 3, 0.0);
  double* part = (double*)pool.push(pz.data(), sizeof(double) * pz.size());
  hipLaunchKernelGGL(pchol_part_kernel, dim3((unsigned)grid), dim3(PC_ROWS), 0, pool.stream, dd,
                     gsize, part, 0);
  ND_HIP(hipGetLastError());
  for (int k0 = 0; k0 < rmax; k0 += PC_NB) {
    const int kb = std::min(PC_NB, rmax - k0);
    for (int kk = 0; kk < kb; ++kk)
      hipLaunchKernelGGL(pchol_col_kernel, dim3((unsigned)grid), dim3(PC_ROWS), 0, pool.stream, dd,
                         trace, state, gsize, part, k0, kk);
    ND_HIP(hipGetLastError());
    // Schur update with this panel's columns for the problems still running
    ND_HIP(hipMemcpyAsync(hstate.data(), state, sizeof(int) * nb, hipMemcpyDeviceToHost,
                          pool.stream));
    ND_HIP(hipStreamSynchronize(pool.stream));
    g.clear();
    bool any = false;
    for (int i = 0; i < nb; ++i) {
      if (!hstate[i]) continue;
      any = true;
      const PcholDesc& q = d[i];
      int kb = std::min(PC_NB, std::min(q.rmax, q.w) - k0);
      if (kb <= 0) continue;
      const double2* Lp = q.L + (int64_t)k0 * q.ldl;
      g.push_back({q.w, q.w, kb, q.ldl, q.ldl, q.ldk, Lp, Lp, q.K, -1.0, 0.0, 1.0, 1});
    }
    if (!any) break;
    gemm_batched<double>(pool, g, OpN, OpC);
  }
  int kend = rmax;
  hipLaunchKernelGGL(pchol_finish_kernel, dim3(nb), dim3(64), 0, pool.stream, dd, state, kend);
  ND_HIP(hipGetLastError());
}

template <typename T>
static void trsv_small(DescPool& pool, const std::vector<TrsDesc<T>>& d, bool ct) {
  if (d.empty()) return;
  int maxr = 0;
  for (auto& q : d) maxr = std::max(maxr, q.nrhs);
  with_descs(pool, d.data(), d.size(), [&](auto dd) {
    using DS = decltype(dd);
    if (ct)
      hipLaunchKernelGGL((trsv_lds_kernel<T, true, DS>), dim3((unsigned)d.size(), maxr), dim3(256),
                         0, pool.stream, dd);
    else
      hipLaunchKernelGGL((trsv_lds_kernel<T, false, DS>), dim3((unsigned)d.size(), maxr),
                         dim3(256), 0, pool.stream, dd);
  });
  ND_HIP(hipGetLastError());
}

// Upper-triangular solves R X = B, or R^H X = B when conj_trans.  Systems of
// order <= TRS_B: one workgroup each.  Larger ones: blocked substitution,
// TRS_B x TRS_B diagonal blocks solved by one workgroup each, the remaining
// rows updated by a matrix-core GEMM (rows above for R, rows below for R^H).
template <typename T>
void trsv_upper_batched(DescPool& pool, const std::vector<TrsDesc<T>>& d, bool conj_trans) {
  constexpr int BS = TRS_B;
  if (hazards_enabled()) {
    std::vector<Region> v;
    const int64_t es = sizeof(cplx<T>);
    for (size_t i = 0; i < d.size(); ++i) {
      const TrsDesc<T>& q = d[i];
      if (q.k <= 0 || q.nrhs <= 0) continue;
      v.push_back(region(q.B, es, q.k, q.nrhs, q.ldb, true, (int)i));
      v.push_back(region(q.R, es, q.k, q.k, q.ldr, false, (int)i));
    }
    check_hazards("trsv", v);
  }
  std::vector<TrsDesc<T>> small, big;
  for (auto& q : d) {
    if (q.k <= 0 || q.nrhs <= 0) continue;
    (q.k <= BS ? small : big).push_back(q);
  }
  trsv_small<T>(pool, small, conj_trans);
  if (big.empty()) return;
  int maxblk = 0;
  for (auto& q : big) maxblk = std::max(maxblk, (q.k + BS - 1) / BS);
  std::vector<TrsDesc<T>> dg;
  std::vector<GemmDesc<T>> gu;
  for (int s = 0; s < maxblk; ++s) {
    dg.clear();
    gu.clear();
    for (auto& q : big) {
      int nblk = (q.k + BS - 1) / BS;
      if (s >= nblk) continue;
      int b = conj_trans ? s : nblk - 1 - s;
      int i0 = b * BS, bs = std::min(BS, q.k - i0);
      dg.push_back({bs, q.nrhs, q.ldr, q.ldb, q.R + i0 + (int64_t)i0 * q.ldr, q.B + i0});
      if (!conj_trans && i0 > 0)
        gu.push_back({i0, q.nrhs, bs, q.ldr, q.ldb, q.ldb, q.R + (int64_t)i0 * q.ldr, q.B + i0,
                      q.B, T(-1), T(0), T(1)});
      int rest = q.k - i0 - bs;
      if (conj_trans && rest > 0)
        gu.push_back({rest, q.nrhs, bs, q.ldr, q.ldb, q.ldb, q.R + i0 + (int64_t)(i0 + bs) * q.ldr,
                      q.B + i0, q.B + i0 + bs, T(-1), T(0), T(1)});
    }
    trsv_small<T>(pool, dg, conj_trans);
    gemm_batched<T>(pool, gu, conj_trans ? OpC : OpN, OpN);
  }
}

// Triangular inversion.  The TRS_B x TRS_B diagonal blocks are inverted by
// the triangular-solve kernel against identity columns (the block is copied
// to the workspace and replaced by I, then solved in place).  Then inverted
// diagonal groups of g blocks are joined pairwise for g = 1, 2, 4, ...:
//   inv([R11 R12; 0 R22]) = [X11, -X11 (R12 X22); 0, X22],  Xii = inv(Rii),
// two batched GEMMs per doubling (T = R12 X22 into the workspace, then
// R12 <- -X11 T), every pair of every matrix in the same launch.
template <typename T>
size_t trtri_workspace(const std::vector<TriDesc<T>>& d) {
  constexpr int BS = TRS_B;
  size_t s0 = 0, s1 = 0;
  for (auto& q : d) {
    if (q.k <= 0) continue;
    const size_t nblk = (q.k + BS - 1) / BS;
    s0 += nblk * BS * BS;
    s1 += (size_t)q.k * q.k / 2 + (size_t)BS * BS;
  }
  return std::max(s0, s1) * sizeof(cplx<T>) + 256;
}

template <typename T>
void trtri_upper_batched(DescPool& pool, const std::vector<TriDesc<T>>& d, void* ws) {
  constexpr int BS = TRS_B;
  if (d.empty()) return;
  cplx<T>* w0 = (cplx<T>*)ws;
  {
    std::vector<CopyDesc<T, T>> cp;
    std::vector<FillDesc<T>> fl;
    std::vector<TrsDesc<T>> ts;
    cplx<T>* w = w0;
    for (auto& q : d) {
      for (int i0 = 0; i0 < q.k; i0 += BS) {
        const int bs = std::min(BS, q.k - i0);
        cplx<T>* Rbb = q.R + i0 + (int64_t)i0 * q.ldr;
        cp.push_back({bs, bs, q.ldr, bs, Rbb, w, 0});
        fl.push_back({bs, bs, q.ldr, Rbb, 1});
        ts.push_back({bs, bs, bs, q.ldr, w, Rbb});
        w += (size_t)BS * BS;
      }
    }
    copy_batched<T, T>(pool, cp);
    fill_batched<T>(pool, fl);
    trsv_upper_batched<T>(pool, ts, false);
  }
  for (int g = 1;; g *= 2) {
    std::vector<GemmDesc<T>> g1, g2;
    cplx<T>* w = w0;
    for (auto& q : d) {
      const int nblk = (q.k + BS - 1) / BS;
      for (int a = 0; a + g < nblk; a += 2 * g) {
        const int r0 = a * BS, r1 = std::min((a + g) * BS, q.k);
        const int r2 = std::min((a + 2 * g) * BS, q.k);
        const int m = r1 - r0, n = r2 - r1;
        cplx<T>* R12 = q.R + r0 + (int64_t)r1 * q.ldr;
        const cplx<T>* X22 = q.R + r1 + (int64_t)r1 * q.ldr;
        const cplx<T>* X11 = q.R + r0 + (int64_t)r0 * q.ldr;
        g1.push_back({m, n, n, q.ldr, q.ldr, m, R12, X22, w, T(1), T(0), T(0)});
        g2.push_back({m, n, m, q.ldr, m, q.ldr, X11, w, R12, T(-1), T(0), T(0)});
        w += (size_t)m * n;
      }
    }
    if (g1.empty()) break;
    gemm_batched<T>(pool, g1, OpN, OpN);
    gemm_batched<T>(pool, g2, OpN, OpN);
  }
}

template size_t trtri_workspace<float>(const std::vector<TriDesc<float>>&);
template size_t trtri_workspace<double>(const std::vector<TriDesc<double>>&);
template void trtri_upper_batched<float>(DescPool&, const std::vector<TriDesc<float>>&, void*);
template void trtri_upper_batched<double>(DescPool&, const std::vector<TriDesc<double>>&, void*);

// workgroups per descriptor of a copy launch: enough for the largest copy's
// work items, with the whole grid held to about 64K workgroups when the batch
// is long (the kernels loop over their items, so any count is correct)
static unsigned copy_grid_x(int64_t items, size_t ndesc) {
  const int64_t cap = std::max<int64_t>(8, 65536 / (int64_t)ndesc);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>({items, cap, 4096}));
}

template <typename TD, typename TS>
void copy_batched(DescPool& pool, const std::vector<CopyDesc<TD, TS>>& d) {
  if (d.empty()) return;
  if (hazards_enabled()) {
    std::vector<Region> v;
    for (size_t i = 0; i < d.size(); ++i) {
      const CopyDesc<TD, TS>& q = d[i];
      if (q.m <= 0 || q.n <= 0) continue;
      v.push_back(region(q.S, sizeof(cplx<TS>), q.m, q.n, q.lds, false, (int)i));
      if (q.conj_trans) v.push_back(region(q.D, sizeof(cplx<TD>), q.n, q.m, q.ldd, true, (int)i));
      else v.push_back(region(q.D, sizeof(cplx<TD>), q.m, q.n, q.ldd, true, (int)i));
    }
    check_hazards("copy", v);
  }
  // plain copies: a grid-stride loop sized by the largest copy; conjugate
  // transposes: LDS tiles
  std::vector<CopyDesc<TD, TS>> pl, ct;
  int64_t maxcnt = 0, maxtiles = 0;
  for (auto& q : d) {
    if (q.m <= 0 || q.n <= 0) continue;
    if (q.conj_trans) {
      ct.push_back(q);
      maxtiles = std::max<int64_t>(maxtiles, (int64_t)((q.m + 31) / 32) * ((q.n + 31) / 32));
    } else {
      pl.push_back(q);
      maxcnt = std::max<int64_t>(maxcnt, (int64_t)q.m * q.n);
    }
  }
  if (!pl.empty())
    with_descs(pool, pl.data(), pl.size(), [&](auto dd) {
      const unsigned gx = copy_grid_x((maxcnt + 2047) / 2048, pl.size());
      hipLaunchKernelGGL((copy_kernel<TD, TS, decltype(dd)>), dim3(gx, (unsigned)pl.size()),
                         dim3(256), 0, pool.stream, dd);
    });
  if (!ct.empty())
    with_descs(pool, ct.data(), ct.size(), [&](auto dd) {
      const unsigned gx = copy_grid_x(maxtiles, ct.size());
      hipLaunchKernelGGL((copy_ct_kernel<TD, TS, decltype(dd)>), dim3(gx, (unsigned)ct.size()),
                         dim3(256), 0, pool.stream, dd);
    });
  ND_HIP(hipGetLastError());
}

template <typename T>
void fill_batched(DescPool& pool, const std::vector<FillDesc<T>>& d) {
  if (d.empty()) return;
  if (hazards_enabled()) {
    std::vector<Region> v;
    for (size_t i = 0; i < d.size(); ++i)
      v.push_back(region(d[i].D, sizeof(cplx<T>), d[i].m, d[i].n, d[i].ld, true, (int)i));
    check_hazards("fill", v);
  }
  with_descs(pool, d.data(), d.size(), [&](auto dd) {
    hipLaunchKernelGGL((fill_kernel<T, decltype(dd)>), dim3(64, (unsigned)d.size()), dim3(256),
                       0, pool.stream, dd);
  });
  ND_HIP(hipGetLastError());
}

#define INST(T)                                                                          \
  template void gemm_batched<T>(DescPool&, const std::vector<GemmDesc<T>>&, Op, Op, int);\
  template size_t qr_workspace<T>(const std::vector<QRDesc<T>>&);                        \
  template void geqrf_batched<T>(DescPool&, const std::vector<QRDesc<T>>&, void*);       \
  template size_t orm_workspace<T>(const std::vector<OrmDesc<T>>&);                      \
  template void ormqr_batched<T>(DescPool&, const std::vector<OrmDesc<T>>&, bool, void*, bool); \
  template void trsv_upper_batched<T>(DescPool&, const std::vector<TrsDesc<T>>&, bool);  \
  template void fill_batched<T>(DescPool&, const std::vector<FillDesc<T>>&);
INST(float)
INST(double)
template void copy_batched<float, double>(DescPool&, const std::vector<CopyDesc<float, double>>&);
template void copy_batched<double, float>(DescPool&, const std::vector<CopyDesc<double, float>>&);
template void copy_batched<double, double>(DescPool&, const std::vector<CopyDesc<double, double>>&);
template void copy_batched<float, float>(DescPool&, const std::vector<CopyDesc<float, float>>&);

}  // namespace nd
