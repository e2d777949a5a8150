// Kernel-tile generation and face-split generator assembly.
//
// * G^x(j, l): the transformed 1D NUDFT matrix A^x (F^x)^{-1} (Section 2.5),
//   entry (1/n) sum_{k<n} exp(-2 pi i k theta), theta = x_j - l/n, evaluated
//   in the Dirichlet form exp(-i pi (n-1) theta) sin(pi n theta) /
//   (n sin(pi theta)) with exact reduction of n theta and (n-1) theta, and
//   the value 1 at theta = 0 (the limit the paper states).
// * 2D leaf blocks D = G(J, K^x x K^y) = D^x . D^y and the face-split leaf
//   bases U_xi = [D^x.U^y | U^x.D^y | U^x.U^y], V_xi = [I(x)V^y | V^x(x)I |
//   V^x(x)V^y] (Theorem 3.3), plus the Kronecker-structured transfer (R, W)
//   and interaction (B) generators of non-leaf nodes.
#include "device_util.h"
#include "gen.h"
#include "hazard.h"

namespace nd {

__device__ inline double2 dirichlet(double x, int l, int n) {
#pragma clang fp contract(off)   // the two-sum reductions below must stay as written
  double t = x - (double)l / (double)n;
  t -= rint(t);
  if (t == 0.0) return mk<double>(1.0, 0.0);
  double dn = (double)n;
  double p = dn * t;
  double e = fma(dn, t, -p);
  double nt = (p - 2.0 * rint(0.5 * p)) + e;
  double r = sinpi(nt) / (dn * sinpi(t));
  double dn1 = (double)(n - 1);
  double p2 = dn1 * t;
  double e2 = fma(dn1, t, -p2);
  double ph = (p2 - 2.0 * rint(0.5 * p2)) + e2;
  double s, c;
  sincospi(ph, &s, &c);
  return mk<double>(c * r, -s * r);
}

namespace {

__global__ void gen_G1_kernel(const double* __restrict__ xs, int64_t M, int n,
                              double2* __restrict__ G, int64_t ld) {
  int64_t cnt = M * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * 256) {
    int64_t j = e % M;
    int l = (int)(e / M);
    G[j + l * ld] = dirichlet(xs[j], l, n);
  }
}

template <typename T>
__global__ void gen_leafD_kernel(const LeafDesc<T>* __restrict__ descs,
                                 const double* __restrict__ pts2d) {
  const LeafDesc<T> d = descs[blockIdx.y];
  int64_t cnt = (int64_t)d.m * d.dx * d.dy;
  int nc = d.dx * d.dy;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * 256) {
    int j = (int)(e % d.m);
    int c = (int)(e / d.m);
    int ix = c / d.dy, iy = c % d.dy;
    int64_t g = d.row0 + j;
    double2 gx = dirichlet(pts2d[2 * g], d.colx0 + ix, d.nx);
    double2 gy = dirichlet(pts2d[2 * g + 1], d.coly0 + iy, d.ny);
    double2 v = cmul(gx, gy);
    d.out[j + (int64_t)(d.coff + c) * d.ld] = mk<T>((T)v.x, (T)v.y);
    (void)nc;
  }
}

template <typename T>
__global__ void gen_leafU_kernel(const LeafDesc<T>* __restrict__ descs,
                                 const double* __restrict__ pts2d,
                                 const int64_t* __restrict__ posx,
                                 const int64_t* __restrict__ posy) {
  const LeafDesc<T> d = descs[blockIdx.y];
  const int w1 = d.dx * d.ry, w2 = d.rx * d.dy, w3 = d.rx * d.ry;
  const int w = w1 + w2 + w3;
  int64_t cnt = (int64_t)d.m * w;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * 256) {
    int j = (int)(e % d.m);
    int c = (int)(e / d.m);
    int64_t g = d.row0 + j;
    double2 v;
    if (c < w1) {
      int ix = c / d.ry, s = c % d.ry;
      double2 gx = dirichlet(pts2d[2 * g], d.colx0 + ix, d.nx);
      double2 uy = d.Uy[(posy[g] - d.rowy0) + (int64_t)s * d.lduy];
      v = cmul(gx, uy);
    } else if (c < w1 + w2) {
      int cc = c - w1;
      int t = cc / d.dy, iy = cc % d.dy;
      double2 ux = d.Ux[(posx[g] - d.rowx0) + (int64_t)t * d.ldux];
      double2 gy = dirichlet(pts2d[2 * g + 1], d.coly0 + iy, d.ny);
      v = cmul(ux, gy);
    } else {
      int cc = c - w1 - w2;
      int t = cc / d.ry, s = cc % d.ry;
      double2 ux = d.Ux[(posx[g] - d.rowx0) + (int64_t)t * d.ldux];
      double2 uy = d.Uy[(posy[g] - d.rowy0) + (int64_t)s * d.lduy];
      v = cmul(ux, uy);
    }
    d.out[j + (int64_t)c * d.ld] = mk<T>((T)v.x, (T)v.y);
  }
}

template <typename T>
__global__ void gen_leafV_kernel(const LeafVDesc<T>* __restrict__ descs) {
  const LeafVDesc<T> d = descs[blockIdx.y];
  const int w1 = d.dx * d.ry, w2 = d.rx * d.dy, w3 = d.rx * d.ry;
  const int w = w1 + w2 + w3;
  const int nr = d.dx * d.dy;
  int64_t cnt = (int64_t)nr * w;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * 256) {
    int row = (int)(e % nr);
    int c = (int)(e / nr);
    int ix = row / d.dy, iy = row % d.dy;
    double2 v = mk<double>(0.0, 0.0);
    if (c < w1) {
      int ix2 = c / d.ry, s = c % d.ry;
      if (ix2 == ix) v = d.Vy[iy + (int64_t)s * d.ldvy];
    } else if (c < w1 + w2) {
      int cc = c - w1;
      int t = cc / d.dy, iy2 = cc % d.dy;
      if (iy2 == iy) v = d.Vx[ix + (int64_t)t * d.ldvx];
    } else {
      int cc = c - w1 - w2;
      int t = cc / d.ry, s = cc % d.ry;
      v = cmul(d.Vx[ix + (int64_t)t * d.ldvx], d.Vy[iy + (int64_t)s * d.ldvy]);
    }
    d.out[row + (int64_t)c * d.ld] = mk<T>((T)v.x, (T)v.y);
  }
}

__device__ inline void split3(int i, int d1, int r2, int r1, int d2, int& blk, int& u, int& v) {
  // block widths: [d1 * r2 | r1 * d2 | r1 * r2]; blk1 index = u * r2 + v (u < d1),
  // blk2 index = u * d2 + v (u < r1), blk3 index = u * r2 + v (u < r1)
  int w1 = d1 * r2, w2 = r1 * d2;
  if (i < w1) { blk = 0; u = i / r2; v = i % r2; }
  else if (i < w1 + w2) { blk = 1; i -= w1; u = i / d2; v = i % d2; }
  else { blk = 2; i -= w1 + w2; u = i / r2; v = i % r2; }
}

template <typename T>
__global__ void gen_asm_kernel(const AsmDesc<T>* __restrict__ descs) {
  const AsmDesc<T> d = descs[blockIdx.y];
  int64_t cnt = (int64_t)d.rows * d.cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * 256) {
    int i = (int)(e % d.rows);
    int j = (int)(e / d.rows);
    int rb, ru, rv, cb, cu, cv;
    split3(i, d.dx, d.ry, d.rx, d.dy, rb, ru, rv);
    split3(j, d.cdx, d.cry, d.crx, d.cdy, cb, cu, cv);
    double2 val = mk<double>(0.0, 0.0);
    if (d.kind == 0) {            // R
      if (rb == 0 && cb == 0) {
        if (cu == d.own_x + ru) val = d.Y[rv + (int64_t)cv * d.ldY];
      } else if (rb == 1 && cb == 1) {
        if (cv == d.own_y + rv) val = d.X[ru + (int64_t)cu * d.ldX];
      } else if (rb == 2 && cb == 0) {
        int q = cu - d.sib_x;
        if (q >= 0 && q < d.dsx)
          val = cmul(d.BX[ru + (int64_t)q * d.ldBX], d.Y[rv + (int64_t)cv * d.ldY]);
      } else if (rb == 2 && cb == 1) {
        int q = cv - d.sib_y;
        if (q >= 0 && q < d.dsy)
          val = cmul(d.X[ru + (int64_t)cu * d.ldX], d.BY[rv + (int64_t)q * d.ldBY]);
      } else if (rb == 2 && cb == 2) {
        val = cmul(d.X[ru + (int64_t)cu * d.ldX], d.Y[rv + (int64_t)cv * d.ldY]);
      }
    } else if (d.kind == 1) {     // W
      if (rb == 0 && cb == 0) {
        if (cu == d.own_x + ru) val = d.Y[rv + (int64_t)cv * d.ldY];
      } else if (rb == 1 && cb == 1) {
        if (cv == d.own_y + rv) val = d.X[ru + (int64_t)cu * d.ldX];
      } else if (rb == 2 && cb == 2) {
        val = cmul(d.X[ru + (int64_t)cu * d.ldX], d.Y[rv + (int64_t)cv * d.ldY]);
      }
    } else {                      // B
      if (d.bcase == 0) {         // same x node: I (x) B^y
        if (rb == 0 && cb == 0 && ru == cu) val = d.Y[rv + (int64_t)cv * d.ldY];
      } else if (d.bcase == 1) {  // same y node: B^x (x) I
        if (rb == 1 && cb == 1 && rv == cv) val = d.X[ru + (int64_t)cu * d.ldX];
      } else {                    // B^x (x) B^y
        if (rb == 2 && cb == 2)
          val = cmul(d.X[ru + (int64_t)cu * d.ldX], d.Y[rv + (int64_t)cv * d.ldY]);
      }
    }
    d.out[i + (int64_t)j * d.ld] = mk<T>((T)val.x, (T)val.y);
  }
}

__global__ void zero_rc_kernel(const ZeroRCDesc* __restrict__ descs) {
  const ZeroRCDesc d = descs[blockIdx.y];
  // zero rows and columns [c0, c0 + w) of an n x n matrix
  int64_t cnt = (int64_t)d.n * d.w;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * 256) {
    int i = (int)(e % d.n);
    int j = d.c0 + (int)(e / d.n);
    d.K[i + (int64_t)j * d.ld] = mk<double>(0.0, 0.0);
    d.K[j + (int64_t)i * d.ld] = mk<double>(0.0, 0.0);
  }
}

__global__ void zero_cols_kernel(const ZeroRCDesc* __restrict__ descs) {
  const ZeroRCDesc d = descs[blockIdx.y];
  // zero columns [c0, c0 + w) of an n-row matrix
  int64_t cnt = (int64_t)d.n * d.w;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * 256) {
    int i = (int)(e % d.n);
    int j = d.c0 + (int)(e / d.n);
    d.K[i + (int64_t)j * d.ld] = mk<double>(0.0, 0.0);
  }
}

__global__ void gather_cols_kernel(const GatherDesc* __restrict__ descs) {
  const GatherDesc d = descs[blockIdx.y];
  int64_t cnt = (int64_t)d.m * d.r;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * 256) {
    int i = (int)(e % d.m);
    int j = (int)(e / d.m);
    d.out[i + (int64_t)j * d.ldo] = d.in[i + (int64_t)d.piv[j] * d.ldi];
  }
}

// y_j += sum_{l in [col0, col0+d)} G(x_j, l) x_l for rows of one 1D leaf
__global__ void diag1d_kernel(const Diag1Desc* __restrict__ descs, const double* __restrict__ xs) {
  const Diag1Desc d = descs[blockIdx.y];
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < d.m;
       j += (int64_t)gridDim.x * 256) {
    double xv = xs[d.row0 + j];
    double2 acc = mk<double>(0.0, 0.0);
    for (int l = 0; l < d.d; ++l) acc = cadd(acc, cmul(dirichlet(xv, d.col0 + l, d.n), d.x[d.col0 + l]));
    d.y[d.row0 - d.m0 + j] = cadd(d.y[d.row0 - d.m0 + j], acc);
  }
}

}  // namespace

static unsigned grid_for(int64_t cnt) {
  int64_t b = (cnt + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 2048));
}

void gen_G1(hipStream_t s, const double* xs, int64_t M, int n, double2* G, int64_t ld) {
  hipLaunchKernelGGL(gen_G1_kernel, dim3(grid_for(M * n)), dim3(256), 0, s, xs, M, n, G, ld);
  ND_HIP(hipGetLastError());
}

template <typename T>
void gen_leafD(DescPool& pool, const std::vector<LeafDesc<T>>& d, const double* pts2d) {
  if (d.empty()) return;
  if (hazards_enabled()) {
    std::vector<Region> v;
    for (size_t i = 0; i < d.size(); ++i)
      v.push_back(region(d[i].out + (int64_t)d[i].coff * d[i].ld, sizeof(cplx<T>), d[i].m,
                         d[i].dx * d[i].dy, d[i].ld, true, (int)i));
    check_hazards("gen_leafD", v);
  }
  int64_t mx = 0;
  for (auto& q : d) mx = std::max<int64_t>(mx, (int64_t)q.m * q.dx * q.dy);
  auto* dd = (LeafDesc<T>*)pool.push(d.data(), sizeof(LeafDesc<T>) * d.size());
  hipLaunchKernelGGL((gen_leafD_kernel<T>), dim3(grid_for(mx), (unsigned)d.size()), dim3(256), 0,
                     pool.stream, dd, pts2d);
  ND_HIP(hipGetLastError());
}

template <typename T>
void gen_leafU(DescPool& pool, const std::vector<LeafDesc<T>>& d, const double* pts2d,
               const int64_t* posx, const int64_t* posy) {
  if (d.empty()) return;
  if (hazards_enabled()) {
    std::vector<Region> v;
    for (size_t i = 0; i < d.size(); ++i) {
      const LeafDesc<T>& q = d[i];
      v.push_back(region(q.out, sizeof(cplx<T>), q.m, q.dx * q.ry + q.rx * q.dy + q.rx * q.ry,
                         q.ld, true, (int)i));
    }
    check_hazards("gen_leafU", v);
  }
  int64_t mx = 0;
  for (auto& q : d)
    mx = std::max<int64_t>(mx, (int64_t)q.m * (q.dx * q.ry + q.rx * q.dy + q.rx * q.ry));
  auto* dd = (LeafDesc<T>*)pool.push(d.data(), sizeof(LeafDesc<T>) * d.size());
  hipLaunchKernelGGL((gen_leafU_kernel<T>), dim3(grid_for(mx), (unsigned)d.size()), dim3(256), 0,
                     pool.stream, dd, pts2d, posx, posy);
  ND_HIP(hipGetLastError());
}

template <typename T>
void gen_leafV(DescPool& pool, const std::vector<LeafVDesc<T>>& d) {
  if (d.empty()) return;
  if (hazards_enabled()) {
    std::vector<Region> v;
    for (size_t i = 0; i < d.size(); ++i) {
      const LeafVDesc<T>& q = d[i];
      v.push_back(region(q.out, sizeof(cplx<T>), q.dx * q.dy,
                         q.dx * q.ry + q.rx * q.dy + q.rx * q.ry, q.ld, true, (int)i));
    }
    check_hazards("gen_leafV", v);
  }
  int64_t mx = 0;
  for (auto& q : d)
    mx = std::max<int64_t>(mx, (int64_t)q.dx * q.dy * (q.dx * q.ry + q.rx * q.dy + q.rx * q.ry));
  auto* dd = (LeafVDesc<T>*)pool.push(d.data(), sizeof(LeafVDesc<T>) * d.size());
  hipLaunchKernelGGL((gen_leafV_kernel<T>), dim3(grid_for(mx), (unsigned)d.size()), dim3(256), 0,
                     pool.stream, dd);
  ND_HIP(hipGetLastError());
}

template <typename T>
void gen_asm(DescPool& pool, const std::vector<AsmDesc<T>>& d) {
  if (d.empty()) return;
  if (hazards_enabled()) {
    std::vector<Region> v;
    for (size_t i = 0; i < d.size(); ++i)
      v.push_back(region(d[i].out, sizeof(cplx<T>), d[i].rows, d[i].cols, d[i].ld, true, (int)i));
    check_hazards("gen_asm", v);
  }
  int64_t mx = 0;
  for (auto& q : d) mx = std::max<int64_t>(mx, (int64_t)q.rows * q.cols);
  if (mx == 0) return;
  auto* dd = (AsmDesc<T>*)pool.push(d.data(), sizeof(AsmDesc<T>) * d.size());
  hipLaunchKernelGGL((gen_asm_kernel<T>), dim3(grid_for(mx), (unsigned)d.size()), dim3(256), 0,
                     pool.stream, dd);
  ND_HIP(hipGetLastError());
}

namespace {

__device__ inline double2 cdiv(double2 a, double2 b) {
  const double r = 1.0 / (b.x * b.x + b.y * b.y);
  return mk<double>((a.x * b.x + a.y * b.y) * r, (a.y * b.x - a.x * b.y) * r);
}

// one thread per row of the block: its near kernel entries and its fADI
// vector entries (a running product over the shifts)
__global__ void fadi_rows_kernel(const FadiDesc* __restrict__ descs) {
#pragma clang fp contract(off)
  const FadiDesc d = descs[blockIdx.y];
  const double2* p = d.pq;
  const double2* q = d.pq + d.s;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < d.m; i += gridDim.x * 256) {
    const double x = d.xs[i];
    for (int c = 0; c < d.b; ++c) {
      d.Z[i + (int64_t)c * d.ldz] = dirichlet(x, (d.hi + c) % d.n, d.n);
      d.Z[i + (int64_t)(d.b + c) * d.ldz] = dirichlet(x, (d.lo - d.b + c + d.n) % d.n, d.n);
    }
    double sx, cx;
    sincospi(2.0 * x, &sx, &cx);
    const double2 g = mk<double>(cx, -sx);
    // u = g^n - 1 = exp(-2 pi i f) - 1, f = n x mod 1: pn + e = n x exactly
    // and pn - rint(pn) is exact (contraction is off in this kernel: fusing
    // n x - rint(pn) into one fma would count e twice)
    const double dn = (double)d.n;
    const double pn = dn * x, e = fma(dn, x, -pn);
    const double f = (pn - rint(pn)) + e;
    double sf, cf;
    sincospi(f, &sf, &cf);
    double2 z = cdiv(mk<double>(-2.0 * sf * sf, -2.0 * sf * cf), csub(g, q[0]));
    double2* out = d.Z + i + (int64_t)(2 * d.b) * d.ldz;
    out[0] = z;
    for (int j = 1; j < d.s; ++j) {
      z = cmul(z, cdiv(csub(g, p[j - 1]), csub(g, q[j])));
      out[(int64_t)j * d.ldz] = z;
    }
  }
}

// one thread per column: W(l, .) = 0 on K_a, a unit entry on a near column,
// the conjugated weighted fADI vector entries on a far one
__global__ void fadi_cols_kernel(const FadiDesc* __restrict__ descs) {
  const FadiDesc d = descs[blockIdx.y];
  const double2* p = d.pq;
  const double2* q = d.pq + d.s;
  const int w = 2 * d.b + d.s;
  for (int l = blockIdx.x * 256 + threadIdx.x; l < d.n; l += gridDim.x * 256) {
    double2* row = d.W + l;
    const int dh = (l - d.hi + d.n) % d.n;
    const int dl = (d.lo - 1 - l + d.n) % d.n;
    const bool own = l >= d.lo && l < d.hi;
    int near = -1;
    if (!own && dh < d.b) near = dh;
    else if (!own && dl < d.b) near = 2 * d.b - 1 - dl;
    for (int c = 0; c < 2 * d.b; ++c)
      row[(int64_t)c * d.ldw] = mk<double>(c == near ? 1.0 : 0.0, 0.0);
    if (own || near >= 0) {
      for (int c = 2 * d.b; c < w; ++c) row[(int64_t)c * d.ldw] = mk<double>(0.0, 0.0);
      continue;
    }
    double sw, cw;
    sincospi(2.0 * (double)l / (double)d.n, &sw, &cw);
    const double2 xi = mk<double>(cw, -sw);
    double2 y = cdiv(mk<double>(cw / d.n, -sw / d.n), csub(xi, p[0]));
    for (int j = 0; j < d.s; ++j) {
      if (j > 0) y = cmul(y, cdiv(csub(xi, q[j - 1]), csub(xi, p[j])));
      row[(int64_t)(2 * d.b + j) * d.ldw] = cconj(cmul(csub(q[j], p[j]), y));
    }
  }
}

}  // namespace

void fadi_factors(DescPool& pool, const std::vector<FadiDesc>& d) {
  if (d.empty()) return;
  if (hazards_enabled()) {
    std::vector<Region> v;
    for (size_t i = 0; i < d.size(); ++i) {
      const int w = 2 * d[i].b + d[i].s;
      v.push_back(region(d[i].Z, 16, d[i].m, w, d[i].ldz, true, (int)i));
      v.push_back(region(d[i].W, 16, d[i].n, w, d[i].ldw, true, (int)i));
    }
    check_hazards("fadi_factors", v);
  }
  int mm = 1, mn = 1;
  for (auto& q : d) {
    ND_CHECK(q.s >= 1 && q.b >= 1 && q.m >= 0 && q.n > 2 * q.b && q.lo >= 0 && q.lo < q.hi &&
                 q.hi <= q.n && q.ldz >= std::max(q.m, 1) && q.ldw >= q.n,
             NUDFT2_E_INTERNAL, "fadi_factors: bad descriptor");
    mm = std::max(mm, q.m);
    mn = std::max(mn, q.n);
  }
  auto* dd = (FadiDesc*)pool.push(d.data(), sizeof(FadiDesc) * d.size());
  hipLaunchKernelGGL(fadi_rows_kernel, dim3(std::min(ceil_div(mm, 256), 256), (unsigned)d.size()),
                     dim3(256), 0, pool.stream, dd);
  ND_HIP(hipGetLastError());
  hipLaunchKernelGGL(fadi_cols_kernel, dim3(std::min(ceil_div(mn, 256), 64), (unsigned)d.size()),
                     dim3(256), 0, pool.stream, dd);
  ND_HIP(hipGetLastError());
}

void zero_rc(DescPool& pool, const std::vector<ZeroRCDesc>& d, bool rows_too) {
  if (d.empty()) return;
  if (hazards_enabled()) {
    std::vector<Region> v;
    for (size_t i = 0; i < d.size(); ++i)
      v.push_back(region(d[i].K, 16, d[i].n, d[i].n, d[i].ld, true, (int)i));
    check_hazards("zero_rc", v);
  }
  int64_t mx = 0;
  for (auto& q : d) mx = std::max<int64_t>(mx, (int64_t)q.n * q.w);
  if (mx == 0) return;
  auto* dd = (ZeroRCDesc*)pool.push(d.data(), sizeof(ZeroRCDesc) * d.size());
  if (rows_too)
    hipLaunchKernelGGL(zero_rc_kernel, dim3(grid_for(mx), (unsigned)d.size()), dim3(256), 0,
                       pool.stream, dd);
  else
    hipLaunchKernelGGL(zero_cols_kernel, dim3(grid_for(mx), (unsigned)d.size()), dim3(256), 0,
                       pool.stream, dd);
  ND_HIP(hipGetLastError());
}

void gather_cols(DescPool& pool, const std::vector<GatherDesc>& d) {
  if (d.empty()) return;
  if (hazards_enabled()) {
    std::vector<Region> v;
    for (size_t i = 0; i < d.size(); ++i)
      v.push_back(region(d[i].out, 16, d[i].m, d[i].r, d[i].ldo, true, (int)i));
    check_hazards("gather_cols", v);
  }
  int64_t mx = 0;
  for (auto& q : d) mx = std::max<int64_t>(mx, (int64_t)q.m * q.r);
  if (mx == 0) return;
  auto* dd = (GatherDesc*)pool.push(d.data(), sizeof(GatherDesc) * d.size());
  hipLaunchKernelGGL(gather_cols_kernel, dim3(grid_for(mx), (unsigned)d.size()), dim3(256), 0,
                     pool.stream, dd);
  ND_HIP(hipGetLastError());
}

void diag1d(DescPool& pool, const std::vector<Diag1Desc>& d, const double* xs) {
  if (d.empty()) return;
  int64_t mx = 0;
  for (auto& q : d) mx = std::max<int64_t>(mx, q.m);
  auto* dd = (Diag1Desc*)pool.push(d.data(), sizeof(Diag1Desc) * d.size());
  hipLaunchKernelGGL(diag1d_kernel, dim3(grid_for(mx), (unsigned)d.size()), dim3(256), 0,
                     pool.stream, dd, xs);
  ND_HIP(hipGetLastError());
}

#define GINST(T)                                                                          \
  template void gen_leafD<T>(DescPool&, const std::vector<LeafDesc<T>>&, const double*);  \
  template void gen_leafU<T>(DescPool&, const std::vector<LeafDesc<T>>&, const double*,   \
                             const int64_t*, const int64_t*);                             \
  template void gen_leafV<T>(DescPool&, const std::vector<LeafVDesc<T>>&);                \
  template void gen_asm<T>(DescPool&, const std::vector<AsmDesc<T>>&);
GINST(float)
GINST(double)

}  // namespace nd
