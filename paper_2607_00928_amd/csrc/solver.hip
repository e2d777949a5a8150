// Offline (factor) and online (solve) drivers, Algorithm 4.1.
//
// factor: 1D HSS of G^x and G^y at eps/10 -> face-splitting assembly ->
//         recompression at eps -> URV factorization (working precision).
// solve:  c = F^{-1} H^+ (conj(phi) o f) by the URV sweeps and a 2D inverse
//         DFT (phi_j = exp(i pi (nx x_j + ny y_j)) maps the paper's 0-based
//         frequencies to the centred ones), optionally refined in FP64 against
//         the exact operator: r = f - A c, c += F^{-1} H^+ (r / ||r||) ||r||.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "device_util.h"
#include "gen.h"
#include "hss.h"
#include "solver.h"

namespace nd {

namespace {

struct PrepDesc {
  int64_t m0, M;
  int nx, ny;
};

// fw[s + r*ldw] = conj(phi_s) f[r][perm2d[s]] * inv_scale[r]   (2D-sorted rows)
template <typename T>
__global__ void prep_rhs_kernel(const PrepDesc* __restrict__ pd, const double* __restrict__ pts2d,
                                const int64_t* __restrict__ perm2d, const double2* __restrict__ f,
                                int64_t ldf, const double* __restrict__ inv_scale,
                                cplx<T>* __restrict__ fw, int64_t ldw, int nrhs) {
  const PrepDesc d = pd[blockIdx.y];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < d.M * nrhs;
       e += (int64_t)gridDim.x * 256) {
    int64_t j = e % d.M;
    int r = (int)(e / d.M);
    int64_t s = d.m0 + j;
    double x = pts2d[2 * s], y = pts2d[2 * s + 1];
    // conj(phi) = exp(-i pi (nx x + ny y)) = expi_kx(nx/2, x) * expi_kx(ny/2, y)
    double2 ph = cmul(expi_kx((double)(d.nx / 2), x), expi_kx((double)(d.ny / 2), y));
    double2 v = cmul(ph, f[r * ldf + perm2d[s]]);
    double sc = inv_scale[r];
    fw[s + r * ldw] = mk<T>((T)(v.x * sc), (T)(v.y * sc));
  }
}

// out[r][colperm[i]] = cw[i + r*ldw] * scale[r]  (FP64)
template <typename T>
__global__ void post_sol_kernel(const cplx<T>* __restrict__ cw, int64_t ldw,
                                const int64_t* __restrict__ colperm, const double* __restrict__ scale,
                                double2* __restrict__ out, int64_t ldo, int64_t N, int nrhs) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N * nrhs;
       e += (int64_t)gridDim.x * 256) {
    int64_t i = e % N;
    int r = (int)(e / N);
    cplx<T> v = cw[i + r * ldw];
    double sc = scale[r];
    out[r * ldo + colperm[i]] = mk<double>((double)v.x * sc, (double)v.y * sc);
  }
}

// inverse DFT matrix F^{-1}(a, b) = exp(2 pi i ab / n) / n, exact phase
__global__ void idft_matrix_kernel(double2* F, int n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.x * 256) {
    int a = (int)(e % n), b = (int)(e / n);
    int64_t t = ((int64_t)a * b) % n;
    double s, c;
    sincospi(2.0 * (double)t / (double)n, &s, &c);
    F[e] = mk<double>(c / n, s / n);
  }
}

// per right-hand side sum of squares (atomics), x: nrhs x n row-major
__global__ void sumsq_kernel(const double2* __restrict__ x, int64_t n, int64_t ldx,
                             double* __restrict__ out) {
  const int r = blockIdx.y;
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double2 v = x[r * ldx + i];
    s += v.x * v.x + v.y * v.y;
  }
  s = warp_sum(s);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out + r, red[0] + red[1] + red[2] + red[3]);
}

// per right-hand side and problem sum of squares (atomics): x is nrhs rows of
// ldx entries, problem p's segment of a row is [m0, m0 + M) (M-vectors) or
// [c0, c0 + nx ny) (N-vectors, ncoef); out[r * nprob + p]
__global__ void seg_sumsq_kernel(const double2* __restrict__ x, int64_t ldx,
                                 const ApplyProb* __restrict__ ap, int nprob, int ncoef,
                                 double* __restrict__ out) {
  const int p = blockIdx.y % nprob, r = blockIdx.y / nprob;
  const ApplyProb q = ap[p];
  const int64_t o = ncoef ? q.c0 : q.m0;
  const int64_t n = ncoef ? (int64_t)q.nx * q.ny : q.M;
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double2 v = x[r * ldx + o + i];
    s += v.x * v.x + v.y * v.y;
  }
  s = warp_sum(s);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out + r * nprob + p, red[0] + red[1] + red[2] + red[3]);
}

// y = a x + b y (complex vectors, real a, b)
__global__ void axpby_kernel(double a, const double2* __restrict__ x, double b,
                             double2* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double2 xv = x[i], yv = y[i];
    y[i] = mk<double>(a * xv.x + b * yv.x, a * xv.y + b * yv.y);
  }
}

__global__ void zero_d_kernel(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0.0;
}

__global__ void inv_kernel(const double* s, double* inv, double* sq, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v = sqrt(s[i]);
    sq[i] = v > 0 ? v : 1.0;
    inv[i] = v > 0 ? 1.0 / v : 1.0;
  }
}

// out[r][perm2d[s]] = phi_s fw[s + r*ldw] scale[r]  (adjoint of prep_rhs_kernel)
template <typename T>
__global__ void prep_adj_kernel(const PrepDesc* __restrict__ pd, const double* __restrict__ pts2d,
                                const int64_t* __restrict__ perm2d, const cplx<T>* __restrict__ fw,
                                int64_t ldw, const double* __restrict__ scale,
                                double2* __restrict__ out, int64_t ldo, int nrhs) {
  const PrepDesc d = pd[blockIdx.y];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < d.M * nrhs;
       e += (int64_t)gridDim.x * 256) {
    int64_t j = e % d.M;
    int r = (int)(e / d.M);
    int64_t s = d.m0 + j;
    double x = pts2d[2 * s], y = pts2d[2 * s + 1];
    double2 ph = cmul(expi_kx((double)(d.nx / 2), x), expi_kx((double)(d.ny / 2), y));
    cplx<T> v = fw[s + r * ldw];
    double2 o = cmul(cconj(ph), mk<double>((double)v.x, (double)v.y));
    double sc = scale[r];
    out[r * ldo + perm2d[s]] = mk<double>(o.x * sc, o.y * sc);
  }
}

// cw[i + r*ldw] = in[r][colperm[i]] inv_scale[r]  (adjoint of post_sol_kernel)
template <typename T>
__global__ void post_adj_kernel(const double2* __restrict__ in, int64_t ldi,
                                const int64_t* __restrict__ colperm,
                                const double* __restrict__ inv_scale, cplx<T>* __restrict__ cw,
                                int64_t ldw, int64_t N, int nrhs) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N * nrhs;
       e += (int64_t)gridDim.x * 256) {
    int64_t i = e % N;
    int r = (int)(e / N);
    double2 v = in[r * ldi + colperm[i]];
    double sc = inv_scale[r];
    cw[i + r * ldw] = mk<T>((T)(v.x * sc), (T)(v.y * sc));
  }
}

struct KDesc {
  int64_t c0, N;
  int nx, ny;
};

// Y = [k^x o c; k^x o z; k^y o c; k^y o z] (each nrhs x Ntot) with the centred
// frequencies of the coefficient index (i = kx' ny + ky')
__global__ void kscale_kernel(const KDesc* __restrict__ kd, const double2* __restrict__ c,
                              const double2* __restrict__ z, double2* __restrict__ Y,
                              int64_t Ntot, int nrhs) {
  const KDesc d = kd[blockIdx.y];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < d.N * nrhs;
       e += (int64_t)gridDim.x * 256) {
    int64_t i = e % d.N;
    int r = (int)(e / d.N);
    double kx = (double)(i / d.ny) - (double)(d.nx / 2);
    double ky = (double)(i % d.ny) - (double)(d.ny / 2);
    int64_t o = r * Ntot + d.c0 + i;
    double2 cv = c[o], zv = z[o];
    int64_t sN = (int64_t)nrhs * Ntot;
    Y[o] = mk<double>(kx * cv.x, kx * cv.y);
    Y[sN + o] = mk<double>(kx * zv.x, kx * zv.y);
    Y[2 * sN + o] = mk<double>(ky * cv.x, ky * cv.y);
    Y[3 * sN + o] = mk<double>(ky * zv.x, ky * zv.y);
  }
}

// dL/dx_j = 2 pi sum_r Im(conj(r_j) t_j - conj(w_j) s_j) with s = A(k^x o c),
// t = A(k^x o z), likewise y with k^y; S4 = A Y (4 nrhs x Mtot)
__global__ void grad_points_kernel(const double2* __restrict__ r, const double2* __restrict__ w,
                                   const double2* __restrict__ S4, double* __restrict__ grad,
                                   int64_t Mtot, int nrhs) {
  const double two_pi = 6.283185307179586476925286766559;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < Mtot;
       j += (int64_t)gridDim.x * 256) {
    double gx = 0, gy = 0;
    const int64_t sM = (int64_t)nrhs * Mtot;
    for (int q = 0; q < nrhs; ++q) {
      int64_t o = q * Mtot + j;
      double2 rv = r[o], wv = w[o];
      double2 sx = S4[o], tx = S4[sM + o], sy = S4[2 * sM + o], ty = S4[3 * sM + o];
      // Im(conj(a) b) = a.x b.y - a.y b.x
      gx += (rv.x * tx.y - rv.y * tx.x) - (wv.x * sx.y - wv.y * sx.x);
      gy += (rv.x * ty.y - rv.y * ty.x) - (wv.x * sy.y - wv.y * sy.x);
    }
    grad[2 * j] = two_pi * gx;
    grad[2 * j + 1] = two_pi * gy;
  }
}

unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

template <typename T>
void factor_t(Plan* P) {
  Ctx cx;
  cx.P = P;
  cx.s = P->stream;
  cx.pool.init(256 << 20, cx.s);
  std::unique_ptr<HSS2<T>> H(new HSS2<T>());
  H->precision = std::is_same<T, float>::value ? 1 : 0;
  ND_HIP(hipStreamSynchronize(cx.s));
  double t0 = now_ms();
  std::vector<Tree1> tx, ty;
  build_1d(cx, 0, P->opts.eps / 10, tx);
  build_1d(cx, 1, P->opts.eps / 10, ty);
  ND_HIP(hipStreamSynchronize(cx.s));
  double t1 = now_ms();
  build_2d<T>(cx, tx, ty, P->opts.eps, *H, 2);
  free_1d(P, tx);
  free_1d(P, ty);
  ND_HIP(hipStreamSynchronize(cx.s));
  double t2 = now_ms();
  urv_factor<T>(cx, *H);
  // inverse DFT matrices
  for (size_t p = 0; p < P->probs.size(); ++p) {
    Prob2<T>& pb = H->probs[p];
    const Problem& q = P->probs[p];
    pb.Fx.r = pb.Fx.c = q.nx;
    pb.Fy.r = pb.Fy.c = q.ny;
    std::vector<Mat<double>*> m{&pb.Fx, &pb.Fy};
    H->mem.push_back(carve(P->arena, m));
    hipLaunchKernelGGL(idft_matrix_kernel, dim3(grid_for((int64_t)q.nx * q.nx)), dim3(256), 0,
                       cx.s, pb.Fx.p, q.nx);
    hipLaunchKernelGGL(idft_matrix_kernel, dim3(grid_for((int64_t)q.ny * q.ny)), dim3(256), 0,
                       cx.s, pb.Fy.p, q.ny);
  }
  cx.pool.check_flag();
  double t3 = now_ms();
  P->info.t_compress_ms = t1 - t0;
  // build_2d timed its face-split assembly; the rest is recompression
  P->info.t_recompress_ms = std::max(0.0, t2 - t1 - P->info.t_facesplit_ms);
  P->info.t_urv_ms = t3 - t2;
  P->info.sweep_bytes = urv_sweep_bytes<T>(*H);
  P->hss.reset(H.release());
  P->factored = true;
}

template <typename T>
struct SolveWs {
  cplx<T>* fw = nullptr;
  cplx<T>* cw = nullptr;
  double2* chat = nullptr;   // natural order, nrhs x Ntot
  double2* tmp = nullptr;    // nrhs x Ntot
  double* sums = nullptr;    // 3 x nrhs
};

// d = F^{-1} H^+ (conj(phi) o r) for nrhs right-hand sides (r: nrhs x Mtot,
// d: nrhs x Ntot), with r normalised per right-hand side by inv_scale.
template <typename T>
void hss_inverse(Ctx& cx, HSS2<T>& H, const double2* r, double2* d, int nrhs, SolveWs<T>& w,
                 const double* scale, const double* inv_scale) {
  Plan* P = cx.P;
  std::vector<PrepDesc> pd;
  int64_t mmax = 0;
  for (auto& q : P->probs) {
    pd.push_back({q.m0, q.M, q.nx, q.ny});
    mmax = std::max(mmax, q.M);
  }
  auto* dpd = (PrepDesc*)cx.pool.push_ro(pd.data(), sizeof(PrepDesc) * pd.size());
  hipLaunchKernelGGL((prep_rhs_kernel<T>), dim3(grid_for(mmax * nrhs), (unsigned)pd.size()),
                     dim3(256), 0, cx.s, dpd, P->pts_2d, P->perm2d, r, P->Mtot, inv_scale, w.fw,
                     P->Mtot, nrhs);
  ND_HIP(hipGetLastError());
  urv_solve<T>(cx, H, w.fw, P->Mtot, w.cw, P->Ntot, nrhs);
  hipLaunchKernelGGL((post_sol_kernel<T>), dim3(grid_for(P->Ntot * nrhs)), dim3(256), 0, cx.s,
                     w.cw, P->Ntot, P->colperm, scale, w.chat, P->Ntot, P->Ntot, nrhs);
  ND_HIP(hipGetLastError());
  // 2D inverse DFT per problem and right-hand side: with the C-order (nx, ny)
  // array seen as the column-major ny x nx matrix X, c = Fy^{-1} X Fx^{-1}.
  std::vector<GemmDesc<double>> g1, g2;
  for (size_t p = 0; p < P->probs.size(); ++p) {
    const Problem& q = P->probs[p];
    Prob2<T>& pb = H.probs[p];
    for (int rr = 0; rr < nrhs; ++rr) {
      const double2* X = w.chat + rr * P->Ntot + q.c0;
      double2* T1 = w.tmp + rr * P->Ntot + q.c0;
      double2* Y = d + rr * P->Ntot + q.c0;
      g1.push_back({q.ny, q.nx, q.ny, pb.Fy.ld, q.ny, q.ny, pb.Fy.p, X, T1, 1.0, 0.0, 0.0});
      g2.push_back({q.ny, q.nx, q.nx, q.ny, pb.Fx.ld, q.ny, T1, pb.Fx.p, Y, 1.0, 0.0, 0.0});
    }
  }
  gemm_batched<double>(cx.pool, g1, OpN, OpN);
  gemm_batched<double>(cx.pool, g2, OpN, OpN);
}

void sumsq(hipStream_t s, const double2* x, int64_t n, int64_t ldx, int nrhs, double* out) {
  hipLaunchKernelGGL(zero_d_kernel, dim3(1), dim3(256), 0, s, out, (int64_t)nrhs);
  hipLaunchKernelGGL(sumsq_kernel, dim3(std::min<int64_t>(grid_for(n), 1024), nrhs), dim3(256), 0,
                     s, x, n, ldx, out);
  ND_HIP(hipGetLastError());
}

// out = S^H v for the solution operator S of hss_inverse (v: nrhs x Ntot,
// natural order; out: nrhs x Mtot, caller order), v normalised per right-hand
// side by inv_scale and the result multiplied by scale.
template <typename T>
void hss_inverse_adj(Ctx& cx, HSS2<T>& H, const double2* v, double2* out, int nrhs,
                     SolveWs<T>& w, const double* scale, const double* inv_scale) {
  Plan* P = cx.P;
  // adjoint 2D inverse DFT: X = Fy^H V Fx^H per problem and right-hand side
  std::vector<GemmDesc<double>> g1, g2;
  for (size_t p = 0; p < P->probs.size(); ++p) {
    const Problem& q = P->probs[p];
    Prob2<T>& pb = H.probs[p];
    for (int rr = 0; rr < nrhs; ++rr) {
      const double2* V = v + rr * P->Ntot + q.c0;
      double2* T1 = w.tmp + rr * P->Ntot + q.c0;
      double2* X = w.chat + rr * P->Ntot + q.c0;
      g1.push_back({q.ny, q.nx, q.ny, pb.Fy.ld, q.ny, q.ny, pb.Fy.p, V, T1, 1.0, 0.0, 0.0});
      g2.push_back({q.ny, q.nx, q.nx, q.ny, pb.Fx.ld, q.ny, T1, pb.Fx.p, X, 1.0, 0.0, 0.0});
    }
  }
  gemm_batched<double>(cx.pool, g1, OpC, OpN);
  gemm_batched<double>(cx.pool, g2, OpN, OpC);
  hipLaunchKernelGGL((post_adj_kernel<T>), dim3(grid_for(P->Ntot * nrhs)), dim3(256), 0, cx.s,
                     w.chat, P->Ntot, P->colperm, inv_scale, w.cw, P->Ntot, P->Ntot, nrhs);
  ND_HIP(hipGetLastError());
  urv_solve_adj<T>(cx, H, w.cw, P->Ntot, w.fw, P->Mtot, nrhs);
  std::vector<PrepDesc> pd;
  int64_t mmax = 0;
  for (auto& q : P->probs) {
    pd.push_back({q.m0, q.M, q.nx, q.ny});
    mmax = std::max(mmax, q.M);
  }
  auto* dpd = (PrepDesc*)cx.pool.push_ro(pd.data(), sizeof(PrepDesc) * pd.size());
  hipLaunchKernelGGL((prep_adj_kernel<T>), dim3(grid_for(mmax * nrhs), (unsigned)pd.size()),
                     dim3(256), 0, cx.s, dpd, P->pts_2d, P->perm2d, w.fw, P->Mtot, scale, out,
                     P->Mtot, nrhs);
  ND_HIP(hipGetLastError());
}

// Shared state of the solve drivers: workspace, the two HSS solution
// operators S (M -> N) and S^H (N -> M), norms, and the refinement iteration
// as a HIP graph.  The operators take the context they launch on: the eager
// one (cx) or the capture context (gcx).
template <typename T>
struct SolveCtx {
  Plan* P;
  HSS2<T>& H;
  Ctx cx;
  int nrhs;
  SolveWs<T> w;
  double* nrm2;
  double* scale;
  double* inv;
  // norms read back by the drivers: 5 slots of nrhs x nprob squared norms,
  // one per right-hand side and problem, so that every problem of a batch
  // plan meets the stopping test on its own
  double* red;
  int nprob;
  int64_t mmax = 0, nmax = 0;   // longest problem segment of an M- / N-vector
  // graph of the iteration body: recorded on a private stream by a context of
  // its own that keeps its descriptors and temporaries while the graph lives
  bool use_graph;
  Ctx gcx;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  SolveCtx(Plan* p, int nr) : P(p), H(*static_cast<HSS2<T>*>(p->hss.get())), nrhs(nr) {
    cx.P = P;
    cx.s = P->stream;
    cx.pool.init(64 << 20, cx.s);
    w.fw = (cplx<T>*)cx.tmp_alloc(sizeof(cplx<T>) * P->Mtot * nrhs);
    w.cw = (cplx<T>*)cx.tmp_alloc(sizeof(cplx<T>) * P->Ntot * nrhs);
    w.chat = (double2*)cx.tmp_alloc(sizeof(double2) * P->Ntot * nrhs);
    w.tmp = (double2*)cx.tmp_alloc(sizeof(double2) * P->Ntot * nrhs);
    nprob = (int)P->probs.size();
    for (auto& q : P->probs) {
      mmax = std::max(mmax, q.M);
      nmax = std::max(nmax, q.N());
    }
    w.sums = (double*)cx.tmp_alloc(sizeof(double) * (3 + 5 * (size_t)nprob) * nrhs);
    nrm2 = w.sums;
    scale = w.sums + nrhs;
    inv = w.sums + 2 * nrhs;
    red = w.sums + 3 * nrhs;
    use_graph = P->opts.graph == 1 && !P->profiling;
  }
  ~SolveCtx() {
    (void)hipStreamSynchronize(cx.s);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) {
      (void)hipStreamSynchronize(cap);
      gcx.s = cx.s;   // the capture stream goes; gcx releases its temporaries on cx.s
      gcx.pool.stream = cx.s;
      (void)hipStreamDestroy(cap);
    } else {
      gcx.s = cx.s;
    }
  }
  double2* vecM() { return (double2*)cx.tmp_alloc(sizeof(double2) * P->Mtot * nrhs); }
  double2* vecN() { return (double2*)cx.tmp_alloc(sizeof(double2) * P->Ntot * nrhs); }
  void zero(double2* x, int64_t n) {
    hipLaunchKernelGGL(zero_d_kernel, dim3(grid_for(2 * n * nrhs)), dim3(256), 0, cx.s,
                       (double*)x, 2 * n * nrhs);
  }
  void copy(const double2* x, double2* y, int64_t n) {
    ND_HIP(hipMemcpyAsync(y, x, sizeof(double2) * n * nrhs, hipMemcpyDeviceToDevice, cx.s));
  }
  void axpby(Ctx& k, double a, const double2* x, double b, double2* y, int64_t n) {
    hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, k.s, a, x, b, y,
                       n * nrhs);
  }
  void axpby(double a, const double2* x, double b, double2* y, int64_t n) {
    axpby(cx, a, x, b, y, n);
  }
  void normalise(Ctx& k, const double2* x, int64_t n) {
    sumsq(k.s, x, n, n, nrhs, nrm2);
    hipLaunchKernelGGL(inv_kernel, dim3(1), dim3(256), 0, k.s, nrm2, inv, scale, nrhs);
  }
  // d = S r (r: nrhs x Mtot -> d: nrhs x Ntot)
  void S(Ctx& k, const double2* r, double2* d) {
    normalise(k, r, P->Mtot);
    hss_inverse<T>(k, H, r, d, nrhs, w, scale, inv);
  }
  void S(const double2* r, double2* d) { S(cx, r, d); }
  // out = S^H v (v: nrhs x Ntot -> out: nrhs x Mtot)
  void SH(Ctx& k, const double2* v, double2* out) {
    normalise(k, v, P->Ntot);
    hss_inverse_adj<T>(k, H, v, out, nrhs, w, scale, inv);
  }
  // squared norms per right-hand side and problem into slot i of red (no
  // wait); x is an M-vector (n == Mtot) or an N-vector (n == Ntot).  Every
  // problem has M_p >= N_p, so Mtot == Ntot only when M_p == N_p for all p,
  // and then both segmentations coincide.
  void norm_into(Ctx& k, int i, const double2* x, int64_t n) {
    double* out = red + (size_t)i * nrhs * nprob;
    const bool coef = n != P->Mtot;
    hipLaunchKernelGGL(zero_d_kernel, dim3(1), dim3(256), 0, k.s, out, (int64_t)nrhs * nprob);
    const int64_t len = coef ? nmax : mmax;
    hipLaunchKernelGGL(seg_sumsq_kernel,
                       dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(grid_for(len), 256)),
                            (unsigned)(nrhs * nprob)),
                       dim3(256), 0, k.s, x, n, P->d_aprob, nprob, coef ? 1 : 0, out);
    ND_HIP(hipGetLastError());
  }
  // read back the first cnt norm slots (synchronises); the eager pool is
  // recycled here
  std::vector<double> read_norms(int cnt) {
    std::vector<double> h((size_t)cnt * nrhs * nprob);
    ND_HIP(hipMemcpyAsync(h.data(), red, sizeof(double) * h.size(), hipMemcpyDeviceToHost,
                          cx.s));
    ND_HIP(hipStreamSynchronize(cx.s));
    cx.pool.sync_reset();
    return h;
  }
  // squared norms per right-hand side of several vectors, read back (synchronises)
  std::vector<double> norms2(std::initializer_list<std::pair<const double2*, int64_t>> xs) {
    int i = 0;
    for (auto& x : xs) norm_into(cx, i++, x.first, x.second);
    return read_norms(i);
  }
  // Run the iteration body: eagerly, or (graph mode) eagerly on the first
  // call, then captured once and replayed on cx.s.  The eager first call
  // leaves the body's temporaries in the arena's free list, so the capture
  // allocates no new device memory.  The body must issue the same work with
  // the same pointers on every call, and launch only on k.s through k.pool.
  int runs = 0;
  template <class F>
  void run(F&& body) {
    if (!use_graph || runs++ == 0) {
      body(cx);
      return;
    }
    if (!gexec) {
      ND_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      gcx.P = P;
      gcx.s = cap;
      gcx.pool.init(64 << 20, cap);
      ND_HIP(hipStreamSynchronize(cap));
      gcx.pool.deferred = true;
      gcx.keep = true;
      Profiler* saved = g_prof;
      g_prof = nullptr;
      ND_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
      try {
        body(gcx);
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cap, &g);
        if (g) (void)hipGraphDestroy(g);
        g_prof = saved;
        throw;
      }
      g_prof = saved;
      ND_HIP(hipStreamEndCapture(cap, &graph));
      ND_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
      // descriptors reach the device before the first replay (same stream)
      gcx.pool.stream = cx.s;
      gcx.pool.flush();
    }
    ND_HIP(hipGraphLaunch(gexec, cx.s));
  }
  // worst ||a|| / ||b|| over the right-hand sides and problems of two norm
  // slots (a problem whose b vanishes counts as converged when a does too)
  double worst_ratio(const std::vector<double>& h, int ia, int ib) const {
    double worst = 0;
    const size_t sl = (size_t)nrhs * nprob;
    for (size_t e = 0; e < sl; ++e)
      worst = std::max(worst, std::sqrt(h[ia * sl + e]) /
                                  std::max(std::sqrt(h[ib * sl + e]), 1e-300));
    return worst;
  }
  // ||x|| of right-hand side r over all problems from one norm slot
  double total(const std::vector<double>& h, int i, int r) const {
    double t = 0;
    for (int p = 0; p < nprob; ++p) t += h[((size_t)i * nrhs + r) * nprob + p];
    return std::sqrt(t);
  }
};

void report(nudft2_solve_info* info, int its, double upd, double res) {
  if (!info) return;
  info->iterations = its;
  info->rel_update = upd;
  info->rel_residual = res;
}

// Least-squares solve.  refine == 0: iterative refinement c += S (f - A c)
// (exact for consistent f); refine == 1: refinement on the normal equations,
// c += S S^H A^H (f - A c), whose fixed point is the least-squares solution
// for any f.  ir_maxit == 0: the direct solution S f.
template <typename T>
void solve_t(Plan* P, const double2* f, double2* c, int nrhs, nudft2_solve_info* info) {
  SolveCtx<T> sc(P, nrhs);
  const int64_t M = P->Mtot, N = P->Ntot;
  const int maxit = P->opts.ir_maxit;
  if (maxit == 0) {
    sc.S(f, c);
    ND_HIP(hipStreamSynchronize(sc.cx.s));
    report(info, 0, 0, -1);
    return;
  }
  const bool ne = P->opts.refine == 1;
  double2* rr = sc.vecM();
  double2* dd = sc.vecN();
  double2* rN = ne ? sc.vecN() : nullptr;
  double2* tM = ne ? sc.vecM() : nullptr;
  sc.copy(f, rr, M);
  sc.zero(c, N);
  const double fn = sc.total(sc.norms2({{f, M}}), 0, 0);
  int it = 1;
  double upd = 0, res = 1;
  bool conv = false;
  // correction of the current iterate from its residual r: d = S r (or
  // S S^H A^H r), c += d, norms of d and c
  auto correct = [&](Ctx& k) {
    if (ne) {
      apply_adj(P, rr, rN, nrhs, k.s);
      sc.SH(k, rN, tM);
      sc.S(k, tM, dd);
    } else {
      sc.S(k, rr, dd);
    }
    sc.axpby(k, 1.0, dd, 1.0, c, N);
    sc.norm_into(k, 0, dd, N);
    sc.norm_into(k, 1, c, N);
  };
  // iterations after the first: the residual r = f - A c of the current
  // iterate, then its correction.  A converged solve thus forms no residual
  // after its last update; the residual reported is that of the iterate
  // before it (the returned c differs from it by rel_update).
  auto body = [&](Ctx& k) {
    apply_fwd(P, c, rr, nrhs, k.s);
    sc.axpby(k, 1.0, f, -1.0, rr, M);
    sc.norm_into(k, 2, rr, M);
    correct(k);
  };
  // first iteration: c = 0, r = f
  correct(sc.cx);
  upd = sc.worst_ratio(sc.read_norms(2), 0, 1);
  conv = upd <= P->opts.ir_tol;
  while (!conv && upd == upd && it < maxit) {   // (upd != upd: NaN, stop)
    ++it;
    sc.run(body);
    std::vector<double> h = sc.read_norms(3);
    upd = sc.worst_ratio(h, 0, 1);
    res = sc.total(h, 2, 0) / std::max(fn, 1e-300);
    conv = upd <= P->opts.ir_tol;
  }
  report(info, it, upd, res);
  if (!conv) throw Error(NUDFT2_E_NOCONV, "refinement did not reach ir_tol");
}

// z = (A^H A)^{-1} g by refinement on the normal equations preconditioned by
// S S^H: z += S S^H (g - A^H A z).  Returns iterations and the last update.
template <typename T>
void normal_solve(SolveCtx<T>& sc, const double2* g, double2* z, int& its, double& upd) {
  Plan* P = sc.P;
  const int64_t M = P->Mtot, N = P->Ntot;
  const int maxit = std::max(P->opts.ir_maxit, 1);
  double2* rz = sc.vecN();
  double2* dd = sc.vecN();
  double2* u = sc.vecM();
  double2* tM = sc.vecM();
  sc.copy(g, rz, N);
  sc.zero(z, N);
  bool conv = false;
  // correction from the residual r: d = S S^H r, z += d, norms of d and z
  auto correct = [&](Ctx& k) {
    sc.SH(k, rz, tM);
    sc.S(k, tM, dd);
    sc.axpby(k, 1.0, dd, 1.0, z, N);
    sc.norm_into(k, 0, dd, N);
    sc.norm_into(k, 1, z, N);
  };
  // later iterations: r = g - A^H A z of the current iterate, then its
  // correction (no residual is formed after the last update)
  auto body = [&](Ctx& k) {
    apply_fwd(P, z, u, sc.nrhs, k.s);
    apply_adj(P, u, rz, sc.nrhs, k.s);
    sc.axpby(k, 1.0, g, -1.0, rz, N);
    correct(k);
  };
  its = 1;
  correct(sc.cx);
  upd = sc.worst_ratio(sc.read_norms(2), 0, 1);
  conv = upd <= P->opts.ir_tol;
  while (!conv && upd == upd && its < maxit) {   // (upd != upd: NaN, stop)
    ++its;
    sc.run(body);
    upd = sc.worst_ratio(sc.read_norms(2), 0, 1);
    conv = upd <= P->opts.ir_tol;
  }
  if (!conv) throw Error(NUDFT2_E_NOCONV, "refinement did not reach ir_tol");
}

// w = (A^+)^H g = A (A^H A)^{-1} g
template <typename T>
void solve_adj_t(Plan* P, const double2* g, double2* w, int nrhs, nudft2_solve_info* info) {
  SolveCtx<T> sc(P, nrhs);
  double2* z = sc.vecN();
  int its = 0;
  double upd = 0;
  normal_solve<T>(sc, g, z, its, upd);
  apply_fwd(P, z, w, nrhs, sc.cx.s);
  ND_HIP(hipStreamSynchronize(sc.cx.s));
  report(info, its, upd, -1);
}

// Backward pass of c = A^+ f for upstream g = dL/dc: grad_f = (A^+)^H g and,
// when grad_pts is given, dL/d(x_j, y_j) (summed over the right-hand sides).
template <typename T>
void lsq_backward_t(Plan* P, const double2* f, const double2* c, const double2* g,
                    double2* grad_f, double* grad_pts, int nrhs, nudft2_solve_info* info) {
  SolveCtx<T> sc(P, nrhs);
  const int64_t M = P->Mtot, N = P->Ntot;
  double2* z = sc.vecN();
  int its = 0;
  double upd = 0;
  normal_solve<T>(sc, g, z, its, upd);
  double2* w = grad_f ? grad_f : sc.vecM();
  apply_fwd(P, z, w, nrhs, sc.cx.s);
  if (grad_pts) {
    double2* r = sc.vecM();
    apply_fwd(P, c, r, nrhs, sc.cx.s);
    sc.axpby(1.0, f, -1.0, r, M);
    double2* Y = (double2*)sc.cx.tmp_alloc(sizeof(double2) * 4 * N * nrhs);
    double2* S4 = (double2*)sc.cx.tmp_alloc(sizeof(double2) * 4 * M * nrhs);
    std::vector<KDesc> kd;
    int64_t nmax = 0;
    for (auto& q : P->probs) {
      kd.push_back({q.c0, q.N(), q.nx, q.ny});
      nmax = std::max<int64_t>(nmax, q.N());
    }
    auto* dkd = (KDesc*)sc.cx.pool.push(kd.data(), sizeof(KDesc) * kd.size());
    hipLaunchKernelGGL(kscale_kernel, dim3(grid_for(nmax * nrhs), (unsigned)kd.size()), dim3(256),
                       0, sc.cx.s, dkd, c, z, Y, N, nrhs);
    ND_HIP(hipGetLastError());
    apply_fwd(P, Y, S4, 4 * nrhs, sc.cx.s);
    hipLaunchKernelGGL(grad_points_kernel, dim3(grid_for(M)), dim3(256), 0, sc.cx.s, r, w, S4,
                       grad_pts, M, nrhs);
    ND_HIP(hipGetLastError());
  }
  ND_HIP(hipStreamSynchronize(sc.cx.s));
  report(info, its, upd, -1);
}

}  // namespace

void factor(Plan* P) {
  if (P->factored) return;
  if (P->opts.precision == 0) factor_t<double>(P);
  else factor_t<float>(P);
}

void solve(Plan* P, const double2* f, double2* c, int nrhs, nudft2_solve_info* info,
           bool adjoint) {
  if (P->hss->precision == 0) {
    if (adjoint) solve_adj_t<double>(P, f, c, nrhs, info);
    else solve_t<double>(P, f, c, nrhs, info);
  } else {
    if (adjoint) solve_adj_t<float>(P, f, c, nrhs, info);
    else solve_t<float>(P, f, c, nrhs, info);
  }
}

void lsq_backward(Plan* P, const double2* f, const double2* c, const double2* g, double2* grad_f,
                  double* grad_pts, int nrhs, nudft2_solve_info* info) {
  if (P->hss->precision == 0) lsq_backward_t<double>(P, f, c, g, grad_f, grad_pts, nrhs, info);
  else lsq_backward_t<float>(P, f, c, g, grad_f, grad_pts, nrhs, info);
}

}  // namespace nd
