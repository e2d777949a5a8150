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

// ---- per-segment FP64 vector kernels of the Krylov refinements.  A
// segment is one problem's part of one right-hand side (blockIdx.y =
// rhs * nprob + problem); coefficient arrays hold one scalar per segment.
struct SegArgs {
  const ApplyProb* ap;
  int nprob;
  int ncoef;     // 1: N-vector segments [c0, c0 + nx ny); 0: M-vector [m0, m0 + M)
  int64_t ld;    // entries per right-hand side (Ntot or Mtot)
};

__device__ inline void seg_range(const SegArgs& a, int64_t& o, int64_t& n) {
  const int p = blockIdx.y % a.nprob, r = blockIdx.y / a.nprob;
  const ApplyProb q = a.ap[p];
  o = r * a.ld + (a.ncoef ? q.c0 : q.m0);
  n = a.ncoef ? (int64_t)q.nx * q.ny : q.M;
}

// out[seg] += Re(x^H y) over the segment (out zeroed beforehand)
__global__ void seg_dot_kernel(SegArgs a, const double2* __restrict__ x,
                               const double2* __restrict__ y, double* __restrict__ out) {
  int64_t o, n;
  seg_range(a, o, n);
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double2 u = x[o + i], v = y[o + i];
    s += u.x * v.x + u.y * v.y;
  }
  s = warp_sum(s);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out + blockIdx.y, red[0] + red[1] + red[2] + red[3]);
}

// y += sgn coef[seg] x
__global__ void seg_axpy_kernel(SegArgs a, const double* __restrict__ coef, double sgn,
                                const double2* __restrict__ x, double2* __restrict__ y) {
  int64_t o, n;
  seg_range(a, o, n);
  const double c = sgn * coef[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double2 u = x[o + i];
    double2 v = y[o + i];
    v.x += c * u.x;
    v.y += c * u.y;
    y[o + i] = v;
  }
}

// y = x + sgn coef[seg] y
__global__ void seg_xpay_kernel(SegArgs a, const double2* __restrict__ x,
                                const double* __restrict__ coef, double sgn,
                                double2* __restrict__ y) {
  int64_t o, n;
  seg_range(a, o, n);
  const double c = sgn * coef[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double2 u = x[o + i], v = y[o + i];
    y[o + i] = mk<double>(u.x + c * v.x, u.y + c * v.y);
  }
}

// y *= coef[seg]
__global__ void seg_scale_kernel(SegArgs a, const double* __restrict__ coef,
                                 double2* __restrict__ y) {
  int64_t o, n;
  seg_range(a, o, n);
  const double c = coef[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double2 v = y[o + i];
    y[o + i] = mk<double>(c * v.x, c * v.y);
  }
}

__global__ void copy_d2_kernel(const double2* __restrict__ x, double2* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    y[i] = x[i];
}

// conjugate gradients: alpha = rho / gamma (gamma = ||A p||^2)
__global__ void pcg_alpha_kernel(const double* rho, const double* gamma, double* alpha, int nseg) {
  for (int e = threadIdx.x; e < nseg; e += blockDim.x)
    alpha[e] = gamma[e] > 0.0 ? rho[e] / gamma[e] : 0.0;
}

// flexible (Polak-Ribiere) beta = (rho_new - r^H z_old) / rho, then rho = rho_new
__global__ void pcg_beta_kernel(double* rho, const double* rho_new, const double* mix,
                                double* beta, int nseg) {
  for (int e = threadIdx.x; e < nseg; e += blockDim.x) {
    beta[e] = rho[e] > 0.0 ? (rho_new[e] - mix[e]) / rho[e] : 0.0;
    rho[e] = rho_new[e];
  }
}

// nrm = sqrt(s2), inv = 1 / nrm (0 for a zero vector)
__global__ void norm_inv_kernel(const double* s2, double* nrm, double* inv, int nseg) {
  for (int e = threadIdx.x; e < nseg; e += blockDim.x) {
    const double v = sqrt(s2[e]);
    nrm[e] = v;
    inv[e] = v > 0.0 ? 1.0 / v : 0.0;
  }
}

// LSQR's plane rotation (Paige and Saunders): from rhobar, phibar and the new
// beta, alpha: rho = |(rhobar, beta)|, c = rhobar / rho, s = beta / rho,
// theta = s alpha, rhobar' = -c alpha, phi = c phibar, phibar' = s phibar;
// the solution moves by (phi / rho) w, then w = v - (theta / rho) w
__global__ void lsqr_rot_kernel(const double* alpha, const double* beta, double* rhobar,
                                double* phibar, double* ax, double* aw, int nseg) {
  for (int e = threadIdx.x; e < nseg; e += blockDim.x) {
    const double rho = hypot(rhobar[e], beta[e]);
    if (rho > 0.0) {
      const double c = rhobar[e] / rho, s = beta[e] / rho;
      const double theta = s * alpha[e];
      rhobar[e] = -c * alpha[e];
      const double phi = c * phibar[e];
      phibar[e] = s * phibar[e];
      ax[e] = phi / rho;
      aw[e] = -theta / rho;
    } else {
      ax[e] = 0.0;
      aw[e] = 0.0;
    }
  }
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
  {
    ProfSite site_(PS_1D);
    build_1d(cx, 0, P->opts.eps / 10, tx);
    build_1d(cx, 1, P->opts.eps / 10, ty);
  }
  ND_HIP(hipStreamSynchronize(cx.s));
  P->arena.check("1D compression");
  double t1 = now_ms();
  build_2d<T>(cx, tx, ty, P->opts.eps, *H, 2);
  free_1d(P, tx);
  free_1d(P, ty);
  ND_HIP(hipStreamSynchronize(cx.s));
  P->arena.check("recompression");
  double t2 = now_ms();
  urv_factor<T>(cx, *H);
  P->arena.check("URV factorization");
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
  {
    ProfSite site_(PS_SOLVE);
    urv_solve<T>(cx, H, w.fw, P->Mtot, w.cw, P->Ntot, nrhs);
  }
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
    if (!P->spool.host) P->spool.init(64 << 20, cx.s);
    cx.pool.adopt(P->spool);
    cx.pool.sync_reset();
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
    // the descriptor pool goes back to the plan for the next solve
    try {
      cx.pool.sync_reset();
    } catch (...) {
      // a failed solve may have left uploads unexecuted: nothing is reusable
      cx.pool.valid = cx.pool.used = 0;
      cx.pool.tainted = false;
    }
    P->spool.adopt(cx.pool);
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
  // ---- segmented vector operations (one scalar per right-hand side and
  // problem), launched on k.s; n is Mtot (M-vectors) or Ntot (N-vectors)
  int nseg() const { return nrhs * nprob; }
  SegArgs seg(int64_t n) const {
    return SegArgs{P->d_aprob, nprob, n != P->Mtot ? 1 : 0, n};
  }
  dim3 seg_grid(int64_t n) const {
    const int64_t len = n != P->Mtot ? nmax : mmax;
    return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(grid_for(len), 256)),
                (unsigned)nseg());
  }
  void seg_zero(Ctx& k, double* out) {
    hipLaunchKernelGGL(zero_d_kernel, dim3(1), dim3(256), 0, k.s, out, (int64_t)nseg());
  }
  void seg_dot(Ctx& k, double* out, const double2* x, const double2* y, int64_t n) {
    seg_zero(k, out);
    hipLaunchKernelGGL(seg_dot_kernel, seg_grid(n), dim3(256), 0, k.s, seg(n), x, y, out);
  }
  void seg_axpy(Ctx& k, const double* coef, double sgn, const double2* x, double2* y, int64_t n) {
    hipLaunchKernelGGL(seg_axpy_kernel, seg_grid(n), dim3(256), 0, k.s, seg(n), coef, sgn, x, y);
  }
  void seg_xpay(Ctx& k, const double2* x, const double* coef, double sgn, double2* y, int64_t n) {
    hipLaunchKernelGGL(seg_xpay_kernel, seg_grid(n), dim3(256), 0, k.s, seg(n), x, coef, sgn, y);
  }
  void seg_scale(Ctx& k, const double* coef, double2* y, int64_t n) {
    hipLaunchKernelGGL(seg_scale_kernel, seg_grid(n), dim3(256), 0, k.s, seg(n), coef, y);
  }
  void copyk(Ctx& k, const double2* x, double2* y, int64_t n) {
    hipLaunchKernelGGL(copy_d2_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, k.s, x, y,
                       n * nrhs);
  }
  // device scalars of the Krylov drivers: slot i holds one value per segment
  double* ks = nullptr;
  double* kslot(int i) {
    if (!ks) ks = (double*)cx.tmp_alloc(sizeof(double) * 32 * (size_t)nseg());
    return ks + (size_t)i * nseg();
  }
  // read back cnt consecutive scalar slots from slot i (synchronises)
  std::vector<double> read_slots(int i, int cnt) {
    std::vector<double> h((size_t)cnt * nseg());
    ND_HIP(hipMemcpyAsync(h.data(), kslot(i), sizeof(double) * h.size(), hipMemcpyDeviceToHost,
                          cx.s));
    ND_HIP(hipStreamSynchronize(cx.s));
    cx.pool.sync_reset();
    return h;
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
  // ||a|| / ||b|| per right-hand side and problem of two norm slots
  std::vector<double> ratios(const std::vector<double>& h, int ia, int ib) const {
    const size_t sl = (size_t)nrhs * nprob;
    std::vector<double> r(sl);
    for (size_t e = 0; e < sl; ++e)
      r[e] = std::sqrt(h[ia * sl + e]) / std::max(std::sqrt(h[ib * sl + e]), 1e-300);
    return r;
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

// Slots of SolveCtx::kslot used by the Krylov drivers.
enum KSlot {
  K_PN2 = 0, K_CN2, K_ALPHA,            // read back together (PCG)
  K_RHO, K_GAMMA, K_BETA, K_RHON, K_MIX,
  K_WN2 = 8, K_LCN2, K_AX, K_PHIBAR, K_BETA1,   // read back together (LSQR)
  K_LA, K_LB, K_RHOBAR, K_AW, K_S2, K_INV
};

// Preconditioned conjugate gradients on the normal equations A^H A c = b
// with the preconditioner S S^H (S the factored solution operator, S^H its
// adjoint sweep), in the flexible Polak-Ribiere form: A^H A is applied
// exactly in FP64 each iteration, while the preconditioner may be the FP32
// sweep, whose rounding makes it vary slightly between applications.  Every
// scalar is per right-hand side and problem (the problems of a batch plan are
// independent).  On entry c holds the first iterate and r = b - A^H A c; on
// exit c is the solution.  Stops when every problem's ||alpha p|| / ||c|| <=
// tol; its counts the iterations taken here.
template <typename T>
bool pcg_normal(SolveCtx<T>& sc, double2* c, double2* r, int maxit, double tol, int& its,
                double& upd) {
  Plan* P = sc.P;
  const int64_t M = P->Mtot, N = P->Ntot;
  const int ns = sc.nseg();
  double2* z = sc.vecN();
  double2* zo = sc.vecN();
  double2* p = sc.vecN();
  double2* q = sc.vecN();
  double2* t = sc.vecM();
  double* pn2 = sc.kslot(K_PN2);
  double* cn2 = sc.kslot(K_CN2);
  double* alpha = sc.kslot(K_ALPHA);
  double* rho = sc.kslot(K_RHO);
  double* gamma = sc.kslot(K_GAMMA);
  double* beta = sc.kslot(K_BETA);
  double* rhon = sc.kslot(K_RHON);
  double* mix = sc.kslot(K_MIX);
  // z = S S^H r, p = z, rho = Re(r^H z)
  sc.SH(sc.cx, r, t);
  sc.S(sc.cx, t, z);
  sc.copyk(sc.cx, z, p, N);
  sc.seg_dot(sc.cx, rho, r, z, N);
  auto body = [&](Ctx& k) {
    op_fwd(P, p, t, sc.nrhs, k.s);                 // t = A p
    sc.seg_dot(k, gamma, t, t, M);                    // gamma = ||A p||^2
    op_adj(P, t, q, sc.nrhs, k.s);                 // q = A^H A p
    hipLaunchKernelGGL(pcg_alpha_kernel, dim3(1), dim3(256), 0, k.s, rho, gamma, alpha, ns);
    sc.seg_dot(k, pn2, p, p, N);
    sc.seg_axpy(k, alpha, 1.0, p, c, N);              // c += alpha p
    sc.seg_axpy(k, alpha, -1.0, q, r, N);             // r -= alpha q
    sc.seg_dot(k, cn2, c, c, N);
    sc.copyk(k, z, zo, N);
    sc.SH(k, r, t);                                   // z = S S^H r
    sc.S(k, t, z);
    sc.seg_dot(k, rhon, r, z, N);
    sc.seg_dot(k, mix, r, zo, N);
    hipLaunchKernelGGL(pcg_beta_kernel, dim3(1), dim3(256), 0, k.s, rho, rhon, mix, beta, ns);
    sc.seg_xpay(k, z, beta, 1.0, p, N);               // p = z + beta p
    ND_HIP(hipGetLastError());
  };
  its = 0;
  upd = 1.0;
  bool conv = false;
  while (!conv && upd == upd && its < maxit) {   // (upd != upd: NaN, stop)
    ++its;
    sc.run(body);
    const std::vector<double> h = sc.read_slots(K_PN2, 3);
    upd = 0;
    for (int e = 0; e < ns; ++e)
      upd = std::max(upd, std::fabs(h[2 * ns + e]) * std::sqrt(h[e]) /
                              std::max(std::sqrt(h[ns + e]), 1e-300));
    conv = upd <= tol;
  }
  return conv;
}

// The paper's plsqr (Section 4.1): LSQR (Paige and Saunders) on the left-
// preconditioned system S A c = S f, with B = S A applied as the exact FP64
// apply followed by the factored sweep and B^H = A^H S^H as the adjoint sweep
// followed by the exact adjoint apply.  Its fixed point is the least-squares
// solution for consistent f (S A is nonsingular), as for plain refinement.
// With FP32 factors the sweep's rounding bounds what one LSQR run can reach
// (about 1e-6 relative), so the run restarts from the exact FP64 residual
// r = f - A c whenever its own residual estimate phibar has fallen by
// cycle_tol; with FP64 factors it is one run.  Scalars per right-hand side
// and problem.  Stops when every problem's ||dc|| / ||c|| <= tol.
template <typename T>
bool plsqr(SolveCtx<T>& sc, const double2* f, double2* c, int maxit, double tol,
           double cycle_tol, int& its, double& upd) {
  Plan* P = sc.P;
  const int64_t M = P->Mtot, N = P->Ntot;
  const int ns = sc.nseg();
  double2* u = sc.vecN();
  double2* v = sc.vecN();
  double2* w = sc.vecN();
  double2* tN = sc.vecN();
  double2* tM = sc.vecM();
  double* wn2 = sc.kslot(K_WN2);
  double* cn2 = sc.kslot(K_LCN2);
  double* ax = sc.kslot(K_AX);
  double* phibar = sc.kslot(K_PHIBAR);
  double* beta1 = sc.kslot(K_BETA1);
  double* la = sc.kslot(K_LA);
  double* lb = sc.kslot(K_LB);
  double* rhobar = sc.kslot(K_RHOBAR);
  double* aw = sc.kslot(K_AW);
  double* s2 = sc.kslot(K_S2);
  double* inv = sc.kslot(K_INV);
  auto normalise_seg = [&](Ctx& k, double2* x, double* nrm) {
    sc.seg_dot(k, s2, x, x, N);
    hipLaunchKernelGGL(norm_inv_kernel, dim3(1), dim3(256), 0, k.s, s2, nrm, inv, ns);
    sc.seg_scale(k, inv, x, N);
  };
  auto body = [&](Ctx& k) {
    op_fwd(P, v, tM, sc.nrhs, k.s);                // tN = B v
    sc.S(k, tM, tN);
    sc.seg_xpay(k, tN, la, -1.0, u, N);               // u = B v - alpha u
    normalise_seg(k, u, lb);                          // beta, u /= beta
    sc.SH(k, u, tM);                                  // tN = B^H u
    op_adj(P, tM, tN, sc.nrhs, k.s);
    sc.seg_xpay(k, tN, lb, -1.0, v, N);               // v = B^H u - beta v
    normalise_seg(k, v, la);                          // alpha, v /= alpha
    hipLaunchKernelGGL(lsqr_rot_kernel, dim3(1), dim3(256), 0, k.s, la, lb, rhobar, phibar,
                       ax, aw, ns);
    sc.seg_dot(k, wn2, w, w, N);
    sc.seg_axpy(k, ax, 1.0, w, c, N);                 // c += (phi / rho) w
    sc.seg_xpay(k, v, aw, 1.0, w, N);                 // w = v - (theta / rho) w
    sc.seg_dot(k, cn2, c, c, N);
    ND_HIP(hipGetLastError());
  };
  sc.zero(c, N);
  its = 0;
  upd = 1.0;
  bool conv = false;
  while (!conv && upd == upd && its < maxit) {
    // a run starts from the exact residual of the current iterate
    Ctx& k = sc.cx;
    op_fwd(P, c, tM, sc.nrhs, k.s);
    sc.axpby(k, 1.0, f, -1.0, tM, M);                 // tM = f - A c
    sc.S(k, tM, u);                                   // beta_1 u = S r
    normalise_seg(k, u, beta1);
    sc.SH(k, u, tM);                                  // alpha_1 v = B^H u
    op_adj(P, tM, v, sc.nrhs, k.s);
    normalise_seg(k, v, la);
    sc.copyk(k, v, w, N);
    ND_HIP(hipMemcpyAsync(phibar, beta1, sizeof(double) * ns, hipMemcpyDeviceToDevice, k.s));
    ND_HIP(hipMemcpyAsync(rhobar, la, sizeof(double) * ns, hipMemcpyDeviceToDevice, k.s));
    while (!conv && upd == upd && its < maxit) {
      ++its;
      sc.run(body);
      const std::vector<double> h = sc.read_slots(K_WN2, 5);
      upd = 0;
      double rres = 0;
      for (int e = 0; e < ns; ++e) {
        upd = std::max(upd, std::fabs(h[2 * ns + e]) * std::sqrt(h[e]) /
                                std::max(std::sqrt(h[ns + e]), 1e-300));
        if (h[4 * ns + e] > 0) rres = std::max(rres, h[3 * ns + e] / h[4 * ns + e]);
      }
      conv = upd <= tol;
      if (rres <= cycle_tol) break;   // restart from the exact residual
    }
  }
  return conv;
}

// Least-squares solve.  refine == 0: iterative refinement c += S (f - A c)
// (exact for consistent f); refine == 1: preconditioned conjugate gradients
// on the normal equations from the direct solution (exact least squares for
// any f); refine == 2: the paper's plsqr (exact for consistent f).
// ir_maxit == 0: the direct solution S f.
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
  const int mode = P->opts.refine;
  if (mode == 1 || mode == 2) {
    const double fn = sc.total(sc.norms2({{f, M}}), 0, 0);
    int its = 0;
    double upd = 0;
    bool conv;
    double2* rM = sc.vecM();
    if (mode == 1) {
      // first iterate: the direct solution; then CG on the normal equations
      double2* r = sc.vecN();
      sc.S(f, c);
      op_fwd(P, c, rM, nrhs, sc.cx.s);
      sc.axpby(1.0, f, -1.0, rM, M);
      op_adj(P, rM, r, nrhs, sc.cx.s);
      conv = pcg_normal<T>(sc, c, r, maxit - 1, P->opts.ir_tol, its, upd);
      ++its;
    } else {
      const double cycle_tol = P->hss->precision == 1 ? 1e-5 : 0.0;
      conv = plsqr<T>(sc, f, c, maxit, P->opts.ir_tol, cycle_tol, its, upd);
    }
    // the residual of the returned solution (first right-hand side)
    op_fwd(P, c, rM, nrhs, sc.cx.s);
    sc.axpby(1.0, f, -1.0, rM, M);
    const double res = sc.total(sc.norms2({{rM, M}}), 0, 0) / std::max(fn, 1e-300);
    report(info, its, upd, res);
    if (!conv) throw Error(NUDFT2_E_NOCONV, "refinement did not reach ir_tol");
    return;
  }
  double2* rr = sc.vecM();
  double2* dd = sc.vecN();
  sc.copy(f, rr, M);
  sc.zero(c, N);
  const double fn = sc.total(sc.norms2({{f, M}}), 0, 0);
  int it = 1;
  double upd = 0, res = 1;
  bool conv = false;
  // correction of the current iterate from its residual r: d = S r, c += d,
  // norms of d and c
  auto correct = [&](Ctx& k) {
    sc.S(k, rr, dd);
    sc.axpby(k, 1.0, dd, 1.0, c, N);
    sc.norm_into(k, 0, dd, N);
    sc.norm_into(k, 1, c, N);
  };
  // iterations after the first: the residual r = f - A c of the current
  // iterate, then its correction.  A converged solve thus forms no residual
  // after its last update; the residual reported is that of the iterate
  // before it (the returned c differs from it by rel_update).
  auto body = [&](Ctx& k) {
    op_fwd(P, c, rr, nrhs, k.s);
    sc.axpby(k, 1.0, f, -1.0, rr, M);
    sc.norm_into(k, 2, rr, M);
    correct(k);
  };
  // Stop test, per right-hand side and problem: the relative update u_k =
  // ||dc_k|| / ||c_k|| is at most ir_tol, or (from the third iteration, whose
  // update and the one before it are both corrections of the direct solution)
  // the error bound of a contraction, q / (1 - q) u_k <= ir_tol, holds with
  // q = 10 u_k / u_{k-1} < 1/2 (ten times the observed contraction).  For
  // e_{k+1} = (I - S A) e_k with ||I - S A|| <= q, ||c_k - c*|| <= q / (1 - q)
  // ||dc_k||; the factor 10 covers an observed ratio below the true one.
  const double tol = P->opts.ir_tol;
  std::vector<double> uprev;
  // the worst relative update (NaN if any is NaN)
  auto worst = [](const std::vector<double>& u) {
    double w = 0;
    for (double x : u) {
      if (!(x == x)) return x;
      w = std::max(w, x);
    }
    return w;
  };
  auto converged = [&](const std::vector<double>& u, bool bound) {
    for (size_t e = 0; e < u.size(); ++e) {
      if (u[e] <= tol) continue;
      if (!bound || !(u[e] == u[e])) return false;
      const double q = 10.0 * u[e] / std::max(uprev[e], 1e-300);
      if (!(q < 0.5) || q / (1.0 - q) * u[e] > tol) return false;
    }
    return true;
  };
  // first iteration: c = 0, r = f
  correct(sc.cx);
  {
    std::vector<double> u = sc.ratios(sc.read_norms(2), 0, 1);
    upd = worst(u);
    conv = converged(u, false);
    uprev = u;
  }
  while (!conv && upd == upd && it < maxit) {   // (upd != upd: NaN, stop)
    ++it;
    sc.run(body);
    std::vector<double> h = sc.read_norms(3);
    std::vector<double> u = sc.ratios(h, 0, 1);
    upd = worst(u);
    res = sc.total(h, 2, 0) / std::max(fn, 1e-300);
    conv = converged(u, it >= 3);
    uprev = u;
  }
  report(info, it, upd, res);
  if (!conv) throw Error(NUDFT2_E_NOCONV, "refinement did not reach ir_tol");
}

// z = (A^H A)^{-1} g by preconditioned conjugate gradients on the normal
// equations, from z = S S^H g.  Returns iterations and the last update.
template <typename T>
void normal_solve(SolveCtx<T>& sc, const double2* g, double2* z, int& its, double& upd) {
  Plan* P = sc.P;
  const int64_t N = P->Ntot;
  const int maxit = std::max(P->opts.ir_maxit, 2);   // at least one CG step
  double2* r = sc.vecN();
  double2* u = sc.vecM();
  sc.SH(sc.cx, g, u);                 // z = S S^H g
  sc.S(sc.cx, u, z);
  op_fwd(P, z, u, sc.nrhs, sc.cx.s);
  op_adj(P, u, r, sc.nrhs, sc.cx.s);
  sc.axpby(1.0, g, -1.0, r, N);       // r = g - A^H A z
  const bool conv = pcg_normal<T>(sc, z, r, maxit - 1, P->opts.ir_tol, its, upd);
  ++its;
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
  op_fwd(P, z, w, nrhs, sc.cx.s);
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
  op_fwd(P, z, w, nrhs, sc.cx.s);
  if (grad_pts) {
    double2* r = sc.vecM();
    op_fwd(P, c, r, nrhs, sc.cx.s);
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
    op_fwd(P, Y, S4, 4 * nrhs, sc.cx.s);
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
