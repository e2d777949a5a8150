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
  int i = threadIdx.x;
  if (i < n) {
    double v = sqrt(s[i]);
    sq[i] = v > 0 ? v : 1.0;
    inv[i] = v > 0 ? 1.0 / v : 1.0;
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
  P->info.t_recompress_ms = t2 - t1;   // face-split assembly + recompression
  P->info.t_facesplit_ms = 0;
  P->info.t_urv_ms = t3 - t2;
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
  auto* dpd = (PrepDesc*)cx.pool.push(pd.data(), sizeof(PrepDesc) * pd.size());
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

template <typename T>
void solve_t(Plan* P, const double2* f, double2* c, int nrhs, nudft2_solve_info* info) {
  HSS2<T>& H = *static_cast<HSS2<T>*>(P->hss.get());
  Ctx cx;
  cx.P = P;
  cx.s = P->stream;
  cx.pool.init(64 << 20, cx.s);
  SolveWs<T> w;
  w.fw = (cplx<T>*)cx.tmp_alloc(sizeof(cplx<T>) * P->Mtot * nrhs);
  w.cw = (cplx<T>*)cx.tmp_alloc(sizeof(cplx<T>) * P->Ntot * nrhs);
  w.chat = (double2*)cx.tmp_alloc(sizeof(double2) * P->Ntot * nrhs);
  w.tmp = (double2*)cx.tmp_alloc(sizeof(double2) * P->Ntot * nrhs);
  w.sums = (double*)cx.tmp_alloc(sizeof(double) * 8 * nrhs);
  double* nrm2 = w.sums;
  double* scale = w.sums + nrhs;
  double* inv = w.sums + 2 * nrhs;
  double* tmp2 = w.sums + 3 * nrhs;
  const int64_t MN = P->Mtot * nrhs, NN = P->Ntot * nrhs;
  const int maxit = P->opts.ir_maxit;
  if (maxit == 0) {
    sumsq(cx.s, f, P->Mtot, P->Mtot, nrhs, nrm2);
    hipLaunchKernelGGL(inv_kernel, dim3(1), dim3(64), 0, cx.s, nrm2, inv, scale, nrhs);
    hss_inverse<T>(cx, H, f, c, nrhs, w, scale, inv);
    if (info) {
      info->iterations = 0;
      info->rel_update = 0;
      info->rel_residual = -1;
    }
    ND_HIP(hipStreamSynchronize(cx.s));
    return;
  }
  double2* rr = (double2*)cx.tmp_alloc(sizeof(double2) * MN);
  double2* dd = (double2*)cx.tmp_alloc(sizeof(double2) * NN);
  ND_HIP(hipMemcpyAsync(rr, f, sizeof(double2) * MN, hipMemcpyDeviceToDevice, cx.s));
  hipLaunchKernelGGL(zero_d_kernel, dim3(grid_for(2 * NN)), dim3(256), 0, cx.s, (double*)c,
                     2 * NN);
  std::vector<double> h(4 * nrhs);
  double fn = 0;
  {
    sumsq(cx.s, f, P->Mtot, P->Mtot, nrhs, nrm2);
    ND_HIP(hipMemcpyAsync(h.data(), nrm2, sizeof(double) * nrhs, hipMemcpyDeviceToHost, cx.s));
    ND_HIP(hipStreamSynchronize(cx.s));
    fn = std::sqrt(h[0]);
  }
  int it = 0;
  double upd = 0, res = 1;
  bool conv = false;
  for (it = 1; it <= maxit; ++it) {
    // d = H^+ r (normalised), c += d
    sumsq(cx.s, rr, P->Mtot, P->Mtot, nrhs, nrm2);
    hipLaunchKernelGGL(inv_kernel, dim3(1), dim3(64), 0, cx.s, nrm2, inv, scale, nrhs);
    hss_inverse<T>(cx, H, rr, dd, nrhs, w, scale, inv);
    hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(NN)), dim3(256), 0, cx.s, 1.0, dd, 1.0, c, NN);
    // r = f - A c
    apply_fwd(P, c, rr, nrhs, cx.s);
    hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(MN)), dim3(256), 0, cx.s, 1.0, f, -1.0, rr, MN);
    sumsq(cx.s, dd, P->Ntot, P->Ntot, nrhs, tmp2);
    sumsq(cx.s, c, P->Ntot, P->Ntot, nrhs, tmp2 + nrhs);
    sumsq(cx.s, rr, P->Mtot, P->Mtot, nrhs, tmp2 + 2 * nrhs);
    ND_HIP(hipMemcpyAsync(h.data(), tmp2, sizeof(double) * 3 * nrhs, hipMemcpyDeviceToHost, cx.s));
    ND_HIP(hipStreamSynchronize(cx.s));
    cx.pool.sync_reset();
    double worst = 0;
    for (int r = 0; r < nrhs; ++r) {
      double u = std::sqrt(h[r]) / std::max(std::sqrt(h[nrhs + r]), 1e-300);
      worst = std::max(worst, u);
    }
    upd = worst;
    res = std::sqrt(h[2 * nrhs]) / std::max(fn, 1e-300);
    if (!(worst == worst)) break;   // NaN: stop
    if (worst <= P->opts.ir_tol) {
      conv = true;
      break;
    }
  }
  if (info) {
    info->iterations = std::min(it, maxit);
    info->rel_update = upd;
    info->rel_residual = res;
  }
  if (!conv) throw Error(NUDFT2_E_NOCONV, "refinement did not reach ir_tol");
}

}  // namespace

void factor(Plan* P) {
  if (P->factored) return;
  if (P->opts.precision == 0) factor_t<double>(P);
  else factor_t<float>(P);
}

void solve(Plan* P, const double2* f, double2* c, int nrhs, nudft2_solve_info* info,
           bool adjoint) {
  ND_CHECK(!adjoint, NUDFT2_E_INTERNAL, "adjoint solve not available yet");
  if (P->hss->precision == 0) solve_t<double>(P, f, c, nrhs, info);
  else solve_t<float>(P, f, c, nrhs, info);
}

}  // namespace nd
