// A c and A^* f by spreading and FFT: the NUFFT the paper's Section 4.1
// iterations use for the exact operator, here written for gfx950 in FP64.
//
// Kernel (exponential of a semicircle, support w fine-grid cells):
//   phi(z) = exp(beta (sqrt(1 - (2 z / w)^2) - 1)) for |z| < w / 2, else 0,
// and its Fourier transform phihat(xi) = int phi(t) cos(2 pi xi t) dt, taken
// by Gauss-Legendre quadrature on the host.  Per axis the fine grid has nf
// points (the smallest power of two >= max(2n, 2w)), so x -> nf x is exact.
//
// Type 1, c = A^* f (c_k = sum_j f_j exp(+2 pi i k x_j)):
//   b_l = sum_j f_j phi(l - nf x_j)  (l taken mod nf; both axes)
//   B_k = sum_l b_l exp(+2 pi i k l / nf)          (2D FFT, + sign)
//   c_k = B_k / (phihat(kx / nfx) phihat(ky / nfy))
// since the trapezoid rule on the fine grid reproduces the Fourier
// coefficients of the periodised convolution sum_j f_j phi(nf (x - x_j)),
// which are c_k phihat(k / nf) / nf on each axis.
// Type 2, f = A c, is the exact adjoint of these three steps:
//   u = deconvolved c zero-padded into the fine grid (slot k mod nf),
//   U_l = sum_k u_k exp(-2 pi i k l / nf)           (2D FFT, - sign),
//   f_j = sum_l U_l phi(l - nf x_j).
//
// The FFT is a radix-2 Stockham transform of each row in LDS with a twiddle
// table per length; the second axis is reached by a tiled transpose, so every
// pass reads and writes whole rows.  Spreading adds into the fine grid with
// FP64 atomics (points in quadtree order, so neighbouring threads touch
// neighbouring cells); interpolation gathers.
#include <algorithm>
#include <cmath>
#include <vector>

#include "device_util.h"
#include "plan.h"
#include "prof.h"

namespace nd {

namespace {

constexpr int FFT_MAX = 2048;   // longest fine-grid axis (LDS: 2 x 2048 complex)
constexpr int NT = 256;

__device__ inline double es_kernel(double z, double beta, double inv_half_w) {
  const double u = z * inv_half_w;
  const double a = 1.0 - u * u;
  return a > 0.0 ? exp(beta * (sqrt(a) - 1.0)) : 0.0;
}

// tw[j] = exp(-2 pi i j / n), j < n / 2
__global__ void twiddle_kernel(double2* tw, int n) {
  for (int j = blockIdx.x * NT + threadIdx.x; j < n / 2; j += gridDim.x * NT) {
    double s, c;
    sincospi(2.0 * (double)j / (double)n, &s, &c);
    tw[j] = make_double2(c, -s);
  }
}

__global__ void zero2_kernel(double2* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    p[i] = make_double2(0.0, 0.0);
}

// Row transforms X_k = sum_j x_j exp(sign 2 pi i j k / n), in place, for
// nrows rows of length n (a power of two, n <= FFT_MAX) stored contiguously.
// Stockham autosort, decimation in frequency: a pass of length len and
// stride s (len s = n) maps butterfly (p, q), p < len / 2, q < s, to
//   y[q + s 2p] = a + b,  y[q + s (2p + 1)] = (a - b) w^p,  w = exp(sign 2 pi i / len)
// with a = x[q + s p], b = x[q + s (p + len / 2)]; w^p = tw[p s] (conjugated
// for the + sign).
__global__ __launch_bounds__(NT) void fft_rows_kernel(double2* __restrict__ data, int n,
                                                      int64_t nrows, double sign,
                                                      const double2* __restrict__ tw) {
  __shared__ double2 buf[2 * FFT_MAX];
  __shared__ double2 tws[FFT_MAX / 2];
  for (int j = threadIdx.x; j < n / 2; j += NT) {
    const double2 t = tw[j];
    tws[j] = make_double2(t.x, sign > 0 ? -t.y : t.y);
  }
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    double2* row = data + r * n;
    double2* x = buf;
    double2* y = buf + n;
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += NT) x[j] = row[j];
    __syncthreads();
    for (int len = n, s = 1; len > 1; len >>= 1, s <<= 1) {
      const int m = len >> 1;
      for (int b = threadIdx.x; b < n / 2; b += NT) {
        const int p = b / s, q = b - p * s;
        const double2 a = x[q + s * p], c = x[q + s * (p + m)];
        const double2 w = tws[p * s];
        const double dx = a.x - c.x, dy = a.y - c.y;
        y[q + 2 * s * p] = make_double2(a.x + c.x, a.y + c.y);
        y[q + s * (2 * p + 1)] = make_double2(dx * w.x - dy * w.y, dx * w.y + dy * w.x);
      }
      __syncthreads();
      double2* t = x;
      x = y;
      y = t;
    }
    for (int j = threadIdx.x; j < n; j += NT) row[j] = x[j];
  }
}

// out[b][c][r] = in[b][r][c] for nb matrices of rows x cols (32 x 32 tiles)
__global__ void transpose_kernel(const double2* __restrict__ in, double2* __restrict__ out,
                                 int rows, int cols) {
  __shared__ double2 t[32][33];
  const int64_t b = blockIdx.z;
  const double2* src = in + b * rows * (int64_t)cols;
  double2* dst = out + b * rows * (int64_t)cols;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) t[k][tx] = src[(int64_t)r * cols + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) dst[(int64_t)c * rows + r] = t[tx][k];
  }
}

// g[r][kx mod nfx][ky mod nfy] = c[r][kx'][ky'] invx[kx'] invy[ky'] (centred
// kx = kx' - nx/2); the rest of g is zero beforehand
__global__ void pad_kernel(const double2* __restrict__ c, int64_t ldc, int64_t c0, int nx, int ny,
                           const double* __restrict__ invx, const double* __restrict__ invy,
                           double2* __restrict__ g, int nfx, int nfy, int nrhs) {
  const int64_t n = (int64_t)nx * ny;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n * nrhs;
       e += (int64_t)gridDim.x * NT) {
    const int r = (int)(e / n);
    const int64_t i = e - r * n;
    const int kx = (int)(i / ny), ky = (int)(i - (int64_t)kx * ny);
    const int sx = (kx - nx / 2 + nfx) % nfx, sy = (ky - ny / 2 + nfy) % nfy;
    const double2 v = c[r * ldc + c0 + i];
    const double d = invx[kx] * invy[ky];
    g[((int64_t)r * nfx + sx) * nfy + sy] = make_double2(v.x * d, v.y * d);
  }
}

// c[r][kx'][ky'] = G[r][ky mod nfy][kx mod nfx] invx[kx'] invy[ky'] (G in
// the transposed layout the second row transform leaves)
__global__ void crop_kernel(const double2* __restrict__ G, int nfx, int nfy, int nx, int ny,
                            const double* __restrict__ invx, const double* __restrict__ invy,
                            double2* __restrict__ c, int64_t ldc, int64_t c0, int nrhs) {
  const int64_t n = (int64_t)nx * ny;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n * nrhs;
       e += (int64_t)gridDim.x * NT) {
    const int r = (int)(e / n);
    const int64_t i = e - r * n;
    const int kx = (int)(i / ny), ky = (int)(i - (int64_t)kx * ny);
    const int sx = (kx - nx / 2 + nfx) % nfx, sy = (ky - ny / 2 + nfy) % nfy;
    const double2 v = G[((int64_t)r * nfy + sy) * nfx + sx];
    const double d = invx[kx] * invy[ky];
    c[r * ldc + c0 + i] = make_double2(v.x * d, v.y * d);
  }
}

constexpr int WMAX = 16;

struct NuProb {
  int64_t m0, M;
  int nfx, nfy;
};

// the w kernel weights of one axis for the point t = nf x: cells l0 + i
__device__ inline int axis_weights(double x, int nf, int w, double beta, double* wt) {
  const double t = x * (double)nf;
  const int l0 = (int)ceil(t - 0.5 * w);
  const double ihw = 2.0 / (double)w;
  for (int i = 0; i < w; ++i) wt[i] = es_kernel((double)(l0 + i) - t, beta, ihw);
  return l0;
}

// f[r][perm[s]] = sum_l G[r][ly][lx] phi(lx - nfx x_s) phi(ly - nfy y_s), for
// the points s of the problem in tree order (G transposed: ly major)
__global__ __launch_bounds__(NT) void interp_kernel(const double* __restrict__ pts2d,
                                                    const int64_t* __restrict__ perm2d,
                                                    NuProb q, int w, double beta,
                                                    const double2* __restrict__ G,
                                                    double2* __restrict__ f, int64_t ldf,
                                                    int nrhs) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < q.M * nrhs;
       e += (int64_t)gridDim.x * NT) {
    const int r = (int)(e / q.M);
    const int64_t s = q.m0 + (e - r * q.M);
    double wx[WMAX], wy[WMAX];
    const int lx0 = axis_weights(pts2d[2 * s], q.nfx, w, beta, wx);
    const int ly0 = axis_weights(pts2d[2 * s + 1], q.nfy, w, beta, wy);
    const double2* Gr = G + (int64_t)r * q.nfx * q.nfy;
    double ar = 0.0, ai = 0.0;
    for (int j = 0; j < w; ++j) {
      const int ly = (ly0 + j + q.nfy) & (q.nfy - 1);
      const double2* row = Gr + (int64_t)ly * q.nfx;
      double sr = 0.0, si = 0.0;
      for (int i = 0; i < w; ++i) {
        const int lx = (lx0 + i + q.nfx) & (q.nfx - 1);
        const double2 v = row[lx];
        sr += wx[i] * v.x;
        si += wx[i] * v.y;
      }
      ar += wy[j] * sr;
      ai += wy[j] * si;
    }
    f[r * ldf + perm2d[s]] = make_double2(ar, ai);
  }
}

// g[r][lx][ly] += f[r][perm[s]] phi(lx - nfx x_s) phi(ly - nfy y_s)
__global__ __launch_bounds__(NT) void spread_kernel(const double* __restrict__ pts2d,
                                                    const int64_t* __restrict__ perm2d,
                                                    NuProb q, int w, double beta,
                                                    const double2* __restrict__ f, int64_t ldf,
                                                    double2* __restrict__ g, int nrhs) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < q.M * nrhs;
       e += (int64_t)gridDim.x * NT) {
    const int r = (int)(e / q.M);
    const int64_t s = q.m0 + (e - r * q.M);
    double wx[WMAX], wy[WMAX];
    const int lx0 = axis_weights(pts2d[2 * s], q.nfx, w, beta, wx);
    const int ly0 = axis_weights(pts2d[2 * s + 1], q.nfy, w, beta, wy);
    const double2 v = f[r * ldf + perm2d[s]];
    double* gr = reinterpret_cast<double*>(g + (int64_t)r * q.nfx * q.nfy);
    for (int i = 0; i < w; ++i) {
      const int lx = (lx0 + i + q.nfx) & (q.nfx - 1);
      const double ax = wx[i] * v.x, ay = wx[i] * v.y;
      double* col = gr + 2 * (int64_t)lx * q.nfy;
      for (int j = 0; j < w; ++j) {
        const int ly = (ly0 + j + q.nfy) & (q.nfy - 1);
        atomic_addg(col + 2 * ly, wy[j] * ax);
        atomic_addg(col + 2 * ly + 1, wy[j] * ay);
      }
    }
  }
}

unsigned grid1(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, 8192));
}

int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on the three-term
// recurrence of the Legendre polynomials)
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& wt) {
  x.assign(q, 0.0);
  wt.assign(q, 0.0);
  const double pi = 3.141592653589793238462643383279502884;
  for (int i = 0; i < (q + 1) / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (q + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_q(z), p0 = P_{q-1}(z)
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= q; ++k) {
      const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = q * (z * p1 - p0) / (z * z - 1.0);
    x[i] = -z;
    x[q - 1 - i] = z;
    wt[i] = wt[q - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// 1 / phihat(k / nf) for the centred k = k' - n/2, k' < n
std::vector<double> deconv_factors(int n, int nf, int w, double beta) {
  std::vector<double> gx, gw;
  const int q = 4 * w + 40;
  gauss_legendre(q, gx, gw);
  const double hw = 0.5 * w, pi = 3.141592653589793238462643383279502884;
  std::vector<double> phi(q), t(q);
  for (int i = 0; i < q; ++i) {
    t[i] = hw * 0.5 * (gx[i] + 1.0);   // nodes on [0, w/2]
    const double u = t[i] / hw;
    phi[i] = std::exp(beta * (std::sqrt(std::max(0.0, 1.0 - u * u)) - 1.0)) * gw[i] * hw * 0.5;
  }
  std::vector<double> inv(n);
  for (int kk = 0; kk < n; ++kk) {
    const double xi = (double)(kk - n / 2) / (double)nf;
    double s = 0.0;
    for (int i = 0; i < q; ++i) s += phi[i] * std::cos(2.0 * pi * xi * t[i]);
    inv[kk] = 1.0 / (2.0 * s);
  }
  return inv;
}

// kernel width and shape for a relative tolerance (upsampling >= 2):
// w = ceil(log10(1/tol)) + 2 cells, beta = 2.30 w
void kernel_params(double tol, int& w, double& beta) {
  w = (int)std::ceil(std::log10(1.0 / tol)) + 2;
  w = std::max(4, std::min(WMAX, w));
  beta = 2.30 * w;
}

void setup(Plan* P, double tol, hipStream_t s) {
  NufftState& S = P->nufft;
  if (S.tol == tol && !S.probs.empty()) return;
  ND_CHECK(tol > 0.0 && tol < 1e-1, NUDFT2_E_INVAL, "NUFFT tolerance must lie in (0, 0.1)");
  ND_HIP(hipStreamSynchronize(s));
  for (auto& q : S.probs) {
    P->arena.release(q.invx);
    P->arena.release(q.invy);
  }
  S.probs.clear();
  S.tol = tol;
  kernel_params(tol, S.w, S.beta);
  for (const Problem& pb : P->probs) {
    NufftProb q;
    q.nfx = std::max(next_pow2(2 * pb.nx), next_pow2(2 * S.w));
    q.nfy = std::max(next_pow2(2 * pb.ny), next_pow2(2 * S.w));
    ND_CHECK(q.nfx <= FFT_MAX && q.nfy <= FFT_MAX, NUDFT2_E_INVAL,
             "the NUFFT handles nx, ny <= 1024");
    const std::vector<double> ix = deconv_factors(pb.nx, q.nfx, S.w, S.beta);
    const std::vector<double> iy = deconv_factors(pb.ny, q.nfy, S.w, S.beta);
    q.invx = (double*)P->arena.alloc(sizeof(double) * ix.size());
    q.invy = (double*)P->arena.alloc(sizeof(double) * iy.size());
    ND_HIP(hipMemcpyAsync(q.invx, ix.data(), sizeof(double) * ix.size(), hipMemcpyHostToDevice, s));
    ND_HIP(hipMemcpyAsync(q.invy, iy.data(), sizeof(double) * iy.size(), hipMemcpyHostToDevice, s));
    for (int n : {q.nfx, q.nfy}) {
      if (S.tw.count(n)) continue;
      double2* t = (double2*)P->arena.alloc(sizeof(double2) * (n / 2));
      hipLaunchKernelGGL(twiddle_kernel, dim3(grid1(n / 2)), dim3(NT), 0, s, t, n);
      S.tw[n] = t;
    }
    S.probs.push_back(q);
  }
  ND_HIP(hipGetLastError());
  ND_HIP(hipStreamSynchronize(s));
}

// the two fine-grid buffers for nrhs right-hand sides of the largest problem
void ensure_grids(Plan* P, int nrhs, hipStream_t s) {
  NufftState& S = P->nufft;
  size_t need = 0;
  for (auto& q : S.probs) need = std::max(need, sizeof(double2) * (size_t)q.nfx * q.nfy * nrhs);
  if (need <= S.gbytes) return;
  if (S.g1) {
    ND_HIP(hipStreamSynchronize(s));
    P->arena.release(S.g1);
    P->arena.release(S.g2);
  }
  S.g1 = S.g2 = nullptr;
  S.gbytes = 0;
  S.g1 = (double2*)P->arena.alloc(need);
  S.g2 = (double2*)P->arena.alloc(need);
  S.gbytes = need;
}

void fft_rows(double2* g, int n, int64_t rows, double sign, const double2* tw, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<int64_t>(rows, 2048);
  hipLaunchKernelGGL(fft_rows_kernel, dim3(blocks), dim3(NT), 0, s, g, n, rows, sign, tw);
}

void transpose(const double2* in, double2* out, int rows, int cols, int nb, hipStream_t s) {
  dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32), (unsigned)nb);
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, s, in, out, rows, cols);
}

}  // namespace

void nufft_fwd(Plan* P, const double2* c, double2* f, int nrhs, double tol, hipStream_t s) {
  setup(P, tol, s);
  ensure_grids(P, nrhs, s);
  NufftState& S = P->nufft;
  for (size_t p = 0; p < P->probs.size(); ++p) {
    const Problem& pb = P->probs[p];
    const NufftProb& q = S.probs[p];
    const int64_t gsz = (int64_t)q.nfx * q.nfy * nrhs;
    hipLaunchKernelGGL(zero2_kernel, dim3(grid1(gsz)), dim3(NT), 0, s, S.g1, gsz);
    hipLaunchKernelGGL(pad_kernel, dim3(grid1(pb.N() * nrhs)), dim3(NT), 0, s, c, P->Ntot, pb.c0,
                       pb.nx, pb.ny, q.invx, q.invy, S.g1, q.nfx, q.nfy, nrhs);
    fft_rows(S.g1, q.nfy, (int64_t)q.nfx * nrhs, -1.0, S.tw[q.nfy], s);
    transpose(S.g1, S.g2, q.nfx, q.nfy, nrhs, s);
    fft_rows(S.g2, q.nfx, (int64_t)q.nfy * nrhs, -1.0, S.tw[q.nfx], s);
    NuProb nq{pb.m0, pb.M, q.nfx, q.nfy};
    hipLaunchKernelGGL(interp_kernel, dim3(grid1(pb.M * nrhs)), dim3(NT), 0, s, P->pts_2d,
                       P->perm2d, nq, S.w, S.beta, S.g2, f, P->Mtot, nrhs);
  }
  ND_HIP(hipGetLastError());
}

void nufft_adj(Plan* P, const double2* f, double2* c, int nrhs, double tol, hipStream_t s) {
  setup(P, tol, s);
  ensure_grids(P, nrhs, s);
  NufftState& S = P->nufft;
  for (size_t p = 0; p < P->probs.size(); ++p) {
    const Problem& pb = P->probs[p];
    const NufftProb& q = S.probs[p];
    const int64_t gsz = (int64_t)q.nfx * q.nfy * nrhs;
    hipLaunchKernelGGL(zero2_kernel, dim3(grid1(gsz)), dim3(NT), 0, s, S.g1, gsz);
    NuProb nq{pb.m0, pb.M, q.nfx, q.nfy};
    hipLaunchKernelGGL(spread_kernel, dim3(grid1(pb.M * nrhs)), dim3(NT), 0, s, P->pts_2d,
                       P->perm2d, nq, S.w, S.beta, f, P->Mtot, S.g1, nrhs);
    fft_rows(S.g1, q.nfy, (int64_t)q.nfx * nrhs, 1.0, S.tw[q.nfy], s);
    transpose(S.g1, S.g2, q.nfx, q.nfy, nrhs, s);
    fft_rows(S.g2, q.nfx, (int64_t)q.nfy * nrhs, 1.0, S.tw[q.nfx], s);
    hipLaunchKernelGGL(crop_kernel, dim3(grid1(pb.N() * nrhs)), dim3(NT), 0, s, S.g2, q.nfx,
                       q.nfy, pb.nx, pb.ny, q.invx, q.invy, c, P->Ntot, pb.c0, nrhs);
  }
  ND_HIP(hipGetLastError());
}

void op_fwd(Plan* P, const double2* c, double2* f, int nrhs, hipStream_t s) {
  if (P->opts.nufft_tol > 0.0) nufft_fwd(P, c, f, nrhs, P->opts.nufft_tol, s);
  else apply_fwd(P, c, f, nrhs, s);
}

void op_adj(Plan* P, const double2* f, double2* c, int nrhs, hipStream_t s) {
  if (P->opts.nufft_tol > 0.0) nufft_adj(P, f, c, nrhs, P->opts.nufft_tol, s);
  else apply_adj(P, f, c, nrhs, s);
}

}  // namespace nd
