// Exact FP64 apply of the 2D type-II NUDFT matrix and of its adjoint.
//
// f_j = sum_{kx,ky} c[kx,ky] exp(-2 pi i (kx x_j + ky y_j))   (Section 1)
//
// Face-splitting form (A = A^x . A^y, Section 3.1): for a tile of rows j,
//   T(j, kx) = sum_ky A^y(j, ky) c[kx, ky]          (matrix-core GEMM, FP64)
//   f_j      = sum_kx A^x(j, kx) T(j, kx)          (row-wise dot, wave shuffles)
// A^x and A^y are generated on the fly: every entry is a product of a per-row
// base phase (one sincospi per 16 frequencies) and a per-row step table, each
// evaluated with exact phase reduction, so entries are accurate to ~2 ulp for
// any frequency.  The adjoint is the GEMM  C = (A^x)^H diag(f) conj(A^y),
// split over chunks of points: every (chunk, coefficient tile) workgroup
// stores its partial tile with plain stores, and a second kernel adds the
// chunks' partials in chunk order, so the result does not depend on the
// order in which workgroups run.
#include <mutex>
#include <string>

#include "device_util.h"
#include "plan.h"
#include "prof.h"

namespace nd {

namespace {

constexpr int TM = 64;    // rows (points) per workgroup
constexpr int TN = 64;    // kx per chunk
constexpr int TKY = 16;   // ky per shared-memory stage

__global__ __launch_bounds__(256, 2) void apply_fwd_kernel(
    const double* __restrict__ pts, const double2* __restrict__ c,
    double2* __restrict__ f, const ApplyProb* __restrict__ probs, int nprob,
    const int* __restrict__ tile_off, int64_t Mtot, int64_t Ntot) {
  __shared__ double2 E1y[TM][TKY + 1];
  __shared__ double2 E1x[TM][17];
  __shared__ double Cr[TKY][TN + 1], Ci[TKY][TN + 1], Cs[TKY][TN + 1];
  __shared__ double2 basey[TM];
  __shared__ double2 basex[TM][TN / 16];
  __shared__ double ptx[TM], pty[TM];

  const int tile = blockIdx.x;
  const int rhs = blockIdx.y;
  int lo = 0, hi = nprob;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (tile_off[mid] <= tile) lo = mid; else hi = mid;
  }
  const ApplyProb pr = probs[lo];
  const int64_t row0 = (int64_t)(tile - tile_off[lo]) * TM;
  const double2* cp = c + rhs * Ntot + pr.c0;
  double2* fp = f + rhs * Mtot + pr.m0;
  const int nx = pr.nx, ny = pr.ny;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  if (tid < TM) {
    int64_t r = row0 + tid;
    double x = 0.0, y = 0.0;
    if (r < pr.M) {
      x = pts[2 * (pr.m0 + r)];
      y = pts[2 * (pr.m0 + r) + 1];
    }
    ptx[tid] = x;
    pty[tid] = y;
  }
  __syncthreads();
  for (int e = tid; e < TM * 16; e += 256) {
    int r = e >> 4, t = e & 15;
    E1y[r][t] = expi_kx((double)t, pty[r]);
    E1x[r][t] = expi_kx((double)t, ptx[r]);
  }

  double facc[4] = {0.0, 0.0, 0.0, 0.0};
  double faci[4] = {0.0, 0.0, 0.0, 0.0};
  const int arow = wave * 16 + (lane & 15);   // A-operand row of this lane
  const int kq = lane >> 4;                   // k index within a 4-step

  for (int kx0 = 0; kx0 < nx; kx0 += TN) {
    // Gauss products: p1 = Ar Cr, p2 = Ai Ci, p3 = (Ar + Ai)(Cr + Ci);
    // Re = p1 - p2, Im = p3 - p1 - p2 (three matrix-core products, not four)
    dbl4 acc1[4], acc2[4], acc3[4];
    for (int t = 0; t < 4; ++t) {
      acc1[t] = dbl4{0, 0, 0, 0};
      acc2[t] = dbl4{0, 0, 0, 0};
      acc3[t] = dbl4{0, 0, 0, 0};
    }
    for (int ky0 = 0; ky0 < ny; ky0 += TKY) {
      __syncthreads();
      {
        int kxl = tid >> 2, part = tid & 3;
        int kx = kx0 + kxl;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          int t = part * 4 + u;
          int ky = ky0 + t;
          double2 v = mk<double>(0.0, 0.0);
          if (kx < nx && ky < ny) v = cp[(int64_t)kx * ny + ky];
          Cr[t][kxl] = v.x;
          Ci[t][kxl] = v.y;
          Cs[t][kxl] = v.x + v.y;
        }
      }
      if (tid < TM) basey[tid] = expi_kx((double)(ky0 - ny / 2), pty[tid]);
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        int t = kk * 4 + kq;
        double2 a = mk<double>(0.0, 0.0);
        if (ky0 + t < ny) a = cmul(basey[arow], E1y[arow][t]);
        const double as = a.x + a.y;
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
          const int kxl = tt * 16 + (lane & 15);
          acc1[tt] = mfma16(a.x, Cr[t][kxl], acc1[tt]);
          acc2[tt] = mfma16(a.y, Ci[t][kxl], acc2[tt]);
          acc3[tt] = mfma16(as, Cs[t][kxl], acc3[tt]);
        }
      }
    }
    // row-wise dot with A^x over this kx chunk
    __syncthreads();
    {
      int r = tid >> 2, tt = tid & 3;
      basex[r][tt] = expi_kx((double)(kx0 + tt * 16 - nx / 2), ptx[r]);
    }
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      int kxl = tt * 16 + (lane & 15);
      bool ok = (kx0 + kxl) < nx;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int r = wave * 16 + mrow<double>(lane, v);
        double2 ax = cmul(basex[r][tt], E1x[r][lane & 15]);
        const double p1 = acc1[tt][v], p2 = acc2[tt][v];
        const double tr = p1 - p2, ti = acc3[tt][v] - p1 - p2;
        if (ok) {
          facc[v] += ax.x * tr - ax.y * ti;
          faci[v] += ax.x * ti + ax.y * tr;
        }
      }
    }
  }
  // reduce over the 16 lanes that share a row group
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    for (int o = 1; o < 16; o <<= 1) {
      facc[v] += __shfl_xor(facc[v], o, 64);
      faci[v] += __shfl_xor(faci[v], o, 64);
    }
  }
  if ((lane & 15) == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int64_t r = row0 + wave * 16 + mrow<double>(lane, v);
      if (r < pr.M) fp[r] = mk<double>(facc[v], faci[v]);
    }
  }
}

constexpr int AT = 64;     // output tile (kx, ky)
constexpr int AK = 16;     // points per stage

// part[(chunk nrhs + rhs) Ntot + c0 + kx ny + ky] =
//     sum_{j in chunk} conj(Ax[j][kx]) f_j conj(Ay[j][ky])
// for the chunk of rows [blockIdx.y rows, (blockIdx.y + 1) rows); every entry
// of the problem's partial vector is stored by exactly one workgroup.
__global__ __launch_bounds__(256, 2) void apply_adj_kernel(
    const double* __restrict__ pts, const double2* __restrict__ f,
    double2* __restrict__ part, ApplyProb pr, int64_t Mtot, int64_t Ntot, int64_t rows,
    int nrhs) {
  __shared__ double Ar[AK][AT + 1], Ai[AK][AT + 1];
  __shared__ double Br[AK][AT + 1], Bi[AK][AT + 1];
  __shared__ double2 bx[AK][AT / 16], by[AK][AT / 16];
  __shared__ double2 sx[AK][16], sy[AK][16];
  __shared__ double2 fv[AK];

  const int ntx = (pr.nx + AT - 1) / AT;
  const int kx0 = (blockIdx.x % ntx) * AT;
  const int ky0 = (blockIdx.x / ntx) * AT;
  const int64_t j0 = (int64_t)blockIdx.y * rows;
  const int rhs = blockIdx.z;
  const double2* fp = f + rhs * Mtot + pr.m0;
  double2* cp = part + ((int64_t)blockIdx.y * nrhs + rhs) * Ntot + pr.c0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;   // wave's 32x32 sub-tile
  const int nx = pr.nx, ny = pr.ny;

  // Gauss products (three per complex multiply-add): p1 = Ar Br, p2 = Ai Bi,
  // p3 = (Ar + Ai)(Br + Bi); Re = p1 - p2, Im = p3 - p1 - p2
  dbl4 acc1[2][2], acc2[2][2], acc3[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      acc1[a][b] = dbl4{0, 0, 0, 0};
      acc2[a][b] = dbl4{0, 0, 0, 0};
      acc3[a][b] = dbl4{0, 0, 0, 0};
    }

  const int64_t jend = min((int64_t)pr.M, j0 + rows);
  for (int64_t js = j0; js < jend; js += AK) {
    __syncthreads();
    // per-point tables: conj phases (exp(+2 pi i k x)) as conj of expi
    {
      int p = tid >> 4, t = tid & 15;   // 16 points x 16 entries
      int64_t j = js + p;
      double x = 0, y = 0;
      bool ok = j < jend;
      if (ok) { x = pts[2 * (pr.m0 + j)]; y = pts[2 * (pr.m0 + j) + 1]; }
      sx[p][t] = expi_kx((double)t, x);
      sy[p][t] = expi_kx((double)t, y);
      if (t < AT / 16) {
        bx[p][t] = expi_kx((double)(kx0 + 16 * t - nx / 2), x);
        by[p][t] = expi_kx((double)(ky0 + 16 * t - ny / 2), y);
      }
      if (t == 0) fv[p] = ok ? fp[j] : mk<double>(0.0, 0.0);
    }
    __syncthreads();
    for (int e = tid; e < AK * AT; e += 256) {
      int p = e / AT, k = e % AT;
      double2 ex = cmul(bx[p][k >> 4], sx[p][k & 15]);   // exp(-2 pi i kx x)
      double2 ey = cmul(by[p][k >> 4], sy[p][k & 15]);
      double2 a = cmulc(ex, fv[p]);                        // conj(ex) f
      bool okx = kx0 + k < nx, oky = ky0 + k < ny;
      Ar[p][k] = okx ? a.x : 0.0;
      Ai[p][k] = okx ? a.y : 0.0;
      Br[p][k] = oky ? ey.x : 0.0;
      Bi[p][k] = oky ? -ey.y : 0.0;                        // conj(ey)
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      int p = kk * 4 + (lane >> 4);
      double ar[2], ai[2], br[2], bi[2];
      for (int a = 0; a < 2; ++a) {
        ar[a] = Ar[p][wm + a * 16 + (lane & 15)];
        ai[a] = Ai[p][wm + a * 16 + (lane & 15)];
        br[a] = Br[p][wn + a * 16 + (lane & 15)];
        bi[a] = Bi[p][wn + a * 16 + (lane & 15)];
      }
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          acc1[a][b] = mfma16(ar[a], br[b], acc1[a][b]);
          acc2[a][b] = mfma16(ai[a], bi[b], acc2[a][b]);
          acc3[a][b] = mfma16(ar[a] + ai[a], br[b] + bi[b], acc3[a][b]);
        }
    }
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int v = 0; v < 4; ++v) {
        int kx = kx0 + wm + a * 16 + mrow<double>(lane, v);
        int ky = ky0 + wn + b * 16 + (lane & 15);
        if (kx < nx && ky < ny) {
          const double p1 = acc1[a][b][v], p2 = acc2[a][b][v];
          cp[(int64_t)kx * ny + ky] = mk<double>(p1 - p2, acc3[a][b][v] - p1 - p2);
        }
      }
}

// c[rhs][c0 + i] = sum over chunks, in chunk order, of the partials
__global__ void adj_reduce_kernel(const double2* __restrict__ part, double2* __restrict__ c,
                                  ApplyProb pr, int nch, int64_t Ntot, int nrhs) {
  const int64_t n = (int64_t)pr.nx * pr.ny;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / n);
    const int64_t i = pr.c0 + e % n;
    double sr = 0.0, si = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
      const double2 v = part[((int64_t)ch * nrhs + r) * Ntot + i];
      sr += v.x;
      si += v.y;
    }
    c[(int64_t)r * Ntot + i] = mk<double>(sr, si);
  }
}

constexpr int64_t ADJ_MIN_ROWS = 2048;   // rows per chunk, at least
constexpr int64_t ADJ_WG_TARGET = 2048;  // workgroups per problem launch wanted

// Row chunks of the adjoint apply for a plan: as many as fill the device
// (about ADJ_WG_TARGET workgroups per problem) but no more than the partial
// buffer of cap bytes holds; 0 when not even one chunk fits.
int adj_chunks(const Plan* P, int nrhs, size_t cap) {
  int64_t want = 1;
  for (const Problem& q : P->probs) {
    const int64_t tiles = (int64_t)ceil_div(q.nx, AT) * ceil_div(q.ny, AT);
    const int64_t by_rows = std::max<int64_t>(1, (q.M + ADJ_MIN_ROWS - 1) / ADJ_MIN_ROWS);
    want = std::max(want, std::min(by_rows, (ADJ_WG_TARGET + tiles - 1) / tiles));
  }
  const size_t per_chunk = sizeof(double2) * (size_t)P->Ntot * (size_t)nrhs;
  const int64_t fit = per_chunk ? (int64_t)(cap / per_chunk) : want;
  return (int)std::min<int64_t>(want, fit);
}

// the adjoint apply with its partials in part (nch chunks, see adj_chunks)
void apply_adj_into(Plan* P, const double2* f, double2* c, int nrhs, double2* part, int nch,
                    hipStream_t s) {
  for (const Problem& q : P->probs) {
    ApplyProb pr{q.m0, q.M, q.c0, q.nx, q.ny};
    const int tiles = ceil_div(q.nx, AT) * ceil_div(q.ny, AT);
    // rows per chunk: a multiple of the stage height, nch chunks cover M
    int64_t rows = std::max<int64_t>(AK, (q.M + nch - 1) / nch);
    rows = (rows + AK - 1) / AK * AK;
    const int nchp = std::max(1, ceil_div(q.M, rows));
    dim3 grid(tiles, nchp, nrhs);
    hipLaunchKernelGGL(apply_adj_kernel, grid, dim3(256), 0, s, P->pts_user, f, part, pr,
                       P->Mtot, P->Ntot, rows, nrhs);
    const int64_t n = q.N() * nrhs;
    hipLaunchKernelGGL(adj_reduce_kernel,
                       dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (n + 255) / 256))),
                       dim3(256), 0, s, part, c, pr, nchp, P->Ntot, nrhs);
  }
  ND_HIP(hipGetLastError());
}

}  // namespace

void apply_fwd(Plan* P, const double2* c, double2* f, int nrhs, hipStream_t s) {
  dim3 grid(P->apply_tiles, nrhs);
  double fl = 0;
  for (auto& q : P->probs) fl += 8.0 * (double)q.M * (double)q.N() * nrhs;
  ProfScope ps(s, KC_APPLY, fl);
  hipLaunchKernelGGL(apply_fwd_kernel, grid, dim3(256), 0, s, P->pts_user, c, f,
                     P->d_aprob, (int)P->probs.size(), P->d_tile_off, P->Mtot,
                     P->Ntot);
  ND_HIP(hipGetLastError());
}

// ------------------------------------------------ no-allocation variant
// The adjoint apply for callers that cannot allocate device memory keeps its
// partial sums in this file-scope array.  Its name is only a host-side stand
// -in: the device address comes from hipGetSymbolAddress, looked up once per
// device with that device current and kept in scratch_addr.  Every call on a
// device shares that device's array, so calls that overlap on one device
// race; nothing in it needs to start at zero (every partial is stored before
// it is read).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) double2 scratch[NOALLOC_SCRATCH_BYTES / sizeof(double2)];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[MAX_DEVICES] = {};

// device address of this device's scratch (the current device must be dev)
double2* scratch_addr(int dev) {
  ND_CHECK(dev >= 0 && dev < MAX_DEVICES, NUDFT2_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      throw Error(NUDFT2_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                       hipGetErrorString(e));
    }
    g_scratch_addr[dev] = ptr;
  }
  return (double2*)g_scratch_addr[dev];
}
}  // namespace

void apply_adj_noalloc(Plan* P, const double2* f, double2* c, int nrhs) {
  const int nch = adj_chunks(P, nrhs, NOALLOC_SCRATCH_BYTES);
  ND_CHECK(nch >= 1, NUDFT2_E_INVAL,
           "nrhs * N * 16 bytes exceeds the 64 MiB scratch of the no-allocation adjoint");
  int cur = -1;
  ND_HIP(hipGetDevice(&cur));
  const bool switch_dev = cur != P->device;
  if (switch_dev) ND_HIP(hipSetDevice(P->device));
  try {
    apply_adj_into(P, f, c, nrhs, scratch_addr(P->device), nch, P->stream);
  } catch (...) {
    if (switch_dev) (void)hipSetDevice(cur);
    throw;
  }
  if (switch_dev) ND_HIP(hipSetDevice(cur));
}

// Partial buffer of the library path: at most 256 MiB (n = 512: 32 chunks of
// 4 MiB per right-hand side), held by the plan and grown on demand.
constexpr size_t ADJ_PART_CAP = size_t(256) << 20;

void apply_adj(Plan* P, const double2* f, double2* c, int nrhs, hipStream_t s) {
  const int nch = std::max(1, adj_chunks(P, nrhs, ADJ_PART_CAP));
  const size_t need = sizeof(double2) * (size_t)P->Ntot * (size_t)nrhs * (size_t)nch;
  if (need > P->adj_part_bytes) {
    if (P->adj_part) {
      ND_HIP(hipStreamSynchronize(s));   // earlier launches may still read it
      P->arena.release(P->adj_part);
    }
    P->adj_part = nullptr;
    P->adj_part_bytes = 0;
    P->adj_part = (double2*)P->arena.alloc(need);
    P->adj_part_bytes = need;
  }
  apply_adj_into(P, f, c, nrhs, P->adj_part, nch, s);
}

}  // namespace nd
