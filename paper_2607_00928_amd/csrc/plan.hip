// Plan construction: validation, point binning (quadtree and 1D trees) and
// upload.  Binning is host code: the caller's points (device memory) are
// copied to the host once, binned by counting sorts, and uploaded in tree
// order.
//
// Trees (Definitions 2.1 and 3.2): both 1D trees bisect [0, 1) dyadically to
// a common depth L = ceil(log2(max(nx, ny) / leaf)); node (l, a) of the x tree
// owns the points with floor(x 2^l) = a and the columns l' with
// floor(l' 2^l / nx) = a (half-open intervals).  The 2D tree is their
// face-splitting product: node (l, a, b) owns the points in the box and the
// columns K^x_a x K^y_b.  Points are sorted by the Morton code of their leaf
// box so that every quadtree node owns a contiguous range of rows, and the
// columns of every node are contiguous in the "quadtree column order"
// (children concatenated in (p, q) order, each leaf kx-major).
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <thread>

#include "hss.h"
#include "plan.h"

namespace nd {

namespace {
constexpr size_t GUARD = 4096;
constexpr unsigned char GUARD_BYTE = 0xA5;
constexpr size_t SLAB = size_t(1) << 30;
bool env_on(const char* name) {
  const char* e = std::getenv(name);
  return e && e[0] == '1';
}
bool guard_on() {
  static const bool on = env_on("NUDFT2_GUARD");
  return on;
}
bool poison_on() {
  static const bool on = env_on("NUDFT2_POISON");
  return on;
}
bool quarantine_on() {
  static const bool on = env_on("NUDFT2_QUARANTINE");
  return on;
}
// first overwritten guard byte after n bytes of the block, or -1
int64_t guard_bad(const void* p, size_t n) {
  std::vector<unsigned char> h(GUARD);
  ND_HIP(hipDeviceSynchronize());
  ND_HIP(hipMemcpy(h.data(), (const char*)p + n, GUARD, hipMemcpyDeviceToHost));
  for (size_t i = 0; i < GUARD; ++i)
    if (h[i] != GUARD_BYTE) return (int64_t)i;
  return -1;
}
std::vector<std::pair<void*, size_t>> g_quarantine;
}  // namespace

void Arena::take_free(std::map<uintptr_t, size_t>::iterator it) {
  auto range = free_by_size.equal_range(it->second);
  for (auto j = range.first; j != range.second; ++j)
    if (j->second == it->first) {
      free_by_size.erase(j);
      break;
    }
  free_by_addr.erase(it);
}

void Arena::add_free(uintptr_t a, size_t n) {
  // coalesce with the neighbours inside the same slab
  auto next = free_by_addr.find(a + n);
  if (next != free_by_addr.end() && !slab_start.count(a + n)) {
    n += next->second;
    take_free(next);
  }
  auto it = free_by_addr.lower_bound(a);
  if (it != free_by_addr.begin() && !slab_start.count(a)) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == a) {
      a = prev->first;
      n += prev->second;
      take_free(prev);
    }
  }
  free_by_addr[a] = n;
  free_by_size.insert({n, a});
}

void* Arena::alloc(size_t n) {
  if (n == 0) n = 1;
  n = (n + 255) & ~size_t(255);
  const size_t span = n + (guard_on() ? GUARD : 0);
  auto fit = free_by_size.lower_bound(span);
  uintptr_t a = 0;
  if (fit != free_by_size.end()) {
    a = fit->second;
    size_t have = fit->first;
    take_free(free_by_addr.find(a));
    if (have > span) add_free(a + span, have - span);
  } else {
    size_t want = std::max(span, SLAB);
    if (cap && reserved + want > cap) want = span;
    if (cap && reserved + want > cap)
      throw Error(NUDFT2_E_NOMEM, "plan memory cap exceeded");
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess && want > span) {
      (void)hipGetLastError();
      want = span;
      e = hipMalloc(&p, want);
    }
    if (e != hipSuccess && trim() > 0) {
      // slabs left entirely free (fragmentation of earlier phases) went back
      // to the device: try once more
      (void)hipGetLastError();
      e = hipMalloc(&p, want);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(NUDFT2_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    slabs.push_back({p, want});
    slab_start.insert((uintptr_t)p);
    reserved += want;
    a = (uintptr_t)p;
    if (want > span) add_free(a + span, want - span);
  }
  void* p = (void*)a;
  if (poison_on()) ND_HIP(hipMemset(p, 0xFF, n));   // debug: NaN everywhere until written
  if (guard_on()) ND_HIP(hipMemset((char*)p + n, GUARD_BYTE, GUARD));
  live[a] = {n, span};
  bytes += n;
  peak = std::max(peak, bytes);
  return p;
}

size_t Arena::trim() {
  // Blocks are released once their last use is ordered on the plan's stream;
  // wait for the device before handing slabs back.
  if (hipDeviceSynchronize() != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  size_t freed = 0;
  for (size_t i = 0; i < slabs.size();) {
    const uintptr_t a = (uintptr_t)slabs[i].first;
    const size_t n = slabs[i].second;
    auto it = free_by_addr.find(a);
    if (it != free_by_addr.end() && it->second == n) {
      take_free(it);
      slab_start.erase(a);
      (void)hipFree(slabs[i].first);
      reserved -= n;
      freed += n;
      slabs.erase(slabs.begin() + i);
    } else {
      ++i;
    }
  }
  return freed;
}

size_t Arena::block_size(const void* p) const {
  auto it = live.find((uintptr_t)p);
  return it == live.end() ? 0 : it->second.first;
}

void Arena::release(void* p) {
  if (!p) return;
  auto it = live.find((uintptr_t)p);
  if (it == live.end()) return;
  const size_t n = it->second.first, span = it->second.second;
  if (guard_on() && guard_bad(p, n) >= 0)
    std::fprintf(stderr, "nudft2: write past the end of a released block of %zu bytes\n", n);
  live.erase(it);
  bytes -= n;
  if (quarantine_on()) {
    ND_HIP(hipDeviceSynchronize());
    ND_HIP(hipMemset(p, 0xFF, n));
    g_quarantine.push_back({p, n});
    return;
  }
  add_free((uintptr_t)p, span);
}

void Arena::check(const char* where) {
  // NUDFT2_MEM_LOG=1: the arena's live, peak and reserved bytes at each check
  static const bool mem_log = env_on("NUDFT2_MEM_LOG");
  if (mem_log)
    std::fprintf(stderr, "[nudft2 mem] %-28s live %8.2f GB  peak %8.2f GB  reserved %8.2f GB\n",
                 where, bytes / 1e9, peak / 1e9, reserved / 1e9);
  if (quarantine_on()) {
    ND_HIP(hipDeviceSynchronize());
    for (auto& q : g_quarantine) {
      std::vector<unsigned char> h(q.second);
      ND_HIP(hipMemcpy(h.data(), q.first, q.second, hipMemcpyDeviceToHost));
      size_t bad = 0;
      for (unsigned char c : h) bad += c != 0xFF;
      if (bad)
        throw Error(NUDFT2_E_INTERNAL, "write into a released block (" + std::to_string(q.second) +
                                           " bytes) detected at " + where);
    }
  }
  if (!guard_on()) return;
  for (auto& b : live) {
    int64_t off = guard_bad((const void*)b.first, b.second.first);
    if (off >= 0)
      throw Error(NUDFT2_E_INTERNAL, std::string("write past the end of a device block (") +
                                         std::to_string(b.second.first) + " bytes, guard offset " +
                                         std::to_string(off) + ") detected at " + where);
  }
}

void Arena::release_all() {
  for (auto& s : slabs) (void)hipFree(s.first);
  slabs.clear();
  slab_start.clear();
  free_by_addr.clear();
  free_by_size.clear();
  live.clear();
  bytes = 0;
  reserved = 0;
}

Plan::~Plan() {
  hss.reset();
  arena.release_all();
}

int tree_depth(int nx, int ny, int leaf) {
  int L = 0;
  while ((int64_t)std::max(nx, ny) > (int64_t)leaf << L) ++L;
  return L;
}

static inline double wrap01(double v) {
  double w = v - std::floor(v);
  if (w >= 1.0) w -= 1.0;
  return w;
}

// f(begin, end, t) over contiguous chunks [begin, end) of [0, n) on up to
// 16 host threads (chunk t before chunk t + 1), serially for small n
template <class F>
static void par_chunks(int64_t n, int nt, F&& f) {
  if (nt <= 1) {
    f((int64_t)0, n, 0);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(nt);
  for (int t = 0; t < nt; ++t) th.emplace_back(f, n * t / nt, n * (t + 1) / nt, t);
  for (auto& x : th) x.join();
}

static int host_threads(int64_t n) {
  if (n < (int64_t)1 << 16) return 1;
  const unsigned hc = std::thread::hardware_concurrency();
  return (int)std::max<unsigned>(1, std::min<unsigned>(hc ? hc : 1, 16));
}

// Stable counting sort of 0 .. n-1 by key(j) in [0, nbins): ord receives the
// indices in key order (ties in index order), cnt (nbins + 1) the prefix
// counts.  Per-thread histograms of contiguous index chunks, then each chunk
// scatters from its own offsets, so the result equals the serial sort.
template <class K>
static void counting_sort(int64_t n, int nbins, K key, std::vector<int64_t>& ord,
                          std::vector<int64_t>& cnt) {
  const int nt = host_threads(n);
  std::vector<std::vector<int64_t>> h(nt, std::vector<int64_t>(nbins, 0));
  par_chunks(n, nt, [&](int64_t a, int64_t b, int t) {
    for (int64_t j = a; j < b; ++j) h[t][key(j)]++;
  });
  cnt.assign(nbins + 1, 0);
  for (int k = 0; k < nbins; ++k) {
    int64_t s = 0;
    for (int t = 0; t < nt; ++t) s += h[t][k];
    cnt[k + 1] = cnt[k] + s;
  }
  // chunk t's first slot in bin k: the bin start plus the earlier chunks'
  for (int k = 0; k < nbins; ++k) {
    int64_t o = cnt[k];
    for (int t = 0; t < nt; ++t) {
      const int64_t c = h[t][k];
      h[t][k] = o;
      o += c;
    }
  }
  ord.resize(n);
  par_chunks(n, nt, [&](int64_t a, int64_t b, int t) {
    for (int64_t j = a; j < b; ++j) ord[h[t][key(j)]++] = j;
  });
}

static inline int bin_of(double v, int level) {
  int b = (int)std::floor(v * (double)(1 << level));
  return std::min(std::max(b, 0), (1 << level) - 1);
}

// Host part of the plan: fills the trees and the orderings (host arrays).
struct HostOrder {
  std::vector<double> pts_user, pts_2d, xs, ys;
  std::vector<int64_t> perm2d, posx, posy, colperm;
};

static void bin_problem(Problem& q, const double* pts, int leaf, HostOrder& H) {
  const int L = q.L;
  const int64_t M = q.M, m0 = q.m0;
  const int nleaf1 = 1 << L;
  const int nleaf2 = 1 << (2 * L);
  std::vector<int> bx(M), by(M);
  std::vector<uint32_t> z(M);
  const int nt = host_threads(M);
  par_chunks(M, nt, [&](int64_t a, int64_t b, int) {
    for (int64_t j = a; j < b; ++j) {
      double x = wrap01(pts[2 * (m0 + j)]), y = wrap01(pts[2 * (m0 + j) + 1]);
      H.pts_user[2 * (m0 + j)] = x;
      H.pts_user[2 * (m0 + j) + 1] = y;
      bx[j] = bin_of(x, L);
      by[j] = bin_of(y, L);
      z[j] = interleave(bx[j], by[j], L);
    }
  });
  // columns of the 1D trees
  q.colx.assign(L + 1, {});
  q.coly.assign(L + 1, {});
  for (int l = 0; l <= L; ++l) {
    int na = 1 << l;
    q.colx[l].resize(na + 1);
    q.coly[l].resize(na + 1);
    for (int a = 0; a <= na; ++a) {
      q.colx[l][a] = (int)(((int64_t)a * q.nx + na - 1) / na);
      q.coly[l][a] = (int)(((int64_t)a * q.ny + na - 1) / na);
    }
  }
  // 2D order: stable counting sort by leaf Morton code
  std::vector<int64_t> cnt2, ord2;
  counting_sort(M, nleaf2, [&](int64_t j) { return (int)z[j]; }, ord2, cnt2);
  q.row2.assign(L + 1, {});
  for (int l = 0; l <= L; ++l) {
    int nn = 1 << (2 * l);
    q.row2[l].resize(nn + 1);
    int sh = 2 * (L - l);
    for (int zz = 0; zz <= nn; ++zz) q.row2[l][zz] = m0 + cnt2[(int64_t)zz << sh];
  }
  // 1D orders
  auto sort1d = [&](const std::vector<int>& b, std::vector<int64_t>& ord,
                    std::vector<std::vector<int64_t>>& rows) {
    std::vector<int64_t> cnt;
    counting_sort(M, nleaf1, [&](int64_t j) { return b[j]; }, ord, cnt);
    rows.assign(L + 1, {});
    for (int l = 0; l <= L; ++l) {
      int na = 1 << l;
      rows[l].resize(na + 1);
      for (int a = 0; a <= na; ++a) rows[l][a] = m0 + cnt[(int64_t)a << (L - l)];
    }
  };
  std::vector<int64_t> ordx, ordy;
  sort1d(bx, ordx, q.rowx);
  sort1d(by, ordy, q.rowy);
  std::vector<int64_t> invx(M), invy(M);
  par_chunks(M, nt, [&](int64_t a, int64_t b, int) {
    for (int64_t i = a; i < b; ++i) {
      invx[ordx[i]] = i;
      invy[ordy[i]] = i;
    }
  });
  par_chunks(M, nt, [&](int64_t a, int64_t b, int) {
    for (int64_t i = a; i < b; ++i) {
      int64_t j = ord2[i];
      H.perm2d[m0 + i] = m0 + j;
      H.pts_2d[2 * (m0 + i)] = H.pts_user[2 * (m0 + j)];
      H.pts_2d[2 * (m0 + i) + 1] = H.pts_user[2 * (m0 + j) + 1];
      H.posx[m0 + i] = m0 + invx[j];
      H.posy[m0 + i] = m0 + invy[j];
      H.xs[m0 + i] = H.pts_user[2 * (m0 + ordx[i])];
      H.ys[m0 + i] = H.pts_user[2 * (m0 + ordy[i]) + 1];
    }
  });
  // quadtree column order
  q.col2.assign(L + 1, {});
  for (int l = 0; l <= L; ++l) {
    int nn = 1 << (2 * l);
    q.col2[l].resize(nn + 1);
    q.col2[l][0] = 0;
    for (int zz = 0; zz < nn; ++zz) {
      uint32_t a, b;
      deinterleave(zz, l, a, b);
      int d = (q.colx[l][a + 1] - q.colx[l][a]) * (q.coly[l][b + 1] - q.coly[l][b]);
      q.col2[l][zz + 1] = q.col2[l][zz] + d;
    }
  }
  for (int zz = 0; zz < nleaf2; ++zz) {
    uint32_t a, b;
    deinterleave(zz, L, a, b);
    int x0 = q.colx[L][a], x1 = q.colx[L][a + 1];
    int y0 = q.coly[L][b], y1 = q.coly[L][b + 1];
    int64_t o = q.c0 + q.col2[L][zz];
    for (int i = x0; i < x1; ++i)
      for (int j = y0; j < y1; ++j) H.colperm[o++] = q.c0 + (int64_t)i * q.ny + j;
  }
}

static void validate(int nprob, const double* points, const int64_t* m_off,
                     const int32_t* nx, const int32_t* ny, const nudft2_opts* o) {
  ND_CHECK(nprob >= 1, NUDFT2_E_INVAL, "nprob must be >= 1");
  ND_CHECK(points && m_off && nx && ny, NUDFT2_E_INVAL, "null pointer argument");
  for (int p = 0; p < nprob; ++p)
    ND_CHECK(m_off[p + 1] >= m_off[p], NUDFT2_E_INVAL, "m_off must be non-decreasing");
  ND_CHECK(m_off[0] == 0, NUDFT2_E_INVAL, "m_off[0] must be 0");
  ND_CHECK(o != nullptr, NUDFT2_E_INVAL, "null options");
  ND_CHECK(o->precision == 0 || o->precision == 1, NUDFT2_E_INVAL, "precision must be 0 or 1");
  ND_CHECK(o->eps > 0.0 && o->eps < 1.0, NUDFT2_E_INVAL, "eps must lie in (0, 1)");
  ND_CHECK(o->leaf >= 2 && o->leaf <= 64, NUDFT2_E_INVAL, "leaf must lie in [2, 64]");
  ND_CHECK(o->ir_maxit >= 0, NUDFT2_E_INVAL, "ir_maxit must be >= 0");
  ND_CHECK(o->ir_tol >= 0.0, NUDFT2_E_INVAL, "ir_tol must be >= 0");
  ND_CHECK(o->refine >= 0 && o->refine <= 2, NUDFT2_E_INVAL, "refine must be 0, 1 or 2");
  ND_CHECK(o->graph == 0 || o->graph == 1, NUDFT2_E_INVAL, "graph must be 0 or 1");
  ND_CHECK(o->fp32_products == 0 || o->fp32_products == 1, NUDFT2_E_INVAL,
           "fp32_products must be 0 or 1");
  ND_CHECK(o->fadi_1d == 0 || o->fadi_1d == 1, NUDFT2_E_INVAL, "fadi_1d must be 0 or 1");
  ND_CHECK(o->nufft_tol == 0.0 || (o->nufft_tol > 0.0 && o->nufft_tol < 0.1), NUDFT2_E_INVAL,
           "nufft_tol must be 0 or lie in (0, 0.1)");
  if (o->nufft_tol > 0.0)
    for (int p = 0; p < nprob; ++p)
      ND_CHECK(nx[p] <= 1024 && ny[p] <= 1024, NUDFT2_E_INVAL,
               "the NUFFT operator needs nx, ny <= 1024");
  for (int p = 0; p < nprob; ++p) {
    ND_CHECK(nx[p] >= 2 && ny[p] >= 2 && nx[p] % 2 == 0 && ny[p] % 2 == 0,
             NUDFT2_E_INVAL, "nx, ny must be even and >= 2");
    ND_CHECK(nx[p] <= 4096 && ny[p] <= 4096, NUDFT2_E_INVAL, "nx, ny must be <= 4096");
    int64_t M = m_off[p + 1] - m_off[p];
    ND_CHECK(M >= (int64_t)nx[p] * ny[p], NUDFT2_E_INVAL, "need M >= nx*ny points");
    int L = tree_depth(nx[p], ny[p], o->leaf);
    ND_CHECK(L <= 10, NUDFT2_E_INVAL, "tree too deep (nx/leaf > 1024)");
  }
}

static double now_ms_plan() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// points_dev: the caller's points (device memory; the copy direction is
// taken from the address, so host memory works as well).  They are copied
// to the host once for the O(M) integer binning, then uploaded in tree order.
Plan* make_plan(int nprob, const double* points_dev, const int64_t* m_off,
                const int32_t* nx, const int32_t* ny, const nudft2_opts* opts) {
  const double t0 = now_ms_plan();
  validate(nprob, points_dev, m_off, nx, ny, opts);
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    throw Error(NUDFT2_E_DEVICE, "no HIP device available");
  }
  const int64_t Mt = m_off[nprob];
  std::vector<double> host_pts((size_t)2 * Mt);
  if (Mt > 0) {
    ND_HIP(hipMemcpyAsync(host_pts.data(), points_dev, sizeof(double) * 2 * Mt, hipMemcpyDefault,
                          (hipStream_t)opts->stream));
    ND_HIP(hipStreamSynchronize((hipStream_t)opts->stream));
  }
  const double* points = host_pts.data();
  for (int64_t j = 0; j < 2 * Mt; ++j)
    ND_CHECK(std::isfinite(points[j]), NUDFT2_E_INVAL, "non-finite point coordinate");
  std::unique_ptr<Plan> P(new Plan());
  P->opts = *opts;
  P->stream = (hipStream_t)opts->stream;
  P->arena.cap = opts->mem_cap;
  ND_HIP(hipGetDevice(&P->device));
  P->Mtot = m_off[nprob];
  P->probs.resize(nprob);
  int64_t c0 = 0;
  for (int p = 0; p < nprob; ++p) {
    Problem& q = P->probs[p];
    q.nx = nx[p];
    q.ny = ny[p];
    q.m0 = m_off[p];
    q.M = m_off[p + 1] - m_off[p];
    q.c0 = c0;
    q.L = tree_depth(q.nx, q.ny, opts->leaf);
    c0 += q.N();
    P->Lmax = std::max(P->Lmax, q.L);
  }
  P->Ntot = c0;
  HostOrder H;
  H.pts_user.resize(2 * P->Mtot);
  H.pts_2d.resize(2 * P->Mtot);
  H.xs.resize(P->Mtot);
  H.ys.resize(P->Mtot);
  H.perm2d.resize(P->Mtot);
  H.posx.resize(P->Mtot);
  H.posy.resize(P->Mtot);
  H.colperm.resize(P->Ntot);
  for (auto& q : P->probs) bin_problem(q, points, opts->leaf, H);

  Arena& A = P->arena;
  P->pts_user = (double*)A.alloc(sizeof(double) * 2 * P->Mtot);
  P->pts_2d = (double*)A.alloc(sizeof(double) * 2 * P->Mtot);
  P->perm2d = (int64_t*)A.alloc(sizeof(int64_t) * P->Mtot);
  P->xs = (double*)A.alloc(sizeof(double) * P->Mtot);
  P->ys = (double*)A.alloc(sizeof(double) * P->Mtot);
  P->posx = (int64_t*)A.alloc(sizeof(int64_t) * P->Mtot);
  P->posy = (int64_t*)A.alloc(sizeof(int64_t) * P->Mtot);
  P->colperm = (int64_t*)A.alloc(sizeof(int64_t) * P->Ntot);
  hipStream_t s = P->stream;
  ND_HIP(hipMemcpyAsync(P->pts_user, H.pts_user.data(), sizeof(double) * 2 * P->Mtot, hipMemcpyHostToDevice, s));
  ND_HIP(hipMemcpyAsync(P->pts_2d, H.pts_2d.data(), sizeof(double) * 2 * P->Mtot, hipMemcpyHostToDevice, s));
  ND_HIP(hipMemcpyAsync(P->perm2d, H.perm2d.data(), sizeof(int64_t) * P->Mtot, hipMemcpyHostToDevice, s));
  ND_HIP(hipMemcpyAsync(P->xs, H.xs.data(), sizeof(double) * P->Mtot, hipMemcpyHostToDevice, s));
  ND_HIP(hipMemcpyAsync(P->ys, H.ys.data(), sizeof(double) * P->Mtot, hipMemcpyHostToDevice, s));
  ND_HIP(hipMemcpyAsync(P->posx, H.posx.data(), sizeof(int64_t) * P->Mtot, hipMemcpyHostToDevice, s));
  ND_HIP(hipMemcpyAsync(P->posy, H.posy.data(), sizeof(int64_t) * P->Mtot, hipMemcpyHostToDevice, s));
  ND_HIP(hipMemcpyAsync(P->colperm, H.colperm.data(), sizeof(int64_t) * P->Ntot, hipMemcpyHostToDevice, s));

  std::vector<ApplyProb> ap(nprob);
  std::vector<int> toff(nprob + 1, 0);
  for (int p = 0; p < nprob; ++p) {
    const Problem& q = P->probs[p];
    ap[p] = ApplyProb{q.m0, q.M, q.c0, q.nx, q.ny};
    toff[p + 1] = toff[p] + ceil_div(q.M, 64);
  }
  P->apply_tiles = toff[nprob];
  P->d_aprob = (ApplyProb*)A.alloc(sizeof(ApplyProb) * nprob);
  P->d_tile_off = (int*)A.alloc(sizeof(int) * (nprob + 1));
  ND_HIP(hipMemcpyAsync(P->d_aprob, ap.data(), sizeof(ApplyProb) * nprob, hipMemcpyHostToDevice, s));
  ND_HIP(hipMemcpyAsync(P->d_tile_off, toff.data(), sizeof(int) * (nprob + 1), hipMemcpyHostToDevice, s));
  ND_HIP(hipStreamSynchronize(s));
  P->info.nprob = nprob;
  P->info.levels = P->Lmax;
  P->info.t_plan_ms = now_ms_plan() - t0;
  return P.release();
}

// Host-only binning used by the test hooks: returns the 2D order (caller
// indices), leaf row offsets (4^L + 1) and the quadtree column permutation.
void host_binning(const double* points, int64_t M, int nx, int ny, int leaf,
                  int64_t* perm2d, int64_t* leaf_rows, int64_t* colperm) {
  Problem q;
  q.nx = nx;
  q.ny = ny;
  q.M = M;
  q.L = tree_depth(nx, ny, leaf);
  HostOrder H;
  H.pts_user.resize(2 * M);
  H.pts_2d.resize(2 * M);
  H.xs.resize(M);
  H.ys.resize(M);
  H.perm2d.resize(M);
  H.posx.resize(M);
  H.posy.resize(M);
  H.colperm.resize(q.N());
  bin_problem(q, points, leaf, H);
  std::copy(H.perm2d.begin(), H.perm2d.end(), perm2d);
  std::copy(q.row2[q.L].begin(), q.row2[q.L].end(), leaf_rows);
  std::copy(H.colperm.begin(), H.colperm.end(), colperm);
}

}  // namespace nd
