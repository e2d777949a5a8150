// C-ABI entry points: argument checks, error mapping, dispatch.
#include <cstring>
#include <mutex>

#include "../../include/nudft2_testing.h"
#include "device_util.h"
#include "gen.h"
#include "hss.h"
#include "la.h"
#include "plan.h"
#include "solver.h"

namespace nd {

static thread_local std::string g_last_error;
thread_local Profiler* g_prof = nullptr;
thread_local int g_prof_site = PS_NONE;

namespace {
std::mutex g_ev_mu;
std::vector<std::vector<hipEvent_t>> g_ev_cache;   // per device; kept until the process ends
}  // namespace

hipEvent_t event_cache_get(int dev) {
  {
    std::lock_guard<std::mutex> lk(g_ev_mu);
    if (dev >= 0 && (size_t)dev < g_ev_cache.size() && !g_ev_cache[dev].empty()) {
      hipEvent_t e = g_ev_cache[dev].back();
      g_ev_cache[dev].pop_back();
      return e;
    }
  }
  hipEvent_t e;
  ND_HIP(hipEventCreate(&e));
  return e;
}

void event_cache_put(int dev, hipEvent_t e) {
  if (!e || dev < 0) return;
  std::lock_guard<std::mutex> lk(g_ev_mu);
  if ((size_t)dev >= g_ev_cache.size()) g_ev_cache.resize(dev + 1);
  g_ev_cache[dev].push_back(e);
}

// Routes kernel timing of the calling thread to the plan's profiler, and
// its FP32 products to the plan's kind, while an entry point runs.
struct PlanProf {
  Profiler* saved;
  bool split;
  explicit PlanProf(Plan* P) : saved(g_prof), split(g_fp32_split) {
    g_prof = P->profiling ? &P->prof : nullptr;
    g_fp32_split = P->opts.fp32_products == 0;
  }
  ~PlanProf() {
    g_prof = saved;
    g_fp32_split = split;
  }
};
// FP32 products of a testing entry point: prec 1 the FP32 instructions,
// prec 2 the bf16 split (prec 0: FP64, unaffected)
struct TestPrec {
  bool split;
  explicit TestPrec(int prec) : split(g_fp32_split) { g_fp32_split = prec == 2; }
  ~TestPrec() { g_fp32_split = split; }
};
void set_last_error(const std::string& msg) { g_last_error = msg; }

template <typename F>
static nudft2_status guard(F&& f) {
  try {
    f();
    g_last_error.clear();
    return NUDFT2_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return NUDFT2_E_NOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return NUDFT2_E_INTERNAL;
  } catch (...) {
    g_last_error = "unknown error";
    return NUDFT2_E_INTERNAL;
  }
}

namespace {
__global__ void mfma_probe_kernel(const double* a, const double* b, double* d) {
  int lane = threadIdx.x;
  double av = a[(lane % 16) * 4 + lane / 16];
  double bv = b[(lane / 16) * 16 + lane % 16];
  dbl4 acc = dbl4{0, 0, 0, 0};
  acc = mfma16(av, bv, acc);
  for (int v = 0; v < 4; ++v) d[((lane / 16) + 4 * v) * 16 + lane % 16] = acc[v];
}
__global__ void mfma_probe32_kernel(const float* a, const float* b, float* d) {
  int lane = threadIdx.x;
  float av = a[(lane % 16) * 4 + lane / 16];
  float bv = b[(lane / 16) * 16 + lane % 16];
  flt4 acc = flt4{0, 0, 0, 0};
  acc = mfma16(av, bv, acc);
  for (int v = 0; v < 4; ++v) d[(4 * (lane / 16) + v) * 16 + lane % 16] = acc[v];
}
template <typename T, typename K>
void run_probe(K kern, const T* a, const T* b, T* d) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    throw Error(NUDFT2_E_DEVICE, "no HIP device available");
  }
  T *da, *db, *dd;
  ND_HIP(hipMalloc(&da, 64 * sizeof(T)));
  ND_HIP(hipMalloc(&db, 64 * sizeof(T)));
  ND_HIP(hipMalloc(&dd, 256 * sizeof(T)));
  ND_HIP(hipMemcpy(da, a, 64 * sizeof(T), hipMemcpyHostToDevice));
  ND_HIP(hipMemcpy(db, b, 64 * sizeof(T), hipMemcpyHostToDevice));
  hipLaunchKernelGGL(kern, dim3(1), dim3(64), 0, nullptr, da, db, dd);
  ND_HIP(hipGetLastError());
  ND_HIP(hipMemcpy(d, dd, 256 * sizeof(T), hipMemcpyDeviceToHost));
  (void)hipFree(da);
  (void)hipFree(db);
  (void)hipFree(dd);
}
}  // namespace

static void need_device() {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    throw Error(NUDFT2_E_DEVICE, "no HIP device available");
  }
}

template <typename T>
static void test_gemm(int opA, int opB, int nb, const int32_t* mnk, const int32_t* ld,
                      const int64_t* ptrs, double ar, double ai, double beta, int splits = 0,
                      float* ms = nullptr) {
  std::vector<GemmDesc<T>> d(nb);
  for (int i = 0; i < nb; ++i)
    d[i] = GemmDesc<T>{mnk[3 * i], mnk[3 * i + 1], mnk[3 * i + 2], ld[3 * i], ld[3 * i + 1],
                       ld[3 * i + 2], (const cplx<T>*)ptrs[3 * i],
                       (const cplx<T>*)ptrs[3 * i + 1], (cplx<T>*)ptrs[3 * i + 2], (T)ar,
                       (T)ai, (T)beta};
  DescPool pool;
  pool.init(std::max<size_t>(1 << 20, sizeof(GemmDesc<T>) * (size_t)nb * 2 + 4096), nullptr);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms) {
    ND_HIP(hipEventCreate(&e0));
    ND_HIP(hipEventCreate(&e1));
    ND_HIP(hipStreamSynchronize(nullptr));
    ND_HIP(hipEventRecord(e0, nullptr));
  }
  gemm_batched<T>(pool, d, (Op)opA, (Op)opB, splits);
  if (ms) {
    ND_HIP(hipEventRecord(e1, nullptr));
    ND_HIP(hipEventSynchronize(e1));
    ND_HIP(hipEventElapsedTime(ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  pool.sync_reset();
}

template <typename T>
static void test_geqrf(int nb, const int32_t* mn, const int32_t* ld, const int64_t* ptrs) {
  std::vector<QRDesc<T>> d(nb);
  for (int i = 0; i < nb; ++i)
    d[i] = QRDesc<T>{mn[2 * i], mn[2 * i + 1], ld[2 * i], ld[2 * i + 1], (cplx<T>*)ptrs[3 * i],
                     (cplx<T>*)ptrs[3 * i + 1], (cplx<T>*)ptrs[3 * i + 2]};
  DescPool pool;
  pool.init(16 << 20, nullptr);
  void* ws;
  ND_HIP(hipMalloc(&ws, qr_workspace<T>(d)));
  geqrf_batched<T>(pool, d, ws);
  pool.sync_reset();
  ND_HIP(hipFree(ws));
}

template <typename T>
static void test_ormqr(int trans, int nb, const int32_t* dims, const int32_t* ld,
                       const int64_t* ptrs) {
  std::vector<OrmDesc<T>> d(nb);
  for (int i = 0; i < nb; ++i)
    d[i] = OrmDesc<T>{dims[3 * i], dims[3 * i + 1], dims[3 * i + 2], ld[2 * i], ld[2 * i + 1],
                      (const cplx<T>*)ptrs[3 * i], (const cplx<T>*)ptrs[3 * i + 1],
                      (cplx<T>*)ptrs[3 * i + 2]};
  DescPool pool;
  pool.init(16 << 20, nullptr);
  void* ws;
  ND_HIP(hipMalloc(&ws, orm_workspace<T>(d)));
  ormqr_batched<T>(pool, d, trans == 1, ws, trans == 2);
  pool.sync_reset();
  ND_HIP(hipFree(ws));
}

template <typename T>
static void test_trsv(int nb, const int32_t* dims, const int32_t* ld, const int64_t* ptrs, bool ct) {
  std::vector<TrsDesc<T>> d(nb);
  for (int i = 0; i < nb; ++i)
    d[i] = TrsDesc<T>{dims[2 * i], dims[2 * i + 1], ld[2 * i], ld[2 * i + 1],
                      (const cplx<T>*)ptrs[2 * i], (cplx<T>*)ptrs[2 * i + 1]};
  DescPool pool;
  pool.init(1 << 20, nullptr);
  trsv_upper_batched<T>(pool, d, ct);
  pool.sync_reset();
}

template <typename TD, typename TS>
static void test_copy(int nb, const int32_t* dims, const int32_t* ld, const int64_t* ptrs,
                      const int32_t* ct) {
  std::vector<CopyDesc<TD, TS>> d(nb);
  for (int i = 0; i < nb; ++i)
    d[i] = CopyDesc<TD, TS>{dims[2 * i], dims[2 * i + 1], ld[2 * i], ld[2 * i + 1],
                            (const cplx<TS>*)ptrs[2 * i], (cplx<TD>*)ptrs[2 * i + 1],
                            ct[i] != 0};
  DescPool pool;
  pool.init(1 << 20, nullptr);
  copy_batched<TD, TS>(pool, d);
  pool.sync_reset();
}

}  // namespace nd

using namespace nd;

extern "C" {

void nudft2_default_opts(nudft2_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = 1;
  o->eps = 1e-4;
  o->leaf = 16;
  o->ir_tol = 1e-12;
  o->ir_maxit = 30;
  o->refine = 0;
  o->stream = nullptr;
  o->mem_cap = 0;
  o->graph = 0;
  o->nufft_tol = 0.0;
  o->fp32_products = 0;
  o->fadi_1d = 1;
}

const char* nudft2_strerror(nudft2_status s) {
  switch (s) {
    case NUDFT2_OK: return "ok";
    case NUDFT2_E_INVAL: return "invalid argument";
    case NUDFT2_E_STATE: return "call out of order";
    case NUDFT2_E_DEVICE: return "device error";
    case NUDFT2_E_NOMEM: return "out of device memory";
    case NUDFT2_E_SINGULAR: return "singular factor";
    case NUDFT2_E_NOCONV: return "refinement did not converge";
    case NUDFT2_E_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* nudft2_last_error(void) { return g_last_error.c_str(); }

nudft2_status nudft2_plan_batch(nudft2_plan_t* out, int32_t nprob, const double* points,
                                const int64_t* m_off, const int32_t* nx, const int32_t* ny,
                                const nudft2_opts* opts) {
  return guard([&] {
    ND_CHECK(out != nullptr, NUDFT2_E_INVAL, "null output handle");
    Plan* p = make_plan(nprob, points, m_off, nx, ny, opts);
    *out = reinterpret_cast<nudft2_plan_t>(p);
  });
}

nudft2_status nudft2_plan(nudft2_plan_t* out, const double* points, int64_t M, int32_t nx,
                          int32_t ny, const nudft2_opts* opts) {
  int64_t off[2] = {0, M};
  if (M < 0) {
    g_last_error = "M must be >= 0";
    return NUDFT2_E_INVAL;
  }
  return nudft2_plan_batch(out, 1, points, off, &nx, &ny, opts);
}

nudft2_status nudft2_factor(nudft2_plan_t plan) {
  return guard([&] {
    ND_CHECK(plan != nullptr, NUDFT2_E_INVAL, "null plan");
    Plan* P = reinterpret_cast<Plan*>(plan);
    PlanProf pp(P);
    factor(P);
  });
}

nudft2_status nudft2_solve(nudft2_plan_t plan, const double* f, double* c, int32_t nrhs,
                           nudft2_solve_info* info) {
  return guard([&] {
    ND_CHECK(plan != nullptr && f != nullptr && c != nullptr, NUDFT2_E_INVAL, "null pointer");
    ND_CHECK(nrhs > 0, NUDFT2_E_INVAL, "nrhs must be positive");
    Plan* P = reinterpret_cast<Plan*>(plan);
    ND_CHECK(P->factored, NUDFT2_E_STATE, "solve before factor");
    PlanProf pp(P);
    solve(P, reinterpret_cast<const double2*>(f), reinterpret_cast<double2*>(c), nrhs, info,
          false);
  });
}

nudft2_status nudft2_solve_adj(nudft2_plan_t plan, const double* g, double* w, int32_t nrhs,
                               nudft2_solve_info* info) {
  return guard([&] {
    ND_CHECK(plan != nullptr && g != nullptr && w != nullptr, NUDFT2_E_INVAL, "null pointer");
    ND_CHECK(nrhs > 0, NUDFT2_E_INVAL, "nrhs must be positive");
    Plan* P = reinterpret_cast<Plan*>(plan);
    ND_CHECK(P->factored, NUDFT2_E_STATE, "solve before factor");
    PlanProf pp(P);
    solve(P, reinterpret_cast<const double2*>(g), reinterpret_cast<double2*>(w), nrhs, info,
          true);
  });
}

nudft2_status nudft2_lsq_backward(nudft2_plan_t plan, const double* f, const double* c,
                                  const double* g, double* grad_f, double* grad_points,
                                  int32_t nrhs, nudft2_solve_info* info) {
  return guard([&] {
    ND_CHECK(plan != nullptr && f != nullptr && c != nullptr && g != nullptr && grad_f != nullptr,
             NUDFT2_E_INVAL, "null pointer");
    ND_CHECK(nrhs > 0, NUDFT2_E_INVAL, "nrhs must be positive");
    Plan* P = reinterpret_cast<Plan*>(plan);
    ND_CHECK(P->factored, NUDFT2_E_STATE, "backward before factor");
    PlanProf pp(P);
    lsq_backward(P, reinterpret_cast<const double2*>(f), reinterpret_cast<const double2*>(c),
                 reinterpret_cast<const double2*>(g), reinterpret_cast<double2*>(grad_f),
                 grad_points, nrhs, info);
  });
}

nudft2_status nudft2_apply(nudft2_plan_t plan, const double* c, double* f, int32_t nrhs) {
  return guard([&] {
    ND_CHECK(plan != nullptr && f != nullptr && c != nullptr, NUDFT2_E_INVAL, "null pointer");
    ND_CHECK(nrhs > 0, NUDFT2_E_INVAL, "nrhs must be positive");
    Plan* P = reinterpret_cast<Plan*>(plan);
    PlanProf pp(P);
    apply_fwd(P, reinterpret_cast<const double2*>(c), reinterpret_cast<double2*>(f), nrhs,
              P->stream);
  });
}

nudft2_status nudft2_apply_adj(nudft2_plan_t plan, const double* f, double* c, int32_t nrhs) {
  return guard([&] {
    ND_CHECK(plan != nullptr && f != nullptr && c != nullptr, NUDFT2_E_INVAL, "null pointer");
    ND_CHECK(nrhs > 0, NUDFT2_E_INVAL, "nrhs must be positive");
    Plan* P = reinterpret_cast<Plan*>(plan);
    PlanProf pp(P);
    apply_adj(P, reinterpret_cast<const double2*>(f), reinterpret_cast<double2*>(c), nrhs,
              P->stream);
  });
}

nudft2_status nudft2_nufft(nudft2_plan_t plan, const double* c, double* f, int32_t nrhs,
                           double tol) {
  return guard([&] {
    ND_CHECK(plan != nullptr && f != nullptr && c != nullptr, NUDFT2_E_INVAL, "null pointer");
    ND_CHECK(nrhs > 0, NUDFT2_E_INVAL, "nrhs must be positive");
    Plan* P = reinterpret_cast<Plan*>(plan);
    nufft_fwd(P, reinterpret_cast<const double2*>(c), reinterpret_cast<double2*>(f), nrhs, tol,
              P->stream);
  });
}

nudft2_status nudft2_nufft_adj(nudft2_plan_t plan, const double* f, double* c, int32_t nrhs,
                               double tol) {
  return guard([&] {
    ND_CHECK(plan != nullptr && f != nullptr && c != nullptr, NUDFT2_E_INVAL, "null pointer");
    ND_CHECK(nrhs > 0, NUDFT2_E_INVAL, "nrhs must be positive");
    Plan* P = reinterpret_cast<Plan*>(plan);
    nufft_adj(P, reinterpret_cast<const double2*>(f), reinterpret_cast<double2*>(c), nrhs, tol,
              P->stream);
  });
}

nudft2_status nudft2_apply_adj_noalloc(nudft2_plan_t plan, const double* f, double* c,
                                       int32_t nrhs) {
  return guard([&] {
    ND_CHECK(plan != nullptr && f != nullptr && c != nullptr, NUDFT2_E_INVAL, "null pointer");
    ND_CHECK(nrhs > 0, NUDFT2_E_INVAL, "nrhs must be positive");
    Plan* P = reinterpret_cast<Plan*>(plan);
    apply_adj_noalloc(P, reinterpret_cast<const double2*>(f), reinterpret_cast<double2*>(c),
                      nrhs);
  });
}

nudft2_status nudft2_get_info(nudft2_plan_t plan, nudft2_info* info) {
  return guard([&] {
    ND_CHECK(plan != nullptr && info != nullptr, NUDFT2_E_INVAL, "null pointer");
    Plan* P = reinterpret_cast<Plan*>(plan);
    ND_HIP(hipStreamSynchronize(P->stream));
    P->prof.collect();
    *info = P->info;
    info->factor_bytes = (int64_t)P->arena.bytes;
    info->peak_bytes = (int64_t)P->arena.peak;
    for (int i = 0; i < KC_COUNT; ++i) {
      info->kernel_ms[i] = P->prof.ms[i];
      info->kernel_flops[i] = P->prof.flops[i];
      info->kernel_launches[i] = P->prof.launches[i];
    }
  });
}

nudft2_status nudft2_set_solve_opts(nudft2_plan_t plan, double ir_tol, int32_t ir_maxit,
                                    int32_t refine) {
  return guard([&] {
    ND_CHECK(plan != nullptr, NUDFT2_E_INVAL, "null plan");
    ND_CHECK(ir_tol >= 0 && ir_maxit >= 0 && refine >= 0 && refine <= 2, NUDFT2_E_INVAL,
             "bad refinement options");
    Plan* P = reinterpret_cast<Plan*>(plan);
    P->opts.ir_tol = ir_tol;
    P->opts.ir_maxit = ir_maxit;
    P->opts.refine = refine;
  });
}

nudft2_status nudft2_set_nufft_tol(nudft2_plan_t plan, double nufft_tol) {
  return guard([&] {
    ND_CHECK(plan != nullptr, NUDFT2_E_INVAL, "null plan");
    ND_CHECK(nufft_tol == 0.0 || (nufft_tol > 0.0 && nufft_tol < 0.1), NUDFT2_E_INVAL,
             "nufft_tol must be 0 or lie in (0, 0.1)");
    Plan* P = reinterpret_cast<Plan*>(plan);
    if (nufft_tol > 0.0)
      for (auto& q : P->probs)
        ND_CHECK(q.nx <= 1024 && q.ny <= 1024, NUDFT2_E_INVAL,
                 "the NUFFT operator needs nx, ny <= 1024");
    P->opts.nufft_tol = nufft_tol;
  });
}

nudft2_status nudft2_set_profiling(nudft2_plan_t plan, int32_t on) {
  return nudft2_set_profiling_classes(plan, on ? (1u << KC_COUNT) - 1 : 0u);
}

nudft2_status nudft2_set_profiling_classes(nudft2_plan_t plan, uint32_t classes) {
  return guard([&] {
    ND_CHECK(plan != nullptr, NUDFT2_E_INVAL, "null plan");
    ND_CHECK(classes < (1u << KC_COUNT), NUDFT2_E_INVAL, "unknown kernel class in the mask");
    Plan* P = reinterpret_cast<Plan*>(plan);
    ND_HIP(hipStreamSynchronize(P->stream));
    P->prof.reset();
    P->prof.mask = classes;
    P->profiling = classes != 0;
  });
}

nudft2_status nudft2_destroy(nudft2_plan_t plan) {
  return guard([&] {
    if (!plan) return;
    Plan* P = reinterpret_cast<Plan*>(plan);
    (void)hipStreamSynchronize(P->stream);
    delete P;
  });
}

nudft2_status nudft2_test_binning(const double* points, int64_t M, int32_t nx, int32_t ny,
                                  int32_t leaf, int64_t* perm2d, int64_t* leaf_rows,
                                  int64_t* colperm, int32_t* depth) {
  return guard([&] {
    ND_CHECK(points && perm2d && leaf_rows && colperm && depth, NUDFT2_E_INVAL, "null pointer");
    ND_CHECK(nx >= 2 && ny >= 2 && leaf >= 2 && M >= 0, NUDFT2_E_INVAL, "bad sizes");
    *depth = tree_depth(nx, ny, leaf);
    host_binning(points, M, nx, ny, leaf, perm2d, leaf_rows, colperm);
  });
}

nudft2_status nudft2_test_mfma_layout(const double* a, const double* b, double* d) {
  return guard([&] {
    ND_CHECK(a && b && d, NUDFT2_E_INVAL, "null pointer");
    run_probe<double>(mfma_probe_kernel, a, b, d);
  });
}

nudft2_status nudft2_test_mfma_layout32(const float* a, const float* b, float* d) {
  return guard([&] {
    ND_CHECK(a && b && d, NUDFT2_E_INVAL, "null pointer");
    run_probe<float>(mfma_probe32_kernel, a, b, d);
  });
}

nudft2_status nudft2_test_gemm(int32_t prec, int32_t opA, int32_t opB, int32_t nb,
                               const int32_t* mnk, const int32_t* ld, const int64_t* ptrs,
                               double ar, double ai, double beta) {
  return guard([&] {
    ND_CHECK(mnk && ld && ptrs && nb > 0, NUDFT2_E_INVAL, "bad arguments");
    need_device();
    TestPrec tp(prec);
    if (prec == 0) test_gemm<double>(opA, opB, nb, mnk, ld, ptrs, ar, ai, beta);
    else test_gemm<float>(opA, opB, nb, mnk, ld, ptrs, ar, ai, beta);
  });
}

nudft2_status nudft2_test_gemm_cfg(int32_t prec, int32_t opA, int32_t opB, int32_t nb,
                                   const int32_t* mnk, const int32_t* ld, const int64_t* ptrs,
                                   double ar, double ai, double beta, int32_t splits,
                                   float* ms) {
  return guard([&] {
    ND_CHECK(mnk && ld && ptrs && nb > 0 && splits >= -6, NUDFT2_E_INVAL, "bad arguments");
    need_device();
    TestPrec tp(prec);
    if (prec == 0) test_gemm<double>(opA, opB, nb, mnk, ld, ptrs, ar, ai, beta, splits, ms);
    else test_gemm<float>(opA, opB, nb, mnk, ld, ptrs, ar, ai, beta, splits, ms);
  });
}

nudft2_status nudft2_test_geqrf(int32_t prec, int32_t nb, const int32_t* mn, const int32_t* ld,
                                const int64_t* ptrs) {
  return guard([&] {
    ND_CHECK(mn && ld && ptrs && nb > 0, NUDFT2_E_INVAL, "bad arguments");
    need_device();
    TestPrec tp(prec);
    if (prec == 0) test_geqrf<double>(nb, mn, ld, ptrs);
    else test_geqrf<float>(nb, mn, ld, ptrs);
  });
}

nudft2_status nudft2_test_ormqr(int32_t prec, int32_t trans, int32_t nb, const int32_t* dims,
                                const int32_t* ld, const int64_t* ptrs) {
  return guard([&] {
    ND_CHECK(dims && ld && ptrs && nb > 0 && trans >= 0 && trans <= 2, NUDFT2_E_INVAL,
             "bad arguments");
    need_device();
    TestPrec tp(prec);
    if (prec == 0) test_ormqr<double>(trans, nb, dims, ld, ptrs);
    else test_ormqr<float>(trans, nb, dims, ld, ptrs);
  });
}

nudft2_status nudft2_test_pchol(int32_t nb, const int32_t* w, const int32_t* rmax,
                                const int64_t* ptrs, double tol2, int32_t* rank_out,
                                int32_t* piv_out) {
  return guard([&] {
    ND_CHECK(w && rmax && ptrs && rank_out && piv_out && nb > 0, NUDFT2_E_INVAL, "bad arguments");
    need_device();
    std::vector<PcholDesc> d(nb);
    std::vector<void*> allocs;
    int* ranks;
    ND_HIP(hipMalloc((void**)&ranks, sizeof(int) * nb));
    int tot = 0;
    for (int i = 0; i < nb; ++i) tot += rmax[i];
    int* piv;
    ND_HIP(hipMalloc((void**)&piv, sizeof(int) * std::max(tot, 1)));
    int off = 0;
    for (int i = 0; i < nb; ++i) {
      double* dw;
      ND_HIP(hipMalloc((void**)&dw, sizeof(double) * std::max(w[i], 1)));
      allocs.push_back(dw);
      d[i] = PcholDesc{w[i], w[i], w[i], rmax[i], (double2*)ptrs[2 * i], (double2*)ptrs[2 * i + 1],
                       dw, piv + off, ranks + i, tol2};
      off += rmax[i];
    }
    DescPool pool;
    pool.init(16 << 20, nullptr);
    pchol_batched(pool, d);
    pool.sync_reset();
    ND_HIP(hipMemcpy(rank_out, ranks, sizeof(int) * nb, hipMemcpyDeviceToHost));
    if (tot > 0) ND_HIP(hipMemcpy(piv_out, piv, sizeof(int) * tot, hipMemcpyDeviceToHost));
    for (void* p : allocs) (void)hipFree(p);
    (void)hipFree(ranks);
    (void)hipFree(piv);
  });
}

nudft2_status nudft2_test_trsv(int32_t prec, int32_t nb, const int32_t* dims, const int32_t* ld,
                               const int64_t* ptrs, int32_t conj_trans) {
  return guard([&] {
    ND_CHECK(dims && ld && ptrs && nb > 0, NUDFT2_E_INVAL, "bad arguments");
    need_device();
    TestPrec tp(prec);
    if (prec == 0) test_trsv<double>(nb, dims, ld, ptrs, conj_trans != 0);
    else test_trsv<float>(nb, dims, ld, ptrs, conj_trans != 0);
  });
}

nudft2_status nudft2_test_trtri(int32_t prec, int32_t nb, const int32_t* k, const int32_t* ld,
                                const int64_t* ptrs) {
  return guard([&] {
    ND_CHECK(k && ld && ptrs && nb > 0, NUDFT2_E_INVAL, "bad arguments");
    need_device();
    TestPrec tp(prec);
    auto run = [&](auto tag) {
      using T = decltype(tag);
      std::vector<TriDesc<T>> d(nb);
      for (int i = 0; i < nb; ++i) {
        ND_CHECK(k[i] >= 0 && ld[i] >= std::max(1, k[i]), NUDFT2_E_INVAL, "bad sizes");
        d[i] = TriDesc<T>{k[i], ld[i], (cplx<T>*)ptrs[i]};
      }
      DescPool pool;
      pool.init(16 << 20, nullptr);
      void* ws;
      ND_HIP(hipMalloc(&ws, trtri_workspace<T>(d)));
      trtri_upper_batched<T>(pool, d, ws);
      pool.sync_reset();
      ND_HIP(hipFree(ws));
    };
    if (prec == 0) run(double());
    else run(float());
  });
}

nudft2_status nudft2_test_copy(int32_t prec_d, int32_t prec_s, int32_t nb, const int32_t* dims,
                               const int32_t* ld, const int64_t* ptrs, const int32_t* conj_trans) {
  return guard([&] {
    ND_CHECK(dims && ld && ptrs && conj_trans && nb > 0, NUDFT2_E_INVAL, "bad arguments");
    ND_CHECK((prec_d == 0 || prec_d == 1) && (prec_s == 0 || prec_s == 1), NUDFT2_E_INVAL,
             "precision must be 0 (complex128) or 1 (complex64)");
    for (int i = 0; i < nb; ++i) {
      const int m = dims[2 * i], n = dims[2 * i + 1];
      ND_CHECK(m >= 0 && n >= 0 && ld[2 * i] >= std::max(1, m) &&
                   ld[2 * i + 1] >= std::max(1, conj_trans[i] ? n : m),
               NUDFT2_E_INVAL, "bad copy dimensions");
    }
    need_device();
    if (prec_d == 0 && prec_s == 0) test_copy<double, double>(nb, dims, ld, ptrs, conj_trans);
    else if (prec_d == 0) test_copy<double, float>(nb, dims, ld, ptrs, conj_trans);
    else if (prec_s == 0) test_copy<float, double>(nb, dims, ld, ptrs, conj_trans);
    else test_copy<float, float>(nb, dims, ld, ptrs, conj_trans);
  });
}

nudft2_status nudft2_test_fadi_block(const double* xs, int64_t m, int32_t n, int32_t level,
                                     int32_t a, double tau, int32_t* plan_out, double* gamma,
                                     double* pq, int32_t smax, double* Z, double* W) {
  return guard([&] {
    ND_CHECK(plan_out && gamma && pq && smax >= 0, NUDFT2_E_INVAL, "bad arguments");
    ND_CHECK(n >= 1 && level >= 1 && level < 31 && a >= 0 && a < (1 << level) && tau > 0.0 &&
                 tau < 1.0 && m >= 0 && m <= INT32_MAX,
             NUDFT2_E_INVAL, "bad block");
    const FadiPlan pl = fadi_plan(n, level, a, tau);
    plan_out[0] = pl.b;
    plan_out[1] = pl.s;
    *gamma = pl.gamma;
    ND_CHECK(pl.s <= smax, NUDFT2_E_INVAL, "more shifts than smax");
    for (int j = 0; j < pl.s; ++j) {
      pq[2 * j] = pl.p[j].x;
      pq[2 * j + 1] = pl.p[j].y;
      pq[2 * (smax + j)] = pl.q[j].x;
      pq[2 * (smax + j) + 1] = pl.q[j].y;
    }
    if (!Z || !W || pl.b == 0) return;
    ND_CHECK(xs || m == 0, NUDFT2_E_INVAL, "xs is NULL");
    need_device();
    std::vector<double2> sh(pl.p);
    sh.insert(sh.end(), pl.q.begin(), pl.q.end());
    DescPool pool;
    pool.init(1 << 20, nullptr);
    const double2* dsh = (const double2*)pool.push_ro(sh.data(), sizeof(double2) * sh.size());
    std::vector<FadiDesc> d{{xs, dsh, (double2*)Z, (double2*)W, (int)m, n, pl.b, pl.s, pl.lo,
                             pl.hi, (int)std::max<int64_t>(m, 1), n}};
    fadi_factors(pool, d);
    pool.sync_reset();
  });
}

nudft2_status nudft2_test_hss1d_matvec(nudft2_plan_t plan, int32_t dim, double tol,
                                       const double* x, double* y, int32_t* ranks,
                                       int32_t prob) {
  return guard([&] {
    ND_CHECK(plan && x && y && (dim == 0 || dim == 1), NUDFT2_E_INVAL, "bad arguments");
    Plan* P = reinterpret_cast<Plan*>(plan);
    ND_CHECK(prob >= 0 && prob < (int)P->probs.size(), NUDFT2_E_INVAL, "problem index out of range");
    Ctx cx;
    cx.P = P;
    cx.s = P->stream;
    cx.pool.init(64 << 20, cx.s);
    std::vector<Tree1> t;
    build_1d(cx, dim, tol, t);
    if (ranks) {
      int L = t[prob].L;
      for (int l = 0; l <= L; ++l) {
        int ru = 0, rv = 0;
        for (auto& nd : t[prob].lv[l]) {
          ru = std::max(ru, nd.rU);
          rv = std::max(rv, nd.rV);
        }
        ranks[2 * l] = ru;
        ranks[2 * l + 1] = rv;
      }
    }
    matvec_1d(cx, dim, t, prob, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y));
    free_1d(P, t);
  });
}

nudft2_status nudft2_test_hss_matvec(nudft2_plan_t plan, const double* x, double* y,
                                     int32_t stages, int32_t prob, int32_t nrhs) {
  return guard([&] {
    ND_CHECK(plan && x && y && nrhs > 0, NUDFT2_E_INVAL, "bad arguments");
    Plan* P = reinterpret_cast<Plan*>(plan);
    ND_CHECK(prob >= 0 && prob < (int)P->probs.size(), NUDFT2_E_INVAL, "problem index out of range");
    Ctx cx;
    cx.P = P;
    cx.s = P->stream;
    cx.pool.init(256 << 20, cx.s);
    std::vector<Tree1> tx, ty;
    build_1d(cx, 0, P->opts.eps / 10, tx);
    build_1d(cx, 1, P->opts.eps / 10, ty);
    auto run = [&](auto& H) {
      build_2d(cx, tx, ty, P->opts.eps, H, stages);
      free_1d(P, tx);
      free_1d(P, ty);
      matvec_2d(cx, H, prob, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y),
                nrhs);
      ND_HIP(hipStreamSynchronize(cx.s));
      for (void* m : H.mem) P->arena.release(m);
      H.mem.clear();
    };
    if (P->opts.precision == 0) {
      HSS2<double> H;
      run(H);
    } else {
      HSS2<float> H;
      run(H);
    }
  });
}

}  // extern "C"
