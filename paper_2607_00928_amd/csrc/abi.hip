// C-ABI entry points: argument checks, error mapping, dispatch.
#include <cstring>

#include "../../include/nudft2_testing.h"
#include "device_util.h"
#include "hss.h"
#include "plan.h"
#include "solver.h"

namespace nd {

static thread_local std::string g_last_error;
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
    solve(P, reinterpret_cast<const double2*>(g), reinterpret_cast<double2*>(w), nrhs, info,
          true);
  });
}

nudft2_status nudft2_apply(nudft2_plan_t plan, const double* c, double* f, int32_t nrhs) {
  return guard([&] {
    ND_CHECK(plan != nullptr && f != nullptr && c != nullptr, NUDFT2_E_INVAL, "null pointer");
    ND_CHECK(nrhs > 0, NUDFT2_E_INVAL, "nrhs must be positive");
    Plan* P = reinterpret_cast<Plan*>(plan);
    apply_fwd(P, reinterpret_cast<const double2*>(c), reinterpret_cast<double2*>(f), nrhs,
              P->stream);
  });
}

nudft2_status nudft2_apply_adj(nudft2_plan_t plan, const double* f, double* c, int32_t nrhs) {
  return guard([&] {
    ND_CHECK(plan != nullptr && f != nullptr && c != nullptr, NUDFT2_E_INVAL, "null pointer");
    ND_CHECK(nrhs > 0, NUDFT2_E_INVAL, "nrhs must be positive");
    Plan* P = reinterpret_cast<Plan*>(plan);
    apply_adj(P, reinterpret_cast<const double2*>(f), reinterpret_cast<double2*>(c), nrhs,
              P->stream);
  });
}

nudft2_status nudft2_get_info(nudft2_plan_t plan, nudft2_info* info) {
  return guard([&] {
    ND_CHECK(plan != nullptr && info != nullptr, NUDFT2_E_INVAL, "null pointer");
    Plan* P = reinterpret_cast<Plan*>(plan);
    ND_HIP(hipStreamSynchronize(P->stream));
    *info = P->info;
    info->factor_bytes = (int64_t)P->arena.bytes;
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

}  // extern "C"
