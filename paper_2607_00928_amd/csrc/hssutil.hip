// Shared HSS helpers: orthonormalisation by Householder QR and batched
// pivoted-Cholesky rank decisions (FP64).
#include <algorithm>

#include "hss.h"

namespace nd {

// Orthonormal basis of the columns of A (destroyed): Q (m x k), k = min(m, c);
// optionally the triangular factor (k x c) into Rout (caller-allocated).
template <typename T>
void orth(Ctx& cx, std::vector<Mat<T>>& A, std::vector<Mat<T>>& Q,
          std::vector<Mat<T>>* Rout) {
  if (A.empty()) return;
  std::vector<QRDesc<T>> qd;
  std::vector<Mat<T>> Rb(A.size()), Tb(A.size());
  std::vector<Mat<T>*> ms;
  for (size_t i = 0; i < A.size(); ++i) {
    int k = std::min(A[i].r, A[i].c);
    Rb[i].r = std::max(k, 1);
    Rb[i].c = std::max(A[i].c, 1);
    Tb[i].r = (int)qr_tsize(A[i].r, A[i].c);
    Tb[i].c = 1;
    ms.push_back(&Rb[i]);
    ms.push_back(&Tb[i]);
  }
  carve(cx.P->arena, ms, &cx.tmp);
  for (size_t i = 0; i < A.size(); ++i)
    qd.push_back({A[i].r, A[i].c, A[i].ld, Rb[i].ld, A[i].p, Rb[i].p, Tb[i].p});
  void* ws = cx.tmp_alloc(qr_workspace<T>(qd));
  geqrf_batched<T>(cx.pool, qd, ws);
  std::vector<FillDesc<T>> fd;
  std::vector<OrmDesc<T>> od;
  std::vector<CopyDesc<T, T>> cd;
  for (size_t i = 0; i < A.size(); ++i) {
    int k = std::min(A[i].r, A[i].c);
    fd.push_back({Q[i].r, Q[i].c, Q[i].ld, Q[i].p, 1});
    od.push_back({A[i].r, k, Q[i].c, A[i].ld, Q[i].ld, A[i].p, Tb[i].p, Q[i].p});
    if (Rout) cd.push_back({k, A[i].c, Rb[i].ld, (*Rout)[i].ld, Rb[i].p, (*Rout)[i].p, 0});
  }
  fill_batched<T>(cx.pool, fd);
  void* ws2 = cx.tmp_alloc(orm_workspace<T>(od));
  ormqr_batched<T>(cx.pool, od, false, ws2, true);
  if (Rout) copy_batched<T, T>(cx.pool, cd);
}
template void orth<float>(Ctx&, std::vector<Mat<float>>&, std::vector<Mat<float>>&,
                          std::vector<Mat<float>>*);
template void orth<double>(Ctx&, std::vector<Mat<double>>&, std::vector<Mat<double>>&,
                           std::vector<Mat<double>>*);

// Pivoted Cholesky of a batch of FP64 Grams (w x w, ld w); returns ranks on
// the host.  K is destroyed.
void pchol_run(Ctx& cx, std::vector<Mat<double>>& K, std::vector<int>& rmax, double tol2,
               std::vector<PcholOut>& out) {
  size_t nb = K.size();
  out.assign(nb, PcholOut());
  if (nb == 0) return;
  std::vector<Mat<double>*> ms;
  for (size_t i = 0; i < nb; ++i) {
    out[i].L.r = K[i].r;
    out[i].L.c = std::max(rmax[i], 1);
    ms.push_back(&out[i].L);
  }
  carve(cx.P->arena, ms, &cx.tmp);
  int tot = 0, totw = 0;
  for (size_t i = 0; i < nb; ++i) {
    tot += std::max(rmax[i], 1);
    totw += std::max(K[i].r, 1);
  }
  int* piv = (int*)cx.tmp_alloc(sizeof(int) * tot);
  int* rank = (int*)cx.tmp_alloc(sizeof(int) * nb);
  double* dw = (double*)cx.tmp_alloc(sizeof(double) * totw);
  std::vector<PcholDesc> pd;
  int po = 0, wo = 0;
  for (size_t i = 0; i < nb; ++i) {
    out[i].piv = piv + po;
    pd.push_back({K[i].r, K[i].ld, out[i].L.ld, rmax[i], (double2*)K[i].p, (double2*)out[i].L.p,
                  dw + wo, piv + po, rank + i, tol2});
    po += std::max(rmax[i], 1);
    wo += std::max(K[i].r, 1);
  }
  pchol_batched(cx.pool, pd);
  std::vector<int> h(nb);
  ND_HIP(hipMemcpyAsync(h.data(), rank, sizeof(int) * nb, hipMemcpyDeviceToHost, cx.s));
  ND_HIP(hipStreamSynchronize(cx.s));
  for (size_t i = 0; i < nb; ++i) out[i].rank = h[i];
}


}  // namespace nd
