// URV factorization and solution of the recompressed HSS matrix (Section 2.4,
// "The URV factorization for HSS matrices"), with separate row and column
// ranks.  Per node (leaf, or a parent after its children were merged):
//
//  size reduction   if mm >= nn + rU:  [U D] = Omega [U' D'; 0 0]  (QR)
//  basis elimination V = Q [0; V2] by a QR of V with the columns of its Q
//                    factor cyclically shifted ("reverse QR"); D~ = D' Q
//  partial decomposition  QR of the first k = nn - rV columns of D~ gives P
//                    and D11; [D12; D22] = P^H D~(:, k:), [U1; U2] = P^H U'
//  merge            D+ = [D22_i on the diagonal, U2_i B_ij V2_j^H off it],
//                    U+ = [U2_i R_i], V+ = [V2_i W_i]; the root is factored
//                    by a QR for the final least-squares problem.
//
// The solve applies Omega^H and P^H bottom up, solves the root least-squares
// problem, and substitutes top down: b_i = R_i b_parent + sum_j B_ij V2_j^H
// c2_j, c1 = D11^{-1}(f1 - D12 c2 - U1 b), c = Q [c1; c2].
//
// Storage per node: W = [D~(:,0:k) | U' | D~(:,k:)] so that one QR of its
// first k columns and one application of P^H to the remaining columns give
// [U1 D12; U2 D22] in place.  Once the factorization is complete, D11 and the
// root's triangle are replaced by their inverses (blocked triangular
// inversion), which is all the solves use: every triangular solve of a sweep
// becomes one batched matrix-vector product.
#include <algorithm>

#include "gen.h"
#include "hss.h"

namespace nd {

namespace {
template <typename T>
int sib_slot(int c, int other) { return other < c ? other : other - 1; }
}  // namespace

template <typename T>
void urv_factor(Ctx& cx, HSS2<T>& H) {
  TmpScope scope_(cx);
  Plan* P = cx.P;
  const int np = (int)H.probs.size();
  int Lmax = 0;
  for (auto& pb : H.probs) Lmax = std::max(Lmax, pb.L);

  // leaves: [U D]
  {
    std::vector<LeafDesc<T>> ld;
    std::vector<CopyDesc<T, T>> cd;
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      const Problem& q = P->probs[p];
      if (pb.L == 0) {
        pb.root_m = (int)q.M;
        pb.root_n = (int)q.N();
        pb.rootA.r = pb.root_m;
        pb.rootA.c = pb.root_n;
        std::vector<Mat<T>*> m1{&pb.rootA};
        H.mem.push_back(carve(P->arena, m1));
        LeafDesc<T> d{};
        d.row0 = q.m0;
        d.m = (int)q.M;
        d.nx = q.nx;
        d.ny = q.ny;
        d.colx0 = 0;
        d.dx = q.nx;
        d.coly0 = 0;
        d.dy = q.ny;
        d.out = pb.rootA.p;
        d.ld = pb.rootA.ld;
        d.coff = 0;
        ld.push_back(d);
        continue;
      }
      std::vector<Mat<T>*> mu;
      for (auto& nd : pb.lv[pb.L]) {
        nd.mm = (int)nd.m;
        nd.nn = nd.n;
        nd.UD.r = nd.mm;
        nd.UD.c = nd.wU + nd.nn;
        mu.push_back(&nd.UD);
      }
      H.mem.push_back(carve(P->arena, mu));
      for (auto& nd : pb.lv[pb.L]) {
        nd.Vm = nd.V;
        if (nd.wU > 0 && nd.mm > 0) cd.push_back({nd.mm, nd.wU, nd.U.ld, nd.UD.ld, nd.U.p, nd.UD.p, 0});
        LeafDesc<T> d{};
        d.row0 = nd.row0;
        d.m = nd.mm;
        d.nx = q.nx;
        d.ny = q.ny;
        d.colx0 = q.colx[pb.L][nd.a];
        d.dx = nd.dx;
        d.coly0 = q.coly[pb.L][nd.b];
        d.dy = nd.dy;
        d.out = nd.UD.p;
        d.ld = nd.UD.ld;
        d.coff = nd.wU;
        if (nd.mm > 0) ld.push_back(d);
      }
    }
    copy_batched<T, T>(cx.pool, cd);
    gen_leafD<T>(cx.pool, ld, P->pts_2d);
  }

  for (int h = 0; h < Lmax; ++h) {
    struct Ref { int p, l, z; };
    std::vector<Ref> nodes;
    for (int p = 0; p < np; ++p) {
      int l = H.probs[p].L - h;
      if (l < 1) continue;
      for (int z = 0; z < (1 << (2 * l)); ++z) nodes.push_back({p, l, z});
    }
    auto N = [&](const Ref& r) -> Node2<T>& { return H.probs[r.p].lv[r.l][r.z]; };
    // ---- allocations of this height
    std::vector<Mat<T>> Rr(nodes.size());
    {
      std::vector<Mat<T>*> mp, mt;
      for (size_t i = 0; i < nodes.size(); ++i) {
        Node2<T>& nd = N(nodes[i]);
        nd.sizered = nd.mm >= nd.nn + nd.wU && nd.mm > 0;
        nd.mchk = nd.sizered ? nd.nn + nd.wU : nd.mm;
        nd.k = std::max(nd.nn - nd.wV, 0);
        nd.nu = nd.nn - nd.k;
        if (nd.mchk < nd.k)
          throw Error(NUDFT2_E_SINGULAR, "a tree node has fewer sample points than unknowns to eliminate");
        nd.pr = nd.mchk - nd.k;
        if (nd.sizered) {
          nd.Tom.r = (int)qr_tsize(nd.mm, nd.wU + nd.nn);
          nd.Tom.c = 1;
          mp.push_back(&nd.Tom);
          Rr[i].r = nd.mchk;
          Rr[i].c = nd.wU + nd.nn;
          mt.push_back(&Rr[i]);
        }
        if (nd.k > 0) {
          nd.Tq.r = (int)qr_tsize(nd.nn, nd.wV);
          nd.Tq.c = 1;
          nd.V2.r = nd.wV;
          nd.V2.c = nd.wV;
          nd.Tp.r = (int)qr_tsize(nd.mchk, nd.k);
          nd.Tp.c = 1;
          nd.D11.r = nd.k;
          nd.D11.c = nd.k;
          mp.push_back(&nd.Tq);
          mp.push_back(&nd.V2);
          mp.push_back(&nd.Tp);
          mp.push_back(&nd.D11);
        }
        nd.Wm.r = nd.mchk;
        nd.Wm.c = nd.nn + nd.wU;
        mp.push_back(&nd.Wm);
      }
      H.mem.push_back(carve(P->arena, mp));
      carve(P->arena, mt, &cx.tmp);
    }
    // ---- size reduction
    {
      ProfSite site_(PS_URV_SIZERED);
      std::vector<QRDesc<T>> qd;
      for (size_t i = 0; i < nodes.size(); ++i) {
        Node2<T>& nd = N(nodes[i]);
        if (nd.sizered)
          qd.push_back({nd.mm, nd.wU + nd.nn, nd.UD.ld, Rr[i].ld, nd.UD.p, Rr[i].p, nd.Tom.p});
      }
      if (!qd.empty()) geqrf_batched<T>(cx.pool, qd, cx.tmp_alloc(qr_workspace<T>(qd)));
    }
    // U' and D' views
    std::vector<Mat<T>> Uc(nodes.size()), Dc(nodes.size());
    for (size_t i = 0; i < nodes.size(); ++i) {
      Node2<T>& nd = N(nodes[i]);
      const Mat<T>& src = nd.sizered ? Rr[i] : nd.UD;
      Uc[i] = src.sub(0, 0, nd.mchk, nd.wU);
      Dc[i] = src.sub(0, nd.wU, nd.mchk, nd.nn);
    }
    // ---- basis elimination: QR of V
    {
      ProfSite site_(PS_URV_VQR);
      std::vector<QRDesc<T>> qd;
      for (size_t i = 0; i < nodes.size(); ++i) {
        Node2<T>& nd = N(nodes[i]);
        if (nd.k > 0) qd.push_back({nd.nn, nd.wV, nd.Vm.ld, nd.V2.ld, nd.Vm.p, nd.V2.p, nd.Tq.p});
        else nd.V2 = nd.Vm;   // nu = nn unknowns pass up unchanged
      }
      if (!qd.empty()) geqrf_batched<T>(cx.pool, qd, cx.tmp_alloc(qr_workspace<T>(qd)));
    }
    // ---- W = [D~(:,0:k) | U' | D~(:,k:)] with D~ = D' Q
    {
      ProfSite site_(PS_URV_DQ);
      std::vector<Mat<T>> X(nodes.size());
      std::vector<Mat<T>*> mx;
      for (size_t i = 0; i < nodes.size(); ++i) {
        Node2<T>& nd = N(nodes[i]);
        if (nd.k > 0) {
          X[i].r = nd.nn;
          X[i].c = nd.mchk;
          mx.push_back(&X[i]);
        }
      }
      carve(P->arena, mx, &cx.tmp);
      std::vector<CopyDesc<T, T>> c1, c2;
      std::vector<OrmDesc<T>> od;
      for (size_t i = 0; i < nodes.size(); ++i) {
        Node2<T>& nd = N(nodes[i]);
        if (nd.k > 0) {
          c1.push_back({nd.mchk, nd.nn, Dc[i].ld, X[i].ld, Dc[i].p, X[i].p, 1});
          od.push_back({nd.nn, nd.wV, nd.mchk, nd.Vm.ld, X[i].ld, nd.Vm.p, nd.Tq.p, X[i].p});
          // W(:, 0:k) = (X'(wV:nn, :))^H ; W(:, k+wU:) = (X'(0:wV, :))^H ; W(:, k:k+wU) = U'
          c2.push_back({nd.k, nd.mchk, X[i].ld, nd.Wm.ld, X[i].p + nd.wV, nd.Wm.p, 1});
          c2.push_back({nd.wV, nd.mchk, X[i].ld, nd.Wm.ld, X[i].p, nd.Wm.at(0, nd.k + nd.wU), 1});
          if (nd.wU > 0) c2.push_back({nd.mchk, nd.wU, Uc[i].ld, nd.Wm.ld, Uc[i].p, nd.Wm.at(0, nd.k), 0});
        } else {
          if (nd.wU > 0) c2.push_back({nd.mchk, nd.wU, Uc[i].ld, nd.Wm.ld, Uc[i].p, nd.Wm.p, 0});
          if (nd.nn > 0) c2.push_back({nd.mchk, nd.nn, Dc[i].ld, nd.Wm.ld, Dc[i].p, nd.Wm.at(0, nd.wU), 0});
        }
      }
      copy_batched<T, T>(cx.pool, c1);
      if (!od.empty()) ormqr_batched<T>(cx.pool, od, true, cx.tmp_alloc(orm_workspace<T>(od)));
      copy_batched<T, T>(cx.pool, c2);
    }
    // ---- partial decomposition
    {
      ProfSite site_(PS_URV_PARTIAL);
      std::vector<QRDesc<T>> qd;
      std::vector<OrmDesc<T>> od;
      for (size_t i = 0; i < nodes.size(); ++i) {
        Node2<T>& nd = N(nodes[i]);
        if (nd.k == 0) continue;
        qd.push_back({nd.mchk, nd.k, nd.Wm.ld, nd.D11.ld, nd.Wm.p, nd.D11.p, nd.Tp.p});
        if (nd.wU + nd.nu > 0)
          od.push_back({nd.mchk, nd.k, nd.wU + nd.nu, nd.Wm.ld, nd.Wm.ld, nd.Wm.p, nd.Tp.p,
                        nd.Wm.at(0, nd.k)});
      }
      if (!qd.empty()) geqrf_batched<T>(cx.pool, qd, cx.tmp_alloc(qr_workspace<T>(qd)));
      if (!od.empty()) ormqr_batched<T>(cx.pool, od, true, cx.tmp_alloc(orm_workspace<T>(od)));
    }
    P->arena.check("URV level");
    // ---- merge into the parents
    {
      ProfSite site_(PS_URV_MERGE);
      struct PRef { int p, l, z; };
      std::vector<PRef> par;
      for (int p = 0; p < np; ++p) {
        int l = H.probs[p].L - h - 1;
        if (l < 0) continue;
        for (int z = 0; z < (1 << (2 * l)); ++z) par.push_back({p, l, z});
      }
      std::vector<Mat<T>*> mp;
      for (auto& r : par) {
        Prob2<T>& pb = H.probs[r.p];
        int mm = 0, nn = 0;
        for (int c = 0; c < 4; ++c) {
          const Node2<T>& ch = pb.lv[r.l + 1][4 * r.z + c];
          mm += ch.pr;
          nn += ch.nu;
        }
        if (r.l == 0) {
          pb.root_m = mm;
          pb.root_n = nn;
          pb.rootA.r = mm;
          pb.rootA.c = nn;
          mp.push_back(&pb.rootA);
        } else {
          Node2<T>& nd = pb.lv[r.l][r.z];
          nd.mm = mm;
          nd.nn = nn;
          nd.UD.r = mm;
          nd.UD.c = nd.wU + nn;
          nd.Vm.r = nn;
          nd.Vm.c = nd.wV;
          mp.push_back(&nd.UD);
          mp.push_back(&nd.Vm);
        }
      }
      H.mem.push_back(carve(P->arena, mp));
      // X_ij = B_ij V2_j^H (rU_i x nu_j), then D+_ij = U2_i X_ij
      std::vector<Mat<T>> Xs;
      std::vector<std::tuple<int, int, int, int>> xref;   // (par idx, i, j, slot)
      for (size_t pi = 0; pi < par.size(); ++pi)
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j)
            if (i != j) xref.push_back({(int)pi, i, j, sib_slot<T>(i, j)});
      Xs.resize(xref.size());
      std::vector<Mat<T>*> mx;
      for (size_t t = 0; t < xref.size(); ++t) {
        auto [pi, i, j, s] = xref[t];
        Prob2<T>& pb = H.probs[par[pi].p];
        const Node2<T>& ci = pb.lv[par[pi].l + 1][4 * par[pi].z + i];
        const Node2<T>& cj = pb.lv[par[pi].l + 1][4 * par[pi].z + j];
        Xs[t].r = ci.wU;
        Xs[t].c = cj.nu;
        mx.push_back(&Xs[t]);
        (void)s;
      }
      carve(P->arena, mx, &cx.tmp);
      std::vector<GemmDesc<T>> gx, gd, gu, gv;
      std::vector<CopyDesc<T, T>> cd;
      for (size_t t = 0; t < xref.size(); ++t) {
        auto [pi, i, j, s] = xref[t];
        Prob2<T>& pb = H.probs[par[pi].p];
        const Node2<T>& ci = pb.lv[par[pi].l + 1][4 * par[pi].z + i];
        const Node2<T>& cj = pb.lv[par[pi].l + 1][4 * par[pi].z + j];
        if (ci.wU > 0 && cj.nu > 0)
          // V2 is the upper-triangular factor of the basis elimination when
          // the node eliminated unknowns (k > 0), else the basis itself
          gx.push_back({ci.wU, cj.nu, cj.wV, ci.B[s].ld, cj.V2.ld, Xs[t].ld, ci.B[s].p, cj.V2.p,
                        Xs[t].p, T(1), T(0), T(0), 0, 0, cj.k > 0 ? 2 : 0});
      }
      gemm_batched<T>(cx.pool, gx, OpN, OpC);
      for (size_t pi = 0; pi < par.size(); ++pi) {
        Prob2<T>& pb = H.probs[par[pi].p];
        const bool root = par[pi].l == 0;
        Mat<T> dst = root ? pb.rootA : pb.lv[par[pi].l][par[pi].z].UD;
        int dcol = root ? 0 : pb.lv[par[pi].l][par[pi].z].wU;
        int roff[5] = {0}, coff[5] = {0};
        for (int c = 0; c < 4; ++c) {
          const Node2<T>& ch = pb.lv[par[pi].l + 1][4 * par[pi].z + c];
          roff[c + 1] = roff[c] + ch.pr;
          coff[c + 1] = coff[c] + ch.nu;
        }
        for (int i = 0; i < 4; ++i) {
          const Node2<T>& ci = pb.lv[par[pi].l + 1][4 * par[pi].z + i];
          Mat<T> U2 = ci.Wm.sub(ci.k, ci.k, ci.pr, ci.wU);
          Mat<T> D22 = ci.Wm.sub(ci.k, ci.k + ci.wU, ci.pr, ci.nu);
          if (ci.pr > 0 && ci.nu > 0)
            cd.push_back({ci.pr, ci.nu, D22.ld, dst.ld, D22.p, dst.at(roff[i], dcol + coff[i]), 0});
          if (!root) {
            const Node2<T>& nd = pb.lv[par[pi].l][par[pi].z];
            if (ci.pr > 0 && nd.wU > 0)
              gu.push_back({ci.pr, nd.wU, ci.wU, U2.ld, ci.R.ld, dst.ld, U2.p, ci.R.p,
                            dst.at(roff[i], 0), T(1), T(0), T(0)});
            if (ci.nu > 0 && nd.wV > 0)
              gv.push_back({ci.nu, nd.wV, ci.wV, ci.V2.ld, ci.W.ld, nd.Vm.ld, ci.V2.p, ci.W.p,
                            nd.Vm.at(coff[i], 0), T(1), T(0), T(0), 0, ci.k > 0 ? 2 : 0});
          }
        }
      }
      for (size_t t = 0; t < xref.size(); ++t) {
        auto [pi, i, j, s] = xref[t];
        (void)s;
        Prob2<T>& pb = H.probs[par[pi].p];
        const bool root = par[pi].l == 0;
        Mat<T> dst = root ? pb.rootA : pb.lv[par[pi].l][par[pi].z].UD;
        int dcol = root ? 0 : pb.lv[par[pi].l][par[pi].z].wU;
        int roff = 0, coff = 0;
        for (int c = 0; c < i; ++c) roff += pb.lv[par[pi].l + 1][4 * par[pi].z + c].pr;
        for (int c = 0; c < j; ++c) coff += pb.lv[par[pi].l + 1][4 * par[pi].z + c].nu;
        const Node2<T>& ci = pb.lv[par[pi].l + 1][4 * par[pi].z + i];
        const Node2<T>& cj = pb.lv[par[pi].l + 1][4 * par[pi].z + j];
        Mat<T> U2 = ci.Wm.sub(ci.k, ci.k, ci.pr, ci.wU);
        if (ci.pr > 0 && cj.nu > 0) {
          if (ci.wU > 0)
            gd.push_back({ci.pr, cj.nu, ci.wU, U2.ld, Xs[t].ld, dst.ld, U2.p, Xs[t].p,
                          dst.at(roff, dcol + coff), T(1), T(0), T(0)});
          else {
            std::vector<FillDesc<T>> f{{ci.pr, cj.nu, dst.ld, dst.at(roff, dcol + coff), 0}};
            fill_batched<T>(cx.pool, f);
          }
        }
      }
      copy_batched<T, T>(cx.pool, cd);
      gemm_batched<T>(cx.pool, gd, OpN, OpN);
      gemm_batched<T>(cx.pool, gu, OpN, OpN);
      gemm_batched<T>(cx.pool, gv, OpN, OpN);
    }
    cx.release_tmp();
    cx.pool.sync_reset();
  }
  // root least squares: QR of the merged root block
  {
    std::vector<QRDesc<T>> qd;
    std::vector<Mat<T>*> mp;
    for (auto& pb : H.probs) {
      if (pb.root_m < pb.root_n)
        throw Error(NUDFT2_E_SINGULAR, "root block has fewer rows than unknowns");
      pb.rootR.r = pb.root_n;
      pb.rootR.c = pb.root_n;
      pb.rootT.r = (int)qr_tsize(pb.root_m, pb.root_n);
      pb.rootT.c = 1;
      mp.push_back(&pb.rootR);
      mp.push_back(&pb.rootT);
    }
    H.mem.push_back(carve(P->arena, mp));
    for (auto& pb : H.probs)
      if (pb.root_n > 0)
        qd.push_back({pb.root_m, pb.root_n, pb.rootA.ld, pb.rootR.ld, pb.rootA.p, pb.rootR.p,
                      pb.rootT.p});
    ProfSite site_(PS_URV_ROOT);
    if (!qd.empty()) geqrf_batched<T>(cx.pool, qd, cx.tmp_alloc(qr_workspace<T>(qd)));
  }
  // The solves need D11^{-1} and R^{-1} only: invert every node's triangle
  // and the root's in place, so that each triangular solve of a sweep is one
  // batched matrix-vector product instead of a chain of blocked substitutions.
  {
    ProfSite site_(PS_URV_INV);
    std::vector<TriDesc<T>> td;
    for (auto& pb : H.probs) {
      for (int l = 1; l <= pb.L; ++l)
        for (auto& nd : pb.lv[l])
          if (nd.k > 0) td.push_back({nd.k, nd.D11.ld, nd.D11.p});
      if (pb.root_n > 0) td.push_back({pb.root_n, pb.rootR.ld, pb.rootR.p});
    }
    if (!td.empty()) trtri_upper_batched<T>(cx.pool, td, cx.tmp_alloc(trtri_workspace<T>(td)));
    cx.release_tmp();
    cx.pool.sync_reset();
  }
}

template <typename T>
void urv_solve(Ctx& cx, HSS2<T>& H, cplx<T>* f, int64_t ldf, cplx<T>* c, int64_t ldc, int nrhs) {
  TmpScope scope_(cx);
  Plan* P = cx.P;
  const int np = (int)H.probs.size();
  int Lmax = 0;
  for (auto& pb : H.probs) Lmax = std::max(Lmax, pb.L);
  // per node right-hand-side buffers: leaves use f in place
  std::vector<std::vector<std::vector<Mat<T>>>> F(np), Cp(np), Bh(np), Z(np);
  for (int p = 0; p < np; ++p) {
    Prob2<T>& pb = H.probs[p];
    F[p].resize(pb.L + 1);
    Cp[p].resize(pb.L + 1);
    Bh[p].resize(pb.L + 1);
    Z[p].resize(pb.L + 1);
    for (int l = 0; l <= pb.L; ++l) {
      size_t nn = (size_t)1 << (2 * l);
      F[p][l].resize(nn);
      Cp[p][l].resize(nn);
      Bh[p][l].resize(nn);
      Z[p][l].resize(nn);
    }
  }
  std::vector<Mat<T>*> mtmp;
  std::vector<Mat<T>> Rt(np);   // the root's R^{-1} Q^H f
  for (int p = 0; p < np; ++p) {
    Rt[p].r = std::max(H.probs[p].root_n, 1);
    Rt[p].c = nrhs;
    mtmp.push_back(&Rt[p]);
  }
  for (int p = 0; p < np; ++p) {
    Prob2<T>& pb = H.probs[p];
    const Problem& q = P->probs[p];
    if (pb.L == 0) {
      Mat<T> m;
      m.p = f + q.m0;
      m.r = (int)q.M;
      m.c = nrhs;
      m.ld = (int)ldf;
      F[p][0][0] = m;
      continue;
    }
    for (auto& nd : pb.lv[pb.L]) {
      Mat<T> m;
      m.p = f + nd.row0;
      m.r = (int)nd.m;
      m.c = nrhs;
      m.ld = (int)ldf;
      F[p][pb.L][nd.z] = m;
      Mat<T> cm;
      cm.p = c + q.c0 + nd.col0;
      cm.r = nd.n;
      cm.c = nrhs;
      cm.ld = (int)ldc;
      Cp[p][pb.L][nd.z] = cm;
    }
    for (int l = 0; l < pb.L; ++l)
      for (int z = 0; z < (1 << (2 * l)); ++z) {
        Mat<T>& m = F[p][l][z];
        m.r = l == 0 ? pb.root_m : pb.lv[l][z].mm;
        m.c = nrhs;
        mtmp.push_back(&m);
        if (l >= 1) {
          Mat<T>& cm = Cp[p][l][z];
          cm.r = pb.lv[l][z].nn;
          cm.c = nrhs;
          mtmp.push_back(&cm);
        }
      }
    for (int l = 1; l <= pb.L; ++l)
      for (int z = 0; z < (1 << (2 * l)); ++z) {
        Mat<T>& b = Bh[p][l][z];
        b.r = pb.lv[l][z].wU;
        b.c = nrhs;
        mtmp.push_back(&b);
        Mat<T>& zz = Z[p][l][z];
        zz.r = pb.lv[l][z].wV;
        zz.c = nrhs;
        mtmp.push_back(&zz);
      }
  }
  carve(P->arena, mtmp, &cx.tmp);

  // ---- bottom-up: Omega^H, P^H, stack f2 into the parent
  for (int h = 0; h < Lmax; ++h) {
    std::vector<OrmDesc<T>> o1, o2;
    std::vector<CopyDesc<T, T>> cd;
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      int l = pb.L - h;
      if (l < 1) continue;
      for (auto& nd : pb.lv[l]) {
        Mat<T>& fm = F[p][l][nd.z];
        if (nd.sizered)
          o1.push_back({nd.mm, nd.mchk, nrhs, nd.UD.ld, fm.ld, nd.UD.p, nd.Tom.p, fm.p});
        if (nd.k > 0) o2.push_back({nd.mchk, nd.k, nrhs, nd.Wm.ld, fm.ld, nd.Wm.p, nd.Tp.p, fm.p});
      }
      for (int z = 0; z < (1 << (2 * (l - 1))); ++z) {
        int off = 0;
        Mat<T>& fp = F[p][l - 1][z];
        for (int c = 0; c < 4; ++c) {
          const Node2<T>& ch = pb.lv[l][4 * z + c];
          Mat<T>& fc = F[p][l][4 * z + c];
          if (ch.pr > 0) cd.push_back({ch.pr, nrhs, fc.ld, fp.ld, fc.at(ch.k, 0), fp.at(off, 0), 0});
          off += ch.pr;
        }
      }
    }
    if (!o1.empty()) ormqr_batched<T>(cx.pool, o1, true, cx.tmp_alloc(orm_workspace<T>(o1)));
    if (!o2.empty()) ormqr_batched<T>(cx.pool, o2, true, cx.tmp_alloc(orm_workspace<T>(o2)));
    copy_batched<T, T>(cx.pool, cd);
  }
  // ---- root least squares: Q^H f, then R^{-1} (stored inverted) through a
  // temporary and back into the root's buffer
  {
    std::vector<OrmDesc<T>> od;
    std::vector<GemmDesc<T>> gr;
    std::vector<CopyDesc<T, T>> cr;
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      Mat<T>& fr = F[p][0][0];
      if (pb.root_n == 0) continue;
      od.push_back({pb.root_m, pb.root_n, nrhs, pb.rootA.ld, fr.ld, pb.rootA.p, pb.rootT.p, fr.p});
      Mat<T>& t = Rt[p];
      gr.push_back({pb.root_n, nrhs, pb.root_n, pb.rootR.ld, fr.ld, t.ld, pb.rootR.p, fr.p, t.p,
                    T(1), T(0), T(0), 0, 2});
      cr.push_back({pb.root_n, nrhs, t.ld, fr.ld, t.p, fr.p, 0});
    }
    ormqr_batched<T>(cx.pool, od, true, cx.tmp_alloc(orm_workspace<T>(od)));
    gemm_batched<T>(cx.pool, gr, OpN, OpN);
    copy_batched<T, T>(cx.pool, cr);
    // L == 0: the root solution is the leaf solution
    std::vector<CopyDesc<T, T>> cd;
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      if (pb.L != 0) continue;
      const Problem& q = P->probs[p];
      cd.push_back({pb.root_n, nrhs, F[p][0][0].ld, (int)ldc, F[p][0][0].p, c + q.c0, 0});
    }
    copy_batched<T, T>(cx.pool, cd);
  }
  // ---- top-down substitution
  for (int l = 1; l <= Lmax; ++l) {
    std::vector<GemmDesc<T>> gz, gbs[3], gbr, g12, gu1, gd1;
    std::vector<CopyDesc<T, T>> cc2;
    std::vector<OrmDesc<T>> oq;
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      if (l > pb.L) continue;
      for (auto& nd : pb.lv[l]) {
        int zp = nd.z >> 2;
        const Mat<T>& cpar = (l == 1) ? F[p][0][0] : Cp[p][l - 1][zp];
        int off = 0;
        for (int c = 0; c < (nd.z & 3); ++c) off += pb.lv[l][(nd.z & ~3) + c].nu;
        Mat<T> c2 = cpar.sub(off, 0, nd.nu, nrhs);
        // z = V2^H c2
        if (nd.wV > 0 && nd.nu > 0)
          gz.push_back({nd.wV, nrhs, nd.nu, nd.V2.ld, c2.ld, Z[p][l][nd.z].ld, nd.V2.p, c2.p,
                        Z[p][l][nd.z].p, T(1), T(0), T(0), 0, nd.k > 0 ? 2 : 0});
        else if (nd.wV > 0) {
          std::vector<FillDesc<T>> fz{{nd.wV, nrhs, Z[p][l][nd.z].ld, Z[p][l][nd.z].p, 0}};
          fill_batched<T>(cx.pool, fz);
        }
        // c+ assembly buffer: [c2; c1] then Q0 (k > 0), or c2 itself (k == 0)
        Mat<T>& cp = Cp[p][l][nd.z];
        if (nd.nu > 0) cc2.push_back({nd.nu, nrhs, c2.ld, cp.ld, c2.p, cp.p, 0});
      }
    }
    gemm_batched<T>(cx.pool, gz, OpC, OpN);
    copy_batched<T, T>(cx.pool, cc2);
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      if (l > pb.L) continue;
      for (auto& nd : pb.lv[l]) {
        Mat<T>& b = Bh[p][l][nd.z];
        if (nd.wU == 0) continue;
        int c = nd.z & 3;
        for (int s = 0; s < 3; ++s) {
          int zs = (nd.z & ~3) | (s < c ? s : s + 1);
          const Node2<T>& sb = pb.lv[l][zs];
          gbs[s].push_back({nd.wU, nrhs, sb.wV, nd.B[s].ld, Z[p][l][zs].ld, b.ld, nd.B[s].p,
                            Z[p][l][zs].p, b.p, T(1), T(0), s == 0 ? T(0) : T(1)});
        }
        if (l >= 2) {
          const Node2<T>& par = pb.lv[l - 1][nd.z >> 2];
          if (par.wU > 0)
            gbr.push_back({nd.wU, nrhs, par.wU, nd.R.ld, Bh[p][l - 1][par.z].ld, b.ld, nd.R.p,
                           Bh[p][l - 1][par.z].p, b.p, T(1), T(0), T(1)});
        }
      }
    }
    for (int s = 0; s < 3; ++s) gemm_batched<T>(cx.pool, gbs[s], OpN, OpN);
    gemm_batched<T>(cx.pool, gbr, OpN, OpN);
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      if (l > pb.L) continue;
      for (auto& nd : pb.lv[l]) {
        if (nd.k == 0) continue;
        Mat<T>& fm = F[p][l][nd.z];
        Mat<T>& cp = Cp[p][l][nd.z];
        Mat<T> U1 = nd.Wm.sub(0, nd.k, nd.k, nd.wU);
        Mat<T> D12 = nd.Wm.sub(0, nd.k + nd.wU, nd.k, nd.nu);
        if (nd.nu > 0)
          g12.push_back({nd.k, nrhs, nd.nu, D12.ld, cp.ld, fm.ld, D12.p, cp.p, fm.p, T(-1), T(0),
                         T(1)});
        if (nd.wU > 0)
          gu1.push_back({nd.k, nrhs, nd.wU, U1.ld, Bh[p][l][nd.z].ld, fm.ld, U1.p,
                         Bh[p][l][nd.z].p, fm.p, T(-1), T(0), T(1)});
        // c1 = D11^{-1} (f1 - D12 c2 - U1 b), straight into the c+ buffer
        gd1.push_back({nd.k, nrhs, nd.k, nd.D11.ld, fm.ld, cp.ld, nd.D11.p, fm.p,
                       cp.at(nd.nu, 0), T(1), T(0), T(0), 0, 2});
        oq.push_back({nd.nn, nd.wV, nrhs, nd.Vm.ld, cp.ld, nd.Vm.p, nd.Tq.p, cp.p});
      }
    }
    gemm_batched<T>(cx.pool, g12, OpN, OpN);
    gemm_batched<T>(cx.pool, gu1, OpN, OpN);
    gemm_batched<T>(cx.pool, gd1, OpN, OpN);
    if (!oq.empty()) ormqr_batched<T>(cx.pool, oq, false, cx.tmp_alloc(orm_workspace<T>(oq)));
  }
  cx.release_tmp();
  cx.pool.sync_reset();
}

// Adjoint of urv_solve: f = S^H c for the linear map S: f -> c of the solve
// above.  The steps run in reverse order with their adjoints: the top-down
// substitution backwards over the levels (Q0^H, D11^{-H}, the transposed B, R,
// V2 and U1, D12 couplings), the root least-squares step (R^{-H}, then Q),
// then the bottom-up sweep forwards (P, then Omega, with the rows dropped by
// the size reduction set to zero).  c (ldc x nrhs, quadtree column order) is
// overwritten; f (ldf x nrhs, 2D-sorted rows) receives the result.
template <typename T>
void urv_solve_adj(Ctx& cx, HSS2<T>& H, cplx<T>* c, int64_t ldc, cplx<T>* f, int64_t ldf,
                   int nrhs) {
  TmpScope scope_(cx);
  Plan* P = cx.P;
  const int np = (int)H.probs.size();
  int Lmax = 0;
  for (auto& pb : H.probs) Lmax = std::max(Lmax, pb.L);
  std::vector<std::vector<std::vector<Mat<T>>>> Fb(np), Cb(np), Bb(np), Zb(np);
  std::vector<Mat<T>*> mtmp;
  std::vector<Mat<T>> Rt(np);   // the root's R^{-H} c
  for (int p = 0; p < np; ++p) {
    Rt[p].r = std::max(H.probs[p].root_n, 1);
    Rt[p].c = nrhs;
    mtmp.push_back(&Rt[p]);
  }
  for (int p = 0; p < np; ++p) {
    Prob2<T>& pb = H.probs[p];
    const Problem& q = P->probs[p];
    Fb[p].resize(pb.L + 1);
    Cb[p].resize(pb.L + 1);
    Bb[p].resize(pb.L + 1);
    Zb[p].resize(pb.L + 1);
    for (int l = 0; l <= pb.L; ++l) {
      size_t nn = (size_t)1 << (2 * l);
      Fb[p][l].resize(nn);
      Cb[p][l].resize(nn);
      Bb[p][l].resize(nn);
      Zb[p][l].resize(nn);
    }
    if (pb.L == 0) {
      Mat<T> m;
      m.p = f + q.m0;
      m.r = (int)q.M;
      m.c = nrhs;
      m.ld = (int)ldf;
      Fb[p][0][0] = m;
      continue;
    }
    for (auto& nd : pb.lv[pb.L]) {
      Mat<T> m;
      m.p = f + nd.row0;
      m.r = (int)nd.m;
      m.c = nrhs;
      m.ld = (int)ldf;
      Fb[p][pb.L][nd.z] = m;
      Mat<T> cm;
      cm.p = c + q.c0 + nd.col0;
      cm.r = nd.n;
      cm.c = nrhs;
      cm.ld = (int)ldc;
      Cb[p][pb.L][nd.z] = cm;
    }
    for (int l = 0; l < pb.L; ++l)
      for (int z = 0; z < (1 << (2 * l)); ++z) {
        Mat<T>& m = Fb[p][l][z];
        m.r = l == 0 ? pb.root_m : pb.lv[l][z].mm;
        m.c = nrhs;
        mtmp.push_back(&m);
        if (l >= 1) {
          Mat<T>& cm = Cb[p][l][z];
          cm.r = pb.lv[l][z].nn;
          cm.c = nrhs;
          mtmp.push_back(&cm);
        }
      }
    for (int l = 1; l <= pb.L; ++l)
      for (int z = 0; z < (1 << (2 * l)); ++z) {
        Mat<T>& b = Bb[p][l][z];
        b.r = pb.lv[l][z].wU;
        b.c = nrhs;
        mtmp.push_back(&b);
        Mat<T>& zz = Zb[p][l][z];
        zz.r = pb.lv[l][z].wV;
        zz.c = nrhs;
        mtmp.push_back(&zz);
      }
  }
  carve(P->arena, mtmp, &cx.tmp);
  {
    std::vector<FillDesc<T>> fz;
    for (int p = 0; p < np; ++p)
      for (int l = 1; l <= H.probs[p].L; ++l)
        for (auto& b : Bb[p][l])
          if (b.r > 0) fz.push_back({b.r, nrhs, b.ld, b.p, 0});
    fill_batched<T>(cx.pool, fz);
  }

  // ---- adjoint of the top-down substitution
  for (int l = Lmax; l >= 1; --l) {
    std::vector<OrmDesc<T>> oq;
    std::vector<CopyDesc<T, T>> cpar;
    std::vector<GemmDesc<T>> gd1, g12, gu1, gz[3], gv, gr[4];
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      if (l > pb.L) continue;
      for (auto& nd : pb.lv[l]) {
        if (nd.k == 0) continue;
        Mat<T>& cb = Cb[p][l][nd.z];
        Mat<T>& fb = Fb[p][l][nd.z];
        oq.push_back({nd.nn, nd.wV, nrhs, nd.Vm.ld, cb.ld, nd.Vm.p, nd.Tq.p, cb.p});
        // f1-bar = D11^{-H} c1-bar (D11 stored inverted)
        gd1.push_back({nd.k, nrhs, nd.k, nd.D11.ld, cb.ld, fb.ld, nd.D11.p, cb.at(nd.nu, 0), fb.p,
                       T(1), T(0), T(0), 0, 2});
        Mat<T> U1 = nd.Wm.sub(0, nd.k, nd.k, nd.wU);
        Mat<T> D12 = nd.Wm.sub(0, nd.k + nd.wU, nd.k, nd.nu);
        if (nd.nu > 0)
          g12.push_back({nd.nu, nrhs, nd.k, D12.ld, fb.ld, cb.ld, D12.p, fb.p, cb.p, T(-1), T(0),
                         T(1)});
        if (nd.wU > 0)
          gu1.push_back({nd.wU, nrhs, nd.k, U1.ld, fb.ld, Bb[p][l][nd.z].ld, U1.p, fb.p,
                         Bb[p][l][nd.z].p, T(-1), T(0), T(1)});
      }
    }
    if (!oq.empty()) ormqr_batched<T>(cx.pool, oq, true, cx.tmp_alloc(orm_workspace<T>(oq)));
    gemm_batched<T>(cx.pool, gd1, OpC, OpN);
    gemm_batched<T>(cx.pool, g12, OpC, OpN);
    gemm_batched<T>(cx.pool, gu1, OpC, OpN);
    // Z-bar of a node: its siblings' b-bar through their interaction blocks
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      if (l > pb.L) continue;
      for (auto& nd : pb.lv[l]) {
        if (nd.wV == 0) continue;
        int cz = nd.z & 3;
        for (int s = 0; s < 3; ++s) {
          int zs = (nd.z & ~3) | (s < cz ? s : s + 1);
          const Node2<T>& sb = pb.lv[l][zs];
          const Mat<T>& Bs = sb.B[sib_slot<T>(zs & 3, cz)];
          gz[s].push_back({nd.wV, nrhs, sb.wU, Bs.ld, Bb[p][l][zs].ld, Zb[p][l][nd.z].ld, Bs.p,
                           Bb[p][l][zs].p, Zb[p][l][nd.z].p, T(1), T(0), s == 0 ? T(0) : T(1)});
        }
        if (nd.nu > 0)
          gv.push_back({nd.nu, nrhs, nd.wV, nd.V2.ld, Zb[p][l][nd.z].ld, Cb[p][l][nd.z].ld,
                        nd.V2.p, Zb[p][l][nd.z].p, Cb[p][l][nd.z].p, T(1), T(0), T(1), 0,
                        nd.k > 0 ? 2 : 0});
      }
    }
    for (int s = 0; s < 3; ++s) gemm_batched<T>(cx.pool, gz[s], OpC, OpN);
    gemm_batched<T>(cx.pool, gv, OpN, OpN);
    // c2-bar into the parent's slice; b-bar into the parent's b-bar
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      if (l > pb.L) continue;
      for (auto& nd : pb.lv[l]) {
        int zp = nd.z >> 2;
        Mat<T>& par = (l == 1) ? Fb[p][0][0] : Cb[p][l - 1][zp];
        int off = 0;
        for (int c2 = 0; c2 < (nd.z & 3); ++c2) off += pb.lv[l][(nd.z & ~3) + c2].nu;
        if (nd.nu > 0)
          cpar.push_back({nd.nu, nrhs, Cb[p][l][nd.z].ld, par.ld, Cb[p][l][nd.z].p, par.at(off, 0),
                          0});
        if (l >= 2) {
          const Node2<T>& pn = pb.lv[l - 1][zp];
          if (pn.wU > 0 && nd.wU > 0)
            gr[nd.z & 3].push_back({pn.wU, nrhs, nd.wU, nd.R.ld, Bb[p][l][nd.z].ld,
                                    Bb[p][l - 1][zp].ld, nd.R.p, Bb[p][l][nd.z].p,
                                    Bb[p][l - 1][zp].p, T(1), T(0), T(1)});
        }
      }
    }
    copy_batched<T, T>(cx.pool, cpar);
    for (int s = 0; s < 4; ++s) gemm_batched<T>(cx.pool, gr[s], OpC, OpN);
  }
  // ---- adjoint of the root least-squares step: f_root = Q [R^{-H} c_root; 0]
  {
    std::vector<CopyDesc<T, T>> cd, cr;
    std::vector<FillDesc<T>> fz;
    std::vector<GemmDesc<T>> gr;
    std::vector<OrmDesc<T>> od;
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      const Problem& q = P->probs[p];
      Mat<T>& fr = Fb[p][0][0];
      if (pb.L == 0) cd.push_back({pb.root_n, nrhs, (int)ldc, fr.ld, c + q.c0, fr.p, 0});
      if (pb.root_m > pb.root_n)
        fz.push_back({pb.root_m - pb.root_n, nrhs, fr.ld, fr.at(pb.root_n, 0), 0});
      if (pb.root_n == 0) continue;
      // R^{-H} (R stored inverted) through a temporary and back
      Mat<T>& t = Rt[p];
      gr.push_back({pb.root_n, nrhs, pb.root_n, pb.rootR.ld, fr.ld, t.ld, pb.rootR.p, fr.p, t.p,
                    T(1), T(0), T(0), 0, 2});
      cr.push_back({pb.root_n, nrhs, t.ld, fr.ld, t.p, fr.p, 0});
      od.push_back({pb.root_m, pb.root_n, nrhs, pb.rootA.ld, fr.ld, pb.rootA.p, pb.rootT.p, fr.p});
    }
    copy_batched<T, T>(cx.pool, cd);
    fill_batched<T>(cx.pool, fz);
    gemm_batched<T>(cx.pool, gr, OpC, OpN);
    copy_batched<T, T>(cx.pool, cr);
    if (!od.empty()) ormqr_batched<T>(cx.pool, od, false, cx.tmp_alloc(orm_workspace<T>(od)));
  }
  // ---- adjoint of the bottom-up sweep: unstack, P, Omega
  for (int l = 1; l <= Lmax; ++l) {
    std::vector<CopyDesc<T, T>> cd;
    std::vector<FillDesc<T>> fz;
    std::vector<OrmDesc<T>> o2, o1;
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      if (l > pb.L) continue;
      for (int z = 0; z < (1 << (2 * (l - 1))); ++z) {
        Mat<T>& fp = Fb[p][l - 1][z];
        int off = 0;
        for (int c2 = 0; c2 < 4; ++c2) {
          const Node2<T>& ch = pb.lv[l][4 * z + c2];
          Mat<T>& fc = Fb[p][l][4 * z + c2];
          if (ch.pr > 0) cd.push_back({ch.pr, nrhs, fp.ld, fc.ld, fp.at(off, 0), fc.at(ch.k, 0), 0});
          off += ch.pr;
        }
      }
      for (auto& nd : pb.lv[l]) {
        Mat<T>& fm = Fb[p][l][nd.z];
        if (nd.mm > nd.mchk) fz.push_back({nd.mm - nd.mchk, nrhs, fm.ld, fm.at(nd.mchk, 0), 0});
        if (nd.k > 0) o2.push_back({nd.mchk, nd.k, nrhs, nd.Wm.ld, fm.ld, nd.Wm.p, nd.Tp.p, fm.p});
        if (nd.sizered)
          o1.push_back({nd.mm, nd.mchk, nrhs, nd.UD.ld, fm.ld, nd.UD.p, nd.Tom.p, fm.p});
      }
    }
    copy_batched<T, T>(cx.pool, cd);
    fill_batched<T>(cx.pool, fz);
    if (!o2.empty()) ormqr_batched<T>(cx.pool, o2, false, cx.tmp_alloc(orm_workspace<T>(o2)));
    if (!o1.empty()) ormqr_batched<T>(cx.pool, o1, false, cx.tmp_alloc(orm_workspace<T>(o1)));
  }
  cx.release_tmp();
  cx.pool.sync_reset();
}

template void urv_factor<float>(Ctx&, HSS2<float>&);
template void urv_factor<double>(Ctx&, HSS2<double>&);
// Stored entries each step of urv_solve reads, without the zeros the
// products skip: the reflector blocks of Omega, P and Q0 (unit lower
// trapezoidal) with their compact-WY factors (upper triangular), V^_2
// (z = V^_2^H c2), the sibling couplings B and the parent transfer R (b^),
// D12 and U1, the inverted triangle D11, and the root's reflectors, factors
// and inverted triangle.
template <typename T>
int64_t urv_sweep_bytes(const HSS2<T>& H) {
  // m x min(m, n) reflectors (lower trapezoid with the unit diagonal) and the
  // upper triangles of their QR_OB-column compact-WY blocks
  auto refl = [](int m, int n) -> double {
    const double k = std::min(m, n);
    double e = (double)m * k - k * (k - 1) / 2;
    for (int j0 = 0; j0 < (int)k; j0 += QR_OB) {
      const double kb = std::min(QR_OB, (int)k - j0);
      e += kb * (kb + 1) / 2;
    }
    return e;
  };
  auto tri = [](int k) -> double { return (double)k * (k + 1) / 2; };
  double e = 0;
  for (const auto& pb : H.probs) {
    for (int l = 1; l <= pb.L; ++l)
      for (const auto& nd : pb.lv[l]) {
        if (nd.sizered) e += refl(nd.mm, nd.mchk);
        if (nd.k > 0) {
          e += refl(nd.mchk, nd.k);
          e += tri(nd.k) + (double)nd.k * nd.nu + (double)nd.k * nd.wU;
        }
        e += nd.k > 0 ? tri(nd.wV) : (double)nd.nu * nd.wV;   // V^_2 triangular when k > 0
        if (nd.wV > 0) e += refl(nd.nn, nd.wV);
        for (int s = 0; s < 3; ++s) e += (double)nd.B[s].r * nd.B[s].c;
        if (l >= 2) e += (double)nd.R.r * nd.R.c;
      }
    if (pb.root_n > 0) e += refl(pb.root_m, pb.root_n) + tri(pb.root_n);
  }
  return (int64_t)(e * sizeof(cplx<T>));
}

template int64_t urv_sweep_bytes<float>(const HSS2<float>&);
template int64_t urv_sweep_bytes<double>(const HSS2<double>&);
template void urv_solve<float>(Ctx&, HSS2<float>&, float2*, int64_t, float2*, int64_t, int);
template void urv_solve<double>(Ctx&, HSS2<double>&, double2*, int64_t, double2*, int64_t, int);
template void urv_solve_adj<float>(Ctx&, HSS2<float>&, float2*, int64_t, float2*, int64_t, int);
template void urv_solve_adj<double>(Ctx&, HSS2<double>&, double2*, int64_t, double2*, int64_t, int);

}  // namespace nd
