// Face-splitting HSS assembly (Theorem 3.3) and recompression (Section 2.3).
//
// Assembly: from the two 1D HSS matrices of G^x and G^y, every quadtree node
// xi = (alpha, beta) gets the generators of H = H^x . H^y on the product tree:
// explicit leaf bases U_xi, V_xi, and Kronecker-structured transfer (R, W) and
// sibling interaction (B) matrices for all four children of a node (the
// paper writes the first child out; the other three follow by selecting the
// child's own / sibling column groups, see gen.hip).
//
// Recompression, stage 1 (bottom-up, exact): thin QR of the leaf bases,
// B <- F B G^H between siblings, thin QR of the stacked [F_c R_c] and
// [G_c W_c] at every non-root node.  Stage 2 (top-down, truncation at eps):
// for every node alpha the row block C^U = [B_{alpha,beta} | R_alpha S_parent]
// and column block C^V = [B_{beta,alpha}^H | W_alpha S_parent] are compressed.
// Where the paper takes a truncated SVD, the rank decision here is a
// diagonally pivoted Cholesky factorization K ~ L L^H of the FP64 Gram
// K = C C^H with the trace rule (relative Frobenius error eps); the new basis
// is P = orth(L) and the weight passed to the children is the triangular
// factor T of L = P T (T T^H = P^H K P up to the discarded part, the role of
// S^2 in the paper).  The updates B <- P^H B Q, R <- P^H R, W <- Q^H W,
// U <- U P, V <- V Q and R_child <- R_child P, W_child <- W_child Q follow the
// paper.
#include <chrono>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <tuple>

#include "gen.h"
#include "hss.h"

namespace nd {

namespace {

template <typename T>
struct Builder {
  Ctx& cx;
  HSS2<T>& H;
  Plan* P;
  std::map<std::tuple<int, int, int>, void*> chunk;   // (problem, level, kind)
  enum { K_U, K_V, K_R, K_W, K_B, K_F, K_G, K_TU, K_TV };

  Builder(Ctx& c, HSS2<T>& h) : cx(c), H(h), P(c.P) {}

  void own(int p, int l, int kind, void* ptr, std::vector<void*>& old) {
    auto key = std::make_tuple(p, l, kind);
    auto it = chunk.find(key);
    if (it != chunk.end() && it->second) old.push_back(it->second);
    chunk[key] = ptr;
  }
  void release(std::vector<void*>& old) {
    ND_HIP(hipStreamSynchronize(cx.s));
    for (void* p : old) P->arena.release(p);
    old.clear();
  }
  Node2<T>& node(int p, int l, int z) { return H.probs[p].lv[l][z]; }

  // nodes of every problem at level l (absolute level)
  template <typename F>
  void each_level(int l, F&& f) {
    for (int p = 0; p < (int)H.probs.size(); ++p) {
      if (l > H.probs[p].L) continue;
      for (int z = 0; z < (1 << (2 * l)); ++z) f(p, z);
    }
  }

  static int sib_child(int c, int s) { return s < c ? s : s + 1; }
  static int sib_slot(int c, int other) { return other < c ? other : other - 1; }
};

}  // namespace

// P = F Z for a face-split transfer matrix Z (kind 0: R, kind 1: W; Theorem
// 3.3) described by k: F is the node's stage-1 factor (ku x the node's basis
// width), P a row slab of the parent's stacked matrix (ku x the parent's
// width).  With the node's row groups g0 | g1 | g2 and the parent's column
// groups G0 | G1 | G2 (see Node2::KronRW), Z has the blocks
//   Z00 = S_own (x) Y,  Z11 = X (x) S_own,  Z22 = X (x) Y   (R and W),
//   Z20 = BX_sib (x) Y, Z21 = X (x) BY_sib                 (R only),
// where S_own places the node's x (y) columns at their offset in the
// parent's and BX_sib (BY_sib) places the sibling term at the sibling's
// columns.  Own and sibling columns partition G0 and G1, so each column of P
// comes from one term; every term is a batch of products with the small 1D
// factors (FP64 factors converted to the working precision first), through
// T1 = F(:, g2) (I (x) Y) and T2 = F(:, g2) (I (x) BY) for the two-factor
// terms.  P is cleared first (W has no sibling terms).
template <typename T>
struct KronJob {
  int kind;
  const typename Node2<T>::KronRW* k;
  Mat<T> F;   // ku x (dx ry + rx dy + rx ry)
  Mat<T> P;   // ku x (cdx cry + crx cdy + crx cry)
};

template <typename T>
static void kron_transfer_products(Ctx& cx, const std::vector<KronJob<T>>& jobs) {
  Plan* P = cx.P;
  const size_t nj = jobs.size();
  std::vector<Mat<T>> Xc(nj), Yc(nj), BXc(nj), BYc(nj), T1(nj), T2(nj);
  std::vector<Mat<T>*> mk;
  for (size_t i = 0; i < nj; ++i) {
    const auto& k = *jobs[i].k;
    const int ku = jobs[i].F.r;
    Xc[i].r = k.rx; Xc[i].c = k.crx;
    Yc[i].r = k.ry; Yc[i].c = k.cry;
    T1[i].r = ku; T1[i].c = k.rx * k.cry;
    mk.push_back(&Xc[i]);
    mk.push_back(&Yc[i]);
    mk.push_back(&T1[i]);
    if (jobs[i].kind == 0) {
      BXc[i].r = k.rx; BXc[i].c = k.dsx;
      BYc[i].r = k.ry; BYc[i].c = k.dsy;
      T2[i].r = ku; T2[i].c = k.rx * k.dsy;
      mk.push_back(&BXc[i]);
      mk.push_back(&BYc[i]);
      mk.push_back(&T2[i]);
    }
  }
  carve(P->arena, mk, &cx.tmp);
  std::vector<FillDesc<T>> fz;
  std::vector<CopyDesc<T, double>> cd;
  std::vector<GemmDesc<T>> g1, g2;
  auto conv = [&](const double2* src, int ld, Mat<T>& dst) {
    if (dst.r > 0 && dst.c > 0) cd.push_back({dst.r, dst.c, ld, dst.ld, src, dst.p, 0});
  };
  // C (m x n, ldc) = A (m x kk, lda) B (kk x n, ldb); skipped when empty
  auto mm = [](std::vector<GemmDesc<T>>& g, int m, int n, int kk, const cplx<T>* A, int64_t lda,
               const cplx<T>* B, int ldb, cplx<T>* C, int64_t ldc) {
    if (m > 0 && n > 0 && kk > 0)
      g.push_back({m, n, kk, (int)lda, ldb, (int)ldc, A, B, C, T(1), T(0), T(0)});
  };
  for (size_t i = 0; i < nj; ++i) {
    const auto& k = *jobs[i].k;
    const Mat<T>& F = jobs[i].F;
    const Mat<T>& Pm = jobs[i].P;
    const int ku = F.r;
    if (ku <= 0 || Pm.c <= 0) continue;
    fz.push_back({Pm.r, Pm.c, Pm.ld, Pm.p, 0});
    conv(k.X, k.ldX, Xc[i]);
    conv(k.Y, k.ldY, Yc[i]);
    const int64_t lf = F.ld, lp = Pm.ld;
    const int g1o = k.dx * k.ry, g2o = k.dx * k.ry + k.rx * k.dy;
    const int G1o = k.cdx * k.cry, G2o = k.cdx * k.cry + k.crx * k.cdy;
    // Z00: P(:, (own_x + u) cry + .) = F(:, u ry + .) Y
    for (int u = 0; u < k.dx; ++u)
      mm(g1, ku, k.cry, k.ry, F.p + (int64_t)u * k.ry * lf, lf, Yc[i].p, Yc[i].ld,
         Pm.p + (int64_t)(k.own_x + u) * k.cry * lp, lp);
    // Z11: P(:, G1 + u' cdy + own_y + v) = sum_u F(:, g1 + u dy + v) X(u, u')
    for (int v = 0; v < k.dy; ++v)
      mm(g1, ku, k.crx, k.rx, F.p + (int64_t)(g1o + v) * lf, (int64_t)k.dy * lf, Xc[i].p,
         Xc[i].ld, Pm.p + (int64_t)(G1o + k.own_y + v) * lp, (int64_t)k.cdy * lp);
    // T1(:, u cry + .) = F(:, g2 + u ry + .) Y
    for (int u = 0; u < k.rx; ++u)
      mm(g1, ku, k.cry, k.ry, F.p + (int64_t)(g2o + u * k.ry) * lf, lf, Yc[i].p, Yc[i].ld,
         T1[i].p + (int64_t)u * k.cry * T1[i].ld, T1[i].ld);
    // Z22: P(:, G2 + u' cry + w) = sum_u T1(:, u cry + w) X(u, u')
    for (int w = 0; w < k.cry; ++w)
      mm(g2, ku, k.crx, k.rx, T1[i].p + (int64_t)w * T1[i].ld, (int64_t)k.cry * T1[i].ld,
         Xc[i].p, Xc[i].ld, Pm.p + (int64_t)(G2o + w) * lp, (int64_t)k.cry * lp);
    if (jobs[i].kind != 0) continue;
    conv(k.BX, k.ldBX, BXc[i]);
    conv(k.BY, k.ldBY, BYc[i]);
    // T2(:, u dsy + .) = F(:, g2 + u ry + .) BY
    for (int u = 0; u < k.rx; ++u)
      mm(g1, ku, k.dsy, k.ry, F.p + (int64_t)(g2o + u * k.ry) * lf, lf, BYc[i].p, BYc[i].ld,
         T2[i].p + (int64_t)u * k.dsy * T2[i].ld, T2[i].ld);
    // Z20: P(:, (sib_x + q) cry + w) = sum_u T1(:, u cry + w) BX(u, q)
    for (int w = 0; w < k.cry; ++w)
      mm(g2, ku, k.dsx, k.rx, T1[i].p + (int64_t)w * T1[i].ld, (int64_t)k.cry * T1[i].ld,
         BXc[i].p, BXc[i].ld, Pm.p + (int64_t)(k.sib_x * k.cry + w) * lp, (int64_t)k.cry * lp);
    // Z21: P(:, G1 + u' cdy + sib_y + q) = sum_u T2(:, u dsy + q) X(u, u')
    for (int q = 0; q < k.dsy; ++q)
      mm(g2, ku, k.crx, k.rx, T2[i].p + (int64_t)q * T2[i].ld, (int64_t)k.dsy * T2[i].ld,
         Xc[i].p, Xc[i].ld, Pm.p + (int64_t)(G1o + k.sib_y + q) * lp, (int64_t)k.cdy * lp);
  }
  fill_batched<T>(cx.pool, fz);
  copy_batched<T, double>(cx.pool, cd);
  gemm_batched<T>(cx.pool, g1, OpN, OpN);
  gemm_batched<T>(cx.pool, g2, OpN, OpN);
}

template <typename T>
void build_2d(Ctx& cx, const std::vector<Tree1>& tx, const std::vector<Tree1>& ty, double eps,
              HSS2<T>& H, int stages) {
  TmpScope scope_(cx);
  Plan* P = cx.P;
  const auto t_start = std::chrono::steady_clock::now();
  Builder<T> bd(cx, H);
  const int np = (int)P->probs.size();
  H.probs.assign(np, Prob2<T>());
  int Lmax = 0;
  for (int p = 0; p < np; ++p) {
    const Problem& q = P->probs[p];
    Prob2<T>& pb = H.probs[p];
    pb.L = q.L;
    Lmax = std::max(Lmax, q.L);
    pb.lv.assign(q.L + 1, {});
    for (int l = 0; l <= q.L; ++l) {
      int nn = 1 << (2 * l);
      pb.lv[l].resize(nn);
      for (int z = 0; z < nn; ++z) {
        Node2<T>& nd = pb.lv[l][z];
        uint32_t a, b;
        deinterleave(z, l, a, b);
        nd.l = l;
        nd.z = z;
        nd.a = a;
        nd.b = b;
        nd.row0 = q.row2[l][z];
        nd.m = q.row2[l][z + 1] - q.row2[l][z];
        nd.col0 = q.col2[l][z];
        nd.n = q.col2[l][z + 1] - q.col2[l][z];
        nd.dx = q.colx[l][a + 1] - q.colx[l][a];
        nd.dy = q.coly[l][b + 1] - q.coly[l][b];
        if (l >= 1) {
          const Node1& ax = tx[p].lv[l][a];
          const Node1& by = ty[p].lv[l][b];
          nd.wU = nd.dx * by.rU + ax.rU * nd.dy + ax.rU * by.rU;
          nd.wV = nd.dx * by.rV + ax.rV * nd.dy + ax.rV * by.rV;
        }
      }
    }
  }
  if (Lmax == 0) return;
  std::vector<void*> old;

  // ------------------------------------------------ face-split assembly
  {
    ProfSite fs_site_(PS_FACESPLIT);
    // leaves
    std::vector<LeafDesc<T>> ud;
    std::vector<LeafVDesc<T>> vd;
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      if (pb.L == 0) continue;
      std::vector<Mat<T>*> mu, mv;
      for (auto& nd : pb.lv[pb.L]) {
        nd.U.r = (int)nd.m;
        nd.U.c = nd.wU;
        nd.V.r = nd.dx * nd.dy;
        nd.V.c = nd.wV;
        mu.push_back(&nd.U);
        mv.push_back(&nd.V);
      }
      bd.own(p, pb.L, Builder<T>::K_U, carve(P->arena, mu), old);
      bd.own(p, pb.L, Builder<T>::K_V, carve(P->arena, mv), old);
      const Problem& q = P->probs[p];
      for (auto& nd : pb.lv[pb.L]) {
        const Node1& ax = tx[p].lv[pb.L][nd.a];
        const Node1& by = ty[p].lv[pb.L][nd.b];
        LeafDesc<T> d{};
        d.row0 = nd.row0;
        d.m = (int)nd.m;
        d.nx = q.nx;
        d.ny = q.ny;
        d.colx0 = ax.col0;
        d.dx = nd.dx;
        d.coly0 = by.col0;
        d.dy = nd.dy;
        d.Ux = ax.U.p;
        d.ldux = ax.U.ld;
        d.rowx0 = ax.row0;
        d.rx = ax.rU;
        d.Uy = by.U.p;
        d.lduy = by.U.ld;
        d.rowy0 = by.row0;
        d.ry = by.rU;
        d.out = nd.U.p;
        d.ld = nd.U.ld;
        d.coff = 0;
        if (nd.m > 0 && nd.wU > 0) ud.push_back(d);
        LeafVDesc<T> v{nd.dx, nd.dy, ax.Vf.p, ax.Vf.ld, ax.rV, by.Vf.p, by.Vf.ld, by.rV, nd.V.p,
                       nd.V.ld};
        if (nd.wV > 0) vd.push_back(v);
      }
    }
    gen_leafU<T>(cx.pool, ud, P->pts_2d, P->posx, P->posy);
    gen_leafV<T>(cx.pool, vd);
    // transfer and interaction matrices
    std::vector<AsmDesc<T>> ad;
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      const Problem& q = P->probs[p];
      for (int l = 1; l <= pb.L; ++l) {
        std::vector<Mat<T>*> mr, mw, mb;
        for (auto& nd : pb.lv[l]) {
          if (l >= 2) {
            const Node2<T>& par = pb.lv[l - 1][nd.z >> 2];
            nd.R.r = nd.wU;
            nd.R.c = par.wU;
            nd.W.r = nd.wV;
            nd.W.c = par.wV;
            mr.push_back(&nd.R);
            mw.push_back(&nd.W);
          }
          int c = nd.z & 3;
          for (int s = 0; s < 3; ++s) {
            const Node2<T>& sb = pb.lv[l][(nd.z & ~3) | Builder<T>::sib_child(c, s)];
            nd.B[s].r = nd.wU;
            nd.B[s].c = sb.wV;
            mb.push_back(&nd.B[s]);
          }
        }
        if (l >= 2) {
          bd.own(p, l, Builder<T>::K_R, carve(P->arena, mr), old);
          bd.own(p, l, Builder<T>::K_W, carve(P->arena, mw), old);
        }
        bd.own(p, l, Builder<T>::K_B, carve(P->arena, mb), old);
        for (auto& nd : pb.lv[l]) {
          const Node1& ax = tx[p].lv[l][nd.a];
          const Node1& by = ty[p].lv[l][nd.b];
          if (l >= 2) {
            const Node2<T>& par = pb.lv[l - 1][nd.z >> 2];
            const Node1& tx_ = tx[p].lv[l - 1][nd.a >> 1];
            const Node1& sy_ = ty[p].lv[l - 1][nd.b >> 1];
            const Node1& axs = tx[p].lv[l][nd.a ^ 1];
            const Node1& bys = ty[p].lv[l][nd.b ^ 1];
            AsmDesc<T> r{};
            r.kind = 0;
            r.rows = nd.wU;
            r.cols = par.wU;
            r.ld = nd.R.ld;
            r.out = nd.R.p;
            r.dx = nd.dx; r.dy = nd.dy; r.rx = ax.rU; r.ry = by.rU;
            r.cdx = par.dx; r.cdy = par.dy; r.crx = tx_.rU; r.cry = sy_.rU;
            r.own_x = ax.col0 - tx_.col0;
            r.own_y = by.col0 - sy_.col0;
            r.sib_x = axs.col0 - tx_.col0;
            r.sib_y = bys.col0 - sy_.col0;
            r.dsx = axs.d;
            r.dsy = bys.d;
            r.X = ax.R.p; r.ldX = ax.R.ld;
            r.Y = by.R.p; r.ldY = by.R.ld;
            r.BX = ax.BV.p; r.ldBX = ax.BV.ld;
            r.BY = by.BV.p; r.ldBY = by.BV.ld;
            ad.push_back(r);
            AsmDesc<T> w = r;
            w.kind = 1;
            w.rows = nd.wV;
            w.cols = par.wV;
            w.ld = nd.W.ld;
            w.out = nd.W.p;
            w.rx = ax.rV; w.ry = by.rV; w.crx = tx_.rV; w.cry = sy_.rV;
            w.X = ax.W.p; w.ldX = ax.W.ld;
            w.Y = by.W.p; w.ldY = by.W.ld;
            ad.push_back(w);
            for (int kind = 0; kind < 2; ++kind) {
              const AsmDesc<T>& a = kind == 0 ? r : w;
              auto& k = kind == 0 ? nd.kr : nd.kw;
              k.dx = a.dx; k.dy = a.dy; k.rx = a.rx; k.ry = a.ry;
              k.cdx = a.cdx; k.cdy = a.cdy; k.crx = a.crx; k.cry = a.cry;
              k.own_x = a.own_x; k.own_y = a.own_y; k.sib_x = a.sib_x; k.sib_y = a.sib_y;
              k.dsx = a.dsx; k.dsy = a.dsy;
              k.X = a.X; k.ldX = a.ldX; k.Y = a.Y; k.ldY = a.ldY;
              k.BX = kind == 0 ? a.BX : nullptr; k.ldBX = a.ldBX;
              k.BY = kind == 0 ? a.BY : nullptr; k.ldBY = a.ldBY;
            }
          }
          int c = nd.z & 3;
          for (int s = 0; s < 3; ++s) {
            const Node2<T>& sb = pb.lv[l][(nd.z & ~3) | Builder<T>::sib_child(c, s)];
            const Node1& axs = tx[p].lv[l][sb.a];
            const Node1& bys = ty[p].lv[l][sb.b];
            AsmDesc<T> b{};
            b.kind = 2;
            b.rows = nd.wU;
            b.cols = sb.wV;
            b.ld = nd.B[s].ld;
            b.out = nd.B[s].p;
            b.dx = nd.dx; b.dy = nd.dy; b.rx = ax.rU; b.ry = by.rU;
            b.cdx = sb.dx; b.cdy = sb.dy; b.crx = axs.rV; b.cry = bys.rV;
            auto& kb = nd.kb[s];
            if (sb.a == nd.a) {
              b.bcase = 0;
              b.Y = by.B.p; b.ldY = by.B.ld;
              kb = {0, 0, b.dx * b.ry, 0, b.cdx * b.cry, b.dx, b.ry, b.cry, by.B.ld, by.B.p};
            } else if (sb.b == nd.b) {
              b.bcase = 1;
              b.X = ax.B.p; b.ldX = ax.B.ld;
              kb = {1, b.dx * b.ry, b.rx * b.dy, b.cdx * b.cry, b.crx * b.cdy, b.dy, b.rx, b.crx,
                    ax.B.ld, ax.B.p};
            } else {
              b.bcase = 2;
              b.X = ax.B.p; b.ldX = ax.B.ld;
              b.Y = by.B.p; b.ldY = by.B.ld;
              kb = {2, b.dx * b.ry + b.rx * b.dy, b.rx * b.ry, b.cdx * b.cry + b.crx * b.cdy,
                    b.crx * b.cry, 1, 0, 0, 0, nullptr};
            }
            ad.push_back(b);
          }
        }
        (void)q;
      }
    }
    gen_asm<T>(cx.pool, ad);
    ND_HIP(hipStreamSynchronize(cx.s));
    cx.pool.sync_reset();
    P->arena.check("face-split assembly");
  }
  // the assembly ends with a synchronisation, so this is its device time
  P->info.t_facesplit_ms = std::chrono::duration<double, std::milli>(
                               std::chrono::steady_clock::now() - t_start)
                               .count();

  // ------------------------------------------------ stage 1 (bottom-up)
  if (stages >= 1) {
    ProfSite site_(PS_S1_PROJ);
    // leaves: U = U~ F, V = V~ G
    std::vector<Mat<T>> A, Q, R;
    std::vector<std::tuple<int, int, int>> who;   // (p, z, 0=U / 1=V)
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      if (pb.L == 0) continue;
      std::vector<Mat<T>*> mq, mf;
      std::vector<Mat<T>> nu(pb.lv[pb.L].size()), nv(pb.lv[pb.L].size());
      for (auto& nd : pb.lv[pb.L]) {
        int ku = std::min((int)nd.m, nd.wU), kv = std::min(nd.dx * nd.dy, nd.wV);
        nu[nd.z].r = (int)nd.m;
        nu[nd.z].c = ku;
        nv[nd.z].r = nd.dx * nd.dy;
        nv[nd.z].c = kv;
        nd.F.r = ku;
        nd.F.c = nd.wU;
        nd.G.r = kv;
        nd.G.c = nd.wV;
        mq.push_back(&nu[nd.z]);
        mq.push_back(&nv[nd.z]);
        mf.push_back(&nd.F);
        mf.push_back(&nd.G);
      }
      void* cq = carve(P->arena, mq);
      bd.own(p, pb.L, Builder<T>::K_F, carve(P->arena, mf), old);
      for (auto& nd : pb.lv[pb.L]) {
        if (nd.m > 0 && nd.wU > 0) {
          A.push_back(nd.U);
          Q.push_back(nu[nd.z]);
          R.push_back(nd.F);
        }
        if (nd.wV > 0) {
          A.push_back(nd.V);
          Q.push_back(nv[nd.z]);
          R.push_back(nd.G);
        }
      }
      {
        ProfSite orth_site_(PS_S1_QR);
        orth<T>(cx, A, Q, &R);
      }
      A.clear(); Q.clear(); R.clear();
      ND_HIP(hipStreamSynchronize(cx.s));
      cx.release_tmp();
      cx.pool.sync_reset();
      for (auto& nd : pb.lv[pb.L]) {
        nd.U = nu[nd.z];
        nd.V = nv[nd.z];
      }
      bd.own(p, pb.L, Builder<T>::K_U, cq, old);
      bd.own(p, pb.L, Builder<T>::K_V, nullptr, old);
      bd.release(old);
      P->arena.check("stage 1, leaves");
    }
    // non-leaf nodes, from the leaves' parents to the root
    for (int h = 1; h <= Lmax; ++h) {
      for (int p = 0; p < np; ++p) {
        Prob2<T>& pb = H.probs[p];
        int l = pb.L - h;
        if (l < 0) continue;
        int lc = l + 1;
        // B~_{ci,cj} = F_ci B_{ci,cj} G_cj^H for the children (level lc).  The
        // face-split B has a single nonzero block Bblk (rows R, columns C),
        // so B~ = F(:, R) Z with Z^H = G(:, C) Bblk^H; for Bblk = I (x) F1 or
        // F1 (x) I, Z^H is a batch of products with the small factor F1.
        std::vector<Mat<T>*> mb, mx, mk;
        const size_t n3 = pb.lv[lc].size() * 3;
        std::vector<Mat<T>> X(n3), NB(n3), Kf(n3);
        for (auto& nd : pb.lv[lc]) {
          int c = nd.z & 3;
          for (int s = 0; s < 3; ++s) {
            const Node2<T>& sb = pb.lv[lc][(nd.z & ~3) | Builder<T>::sib_child(c, s)];
            const size_t i = (size_t)nd.z * 3 + s;
            const auto& kb = nd.kb[s];
            X[i].r = sb.G.r;
            X[i].c = kb.h;
            NB[i].r = nd.F.r;
            NB[i].c = sb.G.r;
            mx.push_back(&X[i]);
            mb.push_back(&NB[i]);
            if (kb.bcase < 2) {
              Kf[i].r = kb.kr;
              Kf[i].c = kb.kc;
              mk.push_back(&Kf[i]);
            }
          }
        }
        carve(P->arena, mx, &cx.tmp);
        carve(P->arena, mk, &cx.tmp);
        void* cb = carve(P->arena, mb);
        std::vector<CopyDesc<T, double>> kcd;
        std::vector<FillDesc<T>> fzb;
        std::vector<GemmDesc<T>> g1, g2;
        for (auto& nd : pb.lv[lc]) {
          int c = nd.z & 3;
          for (int s = 0; s < 3; ++s) {
            const Node2<T>& sb = pb.lv[lc][(nd.z & ~3) | Builder<T>::sib_child(c, s)];
            const size_t i = (size_t)nd.z * 3 + s;
            const auto& kb = nd.kb[s];
            Mat<T>& x = X[i];
            Mat<T>& nb = NB[i];
            if (nb.r <= 0 || nb.c <= 0) continue;
            if (x.c > 0) {
              if (kb.bcase == 2) {
                g1.push_back({x.r, x.c, kb.w, sb.G.ld, nd.B[s].ld, x.ld,
                              sb.G.p + (int64_t)kb.c0 * sb.G.ld, nd.B[s].p + kb.r0 +
                              (int64_t)kb.c0 * nd.B[s].ld, x.p, T(1), T(0), T(0)});
              } else {
                Mat<T>& kf = Kf[i];
                if (kb.kr > 0 && kb.kc > 0) kcd.push_back({kb.kr, kb.kc, kb.ldf, kf.ld, kb.f, kf.p, 0});
                for (int u = 0; u < kb.cnt; ++u) {
                  if (kb.bcase == 0)   // columns u kr .. of Z^H from columns c0 + u kc .. of G
                    g1.push_back({x.r, kb.kr, kb.kc, sb.G.ld, kf.ld, x.ld,
                                  sb.G.p + (int64_t)(kb.c0 + u * kb.kc) * sb.G.ld, kf.p,
                                  x.p + (int64_t)u * kb.kr * x.ld, T(1), T(0), T(0)});
                  else                 // columns u cnt + v of Z^H from columns c0 + u' cnt + v of G
                    g1.push_back({x.r, kb.kr, kb.kc, (int)((int64_t)kb.cnt * sb.G.ld), kf.ld,
                                  (int)((int64_t)kb.cnt * x.ld),
                                  sb.G.p + (int64_t)(kb.c0 + u) * sb.G.ld, kf.p,
                                  x.p + (int64_t)u * x.ld, T(1), T(0), T(0)});
                }
              }
            }
            // F is upper trapezoidal: its columns r0 .. r0 + h - 1 vanish below
            // row r0 + h, and so do the rows of B~ there
            const int mr = std::min(nb.r, kb.r0 + x.c);
            if (mr < nb.r) fzb.push_back({nb.r - mr, nb.c, nb.ld, nb.p + mr, 0});
            g2.push_back({mr, nb.c, x.c, nd.F.ld, x.ld, nb.ld, nd.F.p + (int64_t)kb.r0 * nd.F.ld,
                          x.p, nb.p, T(1), T(0), T(0)});
          }
        }
        copy_batched<T, double>(cx.pool, kcd);
        fill_batched<T>(cx.pool, fzb);
        gemm_batched<T>(cx.pool, g1, OpN, OpC);
        gemm_batched<T>(cx.pool, g2, OpN, OpC);
        std::vector<Mat<T>> SR, SW, QR_, QW_, FR, FW;
        std::vector<Mat<T>*> ms, mnew, mf;
        std::vector<Mat<T>> sr(pb.lv[l].size()), sw(pb.lv[l].size()), qr(pb.lv[l].size()),
            qw(pb.lv[l].size());
        if (l >= 1) {
          // stacked [F_c R_c] and [G_c W_c] of every node at level l
          for (auto& nd : pb.lv[l]) {
            int rows_u = 0, rows_v = 0;
            for (int c = 0; c < 4; ++c) {
              rows_u += pb.lv[lc][4 * nd.z + c].F.r;
              rows_v += pb.lv[lc][4 * nd.z + c].G.r;
            }
            sr[nd.z].r = rows_u;
            sr[nd.z].c = nd.wU;
            sw[nd.z].r = rows_v;
            sw[nd.z].c = nd.wV;
            ms.push_back(&sr[nd.z]);
            ms.push_back(&sw[nd.z]);
            int ku = std::min(rows_u, nd.wU), kv = std::min(rows_v, nd.wV);
            qr[nd.z].r = rows_u;
            qr[nd.z].c = ku;
            qw[nd.z].r = rows_v;
            qw[nd.z].c = kv;
            mnew.push_back(&qr[nd.z]);
            mnew.push_back(&qw[nd.z]);
            nd.F.r = ku;
            nd.F.c = nd.wU;
            nd.G.r = kv;
            nd.G.c = nd.wV;
            mf.push_back(&nd.F);
            mf.push_back(&nd.G);
          }
          carve(P->arena, ms, &cx.tmp);
          {
            std::vector<KronJob<T>> jobs;
            for (auto& nd : pb.lv[l]) {
              int ou = 0, ov = 0;
              for (int c = 0; c < 4; ++c) {
                Node2<T>& ch = pb.lv[lc][4 * nd.z + c];
                jobs.push_back({0, &ch.kr, ch.F, sr[nd.z].sub(ou, 0, ch.F.r, nd.wU)});
                jobs.push_back({1, &ch.kw, ch.G, sw[nd.z].sub(ov, 0, ch.G.r, nd.wV)});
                ou += ch.F.r;
                ov += ch.G.r;
              }
            }
            kron_transfer_products<T>(cx, jobs);
          }
          void* cq = carve(P->arena, mnew);
          void* cf = carve(P->arena, mf);
          std::vector<Mat<T>> A, Q, R;
          for (auto& nd : pb.lv[l]) {
            if (sr[nd.z].r > 0 && nd.wU > 0) {
              A.push_back(sr[nd.z]);
              Q.push_back(qr[nd.z]);
              R.push_back(nd.F);
            }
            if (sw[nd.z].r > 0 && nd.wV > 0) {
              A.push_back(sw[nd.z]);
              Q.push_back(qw[nd.z]);
              R.push_back(nd.G);
            }
          }
          {
            ProfSite orth_site_(PS_S1_QR);
            orth<T>(cx, A, Q, &R);
          }
          bd.own(p, l, Builder<T>::K_F, cf, old);
          bd.own(p, lc, Builder<T>::K_R, cq, old);
          bd.own(p, lc, Builder<T>::K_W, nullptr, old);
        }
        // children: new B, widths, transfer views
        for (auto& nd : pb.lv[lc]) {
          for (int s = 0; s < 3; ++s) nd.B[s] = NB[nd.z * 3 + s];
        }
        if (l >= 1) {
          for (auto& nd : pb.lv[l]) {
            int ou = 0, ov = 0;
            for (int c = 0; c < 4; ++c) {
              Node2<T>& ch = pb.lv[lc][4 * nd.z + c];
              ch.R = qr[nd.z].sub(ou, 0, ch.F.r, qr[nd.z].c);
              ch.W = qw[nd.z].sub(ov, 0, ch.G.r, qw[nd.z].c);
              ou += ch.F.r;
              ov += ch.G.r;
            }
          }
        }
        for (auto& nd : pb.lv[lc]) {
          nd.wU = nd.F.r;
          nd.wV = nd.G.r;
        }
        bd.own(p, lc, Builder<T>::K_B, cb, old);
        bd.own(p, lc, Builder<T>::K_F, nullptr, old);   // children's F/G no longer needed
        cx.release_tmp();
        cx.pool.sync_reset();
        bd.release(old);
        P->arena.check("stage 1, non-leaf level");
      }
    }
    for (int p = 0; p < np; ++p) {
      Prob2<T>& pb = H.probs[p];
      if (pb.L >= 1) {
        for (auto& nd : pb.lv[0]) {
          nd.wU = nd.F.r;
          nd.wV = nd.G.r;
        }
      }
    }
  }

  // ------------------------------------------------ stage 2 (top-down)
  if (stages >= 2) {
    ProfSite s2_site_(PS_S2_UPDATE);
    const double tol2 = eps * eps;
    for (int l = 1; l <= Lmax; ++l) {
      struct Ref { int p, z; };
      std::vector<Ref> nodes;
      bd.each_level(l, [&](int p, int z) { nodes.push_back({p, z}); });
      if (nodes.empty()) continue;
      // Grams K^U = sum_s B_{a,s} B_{a,s}^H + X X^H, K^V = sum_s B_{s,a}^H B_{s,a} + Y Y^H
      // with X = R_a T^U_parent, Y = W_a T^V_parent (levels >= 2), lower
      // triangles only.  They are formed on MFMA in FP32 when T = float and
      // eps >= 5e-3 (the trace threshold eps^2 sits far above FP32 rounding of
      // the Gram entries), else in FP64; the rank decisions (pivoted Cholesky
      // and its trace test) always run on FP64 Grams.
      std::vector<Mat<double>> KU(nodes.size()), KV(nodes.size());
      auto form_grams = [&](auto tag) {
        using G = decltype(tag);
        // a block in the Gram precision: the block itself or a converted copy
        auto conv = [&](const Mat<T>& m) -> Mat<G> {
          Mat<G> o;
          o.r = m.r;
          o.c = m.c;
          if constexpr (std::is_same<T, G>::value) {
            o.p = m.p;
            o.ld = m.ld;
          } else {
            o.ld = std::max(m.r, 1);
            o.p = (cplx<G>*)cx.tmp_alloc(sizeof(cplx<G>) * (size_t)o.ld * std::max(m.c, 1));
            std::vector<CopyDesc<G, T>> cd{{m.r, m.c, m.ld, o.ld, m.p, o.p, 0}};
            if (m.r > 0 && m.c > 0) copy_batched<G, T>(cx.pool, cd);
          }
          return o;
        };
        // the parents' weights T in the Gram precision (one copy per parent)
        std::map<std::pair<int, int>, Mat<G>> tconv;
        auto convT = [&](const Mat<T>& m, int p, int key) -> Mat<G> {
          if constexpr (std::is_same<G, T>::value) {
            (void)p;
            (void)key;
            return m;
          } else {
            auto it = tconv.find({p, key});
            if (it != tconv.end()) return it->second;
            Mat<G> o;
            o.r = m.r;
            o.c = m.c;
            o.ld = std::max(m.r, 1);
            o.p = (cplx<G>*)cx.tmp_alloc(sizeof(cplx<G>) * (size_t)o.ld * std::max(m.c, 1));
            std::vector<CopyDesc<G, T>> cd{{m.r, m.c, m.ld, o.ld, m.p, o.p, 0}};
            if (m.r > 0 && m.c > 0) copy_batched<G, T>(cx.pool, cd);
            tconv[{p, key}] = o;
            return o;
          }
        };
        std::vector<Mat<G>> GU(nodes.size()), GV(nodes.size()), XU(nodes.size()),
            XV(nodes.size());
        std::vector<Mat<G>*> mk;
        for (size_t i = 0; i < nodes.size(); ++i) {
          Node2<T>& nd = bd.node(nodes[i].p, l, nodes[i].z);
          GU[i].r = GU[i].c = nd.wU;
          GV[i].r = GV[i].c = nd.wV;
          mk.push_back(&GU[i]);
          mk.push_back(&GV[i]);
          if (l >= 2) {
            const Node2<T>& par = bd.node(nodes[i].p, l - 1, nodes[i].z >> 2);
            XU[i].r = nd.wU;
            XU[i].c = par.TU.c;
            XV[i].r = nd.wV;
            XV[i].c = par.TV.c;
            mk.push_back(&XU[i]);
            mk.push_back(&XV[i]);
          }
        }
        carve(P->arena, mk, &cx.tmp);
        // one launch per accumulation slot: a batched launch must not hold two
        // descriptors that update the same output matrix
        std::vector<GemmDesc<G>> gx, gnc[4], gcn[4];
        std::vector<FillDesc<G>> fz;
        for (size_t i = 0; i < nodes.size(); ++i) {
          int p = nodes[i].p, z = nodes[i].z;
          Node2<T>& nd = bd.node(p, l, z);
          int c = z & 3;
          if (nd.wU > 0) fz.push_back({nd.wU, nd.wU, GU[i].ld, GU[i].p, 0});
          if (nd.wV > 0) fz.push_back({nd.wV, nd.wV, GV[i].ld, GV[i].p, 0});
          for (int s = 0; s < 3; ++s) {
            int zs = (z & ~3) | Builder<T>::sib_child(c, s);
            Node2<T>& sb = bd.node(p, l, zs);
            Mat<G> b = conv(nd.B[s]);
            if (nd.wU > 0 && b.c > 0)
              gnc[s].push_back({nd.wU, nd.wU, b.c, b.ld, b.ld, GU[i].ld, b.p, b.p, GU[i].p, G(1),
                                G(0), G(1), 1});
            int slot = Builder<T>::sib_slot(zs & 3, c);
            Mat<G> bs = conv(sb.B[slot]);
            if (nd.wV > 0 && bs.r > 0)
              gcn[s].push_back({nd.wV, nd.wV, bs.r, bs.ld, bs.ld, GV[i].ld, bs.p, bs.p, GV[i].p,
                                G(1), G(0), G(1), 1});
          }
          if (l >= 2) {
            const Node2<T>& par = bd.node(p, l - 1, z >> 2);
            Mat<G> r = conv(nd.R), w = conv(nd.W);
            if (nd.wU > 0 && par.TU.c > 0) {
              Mat<G> tu = convT(par.TU, p, 2 * (z >> 2));
              // T^U_parent is upper triangular
              gx.push_back({nd.wU, par.TU.c, r.c, r.ld, tu.ld, XU[i].ld, r.p, tu.p, XU[i].p, G(1),
                            G(0), G(0), 0, 0, 2});
              gnc[3].push_back({nd.wU, nd.wU, XU[i].c, XU[i].ld, XU[i].ld, GU[i].ld, XU[i].p,
                                XU[i].p, GU[i].p, G(1), G(0), G(1), 1});
            }
            if (nd.wV > 0 && par.TV.c > 0) {
              Mat<G> tv = convT(par.TV, p, 2 * (z >> 2) + 1);
              gx.push_back({nd.wV, par.TV.c, w.c, w.ld, tv.ld, XV[i].ld, w.p, tv.p, XV[i].p, G(1),
                            G(0), G(0), 0, 0, 2});
              gnc[3].push_back({nd.wV, nd.wV, XV[i].c, XV[i].ld, XV[i].ld, GV[i].ld, XV[i].p,
                                XV[i].p, GV[i].p, G(1), G(0), G(1), 1});
            }
          }
        }
        fill_batched<G>(cx.pool, fz);
        gemm_batched<G>(cx.pool, gx, OpN, OpN);
        for (int s = 0; s < 4; ++s) {
          gemm_batched<G>(cx.pool, gnc[s], OpN, OpC);
          gemm_batched<G>(cx.pool, gcn[s], OpC, OpN);
        }
        if constexpr (std::is_same<G, double>::value) {
          KU = GU;
          KV = GV;
        } else {
          std::vector<Mat<double>*> mkd;
          for (size_t i = 0; i < nodes.size(); ++i) {
            KU[i].r = KU[i].c = GU[i].r;
            KV[i].r = KV[i].c = GV[i].r;
            mkd.push_back(&KU[i]);
            mkd.push_back(&KV[i]);
          }
          carve(P->arena, mkd, &cx.tmp);
          std::vector<CopyDesc<double, G>> cd;
          for (size_t i = 0; i < nodes.size(); ++i) {
            if (GU[i].r > 0) cd.push_back({GU[i].r, GU[i].c, GU[i].ld, KU[i].ld, GU[i].p, KU[i].p, 0});
            if (GV[i].r > 0) cd.push_back({GV[i].r, GV[i].c, GV[i].ld, KV[i].ld, GV[i].p, KV[i].p, 0});
          }
          copy_batched<double, G>(cx.pool, cd);
        }
      };
      {
        ProfSite gram_site_(PS_S2_GRAM);
        if (std::is_same<T, float>::value && eps >= 5e-3) form_grams(float{});
        else form_grams(double{});
      }
      // rank decisions
      std::vector<Mat<double>> Ks;
      std::vector<int> rmax;
      for (size_t i = 0; i < nodes.size(); ++i) {
        Ks.push_back(KU[i]);
        rmax.push_back(KU[i].r);
        Ks.push_back(KV[i]);
        rmax.push_back(KV[i].r);
      }
      std::vector<PcholOut> po;
      {
        ProfSite pchol_site_(PS_S2_PCHOL);
        pchol_run(cx, Ks, rmax, tol2, po);
      }
      // P = orth(L) and its triangular factor T, in the working precision (the
      // rank decisions above are the FP64 part)
      std::vector<Mat<T>> A, Q, R;
      std::vector<Mat<T>> Pw(nodes.size() * 2);
      std::vector<Mat<T>*> mp, mt;
      for (size_t i = 0; i < nodes.size(); ++i) {
        Node2<T>& nd = bd.node(nodes[i].p, l, nodes[i].z);
        for (int s = 0; s < 2; ++s) {
          int r = po[2 * i + s].rank;
          Pw[2 * i + s].r = s == 0 ? nd.wU : nd.wV;
          Pw[2 * i + s].c = r;
          mp.push_back(&Pw[2 * i + s]);
          Mat<T>& Tm = s == 0 ? nd.TU : nd.TV;
          Tm.r = r;
          Tm.c = r;
          mt.push_back(&Tm);
        }
      }
      carve(P->arena, mp, &cx.tmp);
      // the T matrices persist until the children are processed: one chunk per level
      bd.own(-1, l, Builder<T>::K_TU, carve(P->arena, mt), old);
      std::vector<CopyDesc<T, double>> lcd;
      for (size_t i = 0; i < nodes.size(); ++i) {
        Node2<T>& nd = bd.node(nodes[i].p, l, nodes[i].z);
        for (int s = 0; s < 2; ++s) {
          const PcholOut& pc = po[2 * i + s];
          if (pc.rank == 0) continue;
          Mat<T> a;
          a.r = pc.L.r;
          a.c = pc.rank;
          if constexpr (std::is_same<T, double>::value) {
            a.p = pc.L.p;
            a.ld = pc.L.ld;
          } else {
            a.ld = std::max(a.r, 1);
            a.p = (cplx<T>*)cx.tmp_alloc(sizeof(cplx<T>) * (size_t)a.ld * a.c);
            lcd.push_back({a.r, a.c, pc.L.ld, a.ld, pc.L.p, a.p, 0});
          }
          A.push_back(a);
          Q.push_back(Pw[2 * i + s]);
          R.push_back(s == 0 ? nd.TU : nd.TV);
        }
      }
      copy_batched<T, double>(cx.pool, lcd);
      {
        ProfSite orth_site_(PS_S2_ORTH);
        orth<T>(cx, A, Q, &R);
      }
      ProfSite upd_site_(PS_S2_UPDATE);
      // ---- updates
      // B^_{alpha,s} = P_alpha^H B Q_s
      std::map<int, std::vector<Mat<T>*>> mnb;   // per problem
      std::vector<Mat<T>> NB(nodes.size() * 3), XB(nodes.size() * 3);
      std::vector<Mat<T>*> mxb;
      std::map<std::pair<int, int>, int> idx;
      for (size_t i = 0; i < nodes.size(); ++i) idx[{nodes[i].p, nodes[i].z}] = (int)i;
      for (size_t i = 0; i < nodes.size(); ++i) {
        int p = nodes[i].p, z = nodes[i].z;
        Node2<T>& nd = bd.node(p, l, z);
        int c = z & 3;
        for (int s = 0; s < 3; ++s) {
          int zs = (z & ~3) | Builder<T>::sib_child(c, s);
          int j = idx[{p, zs}];
          XB[3 * i + s].r = nd.B[s].r;
          XB[3 * i + s].c = Pw[2 * j + 1].c;
          NB[3 * i + s].r = Pw[2 * i].c;
          NB[3 * i + s].c = Pw[2 * j + 1].c;
          mxb.push_back(&XB[3 * i + s]);
          mnb[p].push_back(&NB[3 * i + s]);
        }
      }
      carve(P->arena, mxb, &cx.tmp);
      for (auto& kv : mnb) bd.own(kv.first, l, Builder<T>::K_B, carve(P->arena, kv.second), old);
      std::vector<GemmDesc<T>> gb1, gb2;
      for (size_t i = 0; i < nodes.size(); ++i) {
        int p = nodes[i].p, z = nodes[i].z;
        Node2<T>& nd = bd.node(p, l, z);
        int c = z & 3;
        for (int s = 0; s < 3; ++s) {
          int zs = (z & ~3) | Builder<T>::sib_child(c, s);
          int j = idx[{p, zs}];
          Mat<T>& x = XB[3 * i + s];
          Mat<T>& nb = NB[3 * i + s];
          const Mat<T>& q = Pw[2 * j + 1];
          const Mat<T>& pp = Pw[2 * i];
          gb1.push_back({x.r, x.c, nd.B[s].c, nd.B[s].ld, q.ld, x.ld, nd.B[s].p, q.p, x.p, T(1),
                         T(0), T(0)});
          gb2.push_back({nb.r, nb.c, pp.r, pp.ld, x.ld, nb.ld, pp.p, x.p, nb.p, T(1), T(0), T(0)});
        }
      }
      gemm_batched<T>(cx.pool, gb1, OpN, OpN);
      gemm_batched<T>(cx.pool, gb2, OpC, OpN);
      // R^ = P^H R, W^ = Q^H W (l >= 2); leaf bases; children's transfers
      std::map<int, std::vector<Mat<T>*>> mrw, mleaf, mchild;
      std::vector<Mat<T>> NR(nodes.size()), NW(nodes.size()), NU(nodes.size()), NV(nodes.size());
      for (size_t i = 0; i < nodes.size(); ++i) {
        int p = nodes[i].p;
        Node2<T>& nd = bd.node(p, l, nodes[i].z);
        if (l >= 2) {
          NR[i].r = Pw[2 * i].c;
          NR[i].c = nd.R.c;
          NW[i].r = Pw[2 * i + 1].c;
          NW[i].c = nd.W.c;
          mrw[p].push_back(&NR[i]);
          mrw[p].push_back(&NW[i]);
        }
        if (l == H.probs[p].L) {
          NU[i].r = nd.U.r;
          NU[i].c = Pw[2 * i].c;
          NV[i].r = nd.V.r;
          NV[i].c = Pw[2 * i + 1].c;
          mleaf[p].push_back(&NU[i]);
          mleaf[p].push_back(&NV[i]);
        }
      }
      for (auto& kv : mrw) bd.own(kv.first, l, Builder<T>::K_R, carve(P->arena, kv.second), old);
      for (auto& kv : mleaf) bd.own(kv.first, l, Builder<T>::K_U, carve(P->arena, kv.second), old);
      std::vector<GemmDesc<T>> gr, gl;
      for (size_t i = 0; i < nodes.size(); ++i) {
        int p = nodes[i].p;
        Node2<T>& nd = bd.node(p, l, nodes[i].z);
        const Mat<T>& pp = Pw[2 * i];
        const Mat<T>& qq = Pw[2 * i + 1];
        if (l >= 2) {
          gr.push_back({NR[i].r, NR[i].c, pp.r, pp.ld, nd.R.ld, NR[i].ld, pp.p, nd.R.p, NR[i].p,
                        T(1), T(0), T(0)});
          gr.push_back({NW[i].r, NW[i].c, qq.r, qq.ld, nd.W.ld, NW[i].ld, qq.p, nd.W.p, NW[i].p,
                        T(1), T(0), T(0)});
        }
        if (l == H.probs[p].L) {
          gl.push_back({NU[i].r, NU[i].c, pp.r, nd.U.ld, pp.ld, NU[i].ld, nd.U.p, pp.p, NU[i].p,
                        T(1), T(0), T(0)});
          gl.push_back({NV[i].r, NV[i].c, qq.r, nd.V.ld, qq.ld, NV[i].ld, nd.V.p, qq.p, NV[i].p,
                        T(1), T(0), T(0)});
        }
      }
      gemm_batched<T>(cx.pool, gr, OpC, OpN);
      gemm_batched<T>(cx.pool, gl, OpN, OpN);
      // children of non-leaf nodes: R_chi <- R_chi P_alpha, W_chi <- W_chi Q_alpha
      std::vector<Mat<T>> CR, CW;
      std::vector<std::pair<int, int>> cref;   // (problem, child z)
      for (size_t i = 0; i < nodes.size(); ++i) {
        int p = nodes[i].p;
        if (l >= H.probs[p].L) continue;
        for (int c = 0; c < 4; ++c) cref.push_back({p, 4 * nodes[i].z + c});
      }
      CR.resize(cref.size());
      CW.resize(cref.size());
      for (size_t k = 0; k < cref.size(); ++k) {
        Node2<T>& ch = bd.node(cref[k].first, l + 1, cref[k].second);
        int i = idx[{cref[k].first, cref[k].second >> 2}];
        CR[k].r = ch.R.r;
        CR[k].c = Pw[2 * i].c;
        CW[k].r = ch.W.r;
        CW[k].c = Pw[2 * i + 1].c;
        mchild[cref[k].first].push_back(&CR[k]);
        mchild[cref[k].first].push_back(&CW[k]);
      }
      for (auto& kv : mchild)
        bd.own(kv.first, l + 1, Builder<T>::K_R, carve(P->arena, kv.second), old);
      std::vector<GemmDesc<T>> gc;
      for (size_t k = 0; k < cref.size(); ++k) {
        Node2<T>& ch = bd.node(cref[k].first, l + 1, cref[k].second);
        int i = idx[{cref[k].first, cref[k].second >> 2}];
        const Mat<T>& pp = Pw[2 * i];
        const Mat<T>& qq = Pw[2 * i + 1];
        gc.push_back({CR[k].r, CR[k].c, pp.r, ch.R.ld, pp.ld, CR[k].ld, ch.R.p, pp.p, CR[k].p, T(1),
                      T(0), T(0)});
        gc.push_back({CW[k].r, CW[k].c, qq.r, ch.W.ld, qq.ld, CW[k].ld, ch.W.p, qq.p, CW[k].p, T(1),
                      T(0), T(0)});
      }
      gemm_batched<T>(cx.pool, gc, OpN, OpN);
      ND_HIP(hipStreamSynchronize(cx.s));
      // install
      for (size_t i = 0; i < nodes.size(); ++i) {
        int p = nodes[i].p;
        Node2<T>& nd = bd.node(p, l, nodes[i].z);
        for (int s = 0; s < 3; ++s) nd.B[s] = NB[3 * i + s];
        if (l >= 2) {
          nd.R = NR[i];
          nd.W = NW[i];
        }
        if (l == H.probs[p].L) {
          nd.U = NU[i];
          nd.V = NV[i];
        }
        nd.wU = Pw[2 * i].c;
        nd.wV = Pw[2 * i + 1].c;
      }
      for (size_t k = 0; k < cref.size(); ++k) {
        Node2<T>& ch = bd.node(cref[k].first, l + 1, cref[k].second);
        ch.R = CR[k];
        ch.W = CW[k];
      }
      // the parent's T matrices are no longer needed
      if (l >= 2) bd.own(-1, l - 1, Builder<T>::K_TU, nullptr, old);
      cx.release_tmp();
      cx.pool.sync_reset();
      bd.release(old);
      P->arena.check("stage 2 level");
    }
  }
  // hand the remaining chunks to the HSS object
  for (auto& kv : bd.chunk)
    if (kv.second) H.mem.push_back(kv.second);
  // record ranks
  for (int l = 0; l <= Lmax && l < 16; ++l) {
    int ru = 0, rv = 0;
    for (auto& pb : H.probs)
      if (l <= pb.L && l >= 1)
        for (auto& nd : pb.lv[l]) {
          ru = std::max(ru, nd.wU);
          rv = std::max(rv, nd.wV);
        }
    P->info.max_rank_u[l] = ru;
    P->info.max_rank_v[l] = rv;
  }
}

template <typename T>
void matvec_2d(Ctx& cx, HSS2<T>& H, int prob, const double2* x, double2* y, int nrhs) {
  TmpScope scope_(cx);
  // Y = H X for the recompressed HSS of one problem (test hook): X (nrhs x N,
  // natural column order), Y (nrhs x M, caller's point order), FP64.
  Plan* P = cx.P;
  const Problem& q = P->probs[prob];
  Prob2<T>& pb = H.probs[prob];
  const int L = pb.L;
  ND_CHECK(L >= 1, NUDFT2_E_INVAL, "single-node tree");
  const int64_t N = q.N(), M = q.M;
  // X to quadtree order in working precision (host permutation, test sizes)
  std::vector<int64_t> cp(N);
  ND_HIP(hipMemcpy(cp.data(), P->colperm + q.c0, sizeof(int64_t) * N, hipMemcpyDeviceToHost));
  std::vector<double2> hx(N * nrhs);
  ND_HIP(hipMemcpy(hx.data(), x, sizeof(double2) * N * nrhs, hipMemcpyDeviceToHost));
  std::vector<cplx<T>> hxq(N * nrhs);
  for (int r = 0; r < nrhs; ++r)
    for (int64_t i = 0; i < N; ++i) {
      double2 v = hx[r * N + cp[i] - q.c0];
      hxq[r * N + i] = mk<T>((T)v.x, (T)v.y);
    }
  cplx<T>* xq = (cplx<T>*)cx.tmp_alloc(sizeof(cplx<T>) * N * nrhs);
  ND_HIP(hipMemcpy(xq, hxq.data(), sizeof(cplx<T>) * N * nrhs, hipMemcpyHostToDevice));
  std::vector<std::vector<cplx<T>*>> xh(L + 1), yh(L + 1);
  for (int l = 1; l <= L; ++l)
    for (auto& nd : pb.lv[l]) {
      xh[l].push_back((cplx<T>*)cx.tmp_alloc(sizeof(cplx<T>) * std::max(nd.wV, 1) * nrhs));
      yh[l].push_back((cplx<T>*)cx.tmp_alloc(sizeof(cplx<T>) * std::max(nd.wU, 1) * nrhs));
    }
  auto ldv = [](int w) { return std::max(w, 1); };
  std::vector<GemmDesc<T>> g;
  for (auto& nd : pb.lv[L])
    if (nd.wV > 0)
      g.push_back({nd.wV, nrhs, nd.V.r, nd.V.ld, (int)N, nd.wV, nd.V.p, xq + nd.col0,
                   xh[L][nd.z], T(1), T(0), T(0)});
  gemm_batched<T>(cx.pool, g, OpC, OpN);
  for (int l = L - 1; l >= 1; --l) {
    for (int c = 0; c < 4; ++c) {
      std::vector<GemmDesc<T>> gc;
      for (auto& nd : pb.lv[l]) {
        const Node2<T>& ch = pb.lv[l + 1][4 * nd.z + c];
        if (nd.wV == 0) continue;
        gc.push_back({nd.wV, nrhs, ch.wV, ch.W.ld, ldv(ch.wV), nd.wV, ch.W.p, xh[l + 1][ch.z],
                      xh[l][nd.z], T(1), T(0), c == 0 ? T(0) : T(1)});
      }
      gemm_batched<T>(cx.pool, gc, OpC, OpN);
    }
  }
  for (int l = 1; l <= L; ++l) {
    for (int s = 0; s < 3; ++s) {
      std::vector<GemmDesc<T>> gs;
      for (auto& nd : pb.lv[l]) {
        int zs = (nd.z & ~3) | (s < (nd.z & 3) ? s : s + 1);
        const Node2<T>& sb = pb.lv[l][zs];
        if (nd.wU == 0) continue;
        gs.push_back({nd.wU, nrhs, sb.wV, nd.B[s].ld, ldv(sb.wV), nd.wU, nd.B[s].p, xh[l][zs],
                      yh[l][nd.z], T(1), T(0), s == 0 ? T(0) : T(1)});
      }
      gemm_batched<T>(cx.pool, gs, OpN, OpN);
    }
    if (l >= 2) {
      std::vector<GemmDesc<T>> gr;
      for (auto& nd : pb.lv[l]) {
        const Node2<T>& par = pb.lv[l - 1][nd.z >> 2];
        if (nd.wU == 0 || par.wU == 0) continue;
        gr.push_back({nd.wU, nrhs, par.wU, nd.R.ld, par.wU, nd.wU, nd.R.p, yh[l - 1][par.z],
                      yh[l][nd.z], T(1), T(0), T(1)});
      }
      gemm_batched<T>(cx.pool, gr, OpN, OpN);
    }
  }
  // leaves: Y = D X + U yh, in the 2D-sorted order
  cplx<T>* y2 = (cplx<T>*)cx.tmp_alloc(sizeof(cplx<T>) * M * nrhs);
  std::vector<Mat<T>> Ds(pb.lv[L].size());
  std::vector<Mat<T>*> md;
  for (auto& nd : pb.lv[L]) {
    Ds[nd.z].r = (int)nd.m;
    Ds[nd.z].c = nd.n;
    md.push_back(&Ds[nd.z]);
  }
  carve(P->arena, md, &cx.tmp);
  std::vector<LeafDesc<T>> ld;
  std::vector<GemmDesc<T>> gu, gd;
  for (auto& nd : pb.lv[L]) {
    LeafDesc<T> d{};
    d.row0 = nd.row0;
    d.m = (int)nd.m;
    d.nx = q.nx;
    d.ny = q.ny;
    d.colx0 = q.colx[L][nd.a];
    d.dx = nd.dx;
    d.coly0 = q.coly[L][nd.b];
    d.dy = nd.dy;
    d.out = Ds[nd.z].p;
    d.ld = Ds[nd.z].ld;
    if (nd.m == 0) continue;
    ld.push_back(d);
    gu.push_back({(int)nd.m, nrhs, nd.wU, nd.U.ld, ldv(nd.wU), (int)M, nd.U.p, yh[L][nd.z],
                  y2 + (nd.row0 - q.m0), T(1), T(0), T(0)});
    gd.push_back({(int)nd.m, nrhs, nd.n, Ds[nd.z].ld, (int)N, (int)M, Ds[nd.z].p, xq + nd.col0,
                  y2 + (nd.row0 - q.m0), T(1), T(0), T(1)});
  }
  gen_leafD<T>(cx.pool, ld, P->pts_2d);
  gemm_batched<T>(cx.pool, gu, OpN, OpN);
  gemm_batched<T>(cx.pool, gd, OpN, OpN);
  std::vector<cplx<T>> hy(M * nrhs);
  std::vector<int64_t> perm(M);
  ND_HIP(hipMemcpyAsync(hy.data(), y2, sizeof(cplx<T>) * M * nrhs, hipMemcpyDeviceToHost, cx.s));
  ND_HIP(hipMemcpyAsync(perm.data(), P->perm2d + q.m0, sizeof(int64_t) * M, hipMemcpyDeviceToHost,
                        cx.s));
  ND_HIP(hipStreamSynchronize(cx.s));
  std::vector<double2> out(M * nrhs);
  for (int r = 0; r < nrhs; ++r)
    for (int64_t s = 0; s < M; ++s)
      out[r * M + perm[s] - q.m0] = mk<double>(hy[r * M + s].x, hy[r * M + s].y);
  ND_HIP(hipMemcpy(y, out.data(), sizeof(double2) * M * nrhs, hipMemcpyHostToDevice));
  cx.release_tmp();
  cx.pool.sync_reset();
}

template void build_2d<float>(Ctx&, const std::vector<Tree1>&, const std::vector<Tree1>&, double,
                              HSS2<float>&, int);
template void build_2d<double>(Ctx&, const std::vector<Tree1>&, const std::vector<Tree1>&, double,
                               HSS2<double>&, int);
template void matvec_2d<float>(Ctx&, HSS2<float>&, int, const double2*, double2*, int);
template void matvec_2d<double>(Ctx&, HSS2<double>&, int, const double2*, double2*, int);

}  // namespace nd
