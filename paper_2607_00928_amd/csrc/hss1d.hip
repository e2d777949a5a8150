// 1D HSS compression of the transformed NUDFT matrices G^x and G^y.
//
// The paper builds these 1D HSS approximations (tolerance eps/10, Algorithm
// 4.1, first construction step) from the displacement equation of Section
// 2.5, diag(g) G - G diag(xi) = u v^T, with factored ADI (fADI) and an
// interpolative decomposition.  Here every HSS block is compressed with
// nested orthonormal bases (Definition 2.2), bottom up:
//
//  * leaf a, row basis: the columns I selected by a diagonally pivoted
//    Cholesky factorization of the Gram matrix of G(J_a, K_a^c) (a column
//    interpolative decomposition, stopped when the discarded Schur
//    complement has trace <= tol^2 ||G(J_a, K_a^c)||_F^2), orthonormalised:
//    U_a = orth(G(J_a, I)).  With fADI (the default) the Gram matrix is that
//    of the low-rank factor G(J_a, K_a^c) ~= Z W^H, W C W^H with C = Z^H Z:
//    Z holds the exact kernel columns next to the ends of the node's
//    interval and the fADI vectors of the remaining (far) columns, whose
//    Zolotarev shifts on the two arcs of the unit circle reach tol/10
//    entrywise.  This replaces an O(m n^2) product per leaf by O(m w^2 + n^2 w)
//    with w = 2b + s columns (b near columns a side, s shifts).  Without
//    fADI the Gram matrix is formed from the explicit block.
//  * leaf a, column basis: V_a = orth(L) for the pivoted Cholesky factor L of
//    the Gram matrix of G(J_a^c, K_a).
//  * parent t of c1, c2: the stacked projected row blocks [U_c^H G(J_c,
//    K_t^c)] and column blocks [G(J_t^c, K_c) V_c] are compressed the same
//    way; the resulting orthonormal Z = [R_c1; R_c2], Y = [W_c1; W_c2] are the
//    transfer matrices, so U_t = diag(U_c) Z and V_t = diag(V_c) Y.
//  * B_{a,a'} = U_a^H G(J_a, K_a') V_a' for the two siblings of each parent.
//
// Everything in this stage is FP64.  The shifts come from the Moebius map of
// the two arcs onto [-gamma, -1] u [1, gamma] and the elliptic-function
// shifts of that symmetric pair, with the shift count from the bound
// Z_s <= 4 exp(-pi^2 s / log(16 gamma)) on the Zolotarev number.
#include <algorithm>
#include <cmath>
#include <complex>

#include "gen.h"
#include "hss.h"

namespace nd {

namespace {

constexpr int RMAX1D = 128;
constexpr double FADI_TOL_FRACTION = 0.1;   // fADI accuracy / truncation tolerance
constexpr int FADI_MAX_COLS = 64;           // wider factors fall back to the explicit Gram
constexpr int NEAR_COUNTS[] = {1, 2, 3, 4, 6, 8};

typedef std::complex<double> zc;

zc arc_point(double t) { return zc(std::cos(2.0 * M_PI * t), -std::sin(2.0 * M_PI * t)); }

zc cross_ratio(zc z1, zc z2, zc z3, zc z4) {
  return ((z1 - z3) * (z2 - z4)) / ((z1 - z4) * (z2 - z3));
}

// gamma of the image [-gamma, -1] u [1, gamma] of the arcs c([e0, e1]) and
// c([f0, f1]): (-gamma, -1, 1, gamma) has cross-ratio (1 + gamma)^2 / (4 gamma)
double gamma_of(double e0, double e1, double f0, double f1) {
  const double rho = cross_ratio(arc_point(e0), arc_point(e1), arc_point(f0), arc_point(f1)).real();
  return 2.0 * rho - 1.0 + 2.0 * std::sqrt(rho * rho - rho);
}

int shift_count(double gamma, double tau) {
  return std::max(1, (int)std::ceil(std::log(4.0 / tau) * std::log(16.0 * gamma) / (M_PI * M_PI)));
}

// complete elliptic integral K and Jacobi dn for the complementary modulus
// kp = sqrt(1 - k^2), by the arithmetic-geometric mean (Abramowitz and
// Stegun 17.6 and 16.4: descending AGM sequence, then the phase recursion
// phi_{i-1} = (phi_i + asin(c_i sin(phi_i) / a_i)) / 2, dn = cos(phi_0) /
// cos(phi_1 - phi_0))
double ellip_K(double kp) {
  double a = 1.0, b = kp;
  for (int i = 0; i < 64 && std::fabs(a - b) > 1e-16 * a; ++i) {
    const double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return M_PI / (2.0 * a);
}

double jacobi_dn(double u, double kp) {
  double a[66], c[66];
  a[0] = 1.0;
  c[0] = std::sqrt((1.0 - kp) * (1.0 + kp));
  double b = kp;
  int N = 0;
  while (N < 64 && std::fabs(c[N]) > 1e-17) {
    a[N + 1] = 0.5 * (a[N] + b);
    c[N + 1] = 0.5 * (a[N] - b);
    b = std::sqrt(a[N] * b);
    ++N;
  }
  double phi = std::ldexp(1.0, N) * a[N] * u, phi1 = phi;
  for (int i = N; i >= 1; --i) {
    phi1 = phi;
    phi = 0.5 * (phi + std::asin(c[i] * std::sin(phi) / a[i]));
  }
  return std::cos(phi) / std::cos(phi1 - phi);
}

// the optimal shifts of [-gamma, -1] x [1, gamma]: -w_j and w_j, w_j = gamma
// dn((2j - 1) K / (2s)), k' = 1 / gamma; the upper half from the lower one
// through w_j w_{s+1-j} = gamma (dn(u) dn(K - u) = k')
std::vector<double> symmetric_shifts(double gamma, int s) {
  const double kp = 1.0 / gamma, K = ellip_K(kp);
  std::vector<double> w(s);
  for (int j = 1; 2 * j <= s + 1; ++j) {
    w[j - 1] = gamma * jacobi_dn((2 * j - 1) * K / (2.0 * s), kp);
    w[s - j] = gamma / w[j - 1];
  }
  if (s % 2) w[s / 2] = std::sqrt(gamma);
  return w;
}

// z -> 0, 1, infinity for z = z1, z2, z3, and its inverse
zc mob(zc z, zc z1, zc z2, zc z3) { return ((z - z1) * (z2 - z3)) / ((z - z3) * (z2 - z1)); }
zc mob_inv(zc s, zc z1, zc z2, zc z3) {
  const zc k = s * (z2 - z1) / (z2 - z3);
  return (z1 - k * z3) / (1.0 - k);
}

}  // namespace

FadiPlan fadi_plan(int n, int level, int a, double tau) {
  FadiPlan pl;
  const int64_t nl = (int64_t)1 << level;
  pl.lo = (int)((a * (int64_t)n + nl - 1) / nl);
  pl.hi = (int)(((a + 1) * (int64_t)n + nl - 1) / nl);
  const int nc = n - (pl.hi - pl.lo);
  const double e0 = (double)a / (double)nl, e1 = (double)(a + 1) / (double)nl;
  int best = nc;
  double f0b = 0, f1b = 0;
  for (int b : NEAR_COUNTS) {
    if (nc - 2 * b <= 0) break;
    const double f0 = (double)(pl.hi + b) / n, f1 = (double)(pl.lo - b - 1 + n) / n;
    const double g = gamma_of(e0, e1, f0, f1);
    const int s = shift_count(g, tau);
    if (2 * b + s < best) {
      best = 2 * b + s;
      pl.b = b;
      pl.s = s;
      pl.gamma = g;
      f0b = f0;
      f1b = f1;
    }
  }
  if (pl.b == 0) return pl;
  const std::vector<double> w = symmetric_shifts(pl.gamma, pl.s);
  const zc z1 = arc_point(e0), z2 = arc_point(e1), z3 = arc_point(f0b);
  (void)f1b;
  for (int j = 0; j < pl.s; ++j) {
    const zc pj = mob_inv(mob(zc(-w[j], 0.0), -pl.gamma, -1.0, 1.0), z1, z2, z3);
    const zc qj = mob_inv(mob(zc(w[j], 0.0), -pl.gamma, -1.0, 1.0), z1, z2, z3);
    pl.p.push_back(mk<double>(pj.real(), pj.imag()));
    pl.q.push_back(mk<double>(qj.real(), qj.imag()));
  }
  return pl;
}

void free_1d(Plan* P, std::vector<Tree1>& t) {
  for (auto& tr : t)
    for (void* p : tr.mem) P->arena.release(p);
  t.clear();
}

void build_1d(Ctx& cx, int dim, double tol, std::vector<Tree1>& out) {
  TmpScope scope_(cx);
  Plan* P = cx.P;
  const int np = (int)P->probs.size();
  out.assign(np, Tree1());
  const double tol2 = tol * tol;
  // trees
  int Lmax = 0;
  for (int p = 0; p < np; ++p) {
    const Problem& q = P->probs[p];
    Tree1& t = out[p];
    t.n = dim ? q.ny : q.nx;
    t.L = q.L;
    t.M = q.M;
    t.m0 = q.m0;
    t.lv.assign(q.L + 1, {});
    const auto& rows = dim ? q.rowy : q.rowx;
    const auto& cols = dim ? q.coly : q.colx;
    for (int l = 0; l <= q.L; ++l) {
      int na = 1 << l;
      t.lv[l].resize(na);
      for (int a = 0; a < na; ++a) {
        Node1& nd = t.lv[l][a];
        nd.row0 = rows[l][a];
        nd.m = rows[l][a + 1] - rows[l][a];
        nd.col0 = cols[l][a];
        nd.d = cols[l][a + 1] - cols[l][a];
      }
    }
    Lmax = std::max(Lmax, q.L);
  }
  if (Lmax == 0) return;
  const double* axis = dim ? P->ys : P->xs;
  // full G per problem (M x n, ld M)
  std::vector<double2*> Gf(np, nullptr);
  for (int p = 0; p < np; ++p) {
    Tree1& t = out[p];
    if (t.L == 0) continue;
    Gf[p] = (double2*)cx.tmp_alloc(sizeof(double2) * t.M * t.n);
    gen_G1(cx.s, axis + t.m0, t.M, t.n, Gf[p], t.M);
  }
  // per-level projected rows T (sum rU x n) and columns P (M x sum rV)
  std::vector<std::vector<double2*>> Tl(np), Pl(np);
  std::vector<std::vector<int>> ldT(np);
  for (int p = 0; p < np; ++p) {
    Tl[p].assign(out[p].L + 1, nullptr);
    Pl[p].assign(out[p].L + 1, nullptr);
    ldT[p].assign(out[p].L + 1, 0);
  }
  std::vector<std::vector<int>> offU(np), offV(np);   // per node offsets of the current level

  // process heights from the leaves up
  for (int h = 0; h < Lmax; ++h) {
    // nodes at level l = L_p - h >= 1 of every problem
    struct Ref { int p, l, a; };
    std::vector<Ref> nodes;
    for (int p = 0; p < np; ++p) {
      int l = out[p].L - h;
      if (l < 1) continue;
      for (int a = 0; a < (1 << l); ++a) nodes.push_back({p, l, a});
    }
    const bool leaf = (h == 0);
    // ---------------- row side: Grams
    std::vector<Mat<double>> KU(nodes.size());
    std::vector<int> rmaxU(nodes.size());
    {
      std::vector<Mat<double>*> ms;
      for (size_t i = 0; i < nodes.size(); ++i) {
        const Ref& r = nodes[i];
        Tree1& t = out[r.p];
        Node1& nd = t.lv[r.l][r.a];
        int w = leaf ? t.n : (t.lv[r.l + 1][2 * r.a].rU + t.lv[r.l + 1][2 * r.a + 1].rU);
        KU[i].r = w;
        KU[i].c = w;
        rmaxU[i] = leaf ? (int)std::min<int64_t>(std::min(t.n - nd.d, RMAX1D), nd.m)
                        : w;
        ms.push_back(&KU[i]);
      }
      carve(P->arena, ms, &cx.tmp);
    }
    std::vector<GemmDesc<double>> g1, g2;
    std::vector<ZeroRCDesc> zr;
    std::vector<Mat<double>> Stmp(nodes.size());
    if (leaf) {
      // fADI factors Z (m x w), W (n x w) where the plan finds one narrower
      // than FADI_MAX_COLS, else the explicit Gram G(J_a, :)^H G(J_a, :) with
      // the rows and columns of K_a zeroed
      std::vector<FadiPlan> fp(nodes.size());
      std::vector<size_t> fi;
      for (size_t i = 0; i < nodes.size(); ++i) {
        const Ref& r = nodes[i];
        Tree1& t = out[r.p];
        Node1& nd = t.lv[r.l][r.a];
        if (P->opts.fadi_1d && nd.m > 0) {
          fp[i] = fadi_plan(t.n, r.l, r.a, FADI_TOL_FRACTION * tol);
          ND_CHECK(fp[i].b == 0 || (fp[i].lo == nd.col0 && fp[i].hi == nd.col0 + nd.d),
                   NUDFT2_E_INTERNAL, "fADI plan: column range differs from the tree's");
          if (fp[i].b > 0 && 2 * fp[i].b + fp[i].s <= FADI_MAX_COLS) {
            fi.push_back(i);
            continue;
          }
        }
        const double2* Ga = Gf[r.p] + (nd.row0 - t.m0);
        g1.push_back({t.n, t.n, (int)nd.m, (int)t.M, (int)t.M, KU[i].ld, Ga, Ga,
                      (double2*)KU[i].p, 1.0, 0.0, 0.0, 1});
        zr.push_back({t.n, nd.col0, nd.d, KU[i].ld, (double2*)KU[i].p});
      }
      gemm_batched<double>(cx.pool, g1, OpC, OpN);
      zero_rc(cx.pool, zr, true);
      if (!fi.empty()) {
        std::vector<Mat<double>> Zm(fi.size()), Wm(fi.size()), Cm(fi.size()), Tm(fi.size());
        std::vector<Mat<double>*> ms;
        std::vector<double2> shifts;
        for (size_t u = 0; u < fi.size(); ++u) {
          const size_t i = fi[u];
          const Ref& r = nodes[i];
          Tree1& t = out[r.p];
          Node1& nd = t.lv[r.l][r.a];
          const int w = 2 * fp[i].b + fp[i].s;
          Zm[u].r = (int)nd.m;
          Zm[u].c = w;
          Wm[u].r = t.n;
          Wm[u].c = w;
          Cm[u].r = w;
          Cm[u].c = w;
          Tm[u].r = t.n;
          Tm[u].c = w;
          ms.push_back(&Zm[u]);
          ms.push_back(&Wm[u]);
          ms.push_back(&Cm[u]);
          ms.push_back(&Tm[u]);
          shifts.insert(shifts.end(), fp[i].p.begin(), fp[i].p.end());
          shifts.insert(shifts.end(), fp[i].q.begin(), fp[i].q.end());
        }
        carve(P->arena, ms, &cx.tmp);
        const double2* dsh = (const double2*)cx.pool.push_ro(shifts.data(),
                                                             sizeof(double2) * shifts.size());
        std::vector<FadiDesc> fd;
        std::vector<GemmDesc<double>> gc, gt, gk;
        size_t off = 0;
        for (size_t u = 0; u < fi.size(); ++u) {
          const size_t i = fi[u];
          const Ref& r = nodes[i];
          Tree1& t = out[r.p];
          Node1& nd = t.lv[r.l][r.a];
          const FadiPlan& pl = fp[i];
          const int w = 2 * pl.b + pl.s;
          fd.push_back({axis + nd.row0, dsh + off, (double2*)Zm[u].p, (double2*)Wm[u].p, (int)nd.m,
                        t.n, pl.b, pl.s, pl.lo, pl.hi, Zm[u].ld, Wm[u].ld});
          off += 2 * pl.s;
          // C = Z^H Z, T = W C, KU = T W^H (Hermitian: lower triangle)
          gc.push_back({w, w, (int)nd.m, Zm[u].ld, Zm[u].ld, Cm[u].ld, (double2*)Zm[u].p,
                        (double2*)Zm[u].p, (double2*)Cm[u].p, 1.0, 0.0, 0.0});
          gt.push_back({t.n, w, w, Wm[u].ld, Cm[u].ld, Tm[u].ld, (double2*)Wm[u].p,
                        (double2*)Cm[u].p, (double2*)Tm[u].p, 1.0, 0.0, 0.0});
          gk.push_back({t.n, t.n, w, Tm[u].ld, Wm[u].ld, KU[i].ld, (double2*)Tm[u].p,
                        (double2*)Wm[u].p, (double2*)KU[i].p, 1.0, 0.0, 0.0, 1});
        }
        fadi_factors(cx.pool, fd);
        gemm_batched<double>(cx.pool, gc, OpC, OpN);
        gemm_batched<double>(cx.pool, gt, OpN, OpN);
        gemm_batched<double>(cx.pool, gk, OpN, OpC);
      }
    } else {
      // S = [T_c1; T_c2] with the columns of K_t zeroed
      std::vector<Mat<double>*> ms;
      for (size_t i = 0; i < nodes.size(); ++i) {
        const Ref& r = nodes[i];
        Stmp[i].r = KU[i].r;
        Stmp[i].c = out[r.p].n;
        ms.push_back(&Stmp[i]);
      }
      carve(P->arena, ms, &cx.tmp);
      std::vector<CopyDesc<double, double>> cd;
      for (size_t i = 0; i < nodes.size(); ++i) {
        const Ref& r = nodes[i];
        Tree1& t = out[r.p];
        Node1& nd = t.lv[r.l][r.a];
        int lc = r.l + 1;
        int o = offU[r.p][2 * r.a];
        const double2* Tc = Tl[r.p][lc] + o;
        cd.push_back({Stmp[i].r, t.n, ldT[r.p][lc], Stmp[i].ld, Tc, (double2*)Stmp[i].p, 0});
        zr.push_back({Stmp[i].r, nd.col0, nd.d, Stmp[i].ld, (double2*)Stmp[i].p});
        g1.push_back({Stmp[i].r, Stmp[i].r, t.n, Stmp[i].ld, Stmp[i].ld, KU[i].ld,
                      (double2*)Stmp[i].p, (double2*)Stmp[i].p, (double2*)KU[i].p, 1.0, 0.0, 0.0,
                      1});
      }
      copy_batched<double, double>(cx.pool, cd);
      zero_rc(cx.pool, zr, false);
      gemm_batched<double>(cx.pool, g1, OpN, OpC);
    }
    std::vector<PcholOut> pu;
    pchol_run(cx, KU, rmaxU, tol2, pu);
    // ---------------- column side: Grams over the rows outside the node
    std::vector<Mat<double>> KV(nodes.size());
    std::vector<int> rmaxV(nodes.size());
    {
      std::vector<Mat<double>*> ms;
      for (size_t i = 0; i < nodes.size(); ++i) {
        const Ref& r = nodes[i];
        Tree1& t = out[r.p];
        Node1& nd = t.lv[r.l][r.a];
        int w = leaf ? nd.d : (t.lv[r.l + 1][2 * r.a].rV + t.lv[r.l + 1][2 * r.a + 1].rV);
        KV[i].r = w;
        KV[i].c = w;
        rmaxV[i] = w;
        ms.push_back(&KV[i]);
      }
      carve(P->arena, ms, &cx.tmp);
    }
    g1.clear();
    g2.clear();
    for (size_t i = 0; i < nodes.size(); ++i) {
      const Ref& r = nodes[i];
      Tree1& t = out[r.p];
      Node1& nd = t.lv[r.l][r.a];
      const double2* Pc;
      int ldp = (int)t.M;
      if (leaf) Pc = Gf[r.p] + (int64_t)nd.col0 * t.M;
      else Pc = Pl[r.p][r.l + 1] + (int64_t)offV[r.p][2 * r.a] * t.M;
      int w = KV[i].r;
      int k1 = (int)(nd.row0 - t.m0);
      int s2 = (int)(nd.row0 - t.m0 + nd.m);
      int k2 = (int)(t.M - s2);
      g1.push_back({w, w, k1, ldp, ldp, KV[i].ld, Pc, Pc, (double2*)KV[i].p, 1.0, 0.0, 0.0, 1});
      g2.push_back({w, w, k2, ldp, ldp, KV[i].ld, Pc + s2, Pc + s2, (double2*)KV[i].p, 1.0, 0.0, 1.0,
                    1});
    }
    gemm_batched<double>(cx.pool, g1, OpC, OpN);
    gemm_batched<double>(cx.pool, g2, OpC, OpN);
    std::vector<PcholOut> pv;
    pchol_run(cx, KV, rmaxV, tol2, pv);

    // ---------------- orthonormal bases / transfer matrices
    std::vector<Mat<double>> Ain, Qout;
    {
      // row side
      std::vector<Mat<double>*> persist, tmpm;
      std::vector<Mat<double>> Yg(nodes.size());
      for (size_t i = 0; i < nodes.size(); ++i) {
        const Ref& r = nodes[i];
        Tree1& t = out[r.p];
        Node1& nd = t.lv[r.l][r.a];
        int rk = std::max(pu[i].rank, 1);
        nd.rU = pu[i].rank;
        if (leaf) {
          nd.U.r = (int)nd.m;
          nd.U.c = nd.rU;
          persist.push_back(&nd.U);
          Yg[i].r = (int)nd.m;
          Yg[i].c = rk;
          tmpm.push_back(&Yg[i]);
        }
        (void)rk;
      }
      {
        void* ch = carve(P->arena, persist, nullptr);
        if (ch) out[nodes[0].p].mem.push_back(ch);
      }
      carve(P->arena, tmpm, &cx.tmp);
      if (leaf) {
        std::vector<GatherDesc> gd;
        for (size_t i = 0; i < nodes.size(); ++i) {
          const Ref& r = nodes[i];
          Tree1& t = out[r.p];
          Node1& nd = t.lv[r.l][r.a];
          if (nd.rU == 0) continue;
          gd.push_back({(int)nd.m, nd.rU, (int)t.M, Yg[i].ld, Gf[r.p] + (nd.row0 - t.m0),
                        (double2*)Yg[i].p, pu[i].piv});
          Mat<double> a = Yg[i];
          a.c = nd.rU;
          Ain.push_back(a);
          Qout.push_back(nd.U);
        }
        gather_cols(cx.pool, gd);
      } else {
        // Z = orth(L): transfer matrices R_c1, R_c2 (views of one persistent Z)
        std::vector<Mat<double>> Zs(nodes.size());
        std::vector<Mat<double>*> zm;
        for (size_t i = 0; i < nodes.size(); ++i) {
          Zs[i].r = KU[i].r;
          Zs[i].c = std::max(pu[i].rank, 1);
          zm.push_back(&Zs[i]);
        }
        void* ch = carve(P->arena, zm, nullptr);
        out[nodes[0].p].mem.push_back(ch);
        for (size_t i = 0; i < nodes.size(); ++i) {
          const Ref& r = nodes[i];
          Tree1& t = out[r.p];
          Node1& nd = t.lv[r.l][r.a];
          Node1& c1 = t.lv[r.l + 1][2 * r.a];
          Node1& c2 = t.lv[r.l + 1][2 * r.a + 1];
          c1.R = Zs[i].sub(0, 0, c1.rU, nd.rU);
          c2.R = Zs[i].sub(c1.rU, 0, c2.rU, nd.rU);
          if (nd.rU == 0) continue;
          Mat<double> a = pu[i].L;
          a.c = nd.rU;
          Ain.push_back(a);
          Mat<double> q = Zs[i];
          q.c = nd.rU;
          Qout.push_back(q);
        }
      }
    }
    {
      // column side: V (leaf) or Y = [W_c1; W_c2], then the explicit V_f
      std::vector<Mat<double>> Ys(nodes.size());
      std::vector<Mat<double>*> ym, vm;
      for (size_t i = 0; i < nodes.size(); ++i) {
        const Ref& r = nodes[i];
        Tree1& t = out[r.p];
        Node1& nd = t.lv[r.l][r.a];
        nd.rV = pv[i].rank;
        nd.Vf.r = nd.d;
        nd.Vf.c = std::max(nd.rV, 1);
        vm.push_back(&nd.Vf);
        if (!leaf) {
          Ys[i].r = KV[i].r;
          Ys[i].c = std::max(nd.rV, 1);
          ym.push_back(&Ys[i]);
        }
      }
      void* ch = carve(P->arena, vm, nullptr);
      out[nodes[0].p].mem.push_back(ch);
      if (!leaf) {
        ch = carve(P->arena, ym, nullptr);
        out[nodes[0].p].mem.push_back(ch);
      }
      for (size_t i = 0; i < nodes.size(); ++i) {
        const Ref& r = nodes[i];
        Tree1& t = out[r.p];
        Node1& nd = t.lv[r.l][r.a];
        nd.Vf.c = nd.rV;
        if (nd.rV == 0) continue;
        Mat<double> a = pv[i].L;
        a.c = nd.rV;
        Ain.push_back(a);
        if (leaf) {
          Qout.push_back(nd.Vf);
        } else {
          Mat<double> q = Ys[i];
          q.c = nd.rV;
          Qout.push_back(q);
          Node1& c1 = t.lv[r.l + 1][2 * r.a];
          Node1& c2 = t.lv[r.l + 1][2 * r.a + 1];
          c1.W = Ys[i].sub(0, 0, c1.rV, nd.rV);
          c2.W = Ys[i].sub(c1.rV, 0, c2.rV, nd.rV);
        }
      }
      orth<double>(cx, Ain, Qout);
      if (!leaf) {
        // V_f(t) = [V_f(c1) W_c1; V_f(c2) W_c2]
        std::vector<GemmDesc<double>> gv;
        for (size_t i = 0; i < nodes.size(); ++i) {
          const Ref& r = nodes[i];
          Tree1& t = out[r.p];
          Node1& nd = t.lv[r.l][r.a];
          Node1& c1 = t.lv[r.l + 1][2 * r.a];
          Node1& c2 = t.lv[r.l + 1][2 * r.a + 1];
          if (nd.rV == 0) continue;
          gv.push_back({c1.d, nd.rV, c1.rV, c1.Vf.ld, c1.W.ld, nd.Vf.ld, c1.Vf.p, c1.W.p,
                        nd.Vf.p, 1.0, 0.0, 0.0});
          gv.push_back({c2.d, nd.rV, c2.rV, c2.Vf.ld, c2.W.ld, nd.Vf.ld, c2.Vf.p, c2.W.p,
                        nd.Vf.at(c1.d, 0), 1.0, 0.0, 0.0});
        }
        gemm_batched<double>(cx.pool, gv, OpN, OpN);
      }
    }
    // ---------------- projected rows T and columns P of this level
    {
      // offsets
      for (int p = 0; p < np; ++p) {
        int l = out[p].L - h;
        if (l < 1) continue;
        Tree1& t = out[p];
        offU[p].assign(1 << l, 0);
        offV[p].assign(1 << l, 0);
        int su = 0, sv = 0;
        for (int a = 0; a < (1 << l); ++a) {
          offU[p][a] = su;
          offV[p][a] = sv;
          su += t.lv[l][a].rU;
          sv += t.lv[l][a].rV;
        }
        ldT[p][l] = std::max(su, 1);
        Tl[p][l] = (double2*)cx.tmp_alloc(sizeof(double2) * (size_t)std::max(su, 1) * t.n);
        Pl[p][l] = (double2*)cx.tmp_alloc(sizeof(double2) * (size_t)std::max(sv, 1) * t.M);
      }
      std::vector<GemmDesc<double>> gt, gp;
      for (size_t i = 0; i < nodes.size(); ++i) {
        const Ref& r = nodes[i];
        Tree1& t = out[r.p];
        Node1& nd = t.lv[r.l][r.a];
        double2* Tn = Tl[r.p][r.l] + offU[r.p][r.a];
        double2* Pn = Pl[r.p][r.l] + (int64_t)offV[r.p][r.a] * t.M;
        if (leaf) {
          if (nd.rU > 0)
            gt.push_back({nd.rU, t.n, (int)nd.m, nd.U.ld, (int)t.M, ldT[r.p][r.l], nd.U.p,
                          Gf[r.p] + (nd.row0 - t.m0), Tn, 1.0, 0.0, 0.0});
          if (nd.rV > 0)
            gp.push_back({(int)t.M, nd.rV, nd.d, (int)t.M, nd.Vf.ld, (int)t.M,
                          Gf[r.p] + (int64_t)nd.col0 * t.M, nd.Vf.p, Pn, 1.0, 0.0, 0.0});
        }
      }
      if (!leaf) {
        // need the children's offsets: recompute them from the child level
        for (size_t i = 0; i < nodes.size(); ++i) {
          const Ref& r = nodes[i];
          Tree1& t = out[r.p];
          Node1& nd = t.lv[r.l][r.a];
          Node1& c1 = t.lv[r.l + 1][2 * r.a];
          Node1& c2 = t.lv[r.l + 1][2 * r.a + 1];
          int cu = 0, cv = 0;
          for (int a2 = 0; a2 < 2 * r.a; ++a2) {
            cu += t.lv[r.l + 1][a2].rU;
            cv += t.lv[r.l + 1][a2].rV;
          }
          double2* Tn = Tl[r.p][r.l] + offU[r.p][r.a];
          double2* Pn = Pl[r.p][r.l] + (int64_t)offV[r.p][r.a] * t.M;
          if (nd.rU > 0) {
            // T_t = Z^H [T_c1; T_c2]; Z = [R_c1; R_c2] with leading dim of the Z chunk
            gt.push_back({nd.rU, t.n, c1.rU + c2.rU, c1.R.ld, ldT[r.p][r.l + 1], ldT[r.p][r.l],
                          c1.R.p, Tl[r.p][r.l + 1] + cu, Tn, 1.0, 0.0, 0.0});
          }
          if (nd.rV > 0) {
            gp.push_back({(int)t.M, nd.rV, c1.rV + c2.rV, (int)t.M, c1.W.ld, (int)t.M,
                          Pl[r.p][r.l + 1] + (int64_t)cv * t.M, c1.W.p, Pn, 1.0, 0.0, 0.0});
          }
        }
      }
      gemm_batched<double>(cx.pool, gt, OpC, OpN);
      gemm_batched<double>(cx.pool, gp, OpN, OpN);
    }
    // ---------------- sibling interactions at this level
    {
      std::vector<Mat<double>*> bm;
      for (size_t i = 0; i < nodes.size(); ++i) {
        const Ref& r = nodes[i];
        Tree1& t = out[r.p];
        Node1& nd = t.lv[r.l][r.a];
        Node1& sb = t.lv[r.l][r.a ^ 1];
        nd.B.r = nd.rU;
        nd.B.c = std::max(sb.rV, 1);
        nd.BV.r = nd.rU;
        nd.BV.c = std::max(sb.d, 1);
        bm.push_back(&nd.B);
        bm.push_back(&nd.BV);
      }
      void* ch = carve(P->arena, bm, nullptr);
      out[nodes[0].p].mem.push_back(ch);
      std::vector<GemmDesc<double>> gb, gbv;
      for (size_t i = 0; i < nodes.size(); ++i) {
        const Ref& r = nodes[i];
        Tree1& t = out[r.p];
        Node1& nd = t.lv[r.l][r.a];
        Node1& sb = t.lv[r.l][r.a ^ 1];
        nd.B.c = sb.rV;
        nd.BV.c = sb.d;
        if (nd.rU == 0 || sb.rV == 0) {
          std::vector<FillDesc<double>> fz{{std::max(nd.B.r, 1), std::max(nd.B.c, 1), nd.B.ld, nd.B.p, 0},
                                           {std::max(nd.BV.r, 1), std::max(nd.BV.c, 1), nd.BV.ld, nd.BV.p, 0}};
          fill_batched<double>(cx.pool, fz);
          continue;
        }
        const double2* Tsib = Tl[r.p][r.l] + offU[r.p][r.a] + (int64_t)sb.col0 * ldT[r.p][r.l];
        gb.push_back({nd.rU, sb.rV, sb.d, ldT[r.p][r.l], sb.Vf.ld, nd.B.ld, Tsib, sb.Vf.p, nd.B.p,
                      1.0, 0.0, 0.0});
        gbv.push_back({nd.rU, sb.d, sb.rV, nd.B.ld, sb.Vf.ld, nd.BV.ld, nd.B.p, sb.Vf.p, nd.BV.p,
                       1.0, 0.0, 0.0});
      }
      gemm_batched<double>(cx.pool, gb, OpN, OpN);
      gemm_batched<double>(cx.pool, gbv, OpN, OpC);
    }
    // free the previous level's projections
    cx.pool.sync_reset();
    for (int p = 0; p < np; ++p) {
      int l = out[p].L - h;
      if (l + 1 <= out[p].L && l >= 0 && Tl[p][l + 1]) {
        P->arena.release(Tl[p][l + 1]);
        P->arena.release(Pl[p][l + 1]);
        for (auto it = cx.tmp.begin(); it != cx.tmp.end();) {
          if (*it == Tl[p][l + 1] || *it == Pl[p][l + 1]) it = cx.tmp.erase(it);
          else ++it;
        }
        Tl[p][l + 1] = Pl[p][l + 1] = nullptr;
      }
    }
  }
  cx.release_tmp();
}

void matvec_1d(Ctx& cx, int dim, const std::vector<Tree1>& trees, int prob, const double2* x,
               double2* y) {
  TmpScope scope_(cx);
  Plan* P = cx.P;
  const Tree1& t = trees[prob];
  const Problem& q = P->probs[prob];
  ND_CHECK(t.L >= 1, NUDFT2_E_INVAL, "1D tree has a single node");
  // x-hat per node at every level: xh(l, a) = Vf^H x(K_a)
  std::vector<std::vector<double2*>> xh(t.L + 1), yh(t.L + 1);
  for (int l = 1; l <= t.L; ++l)
    for (int a = 0; a < (1 << l); ++a) {
      const Node1& nd = t.lv[l][a];
      xh[l].push_back((double2*)cx.tmp_alloc(sizeof(double2) * std::max(nd.rV, 1)));
      yh[l].push_back((double2*)cx.tmp_alloc(sizeof(double2) * std::max(nd.rU, 1)));
    }
  std::vector<GemmDesc<double>> g;
  for (int l = 1; l <= t.L; ++l)
    for (int a = 0; a < (1 << l); ++a) {
      const Node1& nd = t.lv[l][a];
      if (nd.rV > 0)
        g.push_back({nd.rV, 1, nd.d, nd.Vf.ld, nd.d, nd.rV, nd.Vf.p, x + nd.col0, xh[l][a], 1.0, 0.0, 0.0});
    }
  gemm_batched<double>(cx.pool, g, OpC, OpN);
  for (int l = 1; l <= t.L; ++l) {
    g.clear();
    std::vector<GemmDesc<double>> g2;
    for (int a = 0; a < (1 << l); ++a) {
      const Node1& nd = t.lv[l][a];
      const Node1& sb = t.lv[l][a ^ 1];
      if (nd.rU == 0) continue;
      g.push_back({nd.rU, 1, sb.rV, nd.B.ld, std::max(sb.rV, 1), nd.rU, nd.B.p, xh[l][a ^ 1],
                   yh[l][a], 1.0, 0.0, 0.0});
      if (l >= 2 && t.lv[l - 1][a / 2].rU > 0)
        g2.push_back({nd.rU, 1, t.lv[l - 1][a / 2].rU, nd.R.ld, t.lv[l - 1][a / 2].rU, nd.rU, nd.R.p,
                      yh[l - 1][a / 2], yh[l][a], 1.0, 0.0, 1.0});
    }
    gemm_batched<double>(cx.pool, g, OpN, OpN);
    gemm_batched<double>(cx.pool, g2, OpN, OpN);
  }
  // leaves: y(J_a) = D_a x_a + U_a yh_a, in the axis-sorted order
  double2* ys = (double2*)cx.tmp_alloc(sizeof(double2) * t.M);
  g.clear();
  std::vector<Diag1Desc> dd;
  for (int a = 0; a < (1 << t.L); ++a) {
    const Node1& nd = t.lv[t.L][a];
    g.push_back({(int)nd.m, 1, nd.rU, nd.U.ld, std::max(nd.rU, 1), (int)t.M, nd.U.p, yh[t.L][a],
                 ys + (nd.row0 - t.m0), 1.0, 0.0, 0.0});
    dd.push_back({nd.row0, t.m0, nd.m, nd.col0, nd.d, t.n, x, ys});
  }
  gemm_batched<double>(cx.pool, g, OpN, OpN);
  diag1d(cx.pool, dd, dim ? P->ys : P->xs);
  // to the caller's order: for 2D-sorted s, y_user[perm2d[s]] = ys[pos[s]]
  std::vector<int64_t> perm(q.M), pos(q.M);
  ND_HIP(hipMemcpyAsync(perm.data(), P->perm2d + q.m0, sizeof(int64_t) * q.M, hipMemcpyDeviceToHost, cx.s));
  ND_HIP(hipMemcpyAsync(pos.data(), (dim ? P->posy : P->posx) + q.m0, sizeof(int64_t) * q.M,
                        hipMemcpyDeviceToHost, cx.s));
  std::vector<double2> hy(q.M), out(q.M);
  ND_HIP(hipMemcpyAsync(hy.data(), ys, sizeof(double2) * q.M, hipMemcpyDeviceToHost, cx.s));
  ND_HIP(hipStreamSynchronize(cx.s));
  for (int64_t s = 0; s < q.M; ++s) out[perm[s] - q.m0] = hy[pos[s] - q.m0];
  ND_HIP(hipMemcpy(y, out.data(), sizeof(double2) * q.M, hipMemcpyHostToDevice));
  cx.release_tmp();
}

}  // namespace nd
