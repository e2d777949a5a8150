// HSS data of a plan: 1D trees (FP64), the 2D face-split HSS matrix and its
// URV factors (working precision T = float or double).
#pragma once

#include "la.h"
#include "plan.h"

namespace nd {

template <typename T>
struct Mat {
  cplx<T>* p = nullptr;
  int r = 0, c = 0, ld = 0;
  cplx<T>* at(int64_t i, int64_t j) const { return p + i + j * (int64_t)ld; }
  Mat sub(int i, int j, int rr, int cc) const {
    Mat m;
    m.p = at(i, j);
    m.r = rr;
    m.c = cc;
    m.ld = ld;
    return m;
  }
};

// Execution context: stream, descriptor pool and temporaries.  Temporaries
// are released in scopes: release_tmp() frees what was allocated since the
// innermost TmpScope began.  keep (graph capture): scopes neither wait nor
// release; everything stays until the context is destroyed.
struct Ctx {
  Plan* P = nullptr;
  hipStream_t s = nullptr;
  DescPool pool;
  std::vector<void*> tmp;
  size_t base = 0;
  bool keep = false;
  void* tmp_alloc(size_t bytes) {
    void* p = P->arena.alloc(bytes);
    tmp.push_back(p);
    return p;
  }
  void release_tmp() {
    if (keep) return;
    ND_HIP(hipStreamSynchronize(s));
    for (size_t i = base; i < tmp.size(); ++i) P->arena.release(tmp[i]);
    tmp.resize(base);
  }
  ~Ctx() {
    (void)hipStreamSynchronize(s);
    for (void* p : tmp) P->arena.release(p);
  }
};

struct TmpScope {
  Ctx& c;
  size_t saved;
  explicit TmpScope(Ctx& cx) : c(cx), saved(cx.base) { c.base = c.tmp.size(); }
  ~TmpScope() {
    if (c.keep) {
      c.base = saved;
      return;
    }
    (void)hipStreamSynchronize(c.s);
    for (size_t i = c.base; i < c.tmp.size(); ++i) c.P->arena.release(c.tmp[i]);
    c.tmp.resize(c.base);
    c.base = saved;
  }
};

// Allocate one chunk for a list of matrices (each with ld = max(rows, 1)).
template <typename T>
void* carve(Arena& A, std::vector<Mat<T>*>& ms, std::vector<void*>* track = nullptr) {
  size_t tot = 0;
  for (Mat<T>* m : ms) {
    if (m->ld < m->r) m->ld = m->r;
    if (m->ld < 1) m->ld = 1;
    tot += ((size_t)m->ld * std::max(m->c, 1) + 31) & ~size_t(31);
  }
  if (tot == 0) return nullptr;
  cplx<T>* base = (cplx<T>*)A.alloc(tot * sizeof(cplx<T>));
  if (track) track->push_back(base);
  size_t off = 0;
  for (Mat<T>* m : ms) {
    m->p = base + off;
    off += ((size_t)m->ld * std::max(m->c, 1) + 31) & ~size_t(31);
  }
  return base;
}

// ------------------------------------------------------------------ 1D trees
struct Node1 {
  int64_t row0 = 0, m = 0;   // rows in the axis-sorted order (global)
  int col0 = 0, d = 0;       // columns [col0, col0 + d)
  int rU = 0, rV = 0;
  Mat<double> U;             // leaf: m x rU
  Mat<double> Vf;            // d x rV (explicit nested basis)
  Mat<double> R, W;          // level >= 2: to the parent
  Mat<double> B;             // level >= 1: B_{a, sib(a)}  (rU x rV_sib)
  Mat<double> BV;            // level >= 1: B_{a, sib(a)} Vf_sib^H  (rU x d_sib)
};

struct Tree1 {
  int n = 0, L = 0;
  int64_t M = 0, m0 = 0;
  std::vector<std::vector<Node1>> lv;
  std::vector<void*> mem;    // chunks owned by this tree
};

// ------------------------------------------------------------------ 2D HSS
template <typename T>
struct Node2 {
  int l = 0, z = 0, a = 0, b = 0;
  int64_t row0 = 0, m = 0;   // rows in the 2D-sorted order (global)
  int col0 = 0, n = 0;       // quadtree column range within the problem
  int dx = 0, dy = 0;
  int wU = 0, wV = 0;        // current widths of the row / column bases
  Mat<T> U, V;               // leaves
  Mat<T> R, W;               // l >= 2
  Mat<T> B[3];               // l >= 1: with the siblings in child order
  // Structure of the face-split B[s] (Theorem 3.3) until stage 1 replaces
  // it: one nonzero block, rows [r0, r0 + h) x columns [c0, c0 + w), equal to
  // I (x) F1 (bcase 0, cnt = dx diagonal copies of the kr x kc factor F1),
  // F1 (x) I (bcase 1, index u dy + v, cnt = dy) or F1 (x) F2 (bcase 2, used
  // as the materialised block).  f: the 1D factor F1 (FP64, leading dim ldf).
  struct KronB {
    int bcase = 2, r0 = 0, h = 0, c0 = 0, w = 0, cnt = 0, kr = 0, kc = 0, ldf = 0;
    const double2* f = nullptr;
  } kb[3];
  // Structure of the face-split R (kind 0) and W (kind 1) of a node at level
  // >= 2 until stage 1 consumes them: row blocks [dx ry | rx dy | rx ry] of
  // the node, column blocks [cdx cry | crx cdy | crx cry] of the parent, the
  // node's x / y columns at own_x / own_y of the parent's, its sibling's
  // (dsx / dsy of them) at sib_x / sib_y; X, Y the 1D transfer factors and
  // BX, BY the 1D sibling terms (R only), all FP64.
  struct KronRW {
    int dx = 0, dy = 0, rx = 0, ry = 0, cdx = 0, cdy = 0, crx = 0, cry = 0;
    int own_x = 0, own_y = 0, sib_x = 0, sib_y = 0, dsx = 0, dsy = 0;
    const double2 *X = nullptr, *Y = nullptr, *BX = nullptr, *BY = nullptr;
    int ldX = 0, ldY = 0, ldBX = 0, ldBY = 0;
  } kr, kw;
  Mat<T> F, G;               // stage-1 factors
  Mat<T> TU, TV;             // stage-2 weights (r x r)
  // URV factorization (Section 2.4): the node is a leaf of the (reduced) HSS
  // matrix with mm rows, nn unknowns, row basis U (mm x wU), column basis V
  // (nn x wV) and diagonal block D (mm x nn).
  int mm = 0, nn = 0;
  int mchk = 0;              // rows after the size reduction
  int k = 0;                 // unknowns eliminated at this node
  int nu = 0, pr = 0;        // unknowns / rows passed to the parent
  bool sizered = false;
  Mat<T> UD;                 // [U D]; after the size reduction: reflectors of Omega
  Mat<T> Tom;                // compact-WY blocks of Omega
  Mat<T> Vm;                 // V (nn x wV); after QR: its reflectors (Q0)
  Mat<T> Tq;                 // compact-WY blocks of Q0
  Mat<T> V2;                 // V^_2 (nu x wV)
  Mat<T> Wm;                 // [D~(:,0:k) | U^ | D~(:,k:)] -> [P refl. | U1,U2 | D12,D22]
  Mat<T> Tp;                 // compact-WY blocks of P
  Mat<T> D11;                // k x k upper triangular
};

template <typename T>
struct Prob2 {
  int L = 0;
  std::vector<std::vector<Node2<T>>> lv;   // lv[l][z]
  // root least-squares factor: QR of the merged root block (rm x rn)
  Mat<T> rootA, rootR, rootT;
  int root_m = 0, root_n = 0;
  Mat<double> Fx, Fy;        // inverse DFT matrices (nx x nx, ny x ny), FP64
};

struct HSSFactors {
  int precision = 0;
  virtual ~HSSFactors() = default;
};
using HSSBase = HSSFactors;

template <typename T>
struct HSS2 : HSSBase {
  std::vector<Prob2<T>> probs;
  std::vector<void*> mem;
};

// Orthonormal basis Q (m x min(m,c)) of the columns of each A (destroyed);
// optionally the triangular factors into Rout (caller-allocated, k x c).
template <typename T>
void orth(Ctx& cx, std::vector<Mat<T>>& A, std::vector<Mat<T>>& Q,
          std::vector<Mat<T>>* Rout = nullptr);

struct PcholOut {
  Mat<double> L;
  int* piv = nullptr;
  int rank = 0;
};
// Diagonally pivoted Cholesky with the trace rule on FP64 Grams (destroyed);
// ranks are returned on the host (synchronises).
void pchol_run(Ctx& cx, std::vector<Mat<double>>& K, std::vector<int>& rmax, double tol2,
               std::vector<PcholOut>& out);

int tree_depth(int nx, int ny, int leaf);
void host_binning(const double* points, int64_t M, int nx, int ny, int leaf,
                  int64_t* perm2d, int64_t* leaf_rows, int64_t* colperm);

// 1D compression of G^x (dim 0) or G^y (dim 1) for every problem.
// fADI plan of the HSS row block G(J_a, K_a^c) of node (level, a) of a 1D
// tree with n columns (K_a = [lo, hi)), for relative accuracy tau: b near
// columns on each side of K_a kept exactly and s Zolotarev shifts p (on the
// arc of the node's interval) and q (on the arc of the far columns) for the
// rest; b = 0 when keeping all of K_a^c exactly is no more expensive.
struct FadiPlan {
  int b = 0, s = 0, lo = 0, hi = 0;
  double gamma = 0.0;
  std::vector<double2> p, q;
};
FadiPlan fadi_plan(int n, int level, int a, double tau);

// build_1d compresses the leaf row blocks from their fADI factors when the
// plan's fadi_1d option is set, else from their explicit Gram matrices.
void build_1d(Ctx& cx, int dim, double tol, std::vector<Tree1>& out);
void free_1d(Plan* P, std::vector<Tree1>& t);
// y = H x for a 1D HSS (test hook): x (n, natural columns), y (M, caller order).
void matvec_1d(Ctx& cx, int dim, const std::vector<Tree1>& t, int prob, const double2* x,
               double2* y);

// Face-splitting assembly (Theorem 3.3) + recompression (Section 2.3).
template <typename T>
void build_2d(Ctx& cx, const std::vector<Tree1>& tx, const std::vector<Tree1>& ty, double eps,
              HSS2<T>& H, int stages = 2);
// Y = H X for problem `prob` of a recompressed HSS (test hook); X (nrhs x N)
// natural column order, Y (nrhs x M) caller's point order (FP64, problem-local).
template <typename T>
void matvec_2d(Ctx& cx, HSS2<T>& H, int prob, const double2* x, double2* y, int nrhs);

// URV factorization of the recompressed HSS (bottom-up, root QR).
template <typename T>
void urv_factor(Ctx& cx, HSS2<T>& H);
// Least-squares solve with the URV factors: f (ldf x nrhs, rows in the
// 2D-sorted point order, working precision) -> c (ldc x nrhs, quadtree column
// order, working precision).  f is overwritten.
template <typename T>
void urv_solve(Ctx& cx, HSS2<T>& H, cplx<T>* f, int64_t ldf, cplx<T>* c, int64_t ldc, int nrhs);
// Bytes of the factors one solve sweep reads per pass (the algorithmic HBM
// traffic of urv_solve, right-hand sides excluded).
template <typename T>
int64_t urv_sweep_bytes(const HSS2<T>& H);
// Adjoint of urv_solve: c (ldc x nrhs, quadtree column order, working
// precision, overwritten) -> f (ldf x nrhs, 2D-sorted rows, working precision).
template <typename T>
void urv_solve_adj(Ctx& cx, HSS2<T>& H, cplx<T>* c, int64_t ldc, cplx<T>* f, int64_t ldf,
                   int nrhs);

}  // namespace nd
