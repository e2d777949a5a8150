// Generation / assembly kernels (see gen.hip).
#pragma once

#include "la.h"

namespace nd {

// 2D leaf descriptor (rows in the 2D-sorted order).
template <typename T>
struct LeafDesc {
  int64_t row0;      // first row (global, 2D-sorted)
  int m;             // rows
  int nx, ny;        // problem sizes (kernel periods)
  int colx0, dx, coly0, dy;   // 1D leaf column ranges (0-based frequencies)
  // face-split U only:
  const double2* Ux; int ldux; int64_t rowx0; int rx;
  const double2* Uy; int lduy; int64_t rowy0; int ry;
  cplx<T>* out; int ld;
  int coff;          // D only: first output column
};

template <typename T>
struct LeafVDesc {
  int dx, dy;
  const double2* Vx; int ldvx; int rx;
  const double2* Vy; int ldvy; int ry;
  cplx<T>* out; int ld;
};

// Kronecker-structured generator of a non-leaf node: kind 0 = R (transfer of
// the row basis), 1 = W (column basis), 2 = B (sibling interaction).
// Row blocks have widths [dx*ry | rx*dy | rx*ry], column blocks
// [cdx*cry | crx*cdy | crx*cry].
template <typename T>
struct AsmDesc {
  int kind, bcase;
  int rows, cols, ld;
  cplx<T>* out;
  int dx, dy, rx, ry;
  int cdx, cdy, crx, cry;
  int own_x, own_y, sib_x, sib_y, dsx, dsy;
  const double2* X; int ldX;
  const double2* Y; int ldY;
  const double2* BX; int ldBX;
  const double2* BY; int ldBY;
};

struct ZeroRCDesc {
  int n, c0, w, ld;
  double2* K;
};

struct GatherDesc {
  int m, r, ldi, ldo;
  const double2* in;
  double2* out;
  const int* piv;
};

struct Diag1Desc {
  int64_t row0, m0, m;
  int col0, d, n;
  const double2* x;
  double2* y;
};

// fADI factor of one HSS row block G(J_a, K_a^c) of the 1D matrix (Section
// 2.5's displacement equation diag(g) G - G diag(xi) = u v^T):
// G(J_a, l) ~= sum_j Z(., j) conj(W(l, j)) for l in K_a^c, W(l, .) = 0 on
// K_a = [lo, hi).  Columns 0 .. 2b-1 of Z are the exact kernel columns
// (hi + c) mod n and (lo - b + c) mod n (c < b), with W = 1 there; columns
// 2b .. 2b+s-1 are the fADI vectors z_j = u / (g - q_1) prod_{i<j} (g - p_i) /
// (g - q_{i+1}) and W(l, 2b+j) = conj((q_j - p_j) y_j(l)), y_j = v / (xi - p_1)
// prod_{i<j} (xi - q_i) / (xi - p_{i+1}), on the far columns.
struct FadiDesc {
  const double* xs;      // the block's m row coordinates (device)
  const double2* pq;     // shifts p_1..p_s then q_1..q_s (device)
  double2* Z;            // m x (2b + s), leading dimension ldz
  double2* W;            // n x (2b + s), leading dimension ldw
  int m, n, b, s, lo, hi, ldz, ldw;
};

void gen_G1(hipStream_t s, const double* xs, int64_t M, int n, double2* G, int64_t ld);
void fadi_factors(DescPool& pool, const std::vector<FadiDesc>& d);
template <typename T>
void gen_leafD(DescPool& pool, const std::vector<LeafDesc<T>>& d, const double* pts2d);
template <typename T>
void gen_leafU(DescPool& pool, const std::vector<LeafDesc<T>>& d, const double* pts2d,
               const int64_t* posx, const int64_t* posy);
template <typename T>
void gen_leafV(DescPool& pool, const std::vector<LeafVDesc<T>>& d);
template <typename T>
void gen_asm(DescPool& pool, const std::vector<AsmDesc<T>>& d);
void zero_rc(DescPool& pool, const std::vector<ZeroRCDesc>& d, bool rows_too);
void gather_cols(DescPool& pool, const std::vector<GatherDesc>& d);
void diag1d(DescPool& pool, const std::vector<Diag1Desc>& d, const double* xs);

}  // namespace nd
