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

void gen_G1(hipStream_t s, const double* xs, int64_t M, int n, double2* G, int64_t ld);
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
