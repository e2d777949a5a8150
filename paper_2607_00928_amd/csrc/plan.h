// Plan: problems, trees, point orderings and the factors of the solver.
#pragma once

#include <memory>

#include "common.h"
#include "la.h"
#include "prof.h"

namespace nd {

struct HSSFactors;   // defined in hss.h

// Morton code of a quadtree node (x bit above y bit at every level), so that
// the children of node z are 4z + 2p + q.
inline uint32_t interleave(uint32_t a, uint32_t b, int L) {
  uint32_t z = 0;
  for (int i = 0; i < L; ++i) z |= (((a >> i) & 1u) << (2 * i + 1)) | (((b >> i) & 1u) << (2 * i));
  return z;
}
inline void deinterleave(uint32_t z, int L, uint32_t& a, uint32_t& b) {
  a = b = 0;
  for (int i = 0; i < L; ++i) {
    a |= ((z >> (2 * i + 1)) & 1u) << i;
    b |= ((z >> (2 * i)) & 1u) << i;
  }
}

// Host description of one problem's trees.
//  * 1D trees (x and y), both of depth L: node (l, a) owns the columns
//    [colx[l][a], colx[l][a+1]) and the rows of the x-sorted point order
//    [rowx[l][a], rowx[l][a+1]) (global indices).
//  * 2D quadtree of depth L, nodes of a level in Morton order z (children of
//    z are 4z + 2p + q): node z owns the rows [row2[l][z], row2[l][z+1]) of
//    the 2D-sorted point order (global) and the columns
//    [col2[l][z], col2[l][z+1]) of the quadtree column order (per problem).
struct Problem {
  int nx = 0, ny = 0, L = 0;
  int64_t m0 = 0, M = 0;   // points of this problem: [m0, m0 + M)
  int64_t c0 = 0;          // coefficient offset (complex entries)
  std::vector<std::vector<int>> colx, coly;
  std::vector<std::vector<int64_t>> rowx, rowy;
  std::vector<std::vector<int64_t>> row2;
  std::vector<std::vector<int>> col2;
  int64_t N() const { return (int64_t)nx * ny; }
};

// Device descriptor for the apply kernels.
struct ApplyProb {
  int64_t m0, M, c0;
  int nx, ny;
};

// State of the NUDFT approximation by spreading and FFT (type 2 for A c,
// type 1 for A^* f), built on first use for a tolerance: the kernel width w
// and shape beta, per problem the fine grid nfx x nfy and the deconvolution
// factors 1 / phihat(k / nf) per axis, FFT twiddles per length, and the two
// fine-grid buffers (grown on demand).
struct NufftProb {
  int nfx = 0, nfy = 0;
  double* invx = nullptr;   // nx entries, centred k
  double* invy = nullptr;   // ny entries
};
struct NufftState {
  double tol = 0.0;
  int w = 0;
  double beta = 0.0;
  std::vector<NufftProb> probs;
  std::map<int, double2*> tw;   // FFT length n -> exp(-2 pi i j / n), j < n / 2
  double2* g1 = nullptr;
  double2* g2 = nullptr;
  size_t gbytes = 0;            // bytes of each of g1, g2
};

struct Plan {
  nudft2_opts opts{};
  hipStream_t stream = nullptr;
  int device = 0;
  Arena arena;
  std::vector<Problem> probs;
  int64_t Mtot = 0, Ntot = 0;
  int Lmax = 0;

  // device arrays (global over problems)
  double* pts_user = nullptr;      // Mtot x 2, caller's order
  double* pts_2d = nullptr;        // Mtot x 2, 2D-sorted
  int64_t* perm2d = nullptr;       // 2D-sorted index -> caller index
  double* xs = nullptr;            // x of the x-sorted order (Mtot)
  double* ys = nullptr;            // y of the y-sorted order (Mtot)
  int64_t* posx = nullptr;         // 2D-sorted index -> x-sorted index
  int64_t* posy = nullptr;         // 2D-sorted index -> y-sorted index
  int64_t* colperm = nullptr;      // quadtree column index (global) -> natural index (global)
  ApplyProb* d_aprob = nullptr;
  // partial sums of the adjoint apply (one coefficient vector per row chunk
  // and right-hand side), grown on demand from the arena
  double2* adj_part = nullptr;
  size_t adj_part_bytes = 0;
  NufftState nufft;
  int* d_tile_off = nullptr;       // apply row-tile prefix (nprob + 1)
  int apply_tiles = 0;

  bool factored = false;
  std::unique_ptr<HSSFactors> hss;
  bool profiling = false;
  Profiler prof;
  nudft2_info info{};
  // descriptor pool of the solves, kept between solve calls so that repeated
  // solves find their descriptor lists already on the device
  DescPool spool;

  ~Plan();
};

Plan* make_plan(int nprob, const double* points, const int64_t* m_off,
                const int32_t* nx, const int32_t* ny, const nudft2_opts* opts);

void apply_fwd(Plan* P, const double2* c, double2* f, int nrhs, hipStream_t s);
void apply_adj(Plan* P, const double2* f, double2* c, int nrhs, hipStream_t s);
// apply_adj on the plan's stream with its partial sums in a static device
// array (no device allocation); E_INVAL when they do not fit
void apply_adj_noalloc(Plan* P, const double2* f, double2* c, int nrhs);

// A c and A^* f by spreading and FFT to relative accuracy about tol
// (nufft.hip); the state is built on the first call for a tolerance
void nufft_fwd(Plan* P, const double2* c, double2* f, int nrhs, double tol, hipStream_t s);
void nufft_adj(Plan* P, const double2* f, double2* c, int nrhs, double tol, hipStream_t s);
// the refinement's operators: the NUFFT when opts.nufft_tol > 0, else the
// exact direct sums
void op_fwd(Plan* P, const double2* c, double2* f, int nrhs, hipStream_t s);
void op_adj(Plan* P, const double2* f, double2* c, int nrhs, hipStream_t s);

}  // namespace nd
