// Batched dense complex linear algebra on the matrix cores (gfx950).
//
// All matrices are column-major with a leading dimension; complex numbers are
// interleaved (float2 / double2).  A "batch" is a list of independent
// problems of arbitrary (ragged) sizes executed by one launch.
#pragma once

#include "common.h"

namespace nd {

enum Op { OpN = 0, OpC = 1 };   // none / conjugate transpose

// Descriptor staging: descriptors are written to pinned host memory and
// copied to the device on the stream.  The pool is a bump allocator that is
// recycled only by an explicit sync_reset() (stream synchronisation first),
// so a descriptor is never overwritten while a kernel may still read it.
struct DescPool {
  char* host = nullptr;
  char* dev = nullptr;
  int* flag = nullptr;   // device error flag (set by a cooperative panel whose barrier timed out)
  size_t cap = 0, used = 0;
  hipStream_t stream = nullptr;
  // deferred: push() only stages on the host and sync_reset() does nothing,
  // so a stream capture records no copies and no waits; flush() then uploads
  // everything staged (the descriptors stay valid for the graph's lifetime)
  bool deferred = false;
  void init(size_t bytes, hipStream_t s);
  void destroy();
  void check_flag();   // synchronises; E_INTERNAL if the flag is set
  // copies n bytes to the device, returns the device address
  void* push(const void* src, size_t n);
  // push of read-only kernel arguments: when the pool slot already holds the
  // same bytes from an upload completed before the last sync_reset(), the
  // copy is skipped (repeated sweeps re-push identical descriptor lists).
  // A plain push() may be kernel-modified scratch: it ends reuse until the
  // cycle after the next sync_reset() has uploaded its lists again.
  void* push_ro(const void* src, size_t n);
  // n bytes of device scratch for a kernel, without an upload (the caller
  // initialises them on the stream); ends reuse like push()
  void* reserve(size_t n);
  // Device scratch used by one kernel pair at a time in stream order (the
  // GEMM's partial tiles), apart from the descriptor slots: allocated on first
  // use (a larger request synchronises the stream and replaces it), kept until
  // destroy().  nullptr in deferred mode (nothing is allocated while a stream
  // is captured) or when the allocation fails; the caller then takes a path
  // without it.
  void* stream_scratch(size_t n);
  char* sscr = nullptr;
  size_t sscr_cap = 0;
  size_t valid = 0;        // slots [0, valid) mirror the host staging on the device
  bool tainted = false;    // a plain push happened: no reuse
  void flush();
  void sync_reset();
  // take over o's buffers and state (o is left empty); the current ones are
  // released first
  void adopt(DescPool& o);
  ~DescPool() { destroy(); }
};

template <typename T>
struct GemmDesc {
  int m, n, k;
  int lda, ldb, ldc;
  const cplx<T>* A;
  const cplx<T>* B;
  cplx<T>* C;
  T ar, ai;     // alpha
  T beta;       // real beta
  int lower;    // 1: C (square) is Hermitian, only tiles reaching its lower triangle are computed
  // structure of the stored A and B (zeros are stored; kernels may skip
  // them): 1 = unit lower trapezoidal (explicit Householder reflectors,
  // X(i, j) = 0 for i < j), 2 = upper triangular (X(i, j) = 0 for i > j)
  int tri;
  int trib;
};

// One launch for the whole list.  Two descriptors of one list must not write
// the same output matrix (their tiles run concurrently).  A descriptor with
// lower = 1 leaves the tiles strictly above the diagonal untouched (for
// Hermitian products whose consumer reads the lower triangle only).
// Where the output tiles cannot fill the device, the k loop is shared out
// over workgroups (atomic accumulation into a pre-scaled C): when the
// autotuned table (gemm_tuning.inc, written by tune_gemm.py) or else a
// heuristic calls for a split, the tiles x k stages go in equal stream-K
// shares to the device's workgroup slots.  The table also picks the output
// tile shape of its shape classes: the 64 x 64 tiles, or for A^H B with
// m <= 32 the 32 x 128 or 16/32-square tiles of the small-output kernels.
// splits_force > 0 forces that many plain k splits on the 64 x 64 tiles
// (used by the tuner); -1 runs the tile kernel unsplit, without the table;
// -2 takes the heuristic without the table (the tuner's baseline); -3 takes
// stream-K wherever it applies; -4 takes the partial-tile split wherever the
// pool has room for it; -5 / -6 force the 32 x 128 / square small-output
// tiles (E_INVAL where the shapes do not allow them).
// Long-k products with few output tiles keep their k splits' partial tiles in
// the pool's stream scratch, at most this many bytes a launch; without the
// scratch they take the atomic split instead.
constexpr size_t kGemmPartBytes = size_t(64) << 20;
// FP32 tile products of the calling thread's launches: true (the default) on
// the bf16 matrix cores through a three-way split of each operand entry (six
// bf16 products per real product, FP32-level accuracy, see gemm_tile_bf),
// false on the FP32 matrix instructions.  Set per entry point from the plan.
extern thread_local bool g_fp32_split;
template <typename T>
void gemm_batched(DescPool& pool, const std::vector<GemmDesc<T>>& d, Op opA, Op opB,
                  int splits_force = 0);

// Householder QR of a batch: A (m x n, lda) is overwritten by the explicit
// reflector matrix V (m x kmin, unit lower trapezoidal, zeros above the
// diagonal); R (kmin x n, ldr) receives the triangular factor; Tb receives the
// compact-WY factors of the column blocks of QR_OB reflectors (Q = H_1 ... H_k
// = Q_0 Q_1 ..., Q_b = I - V_b T_b V_b^H).  Block b has kb = min(QR_OB, kmin -
// QR_OB b) columns; its T_b (kb x kb, leading dimension kb) starts at
// Tb + QR_OB^2 b; qr_tsize gives the element count.  The factorization runs in
// QR_NB-column panels (one cooperative launch each) whose updates stay inside
// their half of the block (QR_HB columns); the left half's reflectors then
// update the right half, the block's T joins the two halves' factors, and the
// trailing columns are updated once per block.
// ws: workspace (see qr_workspace).
constexpr int QR_NB = 32;
constexpr int QR_OB = 256;
constexpr int QR_HB = 128;   // the two halves of a block (see geqrf_batched)
template <typename T>
struct QRDesc {
  int m, n;
  int lda, ldr;
  cplx<T>* A;
  cplx<T>* R;
  cplx<T>* Tb;   // qr_tsize(m, n) elements
  cplx<T>* Tw;   // internal: the panels' QR_NB x QR_NB factors of the current block
};
inline int qr_kmin(int m, int n) { return m < n ? m : n; }
inline int qr_nblocks(int m, int n) { return (qr_kmin(m, n) + QR_NB - 1) / QR_NB; }
inline int64_t qr_tsize(int m, int n) {
  const int k = qr_kmin(m, n);
  if (k <= 0) return 1;
  const int nob = (k + QR_OB - 1) / QR_OB;
  const int64_t kl = k - (int64_t)QR_OB * (nob - 1);
  return (int64_t)QR_OB * QR_OB * (nob - 1) + kl * kl;
}
template <typename T>
size_t qr_workspace(const std::vector<QRDesc<T>>& d);   // bytes
template <typename T>
void geqrf_batched(DescPool& pool, const std::vector<QRDesc<T>>& d, void* ws);

// Apply Q (trans = false) or Q^H (trans = true) of a QR from geqrf_batched to
// C (m x nc, ldc) from the left, in place.  Only the first `kuse` reflectors
// of each problem are used when kuse >= 0 (all when kuse < 0).
template <typename T>
struct OrmDesc {
  int m, k, nc;         // rows, reflectors, columns of C
  int ldv, ldc;
  const cplx<T>* V;
  const cplx<T>* Tb;
  cplx<T>* C;
};
template <typename T>
size_t orm_workspace(const std::vector<OrmDesc<T>>& d);
// C <- Q C (trans false) or Q^H C.  from_identity (with trans false): C holds
// [I; 0] on entry (explicit Q formation); block b then updates only the
// columns from its first reflector on, the earlier ones being unit vectors
// its reflectors leave alone.
template <typename T>
void ormqr_batched(DescPool& pool, const std::vector<OrmDesc<T>>& d, bool trans, void* ws,
                   bool from_identity = false);

// Diagonally pivoted Cholesky of Hermitian PSD matrices K (w x w, FP64, only
// the lower triangle is read; overwritten by the Schur complement's lower
// triangle) with a trace stopping rule: stop at the
// first k with sum of the remaining diagonal <= tol2 * trace(K).  Outputs the
// factor L (w x rmax, ldl; columns in pivot order) and the rank (device int).
struct PcholDesc {
  int w, ldk, ldl, rmax;
  double2* K;
  double2* L;
  double* d;       // workspace, w doubles
  int* piv;        // rmax ints
  int* rank;       // output
  double tol2;
};
void pchol_batched(DescPool& pool, const std::vector<PcholDesc>& d);

// Batched upper-triangular solve R X = B in place, or R^H X = B when
// conj_trans (R: k x k, ldr; B: k x nrhs, ldb).
template <typename T>
struct TrsDesc {
  int k, nrhs, ldr, ldb;
  const cplx<T>* R;
  cplx<T>* B;
};
template <typename T>
void trsv_upper_batched(DescPool& pool, const std::vector<TrsDesc<T>>& d,
                        bool conj_trans = false);

// Batched in-place inversion of upper-triangular matrices: R (k x k, ldr) is
// overwritten by R^{-1}.  The strictly lower triangle must hold zeros (it
// stays zero).  ws: trtri_workspace bytes.
template <typename T>
struct TriDesc {
  int k, ldr;
  cplx<T>* R;
};
template <typename T>
size_t trtri_workspace(const std::vector<TriDesc<T>>& d);
template <typename T>
void trtri_upper_batched(DescPool& pool, const std::vector<TriDesc<T>>& d, void* ws);

// Elementwise helpers (batched over descriptors).
template <typename TD, typename TS>
struct CopyDesc {
  int m, n, lds, ldd;
  const cplx<TS>* S;
  cplx<TD>* D;
  int conj_trans;   // 1: D = S^H (D is n x m)
};
template <typename TD, typename TS>
void copy_batched(DescPool& pool, const std::vector<CopyDesc<TD, TS>>& d);

template <typename T>
struct FillDesc {
  int m, n, ld;
  cplx<T>* D;
  int identity;     // 1: identity (ones on the diagonal), 0: zeros
};
template <typename T>
void fill_batched(DescPool& pool, const std::vector<FillDesc<T>>& d);


}  // namespace nd
