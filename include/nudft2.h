/*
 * nudft2 -- direct solver for the 2D type-II inverse NUDFT on AMD MI355X.
 *
 * The problem (Section 1 of Li & Liu, "A superfast direct solver for the 2D
 * type-II inverse NUDFT based on HSS matrices"): given M >= N = nx*ny sample
 * points (x_j, y_j) and values f_j, find coefficients c minimising
 * ||A c - f||_2 with
 *
 *     A(j, (kx, ky)) = exp(-2 pi i (kx x_j + ky y_j)).
 *
 * Frequencies are centred: kx in [-nx/2, nx/2), ky in [-ny/2, ny/2).  A
 * coefficient array is C-order (nx, ny): c[i][j] <-> (kx, ky) =
 * (i - nx/2, j - ny/2); its vectorised column index is ky' + kx' ny with the
 * 0-based kx' = i, ky' = j (the paper's lexicographic ordering).
 *
 * Method (Algorithm 4.1): the transformed matrix G = A F^{-1} (F the 2D DFT)
 * is the face-splitting product G^x . G^y of two 1D transformed NUDFT
 * matrices (Section 3.1).  The library compresses G^x and G^y into HSS form
 * (tolerance eps/10), assembles the HSS form of their face-splitting product
 * (Theorem 3.3), recompresses it (Section 2.3, tolerance eps), factors it by
 * URV (Section 2.4), and solves with one URV sweep plus a 2D inverse DFT.
 * Optionally the solution is refined in FP64 against the exact operator A
 * (r = f - A c; c += F^{-1} H^+ r) until ||dc||/||c|| <= ir_tol, or until
 * the contraction bound on the error (see nudft2_solve) is below ir_tol.
 *
 * Complex data are interleaved (re, im) double pairs, the storage of
 * torch.complex128 / numpy complex128.  Unless stated otherwise pointers to
 * right-hand sides and solutions are DEVICE pointers owned by the caller.
 * Every entry point returns a status code; nothing aborts or throws across
 * this boundary.  Work is enqueued on opts.stream (a hipStream_t; NULL means
 * the default stream) and is asynchronous except where a call must read a
 * result back (factor reads ranks per level, refinement reads one norm per
 * iteration, get_info).  A plan is not re-entrant: calls on one plan must not
 * overlap.
 */
#ifndef NUDFT2_H
#define NUDFT2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NUDFT2_OK = 0,
  NUDFT2_E_INVAL = 1,     /* invalid argument (checked before any device work) */
  NUDFT2_E_STATE = 2,     /* call out of order (e.g. solve before factor)      */
  NUDFT2_E_DEVICE = 3,    /* no usable GPU / HIP runtime error                 */
  NUDFT2_E_NOMEM = 4,     /* device allocation failed or opts.mem_cap exceeded  */
  NUDFT2_E_SINGULAR = 5,  /* a triangular pivot of the URV factors vanished     */
  NUDFT2_E_NOCONV = 6,    /* refinement hit ir_maxit before ir_tol             */
  NUDFT2_E_INTERNAL = 7
} nudft2_status;

typedef struct nudft2_plan_s* nudft2_plan_t;

/* Options.  Fill with nudft2_default_opts() and override fields. */
typedef struct {
  int32_t precision;  /* 0: FP64 HSS factors; 1: FP32 factors, FP64 refinement */
  double eps;         /* HSS tolerance of the recompression (1D stage: eps/10) */
  int32_t leaf;       /* columns per dimension of a leaf (paper: 16)           */
  double ir_tol;      /* refinement stop: ||dc||_2 / ||c||_2 <= ir_tol, or for
                         refine = 0 the error bound of nudft2_solve      */
  int32_t ir_maxit;   /* refinement iterations; 0 = plain direct solve          */
  int32_t refine;     /* with S = F^{-1} H^+ the factored solution operator:
                         0: iterative refinement c += S(f - Ac) (exact for
                            consistent f);
                         1: preconditioned conjugate gradients on the normal
                            equations A^*A c = A^*f, preconditioner S S^*,
                            from the direct solution (exact least squares
                            for any f);
                         2: plsqr (Section 4.1): LSQR on the left-
                            preconditioned system S A c = S f, restarted from
                            the exact residual with FP32 factors (exact for
                            consistent f) */
  void* stream;       /* hipStream_t; NULL = default stream                     */
  size_t mem_cap;     /* device bytes the plan may hold; 0 = no cap             */
  int32_t graph;      /* 1: each solve call runs its first two refinement
                         iterations eagerly, captures the next one (exact apply,
                         residual, HSS solve sweep, update, norms) into a HIP
                         graph and replays it for the rest; 0 (default): eager
                         launches.
                         Kernel profiling (nudft2_set_profiling) runs eagerly. */
  double nufft_tol;   /* operator of the refinement iterations: 0 (default) the
                         exact FP64 direct sums of A and A^*; > 0 their
                         approximation by spreading and FFT (Section 4.1's
                         NUFFT) to about this relative accuracy, in (0, 0.1);
                         nx, ny <= 1024 */
  int32_t fp32_products; /* matrix-core products of the FP32 factorization:
                         0 (default) bf16 instructions on a split of every
                         FP32 entry x into three bf16 parts (x = x0 + x1 + x2
                         exactly), six bf16 products per real product
                         (FP32-level accuracy: the three left out are below
                         2^-23 |a||b|); 1 FP32 instructions.  The FP64
                         factorization ignores it. */
  int32_t fadi_1d;    /* 1D HSS construction of G^x and G^y (Section 2.5):
                         1 (default) the leaf row bases from fADI factors of
                         the displacement equation (Zolotarev shifts on the
                         two arcs of the unit circle, the kernel columns next
                         to each node's interval kept exactly), accurate to a
                         tenth of the 1D tolerance eps/10; 0 from the explicit
                         Gram matrices of the blocks. */
} nudft2_opts;

/* Per-solve report (host memory, may be NULL). */
typedef struct {
  int32_t iterations;     /* refinement iterations taken                     */
  double rel_update;      /* last ||dc|| / ||c||                              */
  double rel_residual;    /* last ||f - A c|| / ||f|| formed (first right-hand
                             side): that of the iterate before the last update,
                             1 after a single iteration                       */
} nudft2_solve_info;

/* Plan-wide report (host memory). */
typedef struct {
  int32_t nprob;          /* problems in the plan                             */
  int32_t levels;         /* depth L of the (deepest) quadtree                */
  int32_t max_rank_u[16]; /* per level 0..L: largest row rank after recompression */
  int32_t max_rank_v[16]; /* per level 0..L: largest column rank                */
  int64_t factor_bytes;   /* device bytes held by the factors                 */
  double factor_flops;    /* flops counted over the factorization's operations */
  int64_t sweep_bytes;    /* factor bytes one solve sweep reads (Algorithm 4.1's
                             bottom-up, root and top-down steps, per pass;
                             right-hand sides excluded): its HBM traffic   */
  /* wall-clock phases (ms): plan (point copy, binning, upload); 1D
   * compression; face-splitting assembly; recompression (both stages); URV
   * factorization.  Each phase ends with a stream synchronisation. */
  double t_plan_ms, t_compress_ms, t_facesplit_ms, t_recompress_ms, t_urv_ms;
  /* kernel timing while profiling is on (nudft2_set_profiling), per class:
   * 0 = exact FP64 apply, 1 = FP32 matrix-core GEMM, 2 = FP64 matrix-core
   * GEMM, 3 = Householder panel, 4 / 5 = FP32 / FP64 skinny products (at
   * most 8 columns, memory bound).  Milliseconds from HIP events recorded on
   * the plan's stream around each launch; algorithmic flops (8 per complex
   * multiply-add of the launch's problems); launch counts. */
  double kernel_ms[6];
  double kernel_flops[6];
  int64_t kernel_launches[6];
  int64_t peak_bytes;     /* most device bytes the plan's arena held at once
                             (factors plus the factorization's workspaces)  */
} nudft2_info;

void nudft2_default_opts(nudft2_opts* opts);

/* Plan for one problem (Section 1: the M >= N sample points of the type-II
 * problem; Section 3.2 and Definition 3.2: the face-splitting product of the
 * two 1D trees that the plan builds).  points: DEVICE pointer to M
 * interleaved (x_j, y_j) doubles, any finite values (wrapped into [0,1));
 * the plan copies them (caller keeps ownership; the copy direction is taken
 * from the address, so a host pointer is accepted too).  Requires nx, ny even
 * and >= 2, M >= nx*ny, all points finite, opts valid (eps in (0,1),
 * leaf >= 2).  Bins the points into the quadtree (host counting sorts after
 * one device-to-host copy) and uploads them in tree order; does not factor.
 * Synchronises with opts.stream.  *out is set only on success.  Errors:
 * E_INVAL, E_DEVICE, E_NOMEM. */
nudft2_status nudft2_plan(nudft2_plan_t* out, const double* points, int64_t M,
                          int32_t nx, int32_t ny, const nudft2_opts* opts);

/* Plan for nprob independent problems solved together (one launch per tree
 * level for all problems; the reuse of one factorization across right-hand
 * sides, Section 5, extended across problems).  points: DEVICE (as in
 * nudft2_plan), concatenated; problem p owns points[2*m_off[p] ..
 * 2*m_off[p+1]).  m_off, nx, ny: HOST arrays (nprob+1, nprob, nprob).
 * Right-hand sides and solutions of a batch plan are concatenated in
 * problem order: f of problem p at f + 2*m_off[p] (per
 * right-hand side stride 2*m_off[nprob] doubles), c of problem p at an offset
 * of sum_{q<p} nx[q]*ny[q] complex entries. */
nudft2_status nudft2_plan_batch(nudft2_plan_t* out, int32_t nprob,
                                const double* points, const int64_t* m_off,
                                const int32_t* nx, const int32_t* ny,
                                const nudft2_opts* opts);

/* The offline stage of Algorithm 4.1: build the HSS approximation of G
 * (1D compression of G^x, G^y at eps/10, Section 2.5; face-splitting
 * assembly, Theorem 3.3; recompression at eps, Section 2.3) and its URV
 * factorization (Section 2.4).  The plan owns every factor.  Idempotent.
 * Synchronises with the stream (ranks are read back per level).  Errors:
 * E_NOMEM, E_SINGULAR, E_DEVICE. */
nudft2_status nudft2_factor(nudft2_plan_t plan);

/* Least-squares solve for nrhs right-hand sides.  f: DEVICE, nrhs x M
 * complex128 (row-major, right-hand side r at f + 2*M*r), in the caller's
 * point order.  c: DEVICE, nrhs x nx x ny complex128 output.  With
 * opts.ir_maxit == 0 returns the direct solution c = S f with S = F^{-1} H^+
 * (Algorithm 4.1); otherwise refines in FP64 against the exact A until
 * ||dc||/||c|| <= ir_tol (per problem and right-hand side): opts.refine = 0
 * iterates c += S(f - A c), whose fixed point is the least-squares solution
 * when f is in the range of A, and also stops, from its third iteration,
 * where q / (1 - q) ||dc_k|| / ||c_k|| <= ir_tol with q = 10 ||dc_k|| /
 * ||dc_{k-1}|| (relative) below 1/2: the error bound of a contraction with
 * ten times the observed rate; refine = 1 runs conjugate gradients on the
 * normal equations preconditioned by S S^* (the least-squares solution for
 * any f); refine = 2 runs the paper's plsqr, LSQR on S A c = S f (Section
 * 4.1; exact for consistent f).  E_NOCONV leaves the last iterate in c.  Errors: E_INVAL
 * (null pointer, nrhs <= 0), E_STATE (not factored), E_NOCONV, E_DEVICE. */
nudft2_status nudft2_solve(nudft2_plan_t plan, const double* f, double* c,
                           int32_t nrhs, nudft2_solve_info* info);

/* Change the refinement options (ir_tol, ir_maxit, refine; meaning as in
 * nudft2_opts) of a plan, factored or not: one factorization serves direct
 * and refined solves.  Errors: E_INVAL (null plan, ir_tol < 0, ir_maxit < 0,
 * refine not 0 or 1). */
nudft2_status nudft2_set_solve_opts(nudft2_plan_t plan, double ir_tol, int32_t ir_maxit,
                                    int32_t refine);

/* Change the refinement's operator of a plan (opts.nufft_tol: 0 the exact
 * direct sums, in (0, 0.1) the NUFFT at that accuracy), factored or not.
 * Errors: E_INVAL (null plan, tolerance out of range, nx or ny > 1024 for a
 * positive tolerance). */
nudft2_status nudft2_set_nufft_tol(nudft2_plan_t plan, double nufft_tol);

/* Adjoint of the least-squares solution operator (Section 4.1 applies the
 * adjoint of the factored solution operator, a 2D FFT followed by the
 * adjoint URV solve; here it preconditions the normal equations):
 * w = (A^+)^* g = A (A^*A)^{-1} g for g of shape nrhs x nx x ny, w of shape
 * nrhs x M (DEVICE, caller-owned).  (A^*A)^{-1} g is obtained by conjugate
 * gradients on the normal equations preconditioned by S S^* (S = F^{-1} H^+
 * the factored solution operator and S^* its adjoint sweep) from
 * z = S S^* g, stopped at ||dz||/||z|| <= ir_tol (at least one step even
 * when ir_maxit < 2).  This is the map that gives
 * dL/df = w for an upstream gradient g = dL/dc of the solution.  Errors:
 * E_INVAL, E_STATE (not factored), E_NOCONV, E_DEVICE. */
nudft2_status nudft2_solve_adj(nudft2_plan_t plan, const double* g, double* w,
                               int32_t nrhs, nudft2_solve_info* info);

/* Backward pass of c = A^+ f (c the least-squares solution for f, as returned
 * by nudft2_solve with refine = 1) for an upstream gradient g = dL/dc (real
 * loss, dL = Re<g, dc>, the convention of PyTorch's complex autograd).  With
 * z = (A^*A)^{-1} g, w = A z, r = f - A c, s = A(k^x o c), t = A(k^x o z):
 *     grad_f = w,
 *     dL/dx_j = 2 pi Im(conj(r_j) t_j - conj(w_j) s_j)   (k^y for dL/dy_j),
 * obtained by differentiating the normal equations A^*A c = A^*f with
 * dA(j,k)/dx_j = -2 pi i k^x A(j,k) (centred k).  f, c, g, grad_f: DEVICE
 * complex128 (nrhs x M, nrhs x nx x ny, nrhs x nx x ny, nrhs x M).
 * grad_points: DEVICE M x 2 doubles in the caller's point order (x, y
 * interleaved) summed over the right-hand sides, or NULL to skip it.  Errors
 * as nudft2_solve_adj. */
nudft2_status nudft2_lsq_backward(nudft2_plan_t plan, const double* f, const double* c,
                                  const double* g, double* grad_f, double* grad_points,
                                  int32_t nrhs, nudft2_solve_info* info);

/* f = A c exactly in FP64 (Section 1 sum).  c: DEVICE nrhs x nx x ny, f:
 * DEVICE nrhs x M.  Does not need the factorization.  Errors: E_INVAL. */
nudft2_status nudft2_apply(nudft2_plan_t plan, const double* c, double* f,
                           int32_t nrhs);

/* c = A^* f exactly in FP64 (the adjoint of the Section 1 sum, which the
 * least-squares iterations of Section 4.1 apply).  f: DEVICE nrhs x M, c:
 * DEVICE nrhs x nx x ny.  Does not need the factorization.  Errors: E_INVAL. */
nudft2_status nudft2_apply_adj(nudft2_plan_t plan, const double* f, double* c,
                               int32_t nrhs);

/* nudft2_apply_adj without device allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, result and kernels as
 * nudft2_apply_adj (the same summation order whenever both split the rows
 * into the same number of chunks); its partial sums live in a static 64 MiB
 * device array per GPU instead of plan memory, so it needs
 * nrhs * nx * ny * 16 bytes <= 64 MiB (summed over the problems of a batch
 * plan), else E_INVAL; larger inputs run with fewer, longer row chunks.  Each
 * GPU's array is shared by every call on that GPU and held until the process
 * ends: calls that overlap on one GPU race (serialise them, e.g. on one
 * stream).  Runs on the plan's stream with the plan's device current.
 * Errors: E_INVAL, E_DEVICE. */
nudft2_status nudft2_apply_adj_noalloc(nudft2_plan_t plan, const double* f, double* c,
                                       int32_t nrhs);

/* f ~= A c (type-2 NUFFT) and c ~= A^* f (type-1 NUFFT) by spreading with an
 * exponential-of-semicircle kernel and FFTs on a twice-oversampled grid (the
 * NUFFT with which Section 4.1 applies A and its adjoint inside the Krylov
 * iterations), in FP64, to relative accuracy about tol (0 < tol < 0.1; the
 * kernel spans ceil(log10(1/tol)) + 2 cells, at most 16).  Shapes and
 * pointers as nudft2_apply / nudft2_apply_adj.  Needs nx, ny <= 1024 and no
 * factorization.  The plan keeps the NUFFT state of the last tol.  Errors:
 * E_INVAL, E_NOMEM, E_DEVICE. */
nudft2_status nudft2_nufft(nudft2_plan_t plan, const double* c, double* f, int32_t nrhs,
                           double tol);
nudft2_status nudft2_nufft_adj(nudft2_plan_t plan, const double* f, double* c, int32_t nrhs,
                               double tol);

/* Fill *info (HOST).  Synchronises with the plan's stream. */
nudft2_status nudft2_get_info(nudft2_plan_t plan, nudft2_info* info);

/* Turn per-kernel-class event timing on (1: every class) or off (0); resets
 * the totals.  Synchronises with the plan's stream. */
nudft2_status nudft2_set_profiling(nudft2_plan_t plan, int32_t on);
/* Event timing for the classes whose bits are set in `classes` (bit c =
 * class c of nudft2_info.kernel_ms; 0 turns timing off): launches of the
 * other classes record no events.  Resets the totals; synchronises with the
 * plan's stream.  E_INVAL for bits beyond the last class. */
nudft2_status nudft2_set_profiling_classes(nudft2_plan_t plan, uint32_t classes);

/* Release every device buffer of the plan.  NULL is accepted. */
nudft2_status nudft2_destroy(nudft2_plan_t plan);

/* Static description of a status code. */
const char* nudft2_strerror(nudft2_status s);

#ifdef __cplusplus
}
#endif

#endif /* NUDFT2_H */
