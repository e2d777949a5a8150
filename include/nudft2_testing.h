/*
 * Test hooks of the nudft2 library.  Not part of the solver's interface:
 * these entry points expose internal building blocks so that the test-suite
 * can check them one by one.  Same conventions as nudft2.h (status codes, no
 * exceptions across the boundary).
 */
#ifndef NUDFT2_TESTING_H
#define NUDFT2_TESTING_H

#include "nudft2.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Message of the last error raised inside the library (thread-local, static
 * storage; "" if none). */
const char* nudft2_last_error(void);

/* Host-only binning of one problem (no device work).  points: HOST M x 2.
 * Outputs (HOST, caller-allocated): perm2d[M] = caller index of the i-th point
 * in quadtree order; leaf_rows[4^L + 1] = row offsets of the leaves in Morton
 * order; colperm[nx*ny] = natural column index (ky + kx ny, 0-based kx, ky) of
 * the i-th column in quadtree column order.  Returns the depth L via *depth. */
nudft2_status nudft2_test_binning(const double* points, int64_t M, int32_t nx,
                                  int32_t ny, int32_t leaf, int64_t* perm2d,
                                  int64_t* leaf_rows, int64_t* colperm,
                                  int32_t* depth);

/* One 16x16x4 FP64 matrix-core step on the device with A[i][k] = a[i*4+k],
 * B[k][j] = b[k*16+j] (HOST inputs); writes D = A B (16 x 16, row-major) to
 * the HOST array d, writing accumulator register v of lane l to row l/16+4v,
 * column l%16 (the interleaved row layout of the FP64 instruction). */
nudft2_status nudft2_test_mfma_layout(const double* a, const double* b, double* d);

/* Same for the FP32 16x16x4 step.  The probe writes the accumulator register
 * v of lane l to row 4(l/16)+v, column l%16 of d, so d equals A B exactly when
 * the instruction uses that (blocked) row layout. */
nudft2_status nudft2_test_mfma_layout32(const float* a, const float* b, float* d);

/* Batched dense building blocks on DEVICE data (complex128 when prec == 0,
 * complex64 when prec == 1 or 2; column-major with leading dimensions).
 * complex64 tile products run on the FP32 matrix instructions with prec 1
 * and on the bf16 ones through the three-way split (nudft2_opts
 * fp32_products = 0) with prec 2.  Per
 * problem sizes, leading dimensions and device addresses are HOST arrays;
 * all work runs on the default stream and is finished on return.
 *
 * gemm:  C_i = alpha op(A_i) op(B_i) + beta C_i; op 0 = none, 1 = conj
 *        transpose; mnk = (m, n, k) per problem, ld = (lda, ldb, ldc),
 *        ptrs = (A, B, C).
 * geqrf: Householder QR; mn = (m, n), ld = (lda, ldr), ptrs = (A, R, Tb).
 *        A returns the explicit unit lower-trapezoidal reflectors V, R the
 *        triangular factor, Tb the compact-WY factors of the column blocks
 *        of 256 reflectors (Q = prod_b (I - V_b T_b V_b^H)): with
 *        k = min(m, n), block b has kb = min(256, k - 256 b) columns and its
 *        kb x kb factor T_b (leading dimension kb) starts at element
 *        256^2 b of Tb (Tb holds 256^2 (nb - 1) + kb_last^2 elements).
 * ormqr: C <- Q C (trans = 0) or Q^H C (trans = 1) with dims = (m, k, nc),
 *        ld = (ldv, ldc), ptrs = (V, Tb, C); trans = 2: C <- Q C for C
 *        holding [I; 0] on entry (explicit Q formation, which skips the
 *        columns each block leaves unchanged).
 * pchol: diagonally pivoted Cholesky of Hermitian PSD K_i (w_i x w_i,
 *        complex128, leading dimension w_i, overwritten) into L_i (w_i x
 *        rmax_i), stopping when the remaining Schur-complement trace is at
 *        most tol2 * trace(K_i).  rank_out (HOST, nb) and piv_out (HOST,
 *        sum rmax_i) receive the ranks and pivot rows.
 * trsv:  R_i X_i = B_i (conj_trans = 0) or R_i^H X_i = B_i (conj_trans = 1)
 *        in place, R upper triangular; dims = (k, nrhs), ld = (ldr, ldb),
 *        ptrs = (R, B). */
nudft2_status nudft2_test_gemm(int32_t prec, int32_t opA, int32_t opB, int32_t nb,
                               const int32_t* mnk, const int32_t* ld, const int64_t* ptrs,
                               double alpha_re, double alpha_im, double beta);
/* gemm with a forced k split or tile shape (splits >= 1: that many plain k
 * splits of the 64 x 64 output tiles; 0 = the library's choice; -1 = the tile
 * kernel without splitting and without the tuned table; -2 = the library's
 * heuristic without the tuned table; -3 = stream-K shares of the tiles' k
 * stages wherever the batch allows; -4 = k splits into partial tiles summed
 * in split order by a second kernel; -5 = 32 x 128 output tiles, -6 = 16- or
 * 32-square output tiles, both for opA = 1, opB = 0, m <= 32 and 8 < n <=
 * 128 (-5) or <= 32 (-6), else NUDFT2_E_INVAL) and the
 * launch's duration in milliseconds (HIP events on the null stream) written to
 * *ms (HOST, may be NULL): the measurement hook of the GEMM autotuner. */
nudft2_status nudft2_test_gemm_cfg(int32_t prec, int32_t opA, int32_t opB, int32_t nb,
                                   const int32_t* mnk, const int32_t* ld, const int64_t* ptrs,
                                   double alpha_re, double alpha_im, double beta,
                                   int32_t splits, float* ms);
nudft2_status nudft2_test_geqrf(int32_t prec, int32_t nb, const int32_t* mn,
                                const int32_t* ld, const int64_t* ptrs);
nudft2_status nudft2_test_ormqr(int32_t prec, int32_t trans, int32_t nb,
                                const int32_t* dims, const int32_t* ld,
                                const int64_t* ptrs);
nudft2_status nudft2_test_pchol(int32_t nb, const int32_t* w, const int32_t* rmax,
                                const int64_t* ptrs, double tol2, int32_t* rank_out,
                                int32_t* piv_out);
nudft2_status nudft2_test_trsv(int32_t prec, int32_t nb, const int32_t* dims,
                               const int32_t* ld, const int64_t* ptrs, int32_t conj_trans);
/* in-place inversion of nb upper-triangular matrices (zeros below the
 * diagonal): k[i], ld[i], ptrs[i] (DEVICE); R_i <- R_i^{-1} */
nudft2_status nudft2_test_trtri(int32_t prec, int32_t nb, const int32_t* k, const int32_t* ld,
                                const int64_t* ptrs);
/* copy with precision change: D_i = S_i (conj_trans[i] = 0, D_i m x n) or
 * D_i = S_i^H (conj_trans[i] != 0, D_i n x m), S_i m x n; prec_d / prec_s
 * select complex128 (0) or complex64 (1) for D and S; dims = (m, n),
 * ld = (lds, ldd), ptrs = (S, D); conj_trans is a HOST array of nb ints.
 * Sources and destinations must not overlap.  NUDFT2_E_INVAL on a
 * precision other than 0 / 1, negative sizes or leading dimensions too
 * small for the stated shapes. */
nudft2_status nudft2_test_copy(int32_t prec_d, int32_t prec_s, int32_t nb, const int32_t* dims,
                               const int32_t* ld, const int64_t* ptrs,
                               const int32_t* conj_trans);

/* 1D HSS compression of G^x (dim 0) or G^y (dim 1) of every problem of the
 * plan at tolerance tol (no factorization needed), then y = H x for problem
 * `prob` with x: DEVICE n complex128 in natural column order (0-based
 * frequency l), y: DEVICE M_prob complex128, the problem's points in the
 * caller's order.  ranks (HOST, 2*(L+1) ints, may be
 * NULL) receives the largest row / column rank per level. */
/* fADI factor of the HSS row block G(J_a, K_a^c) of node (level, a) of a 1D
 * tree with n columns (K_a = the columns l with l/n in [a/2^level,
 * (a+1)/2^level)), relative accuracy tau (the library uses a tenth of the 1D
 * tolerance).  Writes (b, s) to HOST plan_out[2] (b near columns a side,
 * s shifts; b = 0: the library keeps all of K_a^c exactly), the gamma of the
 * arcs' symmetric image to *gamma, and the shifts to HOST pq (complex128
 * pairs): p_j at pq[2j], q_j at pq[2(smax + j)], j < s.  When Z and W are
 * not NULL and b > 0, also fills DEVICE Z (m x (2b+s), leading dimension
 * max(m, 1)) and W (n x (2b+s), leading dimension n), complex128, from the
 * DEVICE row coordinates xs[m]: G(J_a, l) ~= sum_j Z(., j) conj(W(l, j)) for
 * l outside K_a; Z's first 2b columns are the kernel columns (hi + c) mod n,
 * then (lo - b + c) mod n, c < b, with unit W entries; the next s are the fADI
 * vectors and W carries the conjugated weighted column vectors.
 * NUDFT2_E_INVAL if s > smax (plan_out and gamma are still written). */
nudft2_status nudft2_test_fadi_block(const double* xs, int64_t m, int32_t n, int32_t level,
                                     int32_t a, double tau, int32_t* plan_out, double* gamma,
                                     double* pq, int32_t smax, double* Z, double* W);

nudft2_status nudft2_test_hss1d_matvec(nudft2_plan_t plan, int32_t dim, double tol,
                                       const double* x, double* y, int32_t* ranks,
                                       int32_t prob);

/* Build the recompressed HSS approximation of G (1D stage at eps/10,
 * face-splitting assembly, recompression at eps) of every problem of the plan
 * in the plan's precision, then Y = H X for problem `prob` (X: DEVICE nrhs x
 * N_prob complex128, each row in natural column order l^y + l^x ny, 0-based;
 * Y: DEVICE nrhs x M_prob complex128, the problem's points in the caller's
 * order).  stages: 0 = face-splitting generators only, 1 = after the exact
 * orthogonalisation stage, 2 = fully recompressed.  The ranks per level are
 * left in the plan's info. */
nudft2_status nudft2_test_hss_matvec(nudft2_plan_t plan, const double* x, double* y,
                                     int32_t stages, int32_t prob, int32_t nrhs);

#ifdef __cplusplus
}
#endif

#endif /* NUDFT2_TESTING_H */
