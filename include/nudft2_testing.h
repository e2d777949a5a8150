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

#ifdef __cplusplus
}
#endif

#endif /* NUDFT2_TESTING_H */
