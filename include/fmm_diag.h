/*
 * fmm_diag.h -- diagnostics of the MI355X (gfx950) FMM library that are not
 * part of the evaluation interface of fmm.h.
 *
 * They compute nothing of the method; they exist so that a test can check,
 * on the device at hand, a hardware property the kernels rely on.  Same
 * status codes and conventions as fmm.h.
 */
#ifndef FMM_DIAG_H_
#define FMM_DIAG_H_

#include "fmm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Matrix-core lane layout the batched M2L relies on: runs one 16x16x4 MFMA
 * on the current device (f64 = 1: float64, 0: float32) with
 * A[i][k] = i + 1 + 100 k, B[0][j] = 1 + 1000 j, B[k>0][j] = 0 and copies the
 * 64 lanes x 4 accumulators (lane-major; 256 floats or doubles) to the HOST
 * buffer out_host.  Lane l, slot e holds (i + 1)(1 + 1000 j) with j = l % 16
 * and i = 4 (l / 16) + e (float32) or l / 16 + 4 e (float64), as measured on
 * gfx950.  f64 = 2: one float32 4x4x1 MFMA (sixteen 4x4 blocks, the short
 * last row tile of the M2L) with A_b[i] = i + 1 + 16 b on lane 4 b + i and
 * B_b[jj] = 1 + 1000 jj on lane 4 b + jj; lane 4 b + jj, slot e is expected
 * to hold (e + 1 + 16 b)(1 + 1000 jj).  Errors: FMM_ERR_INVALID (NULL
 * out_host, f64 outside 0..2), FMM_ERR_DEVICE. */
FMM_API fmm_status fmm_debug_mfma_layout(int32_t f64, void *out_host);

#ifdef __cplusplus
}
#endif
#endif /* FMM_DIAG_H_ */
