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
 * on the current device (f64 != 0: float64, else float32) with
 * A[i][k] = i + 1 + 100 k, B[0][j] = 1 + 1000 j, B[k>0][j] = 0 and copies the
 * 64 lanes x 4 accumulators (lane-major; 256 floats or doubles) to the HOST
 * buffer out_host.  Lane l, slot e holds (i + 1)(1 + 1000 j) with j = l % 16
 * and i = 4 (l / 16) + e (float32) or l / 16 + 4 e (float64), as measured on
 * gfx950.  Errors: FMM_ERR_INVALID (NULL out_host), FMM_ERR_DEVICE. */
FMM_API fmm_status fmm_debug_mfma_layout(int32_t f64, void *out_host);

#ifdef __cplusplus
}
#endif
#endif /* FMM_DIAG_H_ */
