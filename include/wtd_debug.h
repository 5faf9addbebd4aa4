/*
 * wtd_debug.h - test hooks of libwtd.so (not part of the operator API).
 *
 * These entry points run single internal kernels so that tests can check them
 * in isolation.  Pointers are device memory; calls are asynchronous on the
 * given HIP stream; the return value is a wtd_status (wtd.h).
 */
#ifndef WTD_DEBUG_H
#define WTD_DEBUG_H

#include "wtd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C[m][n] = sum_k A[m*lda + k] * B(k, n) with the library's MFMA GEMM kernel;
 * B(k, n) = B[n*ldb + k] if b_kmajor, else B[k*ldb + n].  prec selects FP64 or
 * FP32 arrays.  Errors: WTD_ERR_ARG for null pointers or negative sizes.     */
wtd_status wtd_debug_gemm(wtd_precision prec, int32_t m, int32_t n, int32_t k, const void *a,
                          int32_t lda, const void *b, int32_t ldb, int32_t b_kmajor, void *c,
                          int32_t ldc, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* WTD_DEBUG_H */
