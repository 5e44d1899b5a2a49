/*
 * Test hook of libharp (not part of the solver's boundary): exposes the
 * batched complex MFMA GEMM used inside reduced_factor / reduced_solve so that
 * tests can check it in isolation.
 *
 * D = beta * C + alpha * A * B for `batch` column-major interleaved-complex
 * matrices (A: M x K, B: K x N, C and D: M x N; all device memory owned by
 * the caller; D may alias C).  dtype as in harp.h.  Strides and leading
 * dimensions in complex elements.  Returns HARP_E_ARG on inconsistent sizes.
 */
#ifndef HARP_DEBUG_H
#define HARP_DEBUG_H

#include "harp.h"

#ifdef __cplusplus
extern "C" {
#endif

harp_status harp_debug_cgemm(harp_dtype dtype, int32_t M, int32_t N, int32_t K, int32_t batch, double alpha,
                             const void *d_A, int64_t lda, int64_t sA, const void *d_B, int64_t ldb, int64_t sB,
                             double beta, const void *d_C, int64_t ldc, int64_t sC, void *d_D, int64_t ldd,
                             int64_t sD, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HARP_DEBUG_H */
