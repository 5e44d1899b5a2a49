/*
 * Kernel-class timers of libharp (instrumentation, not part of the solver's
 * boundary).  When enabled, every launch of the library's kernels is
 * bracketed by two HIP events recorded on the launch's own stream, and the
 * launch's algorithmic work (flops, bytes) is attached to it.  Reading a class
 * synchronises on its events and returns totals over the launches recorded
 * since the last harp_prof_enable(1).
 *
 * For callers that time whole passes: enable, run, read, disable.  Not for
 * use under stream capture; not thread-safe (one profiling thread).
 *
 * Algorithmic work per launch: complex GEMM 8 M N K flops (per matrix of the
 * batch that is active); rank-w update 8 M N w flops and the bytes of one
 * read and one write of the updated block plus one read of its two factors;
 * fill 8 / 16 / 24 bytes written per entry (complex64
 * / complex128 / both) and 0 flops (its flops, (2P+1)(2Q+4) * 2 per
 * model-evaluated entry, depend on each model's order, which the caller
 * knows); other classes report 0.
 */
#ifndef HARP_PROF_H
#define HARP_PROF_H

#include "harp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HARP_K_FILL = 0,      /* harp_fill kernels */
    HARP_K_GETF2 = 1,     /* pivoting panel factorisation */
    HARP_K_TRSM_L = 2,    /* row exchanges + unit-lower block solve */
    HARP_K_TRSM_U = 3,    /* upper block solve */
    HARP_K_GEMM32 = 4,    /* complex64 MFMA GEMM */
    HARP_K_GEMM64 = 5,    /* complex128 MFMA GEMM */
    HARP_K_AUX = 6,       /* conversions, norms, axpy, ports, info reset */
    HARP_K_RANK = 7,      /* rank-w update of an outer block after a panel */
    HARP_K_COUNT = 8
} harp_kernel_class;

/* Call sites of the matrix-core GEMM classes (HARP_K_GEMM32 / GEMM64), read
 * with harp_prof_read_site. */
typedef enum {
    HARP_SITE_OTHER = 0,          /* harp_cgemm and the adjoint's products */
    HARP_SITE_TRAILING = 1,       /* LU trailing update of a super-block */
    HARP_SITE_CATCH_UP = 2,       /* LU: earlier blocks of the super-block on an outer block's columns */
    HARP_SITE_DEFERRED_ROWS = 3,  /* LU: the same on an outer block's row block */
    HARP_SITE_BLOCK_ROW = 4,      /* LU: block row U12 = L11^-1 A12 */
    HARP_SITE_TRI_INVERSE = 5,    /* inverses of the solve groups' diagonal blocks */
    HARP_SITE_SOLVE_DIAG = 6,     /* solve: a group's inverse diagonal block */
    HARP_SITE_SOLVE_UPDATE = 7,   /* solve: update of the rows below / above a group */
    HARP_SITE_RESIDUAL = 8,       /* refinement residual B - Z X */
    HARP_SITE_RESIDUAL_UPDATE = 9, /* refinement: Z D of a correction (complex64, K slices) */
    HARP_SITE_COUNT = 10
} harp_gemm_site;

/* on != 0: clear the records and start recording; on == 0: stop. */
harp_status harp_prof_enable(int32_t on);

/* Stop recording and destroy the pooled events (call before the HIP runtime
 * shuts down, e.g. from an interpreter exit hook; the library keeps no
 * static object whose destructor would do it at process exit). */
harp_status harp_prof_release(void);

/* Totals of one class: launches, summed event time (ms), flops, bytes. */
harp_status harp_prof_read(int32_t cls, int64_t *launches, double *ms, double *flops, double *bytes);

/* The same totals restricted to one call site of a GEMM class. */
harp_status harp_prof_read_site(int32_t cls, int32_t site, int64_t *launches, double *ms, double *flops,
                                double *bytes);

#ifdef __cplusplus
}
#endif

#endif /* HARP_PROF_H */
