/*
 * ozaki_blas.h - host-BLAS entry points of libozaki_blas.so, the interposer
 * that serves standard Fortran-BLAS DGEMM/ZGEMM calls with the emulated GEMMs
 * of libozaki.so.
 *
 * The paper runs the emulation under an unmodified application by intercepting
 * its standard BLAS GEMM calls (Section 3.1). On a discrete MI355X the operands
 * live in host memory, so each call copies op(A), op(B) (and C when beta != 0)
 * to the GPU, runs ozaki_zgemm / ozaki_dgemm (or the Ozaki-II entry points),
 * and copies C back before returning. Load it ahead of the host BLAS
 * (LD_PRELOAD=libozaki_blas.so, or link it first); every DGEMM/ZGEMM of the
 * process then runs on the GPU. There is no host fallback: every call, small
 * or large, runs on the GPU.
 *
 * Configuration (read at every call, so a process may change it between calls):
 *   OZAKI_BLAS_SLICES   Ozaki-I slice count (1..OZAKI_S_MAX, default 7)
 *   OZAKI_BLAS_MODULI   if set (2..OZAKI2_MODULI_MAX), use Ozaki-II with this
 *                       many moduli instead
 *   ozaki_blas_config() overrides both environment variables (0 = unset).
 *
 * Arguments follow reference BLAS (Fortran calling convention: every scalar by
 * reference, column-major host arrays, hidden character-length arguments not
 * read). An illegal argument prints the reference message naming its number
 * to stderr and returns with C untouched. A device failure prints the
 * library's status and aborts the process (a BLAS routine has no error
 * return, and silently unchanged results are worse than a stop).
 * Device buffers are grow-only and kept until ozaki_blas_release(); calls are
 * not thread safe.
 */
#ifndef OZAKI_BLAS_H
#define OZAKI_BLAS_H

#include "ozaki.h"

#ifdef __cplusplus
extern "C" {
#endif

void dgemm_(const char *transa, const char *transb, const int *m, const int *n, const int *k,
            const double *alpha, const double *A, const int *lda, const double *B,
            const int *ldb, const double *beta, double *C, const int *ldc);
void zgemm_(const char *transa, const char *transb, const int *m, const int *n, const int *k,
            const ozaki_z *alpha, const ozaki_z *A, const int *lda, const ozaki_z *B,
            const int *ldb, const ozaki_z *beta, ozaki_z *C, const int *ldc);

/* slices > 0 selects Ozaki-I with that many slices, else moduli > 0 selects
 * Ozaki-II; both 0 returns to the environment variables. Returns 0, or -1 / -2
 * for a slice / moduli count out of range. */
int ozaki_blas_config(int slices, int moduli);
/* Frees the interposer's device staging buffers. */
int ozaki_blas_release(void);

#ifdef __cplusplus
}
#endif

#endif
