// Host-BLAS interposer: Fortran DGEMM/ZGEMM served by libozaki on the GPU.
// The paper reaches the emulation through intercepted standard BLAS calls
// (Section 3.1); on a discrete GPU that means staging the host operands in
// HBM around each call. See include/ozaki_blas.h for the contract.
#include <hip/hip_runtime.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "../../../include/ozaki_blas.h"

namespace {

struct Staging {
  void *buf[3] = {nullptr, nullptr, nullptr};  // A, B, C
  size_t cap[3] = {0, 0, 0};
};
Staging g_stage;
int g_slices = 0, g_moduli = 0;

char up(char c) { return (char)std::toupper((unsigned char)c); }

int env_int(const char *name) {
  const char *v = std::getenv(name);
  return (v != nullptr && *v) ? std::atoi(v) : 0;
}

void fail(const char *routine, const char *what, int status) {
  std::fprintf(stderr, "ozaki_blas: %s: %s (status %d: %s)\n", routine, what, status,
               ozaki_status_string(status));
  std::abort();
}

void *stage(int which, size_t bytes, const char *routine) {
  if (bytes == 0) bytes = 16;
  if (g_stage.cap[which] < bytes) {
    if (g_stage.buf[which] != nullptr) (void)hipFree(g_stage.buf[which]);
    g_stage.buf[which] = nullptr;
    g_stage.cap[which] = 0;
    if (hipMalloc(&g_stage.buf[which], bytes) != hipSuccess) fail(routine, "hipMalloc", OZAKI_ERR_ALLOC);
    g_stage.cap[which] = bytes;
  }
  return g_stage.buf[which];
}

// Copy the rows x cols column-major block at host (leading dimension ld) into
// a packed device buffer, or back: one linear copy when the columns are
// contiguous (ld == rows), else a pitched copy of exactly the block (the rows
// between `rows` and `ld` are neither read nor written).
void to_device(void *dst, const void *src, int64_t rows, int64_t cols, int64_t ld, size_t esz,
               const char *routine) {
  if (rows == 0 || cols == 0) return;
  const hipError_t e =
      ld == rows ? hipMemcpy(dst, src, rows * cols * esz, hipMemcpyHostToDevice)
                 : hipMemcpy2D(dst, rows * esz, src, ld * esz, rows * esz, cols, hipMemcpyHostToDevice);
  if (e != hipSuccess) fail(routine, "copy to device", OZAKI_ERR_HIP);
}
void to_host(void *dst, const void *src, int64_t rows, int64_t cols, int64_t ld, size_t esz,
             const char *routine) {
  if (rows == 0 || cols == 0) return;
  const hipError_t e =
      ld == rows ? hipMemcpy(dst, src, rows * cols * esz, hipMemcpyDeviceToHost)
                 : hipMemcpy2D(dst, ld * esz, src, rows * esz, rows * esz, cols, hipMemcpyDeviceToHost);
  if (e != hipSuccess) fail(routine, "copy to host", OZAKI_ERR_HIP);
}

// Reference-BLAS argument checks; returns the number of the first illegal
// argument or 0.
int check(char ta, char tb, int m, int n, int k, int lda, int ldb, int ldc) {
  ta = up(ta);
  tb = up(tb);
  const bool oka = ta == 'N' || ta == 'T' || ta == 'C';
  const bool okb = tb == 'N' || tb == 'T' || tb == 'C';
  const int nrowa = ta == 'N' ? m : k;
  const int nrowb = tb == 'N' ? k : n;
  if (!oka) return 1;
  if (!okb) return 2;
  if (m < 0) return 3;
  if (n < 0) return 4;
  if (k < 0) return 5;
  if (lda < (nrowa > 1 ? nrowa : 1)) return 8;
  if (ldb < (nrowb > 1 ? nrowb : 1)) return 10;
  if (ldc < (m > 1 ? m : 1)) return 13;
  return 0;
}

template <typename T>
void gemm(bool cplx, const char *routine, char ta, char tb, int m, int n, int k, T alpha,
          const T *A, int lda, const T *B, int ldb, T beta, T *C, int ldc, bool alpha_zero,
          bool beta_zero, bool beta_one) {
  const int info = check(ta, tb, m, n, k, lda, ldb, ldc);
  if (info != 0) {
    std::fprintf(stderr, " ** On entry to %s parameter number %d had an illegal value\n", routine,
                 info);
    return;
  }
  if (m == 0 || n == 0 || ((alpha_zero || k == 0) && beta_one)) return;
  const size_t esz = sizeof(T);
  ta = up(ta);
  tb = up(tb);
  const int64_t rowsA = ta == 'N' ? m : k, colsA = ta == 'N' ? k : m;
  const int64_t rowsB = tb == 'N' ? k : n, colsB = tb == 'N' ? n : k;
  const bool need_ab = !alpha_zero && k > 0;
  T *dA = static_cast<T *>(stage(0, need_ab ? rowsA * colsA * esz : 0, routine));
  T *dB = static_cast<T *>(stage(1, need_ab ? rowsB * colsB * esz : 0, routine));
  T *dC = static_cast<T *>(stage(2, (size_t)m * n * esz, routine));
  if (need_ab) {
    to_device(dA, A, rowsA, colsA, lda, esz, routine);
    to_device(dB, B, rowsB, colsB, ldb, esz, routine);
  }
  if (!beta_zero) to_device(dC, C, m, n, ldc, esz, routine);
  const int64_t ldA = rowsA > 1 ? rowsA : 1, ldB = rowsB > 1 ? rowsB : 1;
  int slices = g_slices, moduli = g_moduli;
  if (slices == 0 && moduli == 0) {
    moduli = env_int("OZAKI_BLAS_MODULI");
    slices = moduli > 0 ? 0 : env_int("OZAKI_BLAS_SLICES");
    if (slices == 0 && moduli == 0) slices = 7;
  }
  int rc;
  if constexpr (sizeof(T) == sizeof(ozaki_z)) {
    rc = slices > 0 ? ozaki_zgemm(ta, tb, m, n, k, alpha, dA, ldA, dB, ldB, beta, dC, m, slices)
                    : ozaki2_zgemm(ta, tb, m, n, k, alpha, dA, ldA, dB, ldB, beta, dC, m, moduli);
  } else {
    rc = slices > 0 ? ozaki_dgemm(ta, tb, m, n, k, alpha, dA, ldA, dB, ldB, beta, dC, m, slices)
                    : ozaki2_dgemm(ta, tb, m, n, k, alpha, dA, ldA, dB, ldB, beta, dC, m, moduli);
  }
  (void)cplx;
  if (rc != 0) fail(routine, "emulated GEMM", rc);
  if (hipDeviceSynchronize() != hipSuccess) fail(routine, "synchronize", OZAKI_ERR_HIP);
  to_host(C, dC, m, n, ldc, esz, routine);
}

}  // namespace

extern "C" {

void dgemm_(const char *transa, const char *transb, const int *m, const int *n, const int *k,
            const double *alpha, const double *A, const int *lda, const double *B,
            const int *ldb, const double *beta, double *C, const int *ldc) {
  gemm<double>(false, "DGEMM ", *transa, *transb, *m, *n, *k, *alpha, A, *lda, B, *ldb, *beta, C,
               *ldc, *alpha == 0.0, *beta == 0.0, *beta == 1.0);
}

void zgemm_(const char *transa, const char *transb, const int *m, const int *n, const int *k,
            const ozaki_z *alpha, const ozaki_z *A, const int *lda, const ozaki_z *B,
            const int *ldb, const ozaki_z *beta, ozaki_z *C, const int *ldc) {
  gemm<ozaki_z>(true, "ZGEMM ", *transa, *transb, *m, *n, *k, *alpha, A, *lda, B, *ldb, *beta, C,
                *ldc, alpha->re == 0.0 && alpha->im == 0.0, beta->re == 0.0 && beta->im == 0.0,
                beta->re == 1.0 && beta->im == 0.0);
}

int ozaki_blas_config(int slices, int moduli) {
  if (slices < 0 || slices > OZAKI_S_MAX) return -1;
  if (moduli != 0 && (moduli < OZAKI2_MODULI_MIN || moduli > OZAKI2_MODULI_MAX)) return -2;
  g_slices = slices;
  g_moduli = slices > 0 ? 0 : moduli;
  return 0;
}

int ozaki_blas_release(void) {
  int rc = 0;
  for (int w = 0; w < 3; ++w) {
    if (g_stage.buf[w] != nullptr && hipFree(g_stage.buf[w]) != hipSuccess) rc = OZAKI_ERR_HIP;
    g_stage.buf[w] = nullptr;
    g_stage.cap[w] = 0;
  }
  return rc;
}

}  // extern "C"
