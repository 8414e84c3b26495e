// ozaki_zgemm_noalloc: the emulated ZGEMM for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc). Its scratch (exponent codes, packed slices and the
// int64 carry space of long contractions) is one file-scope device array of
// OZAKI_NOALLOC_SCRATCH_BYTES, which each device holds from the moment the
// library's code is loaded on it until the process ends.
//
// The array's name is only a host-side stand-in for the device symbol. Its
// device address is taken once per device with hipGetSymbolAddress (with that
// device current) on the entry point's first call there, kept per device, and
// only that address is handed to the kernels.
#include "../../include/ozaki.h"
#include "ozaki_internal.hpp"

namespace {

constexpr int kMaxDevices = 16;
constexpr size_t kScratchBytes = OZAKI_NOALLOC_SCRATCH_BYTES;

__device__ __align__(256) char scratch[kScratchBytes];

// Device address of `scratch` on each device (nullptr: not looked up yet).
char *g_scratch_ptr[kMaxDevices] = {};

int scratch_address(char **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return OZAKI_ERR_NO_DEVICE;
  if (g_scratch_ptr[dev] == nullptr) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return OZAKI_ERR_HIP;
    }
    g_scratch_ptr[dev] = static_cast<char *>(p);
  }
  *out = g_scratch_ptr[dev];
  return OZAKI_OK;
}

}  // namespace

extern "C" {

int ozaki_zgemm_noalloc(char transa, char transb, int64_t m, int64_t n, int64_t k, ozaki_z alpha,
                        const ozaki_z *A, int64_t lda, const ozaki_z *B, int64_t ldb, ozaki_z beta,
                        ozaki_z *C, int64_t ldc, int slices) {
  return oz::zgemm_fixed_scratch(transa, transb, m, n, k, alpha.re, alpha.im, A, lda, B, ldb,
                                 beta.re, beta.im, C, ldc, slices, scratch_address, kScratchBytes);
}

}  // extern "C"
