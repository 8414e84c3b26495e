// Blocked LU with partial pivoting and the inverse of a complex matrix: the
// kernels around the trailing-update GEMMs. The paper's solver inverts the
// multiple-scattering matrix by LU (Section 3.2: ZGEMM and ZTRSM take most of
// its time), so the emulated ZGEMM sits inside this factorization. Every
// complex operation is written out with separately rounded real operations
// (no fused multiply-adds) in a fixed order, so the CPU model repeats it bit
// for bit:
//   product   (ar br - ai bi, ar bi + ai br)
//   quotient  d = br br + bi bi, ((ar br + ai bi) / d, (ai br - ar bi) / d)
//   pivot     the first row of the largest |Re| + |Im| in the column
#include "ozaki_internal.hpp"

namespace oz {
namespace {

struct Z {
  double re, im;
};

__device__ __forceinline__ Z ld(const double2 *p) {
  const double2 v = *p;
  return Z{v.x, v.y};
}
__device__ __forceinline__ void st(double2 *p, Z z) { *p = make_double2(z.re, z.im); }

__device__ __forceinline__ Z zmul(Z a, Z b) {
  return Z{sub_rn(mul_rn(a.re, b.re), mul_rn(a.im, b.im)), add_rn(mul_rn(a.re, b.im), mul_rn(a.im, b.re))};
}
__device__ __forceinline__ Z zsub(Z a, Z b) { return Z{sub_rn(a.re, b.re), sub_rn(a.im, b.im)}; }
__device__ __forceinline__ Z zdiv(Z a, Z b) {
  const double d = add_rn(mul_rn(b.re, b.re), mul_rn(b.im, b.im));
  return Z{__ddiv_rn(add_rn(mul_rn(a.re, b.re), mul_rn(a.im, b.im)), d),
           __ddiv_rn(sub_rn(mul_rn(a.im, b.re), mul_rn(a.re, b.im)), d)};
}
__device__ __forceinline__ double cabs1(Z a) { return add_rn(fabs(a.re), fabs(a.im)); }

// Pivot of column c (rows c..n-1), then the swap of rows c and the pivot row
// over the panel columns [p0, p1). One workgroup of 1024 threads. A zero
// pivot column is recorded in *singular (the smallest such column). When
// c > p0 the workgroup first stores the multipliers of column c - 1
// (l_i = a_i,c-1 / a_c-1,c-1 for i >= c), which the panel update of that
// column has finished using.
__global__ void __launch_bounds__(1024) k_pivot_swap(double2 *A, int64_t lda, int64_t n, int64_t c,
                                                     int64_t p0, int64_t p1, int64_t *ipiv,
                                                     int64_t *singular) {
  __shared__ double sv[1024];
  __shared__ int64_t si[1024];
  const int t = threadIdx.x;
  if (c > p0) {
    const int64_t q = c - 1;
    const Z p = ld(A + q + q * lda);
    for (int64_t i = c + t; i < n; i += 1024) st(A + i + q * lda, zdiv(ld(A + i + q * lda), p));
    __syncthreads();
  }
  double best = -1.0;
  int64_t bi = n;
  for (int64_t i = c + t; i < n; i += 1024) {
    const double v = cabs1(ld(A + i + c * lda));
    if (v > best) {  // rows visited in increasing order: ties keep the first
      best = v;
      bi = i;
    }
  }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) {
      const double vo = sv[t + w];
      const int64_t io = si[t + w];
      if (vo > sv[t] || (vo == sv[t] && io < si[t])) {
        sv[t] = vo;
        si[t] = io;
      }
    }
    __syncthreads();
  }
  const int64_t piv = si[0];
  if (t == 0) {
    ipiv[c] = piv;
    if (!(sv[0] > 0.0)) atomicMin(reinterpret_cast<unsigned long long *>(singular),
                                  (unsigned long long)c);
  }
  if (piv != c) {
    for (int64_t k = p0 + t; k < p1; k += 1024) {
      const Z a = ld(A + c + k * lda), b = ld(A + piv + k * lda);
      st(A + c + k * lda, b);
      st(A + piv + k * lda, a);
    }
  }
}

// Panel update after the pivot of column c: a_ik -= (a_ic / a_cc) a_ck for
// rows i > c and panel columns c < k < p1, one thread per element (each
// recomputes its row's multiplier). The multipliers l_i = a_ic / a_cc are
// stored afterwards: by the next column's pivot workgroup, or by k_panel_mult
// for the last column of the panel.
__global__ void __launch_bounds__(256) k_panel_update(double2 *A, int64_t lda, int64_t n, int64_t c) {
  const int64_t i = c + 1 + (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t k = c + 1 + blockIdx.y;
  if (i >= n) return;
  const Z l = zdiv(ld(A + i + c * lda), ld(A + c + c * lda));
  st(A + i + k * lda, zsub(ld(A + i + k * lda), zmul(l, ld(A + c + k * lda))));
}

__global__ void __launch_bounds__(256) k_panel_mult(double2 *A, int64_t lda, int64_t n, int64_t c) {
  const int64_t i = c + 1 + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  st(A + i + c * lda, zdiv(ld(A + i + c * lda), ld(A + c + c * lda)));
}

// Row interchanges ipiv[c0..c1) applied in order to the columns [q0, q1) of A.
__global__ void __launch_bounds__(256) k_laswp(double2 *A, int64_t lda, int64_t c0, int64_t c1,
                                               const int64_t *ipiv, int64_t q0, int64_t q1) {
  const int64_t k = q0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= q1) return;
  for (int64_t c = c0; c < c1; ++c) {
    const int64_t p = ipiv[c];
    if (p == c) continue;
    const Z a = ld(A + c + k * lda), b = ld(A + p + k * lda);
    st(A + c + k * lda, b);
    st(A + p + k * lda, a);
  }
}

// X <- T^-1 X for the nb x nb triangle T (at T, leading dimension ldt) on
// ncols columns of X, column-oriented: one workgroup per column, thread r
// holds x_r. Unit lower (forward): for k = 0, 1, ..., x_k is final and every
// x_r with r > k takes x_r -= t_rk x_k. Non-unit upper (backward): for
// k = nb-1 down to 0, x_k = x_k / t_kk is final and every x_r with r < k takes
// x_r -= t_rk x_k. Each x_r thus subtracts its terms in the order of k (forward:
// increasing, backward: decreasing). One barrier per step; the final x_k goes
// through LDS slot k.
template <bool UPPER>
__global__ void __launch_bounds__(1024) k_trsm(const double2 *T, int64_t ldt, int nb, double2 *X,
                                               int64_t ldx) {
  __shared__ double2 xs[1024];
  const int r = threadIdx.x;
  double2 *x = X + (int64_t)blockIdx.x * ldx;
  Z xr = r < nb ? ld(x + r) : Z{0.0, 0.0};
  if constexpr (!UPPER) {
    for (int k = 0; k < nb - 1; ++k) {
      if (r == k) xs[k] = make_double2(xr.re, xr.im);
      __syncthreads();
      if (r > k && r < nb) {
        const double2 v = xs[k];
        xr = zsub(xr, zmul(ld(T + r + (int64_t)k * ldt), Z{v.x, v.y}));
      }
    }
  } else {
    for (int k = nb - 1; k >= 0; --k) {
      if (r == k) {
        xr = zdiv(xr, ld(T + r + (int64_t)r * ldt));
        xs[k] = make_double2(xr.re, xr.im);
      }
      __syncthreads();
      if (r < k) {
        const double2 v = xs[k];
        xr = zsub(xr, zmul(ld(T + r + (int64_t)k * ldt), Z{v.x, v.y}));
      }
    }
  }
  if (r < nb) st(x + r, xr);
}

// X = identity (n x n, leading dimension ldx).
__global__ void __launch_bounds__(256) k_identity(double2 *X, int64_t ldx, int64_t n) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx % n, j = idx / n;
  X[i + j * ldx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
}

__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, st, p, v);
  return hipGetLastError();
}

hipError_t launch_lu_column(double2 *A, int64_t lda, int64_t n, int64_t c, int64_t p0, int64_t p1,
                            int64_t *ipiv, int64_t *singular, hipStream_t st) {
  hipLaunchKernelGGL(k_pivot_swap, dim3(1), dim3(1024), 0, st, A, lda, n, c, p0, p1, ipiv, singular);
  if (c + 1 < n) {
    if (c + 1 < p1)
      hipLaunchKernelGGL(k_panel_update, dim3(blocks(n - c - 1), (unsigned)(p1 - c - 1)), dim3(256), 0,
                         st, A, lda, n, c);
    else
      hipLaunchKernelGGL(k_panel_mult, dim3(blocks(n - c - 1)), dim3(256), 0, st, A, lda, n, c);
  }
  return hipGetLastError();
}

hipError_t launch_laswp(double2 *A, int64_t lda, int64_t c0, int64_t c1, const int64_t *ipiv,
                        int64_t q0, int64_t q1, hipStream_t st) {
  if (q1 <= q0 || c1 <= c0) return hipSuccess;
  hipLaunchKernelGGL(k_laswp, dim3(blocks(q1 - q0)), dim3(256), 0, st, A, lda, c0, c1, ipiv, q0, q1);
  return hipGetLastError();
}

hipError_t launch_trsm(bool upper, const double2 *T, int64_t ldt, int64_t nb, double2 *X,
                       int64_t ldx, int64_t ncols, hipStream_t st) {
  if (ncols <= 0 || nb <= 0) return hipSuccess;
  if (nb > kLuMaxBlock || ncols > 0x7fffffffll) return hipErrorInvalidValue;
  const dim3 block((unsigned)((nb + 63) / 64 * 64));
  if (upper)
    hipLaunchKernelGGL(k_trsm<true>, dim3((unsigned)ncols), block, 0, st, T, ldt, (int)nb, X, ldx);
  else
    hipLaunchKernelGGL(k_trsm<false>, dim3((unsigned)ncols), block, 0, st, T, ldt, (int)nb, X, ldx);
  return hipGetLastError();
}

hipError_t launch_identity(double2 *X, int64_t ldx, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_identity, dim3(blocks(n * n)), dim3(256), 0, st, X, ldx, n);
  return hipGetLastError();
}

}  // namespace oz
