// Randomized FP64 residual probe of an emulated product (gfx950).
//
// The emulation's error is not observable without a reference, so the
// selector's choice of slice count is checked with a Freivalds-style probe:
// for sign vectors x_v (entries +-1),
//   r_v = C x_v - op(A) (op(B) x_v),
// computed with compensated dot products (Ogita, Rump and Oishi 2005: TwoSum
// accumulation, TwoProd through fma) and kept as unevaluated double-double
// pairs, so that r_v is accurate even though it is ~1e-13 of C x_v. With
// u = |op(A)| (|op(B)| 1) the per-row statistic
//   est_i = sqrt(mean_v |r_v,i|^2) * sqrt(n) / u_i
// estimates the componentwise error scale |C - C*|_ij / (|A||B|)_ij of row i
// (random signs make |r_v,i| ~ rms error * u_i / sqrt(n)). The paper states
// that accuracy depends on the arithmetic precision and on properties of the
// operator (abstract, and Section 4); the probe measures the second part at
// O(mk + kn + mn) cost instead of predicting it.
//
// Sign vectors: x_v[j] = +1 or -1 by the top bit of SplitMix64(seed + v*n + j)
// (Steele, Lea and Flood 2014; the finalizer constants of Vigna's published
// splitmix64).
#include "ozaki_internal.hpp"

namespace oz {

namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double sign_of(uint64_t seed, int v, int64_t n, int64_t j) {
  return (splitmix64(seed + (uint64_t)v * (uint64_t)n + (uint64_t)j) >> 63) ? -1.0 : 1.0;
}

// Compensated accumulator: value = hi + lo (unevaluated).
struct Dd {
  double hi = 0.0, lo = 0.0;
};

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = add_rn(a, b);
  const double z = sub_rn(s, a);
  e = add_rn(sub_rn(a, sub_rn(s, z)), sub_rn(b, z));
}

// acc += a (a exact)
__device__ __forceinline__ void acc_add(Dd &acc, double a) {
  double s, e;
  two_sum(acc.hi, a, s, e);
  acc.hi = s;
  acc.lo = add_rn(acc.lo, e);
}

// acc += a * b (TwoProd via fma)
__device__ __forceinline__ void acc_mac(Dd &acc, double a, double b) {
  const double p = mul_rn(a, b);
  const double pe = __fma_rn(a, b, -p);
  acc_add(acc, p);
  acc.lo = add_rn(acc.lo, pe);
}

constexpr int kMaxVec = 4;

template <bool CPLX>
__device__ __forceinline__ double2 ld(const View &v, int64_t r, int64_t l) {
  if (CPLX) {
    double2 z = reinterpret_cast<const double2 *>(v.base)[r * v.sr + l * v.sl];
    if (v.conj) z.y = -z.y;
    return z;
  }
  return make_double2(reinterpret_cast<const double *>(v.base)[r * v.sr + l * v.sl], 0.0);
}

// w_v[l] = sum_j op(B)(l, j) x_v[j] and ub[l] = sum_j |op(B)(l, j)|, one thread
// per l. vb views op(B) with rows = columns j and contraction = l, so
// op(B)(l, j) = vb(j, l). Output per l: [v][re.hi, re.lo, im.hi, im.lo].
template <bool CPLX>
__device__ void probe_bx(const View &vb, int nv, uint64_t seed, double *w, double *ub, int64_t l) {
  const int64_t K = vb.L, N = vb.R;
  if (l >= K) return;
  Dd re[kMaxVec], im[kMaxVec];
  double u = 0.0;
  for (int64_t j = 0; j < N; ++j) {
    const double2 b = ld<CPLX>(vb, j, l);
    u = add_rn(u, CPLX ? hypot(b.x, b.y) : fabs(b.x));
    for (int v = 0; v < nv; ++v) {
      const double s = sign_of(seed, v, N, j);
      acc_add(re[v], mul_rn(s, b.x));
      if (CPLX) acc_add(im[v], mul_rn(s, b.y));
    }
  }
  for (int v = 0; v < nv; ++v) {
    double *o = w + (l * kMaxVec + v) * 4;
    o[0] = re[v].hi;
    o[1] = re[v].lo;
    o[2] = im[v].hi;
    o[3] = im[v].lo;
  }
  ub[l] = u;
}

template <bool CPLX>
__global__ void __launch_bounds__(256) k_probe_bx(View vb, int nv, uint64_t seed, double *w,
                                                  double *ub) {
  probe_bx<CPLX>(vb, nv, seed, w, ub, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// Per row i: z_v = sum_l op(A)(i, l) w_v[l] (w as hi + lo), y_v = sum_j C(i, j)
// x_v[j], u = sum_l |op(A)(i, l)| ub[l]; est[i] as described above.
template <bool CPLX>
__device__ void probe_rows(const View &va, const void *C, int64_t ldc, int64_t n, int nv,
                           uint64_t seed, const double *w, const double *ub, double *est,
                           int64_t i) {
  const int64_t M = va.R, K = va.L;
  if (i >= M) return;
  Dd zr[kMaxVec], zi[kMaxVec], yr[kMaxVec], yi[kMaxVec];
  double u = 0.0;
  for (int64_t l = 0; l < K; ++l) {
    const double2 a = ld<CPLX>(va, i, l);
    u = add_rn(u, mul_rn(CPLX ? hypot(a.x, a.y) : fabs(a.x), ub[l]));
    for (int v = 0; v < nv; ++v) {
      const double *o = w + (l * kMaxVec + v) * 4;
      // (ar + i ai)(wr + i wi) with w = hi + lo in both parts
      acc_mac(zr[v], a.x, o[0]);
      acc_mac(zr[v], a.x, o[1]);
      if (CPLX) {
        acc_mac(zr[v], -a.y, o[2]);
        acc_mac(zr[v], -a.y, o[3]);
        acc_mac(zi[v], a.x, o[2]);
        acc_mac(zi[v], a.x, o[3]);
        acc_mac(zi[v], a.y, o[0]);
        acc_mac(zi[v], a.y, o[1]);
      }
    }
  }
  for (int64_t j = 0; j < n; ++j) {
    double cr, ci = 0.0;
    if (CPLX) {
      const double2 c = reinterpret_cast<const double2 *>(C)[i + j * ldc];
      cr = c.x;
      ci = c.y;
    } else {
      cr = reinterpret_cast<const double *>(C)[i + j * ldc];
    }
    for (int v = 0; v < nv; ++v) {
      const double s = sign_of(seed, v, n, j);
      acc_add(yr[v], mul_rn(s, cr));
      if (CPLX) acc_add(yi[v], mul_rn(s, ci));
    }
  }
  double ss = 0.0;
  bool finite = true;
  for (int v = 0; v < nv; ++v) {
    // hi parts agree to within the emulation error, so their difference is
    // exact (Sterbenz); the lo parts add the compensation.
    const double rr = add_rn(sub_rn(yr[v].hi, zr[v].hi), sub_rn(yr[v].lo, zr[v].lo));
    const double ri = add_rn(sub_rn(yi[v].hi, zi[v].hi), sub_rn(yi[v].lo, zi[v].lo));
    finite = finite && isfinite(rr) && isfinite(ri);
    ss = add_rn(ss, add_rn(mul_rn(rr, rr), mul_rn(ri, ri)));
  }
  double e;
  if (!finite || !isfinite(u))
    e = qnan();
  else if (u == 0.0)
    e = ss == 0.0 ? 0.0 : __longlong_as_double(0x7ff0000000000000ll);
  else
    e = sqrt(ss / nv) * sqrt((double)n) / u;
  est[i] = e;
}

template <bool CPLX>
__global__ void __launch_bounds__(256) k_probe_rows(View va, const void *C, int64_t ldc, int64_t n,
                                                    int nv, uint64_t seed, const double *w,
                                                    const double *ub, double *est) {
  probe_rows<CPLX>(va, C, ldc, n, nv, seed, w, ub, est, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

__device__ __forceinline__ int find_task3(const int64_t *start, int ntasks, int64_t b) {
  int lo = 0, hi = ntasks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Batched forms: task t owns blocks start[t] .. start[t+1]-1 (k / 256 blocks
// for the first kernel, m / 256 for the second).
__global__ void __launch_bounds__(256) k_probe_bx_batched(const ProbeTask *tasks,
                                                          const int64_t *start, int ntasks) {
  const int t = find_task3(start, ntasks, blockIdx.x);
  const ProbeTask tk = tasks[t];
  const int64_t l = (blockIdx.x - start[t]) * 256 + threadIdx.x;
  if (tk.cplx)
    probe_bx<true>(tk.vb, tk.nv, tk.seed, tk.w, tk.ub, l);
  else
    probe_bx<false>(tk.vb, tk.nv, tk.seed, tk.w, tk.ub, l);
}

__global__ void __launch_bounds__(256) k_probe_rows_batched(const ProbeTask *tasks,
                                                            const int64_t *start, int ntasks) {
  const int t = find_task3(start, ntasks, blockIdx.x);
  const ProbeTask tk = tasks[t];
  const int64_t i = (blockIdx.x - start[t]) * 256 + threadIdx.x;
  if (tk.cplx)
    probe_rows<true>(tk.va, tk.C, tk.ldc, tk.vb.R, tk.nv, tk.seed, tk.w, tk.ub, tk.est, i);
  else
    probe_rows<false>(tk.va, tk.C, tk.ldc, tk.vb.R, tk.nv, tk.seed, tk.w, tk.ub, tk.est, i);
}

// C_p = alpha_p P_p + beta_p C_p for complex problems, the epilogue formula of
// the fused GEMM (every product and sum rounded on its own); one thread per
// entry, task t owns blocks start[t] ..
__global__ void __launch_bounds__(256) k_axpby_batched(const AxpbyTask *tasks, const int64_t *start,
                                                       int ntasks) {
  const int t = find_task3(start, ntasks, blockIdx.x);
  const AxpbyTask tk = tasks[t];
  const int64_t idx = (blockIdx.x - start[t]) * 256 + threadIdx.x;
  if (idx >= tk.m * tk.n) return;
  const int64_t i = idx % tk.m, j = idx / tk.m;
  const double2 p = reinterpret_cast<const double2 *>(tk.P)[i + j * tk.m];
  double2 *cp = reinterpret_cast<double2 *>(tk.C) + i + j * tk.ldc;
  double re = sub_rn(mul_rn(tk.ar, p.x), mul_rn(tk.ai, p.y));
  double im = add_rn(mul_rn(tk.ar, p.y), mul_rn(tk.ai, p.x));
  if (!tk.beta_zero) {
    const double2 z = *cp;
    re = add_rn(re, sub_rn(mul_rn(tk.br, z.x), mul_rn(tk.bi, z.y)));
    im = add_rn(im, add_rn(mul_rn(tk.br, z.y), mul_rn(tk.bi, z.x)));
  }
  *cp = make_double2(re, im);
}

}  // namespace

int64_t probe_task_blocks_k(const ProbeTask &t) { return (t.vb.L + 255) / 256; }
int64_t probe_task_blocks_m(const ProbeTask &t) { return (t.va.R + 255) / 256; }
int64_t axpby_task_blocks(const AxpbyTask &t) { return (t.m * t.n + 255) / 256; }

hipError_t launch_probe_batched(const ProbeTask *tasks, const int64_t *start_k, int64_t nblk_k,
                                const int64_t *start_m, int64_t nblk_m, int ntasks, hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  if (nblk_k > 0)
    hipLaunchKernelGGL(k_probe_bx_batched, dim3((unsigned)nblk_k), dim3(256), 0, st, tasks, start_k,
                       ntasks);
  if (nblk_m > 0)
    hipLaunchKernelGGL(k_probe_rows_batched, dim3((unsigned)nblk_m), dim3(256), 0, st, tasks,
                       start_m, ntasks);
  return hipGetLastError();
}

hipError_t launch_axpby_batched(const AxpbyTask *tasks, const int64_t *start, int ntasks,
                                int64_t nblocks, hipStream_t st) {
  if (ntasks <= 0 || nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpby_batched, dim3((unsigned)nblocks), dim3(256), 0, st, tasks, start, ntasks);
  return hipGetLastError();
}

size_t probe_workspace_bytes(int64_t k) { return (size_t)k * (kMaxVec * 4 + 1) * sizeof(double) + 256; }
int probe_max_vectors() { return kMaxVec; }

hipError_t launch_probe(const View &va, const View &vb, bool cplx, const void *C, int64_t ldc,
                        int64_t m, int64_t n, int64_t k, int nv, uint64_t seed, void *ws, double *est,
                        hipStream_t st) {
  if (m <= 0) return hipSuccess;
  double *w = static_cast<double *>(ws);
  double *ub = w + (size_t)k * kMaxVec * 4;
  if (k > 0) {
    const dim3 g((unsigned)((k + 255) / 256));
    if (cplx)
      hipLaunchKernelGGL(k_probe_bx<true>, g, dim3(256), 0, st, vb, nv, seed, w, ub);
    else
      hipLaunchKernelGGL(k_probe_bx<false>, g, dim3(256), 0, st, vb, nv, seed, w, ub);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  (void)n;
  const dim3 g((unsigned)((m + 255) / 256));
  if (cplx)
    hipLaunchKernelGGL(k_probe_rows<true>, g, dim3(256), 0, st, va, C, ldc, n, nv, seed, w, ub, est);
  else
    hipLaunchKernelGGL(k_probe_rows<false>, g, dim3(256), 0, st, va, C, ldc, n, nv, seed, w, ub, est);
  return hipGetLastError();
}

}  // namespace oz
