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
#include <algorithm>

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
constexpr int kBatch = 4;  // entries whose loads are issued together in the chunk loops

template <bool CPLX>
__device__ __forceinline__ double2 ld(const View &v, int64_t r, int64_t l) {
  if (CPLX) {
    double2 z = reinterpret_cast<const double2 *>(v.base)[r * v.sr + l * v.sl];
    if (v.conj) z.y = -z.y;
    return z;
  }
  return make_double2(reinterpret_cast<const double *>(v.base)[r * v.sr + l * v.sl], 0.0);
}

// The sums run in chunks so that a problem spreads over many threads (one
// thread per output and chunk, each chunk's compensated sum written out as a
// partial record, then one thread per output adding the records in chunk
// order): a thread per output alone would leave the GPU mostly idle behind
// k + n long dependent chains. A record holds, for every vector v, the two
// compensated sums (re.hi, re.lo, im.hi, im.lo) and one plain sum.
constexpr int kRec = kMaxVec * 4 + 1;

template <int NV>
__device__ __forceinline__ void put_rec(double *o, const Dd *re, const Dd *im, double u) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    o[v * 4 + 0] = re[v].hi;
    o[v * 4 + 1] = re[v].lo;
    o[v * 4 + 2] = im[v].hi;
    o[v * 4 + 3] = im[v].lo;
  }
  o[kMaxVec * 4] = u;
}

template <int NV>
__device__ __forceinline__ void add_rec(const double *o, Dd *re, Dd *im, double &u) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    acc_add(re[v], o[v * 4 + 0]);
    re[v].lo = add_rn(re[v].lo, o[v * 4 + 1]);
    acc_add(im[v], o[v * 4 + 2]);
    im[v].lo = add_rn(im[v].lo, o[v * 4 + 3]);
  }
  u = add_rn(u, o[kMaxVec * 4]);
}

// Stage 1, thread (l, chunk c of columns j): partial w_v[l] = sum_j op(B)(l, j)
// x_v[j] and ub[l] = sum_j |op(B)(l, j)|. vb views op(B) with rows = columns
// j and contraction = l, so op(B)(l, j) = vb(j, l).
template <bool CPLX, int NV>
__device__ void bx_part(const ProbeTask &tk, int64_t idx) {
  const int64_t K = tk.vb.L, N = tk.vb.R;
  if (idx >= K * tk.ncj) return;
  const int64_t l = idx % K, c = idx / K;
  const int64_t j0 = c * tk.chj, j1 = j0 + tk.chj < N ? j0 + tk.chj : N;
  Dd re[kMaxVec], im[kMaxVec];
  double u = 0.0;
  for (int64_t jb = j0; jb < j1; jb += kBatch) {
    double2 bq[kBatch];  // the batch's loads first (past j1: the last entry again)
#pragma unroll
    for (int q = 0; q < kBatch; ++q) bq[q] = ld<CPLX>(tk.vb, jb + q < j1 ? jb + q : j1 - 1, l);
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int64_t j = jb + q;
      if (j >= j1) break;
      const double2 b = bq[q];
      u = add_rn(u, CPLX ? hypot(b.x, b.y) : fabs(b.x));
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double s = sign_of(tk.seed, v, N, j);
        acc_add(re[v], mul_rn(s, b.x));
        if (CPLX) acc_add(im[v], mul_rn(s, b.y));
      }
    }
  }
  put_rec<NV>(tk.p1 + (c * K + l) * kRec, re, im, u);
}

// Stage 2, thread l: w[l] (per v: re.hi, re.lo, im.hi, im.lo) and ub[l] from
// the chunk records in order.
template <int NV>
__device__ void bx_sum(const ProbeTask &tk, int64_t l) {
  const int64_t K = tk.vb.L;
  if (l >= K) return;
  Dd re[kMaxVec], im[kMaxVec];
  double u = 0.0;
#pragma unroll 4
  for (int64_t c = 0; c < tk.ncj; ++c) add_rec<NV>(tk.p1 + (c * K + l) * kRec, re, im, u);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double *o = tk.w + (l * kMaxVec + v) * 4;
    o[0] = re[v].hi;
    o[1] = re[v].lo;
    o[2] = im[v].hi;
    o[3] = im[v].lo;
  }
  tk.ub[l] = u;
}

// Stage 3, thread (i, chunk c): for c < ncl the partial z_v = sum_l op(A)(i, l)
// w_v[l] (w as hi + lo) and u = sum_l |op(A)(i, l)| ub[l] over a chunk of l;
// for c >= ncl the partial y_v = sum_j C(i, j) x_v[j] over a chunk of j.
template <bool CPLX, int NV>
__device__ void rows_part(const ProbeTask &tk, int64_t idx) {
  const int64_t M = tk.va.R, K = tk.va.L, N = tk.vb.R;
  if (idx >= M * (tk.ncl + tk.ncj)) return;
  const int64_t i = idx % M, c = idx / M;
  Dd xr[kMaxVec], xi[kMaxVec];
  double u = 0.0;
  if (c < tk.ncl) {
    const int64_t l0 = c * tk.chl, l1 = l0 + tk.chl < K ? l0 + tk.chl : K;
    for (int64_t lb = l0; lb < l1; lb += kBatch) {
      // the batch's loads first (past l1: the last entry again)
      double2 aq[kBatch];
      double ubq[kBatch], oq[kBatch][NV][4];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int64_t lq = lb + q < l1 ? lb + q : l1 - 1;
        aq[q] = ld<CPLX>(tk.va, i, lq);
        ubq[q] = tk.ub[lq];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e) oq[q][v][e] = tk.w[(lq * kMaxVec + v) * 4 + e];
      }
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        if (lb + q >= l1) break;
        const double2 a = aq[q];
        u = add_rn(u, mul_rn(CPLX ? hypot(a.x, a.y) : fabs(a.x), ubq[q]));
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double *o = oq[q][v];
          // (ar + i ai)(wr + i wi) with w = hi + lo in both parts
          acc_mac(xr[v], a.x, o[0]);
          acc_mac(xr[v], a.x, o[1]);
          if (CPLX) {
            acc_mac(xr[v], -a.y, o[2]);
            acc_mac(xr[v], -a.y, o[3]);
            acc_mac(xi[v], a.x, o[2]);
            acc_mac(xi[v], a.x, o[3]);
            acc_mac(xi[v], a.y, o[0]);
            acc_mac(xi[v], a.y, o[1]);
          }
        }
      }
    }
  } else {
    const int64_t j0 = (c - tk.ncl) * tk.chj, j1 = j0 + tk.chj < N ? j0 + tk.chj : N;
    const int ea = tk.codeA != nullptr ? code_exp(tk.codeA[i]) : 0;
    for (int64_t jb = j0; jb < j1; jb += kBatch) {
      // the batch's loads first (past j1: the last entry again)
      double crq[kBatch], ciq[kBatch];
      int cbq[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int64_t jq = jb + q < j1 ? jb + q : j1 - 1;
        if (CPLX) {
          const double2 cz = reinterpret_cast<const double2 *>(tk.C)[i + jq * tk.ldc];
          crq[q] = cz.x;
          ciq[q] = cz.y;
        } else {
          crq[q] = reinterpret_cast<const double *>(tk.C)[i + jq * tk.ldc];
          ciq[q] = 0.0;
        }
        cbq[q] = tk.codeA != nullptr ? tk.codeB[jq] : 0;
      }
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int64_t j = jb + q;
        if (j >= j1) break;
        double cr = crq[q], ci = ciq[q];
        if (tk.codeA != nullptr) {
          const int sc = ea + code_exp(cbq[q]);
          cr = ldexp(cr, sc);
          ci = ldexp(ci, sc);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double s = sign_of(tk.seed, v, N, j);
          acc_add(xr[v], mul_rn(s, cr));
          if (CPLX) acc_add(xi[v], mul_rn(s, ci));
        }
      }
    }
  }
  put_rec<NV>(tk.p2 + (c * M + i) * kRec, xr, xi, u);
}

// Stage 4, thread i: z, y and u from the records in chunk order; est[i].
template <int NV>
__device__ void rows_sum(const ProbeTask &tk, int64_t i) {
  const int64_t M = tk.va.R, N = tk.vb.R;
  if (i >= M) return;
  Dd zr[kMaxVec], zi[kMaxVec], yr[kMaxVec], yi[kMaxVec];
  double u = 0.0, unused = 0.0;
#pragma unroll 4
  for (int64_t c = 0; c < tk.ncl; ++c) add_rec<NV>(tk.p2 + (c * M + i) * kRec, zr, zi, u);
#pragma unroll 4
  for (int64_t c = tk.ncl; c < tk.ncl + tk.ncj; ++c)
    add_rec<NV>(tk.p2 + (c * M + i) * kRec, yr, yi, unused);
  double ss = 0.0;
  bool finite = true;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
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
    e = sqrt(ss / NV) * sqrt((double)N) / u;
  tk.est[i] = e;
}

template <int NV>
__device__ __forceinline__ void run_stage_nv(const ProbeTask &tk, int stage, int64_t idx) {
  switch (stage) {
    case 0:
      if (tk.cplx) bx_part<true, NV>(tk, idx); else bx_part<false, NV>(tk, idx);
      break;
    case 1: bx_sum<NV>(tk, idx); break;
    case 2:
      if (tk.cplx) rows_part<true, NV>(tk, idx); else rows_part<false, NV>(tk, idx);
      break;
    default: rows_sum<NV>(tk, idx); break;
  }
}

// The vector count is a template parameter so that every per-vector sum lives
// in registers (a runtime count would put them in scratch memory).
__device__ __forceinline__ void run_stage(const ProbeTask &tk, int stage, int64_t idx) {
  switch (tk.nv) {
    case 1: run_stage_nv<1>(tk, stage, idx); break;
    case 2: run_stage_nv<2>(tk, stage, idx); break;
    case 3: run_stage_nv<3>(tk, stage, idx); break;
    default: run_stage_nv<4>(tk, stage, idx); break;
  }
}

// One problem: the task by value.
__global__ void __launch_bounds__(256) k_probe_stage(ProbeTask tk, int stage) {
  run_stage(tk, stage, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// Batched: task t owns blocks tasks[t].blk[stage] .. tasks[t+1].blk[stage]-1.
__global__ void __launch_bounds__(256) k_probe_stage_batched(const ProbeTask *tasks, int ntasks,
                                                             int stage) {
  int lo = 0, hi = ntasks - 1;
  const int64_t b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].blk[stage] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  const ProbeTask &tk = tasks[lo];
  if (tk.flag != nullptr && tk.flag[tk.id] != 1) return;
  run_stage(tk, stage, (b - tk.blk[stage]) * 256 + threadIdx.x);
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

// out[t] = max_i est_t[i] over the rows of task t (NaN if any row is NaN);
// one workgroup per task.
__global__ void __launch_bounds__(256) k_probe_max_batched(const ProbeTask *tasks, double *out) {
  const ProbeTask &tk = tasks[blockIdx.x];
  if (tk.flag != nullptr && tk.flag[tk.id] != 1) return;
  const int64_t M = tk.va.R;
  double mx = 0.0;
  bool nan = false;
  for (int64_t i = threadIdx.x; i < M; i += 256) {
    const double e = tk.est[i];
    if (isnan(e))
      nan = true;
    else
      mx = fmax(mx, e);
  }
  __shared__ double smax[256];
  __shared__ int snan[256];
  smax[threadIdx.x] = mx;
  snan[threadIdx.x] = nan ? 1 : 0;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      snan[threadIdx.x] |= snan[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = snan[0] ? qnan() : smax[0];
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
  double2 p = reinterpret_cast<const double2 *>(tk.P)[i + j * tk.m];
  if (tk.codeA != nullptr) {
    const int sc = code_exp(tk.codeA[i]) + code_exp(tk.codeB[j]);
    p = make_double2(ldexp(p.x, sc), ldexp(p.y, sc));
  }
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

__global__ void __launch_bounds__(256) k_probe_decide(const double *emax, int64_t n, double kappa,
                                                      double target, int smax, int *s,
                                                      const int *cap, int *flag, int first) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  if (!first && flag[e] != 1) return;
  const double mx = emax[e];  // NaN: non-finite inputs, nothing to raise
  const bool miss = !isnan(mx) && mx * kappa > target;
  int f = 0;
  if (miss && s[e] < cap[e]) {
    f = 1;
    s[e] += 1;
  } else if (miss && s[e] < smax) {
    f = 2;
  }
  flag[e] = f;
}

}  // namespace

namespace {

int64_t chunk_len(int64_t len) { return std::max<int64_t>(32, (len + 31) / 32); }
int64_t chunks(int64_t len, int64_t ch) { return len <= 0 ? 0 : (len + ch - 1) / ch; }
int64_t blocks(int64_t threads) { return (threads + 255) / 256; }

}  // namespace

size_t probe_workspace_bytes(int64_t m, int64_t n, int64_t k) {
  const int64_t ncl = chunks(k, chunk_len(k)), ncj = chunks(n, chunk_len(n));
  const size_t recs = (size_t)k + (size_t)ncj * k + (size_t)(ncl + ncj) * m;
  return recs * kRec * sizeof(double) + 4 * 256;
}

ProbeTask probe_task(const View &va, const View &vb, bool cplx, const void *C, int64_t ldc, int nv,
                     uint64_t seed, void *ws, double *est) {
  ProbeTask t{};
  t.va = va;
  t.vb = vb;
  t.C = C;
  t.ldc = ldc;
  t.cplx = cplx ? 1 : 0;
  t.nv = nv;
  t.seed = seed;
  t.est = est;
  const int64_t K = va.L, N = vb.R;
  t.chl = chunk_len(K);
  t.chj = chunk_len(N);
  t.ncl = chunks(K, t.chl);
  t.ncj = chunks(N, t.chj);
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  char *p = static_cast<char *>(ws);
  t.w = reinterpret_cast<double *>(p);  // w (16 per l) and ub (1 per l) share one record each
  t.ub = t.w + (size_t)K * kMaxVec * 4;
  p += al((size_t)K * kRec * sizeof(double));
  t.p1 = reinterpret_cast<double *>(p);
  p += al((size_t)t.ncj * K * kRec * sizeof(double));
  t.p2 = reinterpret_cast<double *>(p);
  return t;
}

int64_t axpby_task_blocks(const AxpbyTask &t) { return (t.m * t.n + 255) / 256; }

int64_t probe_stage_blocks(const ProbeTask &t, int stage) {
  const int64_t M = t.va.R, K = t.va.L;
  switch (stage) {
    case 0: return blocks(K * t.ncj);
    case 1: return blocks(K);
    case 2: return blocks(M * (t.ncl + t.ncj));
    default: return blocks(M);
  }
}

hipError_t launch_probe_batched(const ProbeTask *tasks, int ntasks, const int64_t *nblk,
                                hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  for (int stage = 0; stage < 4; ++stage) {
    if (nblk[stage] <= 0) continue;
    hipLaunchKernelGGL(k_probe_stage_batched, dim3((unsigned)nblk[stage]), dim3(256), 0, st, tasks,
                       ntasks, stage);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_probe_max_batched(const ProbeTask *tasks, int ntasks, double *out,
                                    hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_probe_max_batched, dim3((unsigned)ntasks), dim3(256), 0, st, tasks, out);
  return hipGetLastError();
}

hipError_t launch_axpby_batched(const AxpbyTask *tasks, const int64_t *start, int ntasks,
                                int64_t nblocks, hipStream_t st) {
  if (ntasks <= 0 || nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpby_batched, dim3((unsigned)nblocks), dim3(256), 0, st, tasks, start, ntasks);
  return hipGetLastError();
}

int probe_max_vectors() { return kMaxVec; }

hipError_t launch_probe_decide(const double *emax, int64_t n, double kappa, double target,
                               int smax, int *s, const int *cap, int *flag, int first,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_probe_decide, dim3((unsigned)blocks(n)), dim3(256), 0, st, emax, n, kappa,
                     target, smax, s, cap, flag, first);
  return hipGetLastError();
}

hipError_t launch_probe(const View &va, const View &vb, bool cplx, const void *C, int64_t ldc,
                        int nv, uint64_t seed, void *ws, double *est, hipStream_t st) {
  if (va.R <= 0) return hipSuccess;
  const ProbeTask t = probe_task(va, vb, cplx, C, ldc, nv, seed, ws, est);
  for (int stage = 0; stage < 4; ++stage) {
    const int64_t nb = probe_stage_blocks(t, stage);
    if (nb <= 0) continue;
    hipLaunchKernelGGL(k_probe_stage, dim3((unsigned)nb), dim3(256), 0, st, t, stage);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace oz
