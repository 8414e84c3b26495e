// Learned slice-count selector of libozaki (gfx950): exponent-statistics
// features and a 64 -> 128 -> 128 -> 1 ReLU MLP with BF16 weights and FP32
// accumulation, trained on the GPU by these kernels (forward, backward, Adam).
//
// The paper observes that emulation accuracy depends on both the arithmetic
// precision and properties of the operator (abstract; Section 4), and tunes the
// precision per run by hand. The selector predicts the number of slices a
// product needs from the one property the slicing is sensitive to: how far
// the entries sit below their row (column) maximum in binary exponent, since
// an entry delta binades below the maximum keeps only 7s - delta bits.
//
// Features of a product (64 floats):
//   [0..31]  fraction of entries of op(A) with delta = e_i - E(a_il) in bin
//            min(delta, 30), bin 31 = zero entries (E = frexp exponent, the
//            larger of the real and imaginary parts for complex data)
//   [32..62] the same for the columns of op(B): bins min(delta, 29), bin 30 =
//            zero entries
//   [63]     log2(k) / 16
//
// MLP parameters (P = 24961 floats, FP32 master copy), in this order:
//   W1 [128 x 64], b1 [128], W2 [128 x 128], b2 [128], w3 [128], b3 [1];
//   y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3. W1, W2 and w3 are used as
//   BF16 (round to nearest even), so are the layer inputs fed to the matrix
//   cores; every product is accumulated in FP32 by v_mfma_f32_32x32x16_bf16.
#include "ozaki_internal.hpp"

namespace oz {

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------- features
template <bool CPLX>
__device__ __forceinline__ int elem_code2(const void *base, int64_t off) {
  if (CPLX) {
    const double2 z = reinterpret_cast<const double2 *>(base)[off];
    return max(expo_code(z.x), expo_code(z.y));
  }
  return expo_code(reinterpret_cast<const double *>(base)[off]);
}

// Histogram bin of an entry with code c in a row with code rc (nbins bins;
// the last one counts zeros, the one before collects delta >= nbins - 2).
__device__ __forceinline__ int feat_bin(int c, int rc, int nbins) {
  if (c == 0 || code_bad(c) || code_bad(rc)) return nbins - 1;
  const int d = rc - c;
  return min(max(d, 0), nbins - 2);
}

// One block per task and row group: 256 threads walk the rows of the group
// (64 rows with 4 threads each when rows are unit-stride, else 4 rows with a
// wave each) over the whole contraction, into an LDS histogram; the loads of
// four entries are issued together.
template <bool CPLX>
__device__ void feat_block(const FeatTask &t, int64_t rb) {
  __shared__ int hist[32];
  const int tid = threadIdx.x;
  if (tid < 32) hist[tid] = 0;
  __syncthreads();
  const View &v = t.v;
  int64_t r, l, step, off0, stride;
  if (t.rows_fast) {
    r = rb * 64 + (tid & 63);
    l = tid >> 6;
    step = 4;
    off0 = r;
    stride = v.sl;
  } else {
    r = rb * 4 + (tid >> 6);
    l = tid & 63;
    step = 64;
    off0 = r * v.sr;
    stride = 1;
  }
  if (r < v.R) {
    const int rc = t.code[r];
    for (; l + 3 * step < v.L; l += 4 * step) {
      int cq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) cq[q] = elem_code2<CPLX>(v.base, off0 + (l + q * step) * stride);
#pragma unroll
      for (int q = 0; q < 4; ++q) atomicAdd(&hist[feat_bin(cq[q], rc, t.nbins)], 1);
    }
    for (; l < v.L; l += step)
      atomicAdd(&hist[feat_bin(elem_code2<CPLX>(v.base, off0 + l * stride), rc, t.nbins)], 1);
  }
  __syncthreads();
  if (tid < t.nbins && hist[tid] != 0) atomicAdd(t.hist + tid, hist[tid]);
}

__device__ __forceinline__ int find_task2(const int64_t *start, int ntasks, int64_t b) {
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

__global__ void __launch_bounds__(256) k_feat_hist(const FeatTask *tasks, const int64_t *start,
                                                   int ntasks) {
  const int64_t b = blockIdx.x;
  const int t = find_task2(start, ntasks, b);
  const FeatTask tk = tasks[t];
  if (tk.cplx)
    feat_block<true>(tk, b - start[t]);
  else
    feat_block<false>(tk, b - start[t]);
}

// feat[p][0..63] from the integer histograms hist[p][0..63] (A bins 0..31,
// B bins 32..62) and the problem's m, n, k.
__global__ void __launch_bounds__(64) k_feat_finish(const int *hist, const int64_t *dims, float *feat,
                                                    int64_t np) {
  const int64_t p = blockIdx.x;
  const int j = threadIdx.x;
  if (p >= np) return;
  const int64_t m = dims[3 * p], n = dims[3 * p + 1], k = dims[3 * p + 2];
  float v;
  if (j < 32)
    v = (float)hist[p * 64 + j] / (float)(m * k);
  else if (j < 63)
    v = (float)hist[p * 64 + j] / (float)(k * n);
  else
    v = (float)(log2((double)k) / 16.0);
  feat[p * 64 + j] = v;
}

// ---------------------------------------------------------------- MLP
constexpr int kIn = 64, kH = 128;
constexpr int64_t kP = (int64_t)kH * kIn + kH + (int64_t)kH * kH + kH + kH + 1;  // 24961
// offsets of the parameters in the FP32 vector
constexpr int64_t oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH,
                  oW3 = oB2 + kH, oB3 = oW3 + kH;

// State layout (bytes): theta, adam m, adam v, grad (FP32, P each), then the
// BF16 copies W1 [128 x 64], W2 [128 x 128], W2^T [128 x 128], w3 [128].
constexpr size_t kStF32 = (size_t)kP * 4;
constexpr size_t sTheta = 0, sM = kStF32, sV = 2 * kStF32, sG = 3 * kStF32;
constexpr size_t sW1h = 4 * kStF32 + 64;  // keep 16-byte alignment (P*4 = 99844)
constexpr size_t sW2h = sW1h + (size_t)kH * kIn * 2;
constexpr size_t sW2th = sW2h + (size_t)kH * kH * 2;
constexpr size_t sW3h = sW2th + (size_t)kH * kH * 2;
constexpr size_t kStateBytes = sW3h + (size_t)kH * 2 + 64;

__device__ __forceinline__ float bf_round(float x) { return (float)(__bf16)x; }

// C (M x N, FP32, row-major) = A (M x K, BF16, row-major) * Bt (N x K, BF16,
// row-major)^T. One wave per 32 x 32 output tile; M, N multiples of 32, K a
// multiple of 16. The MFMA's lane l reads 8 consecutive BF16 of row l % 32
// from contraction offset 8 * (l / 32), and leaves D[8(r/4) + 4(l/32) + r%4][l%32]
// in register r. Epilogue per `mode`:
//   0: C = acc
//   1: H = relu(acc + bias[col]): Cf (FP32), Ch (BF16 row-major), Cht (BF16
//      transposed, ldt = M)
//   2: G = acc * [mask[row][col] > 0]: Ch (BF16 row-major) and Cht (BF16 transposed)
struct MmArgs {
  const __bf16 *A;
  const __bf16 *Bt;
  int64_t M, N, K;
  int mode;
  float *Cf;
  const float *bias;
  const float *mask;
  __bf16 *Ch;
  __bf16 *Cht;
};

__global__ void __launch_bounds__(256) k_mm_bf16(MmArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t ntn = a.N / 32;
  if (tile >= (a.M / 32) * ntn) return;
  const int64_t r0 = (tile / ntn) * 32, c0 = (tile % ntn) * 32;
  v16f acc = {0};
  const __bf16 *pa = a.A + (r0 + (lane & 31)) * a.K + 8 * (lane >> 5);
  const __bf16 *pb = a.Bt + (c0 + (lane & 31)) * a.K + 8 * (lane >> 5);
  for (int64_t k0 = 0; k0 < a.K; k0 += 16) {
    const v8bf x = *reinterpret_cast<const v8bf *>(pa + k0);
    const v8bf y = *reinterpret_cast<const v8bf *>(pb + k0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc, 0, 0, 0);
  }
  const int64_t col = c0 + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t row = r0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    float v = acc[r];
    if (a.mode == 0) {
      a.Cf[row * a.N + col] = v;
    } else if (a.mode == 1) {
      v = fmaxf(v + a.bias[col], 0.0f);
      a.Cf[row * a.N + col] = v;
      a.Ch[row * a.N + col] = (__bf16)v;
      a.Cht[col * a.M + row] = (__bf16)v;
    } else {
      if (!(a.mask[row * a.N + col] > 0.0f)) v = 0.0f;
      a.Ch[row * a.N + col] = (__bf16)v;
      a.Cht[col * a.M + row] = (__bf16)v;
    }
  }
}

// X (b x 64 FP32) -> Xh (bp x 64 BF16) and Xht (64 x bp), zero rows b..bp-1.
__global__ void __launch_bounds__(256) k_pack_x(const float *X, int64_t b, int64_t bp, __bf16 *Xh,
                                                __bf16 *Xht) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= bp * kIn) return;
  const int64_t r = idx / kIn, c = idx % kIn;
  const __bf16 v = (__bf16)(r < b ? X[r * kIn + c] : 0.0f);
  Xh[r * kIn + c] = v;
  Xht[c * bp + r] = v;
}

// y[r] = b3 + sum_k bf16(w3[k]) * H2[r][k]   (FP32, sequential in k)
__global__ void __launch_bounds__(256) k_head_fwd(const float *H2, const float *theta,
                                                  const __bf16 *w3h, int64_t b, float *y) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= b) return;
  float s = 0.0f;
  for (int k = 0; k < kH; ++k) s = fmaf((float)w3h[k], H2[r * kH + k], s);
  y[r] = s + theta[oB3];
}

// Loss L = (1/b) sum_r w_r (y_r - t_r)^2 with w_r = under (y_r < t_r) or 1;
// dy_r = (2/b) w_r (y_r - t_r). dH2[r][k] = dy_r * bf16(w3[k]) * [H2 > 0]
// (BF16, row-major and transposed, zero for padded rows); dw3 and db3 are
// atomically accumulated into the gradient.
__global__ void __launch_bounds__(256) k_head_bwd(const float *H2, const float *y, const float *t,
                                                  const __bf16 *w3h, int64_t b, int64_t bp,
                                                  float under, float *grad, float *loss,
                                                  __bf16 *dH2h, __bf16 *dH2ht) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= bp) return;
  float dy = 0.0f;
  if (r < b) {
    const float e = y[r] - t[r];
    const float w = y[r] < t[r] ? under : 1.0f;
    dy = 2.0f * w * e / (float)b;
    if (loss) atomicAdd(loss, w * e * e / (float)b);
    atomicAdd(grad + oB3, dy);
  }
  for (int k = 0; k < kH; ++k) {
    const float h = r < b ? H2[r * kH + k] : 0.0f;
    const float g = h > 0.0f ? dy * (float)w3h[k] : 0.0f;
    dH2h[r * kH + k] = (__bf16)g;
    dH2ht[k * bp + r] = (__bf16)g;
    if (r < b && dy != 0.0f) atomicAdd(grad + oW3 + k, dy * h);
  }
}

// bias gradient: grad[off + c] += sum_r G[r][c] (G BF16 row-major, rows < bp)
__global__ void __launch_bounds__(128) k_colsum(const __bf16 *G, int64_t bp, int cols, float *out) {
  const int c = threadIdx.x;
  if (c >= cols) return;
  float s = 0.0f;
  for (int64_t r = 0; r < bp; ++r) s += (float)G[r * cols + c];
  out[c] += s;
}

__global__ void __launch_bounds__(256) k_zero_f32(float *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// BF16 copies of W1, W2, W2^T and w3 from theta.
__global__ void __launch_bounds__(256) k_refresh_bf16(char *state) {
  const float *th = reinterpret_cast<const float *>(state + sTheta);
  __bf16 *W1h = reinterpret_cast<__bf16 *>(state + sW1h);
  __bf16 *W2h = reinterpret_cast<__bf16 *>(state + sW2h);
  __bf16 *W2th = reinterpret_cast<__bf16 *>(state + sW2th);
  __bf16 *w3h = reinterpret_cast<__bf16 *>(state + sW3h);
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < kH * kIn) W1h[i] = (__bf16)th[oW1 + i];
  if (i < kH * kH) {
    const int64_t r = i / kH, c = i % kH;
    W2h[i] = (__bf16)th[oW2 + i];
    W2th[c * kH + r] = (__bf16)th[oW2 + i];
  }
  if (i < kH) w3h[i] = (__bf16)th[oW3 + i];
}

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// He-uniform initialisation: W ~ U(-sqrt(6/fan_in), +sqrt(6/fan_in)) from
// SplitMix64(seed + index), biases 0; Adam moments 0.
__global__ void __launch_bounds__(256) k_init(char *state, uint64_t seed) {
  float *th = reinterpret_cast<float *>(state + sTheta);
  float *m = reinterpret_cast<float *>(state + sM);
  float *v = reinterpret_cast<float *>(state + sV);
  float *g = reinterpret_cast<float *>(state + sG);
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= kP) return;
  const double u = (double)(mix64(seed + (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);  // [0,1)
  float val = 0.0f;
  if (i < oB1)
    val = (float)((2.0 * u - 1.0) * sqrt(6.0 / kIn));
  else if (i >= oW2 && i < oB2)
    val = (float)((2.0 * u - 1.0) * sqrt(6.0 / kH));
  else if (i >= oW3 && i < oB3)
    val = (float)((2.0 * u - 1.0) * sqrt(6.0 / kH));
  th[i] = val;
  m[i] = 0.0f;
  v[i] = 0.0f;
  g[i] = 0.0f;
}

// Adam (Kingma and Ba 2015) with bias correction at step t >= 1.
__global__ void __launch_bounds__(256) k_adam(char *state, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  float *th = reinterpret_cast<float *>(state + sTheta);
  float *m = reinterpret_cast<float *>(state + sM);
  float *v = reinterpret_cast<float *>(state + sV);
  const float *g = reinterpret_cast<const float *>(state + sG);
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= kP) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Scratch layout for a batch padded to bp rows (all offsets 256-aligned).
struct Scratch {
  size_t xh, xht, h1, h1h, h1ht, h2, h2h, h2ht, dh2h, dh2ht, dh1h, dh1ht, total;
};
Scratch scratch_layout(int64_t bp) {
  Scratch s{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  s.xh = take(bp * kIn * 2);
  s.xht = take(bp * kIn * 2);
  s.h1 = take(bp * kH * 4);
  s.h1h = take(bp * kH * 2);
  s.h1ht = take(bp * kH * 2);
  s.h2 = take(bp * kH * 4);
  s.h2h = take(bp * kH * 2);
  s.h2ht = take(bp * kH * 2);
  s.dh2h = take(bp * kH * 2);
  s.dh2ht = take(bp * kH * 2);
  s.dh1h = take(bp * kH * 2);
  s.dh1ht = take(bp * kH * 2);
  s.total = off;
  return s;
}

}  // namespace

int64_t mlp_params() { return kP; }
size_t mlp_state_bytes() { return kStateBytes; }
size_t mlp_scratch_bytes(int64_t batch) { return scratch_layout((batch + 31) / 32 * 32).total; }

hipError_t launch_feat_hist(const FeatTask *tasks, const int64_t *start, int ntasks, int64_t nblocks,
                            hipStream_t st) {
  if (ntasks <= 0 || nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_feat_hist, dim3((unsigned)nblocks), dim3(256), 0, st, tasks, start, ntasks);
  return hipGetLastError();
}

int64_t feat_task_blocks(const FeatTask &t) {
  return t.rows_fast ? (t.v.R + 63) / 64 : (t.v.R + 3) / 4;
}

hipError_t launch_feat_finish(const int *hist, const int64_t *dims, float *feat, int64_t np,
                              hipStream_t st) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_feat_finish, dim3((unsigned)np), dim3(64), 0, st, hist, dims, feat, np);
  return hipGetLastError();
}

hipError_t mlp_init(void *state, uint64_t seed, hipStream_t st) {
  char *s = static_cast<char *>(state);
  hipLaunchKernelGGL(k_init, dim3(blocks(kP, 256)), dim3(256), 0, st, s, seed);
  hipLaunchKernelGGL(k_refresh_bf16, dim3(blocks(kH * kH, 256)), dim3(256), 0, st, s);
  return hipGetLastError();
}

hipError_t mlp_refresh(void *state, hipStream_t st) {
  hipLaunchKernelGGL(k_refresh_bf16, dim3(blocks(kH * kH, 256)), dim3(256), 0, st,
                     static_cast<char *>(state));
  return hipGetLastError();
}

hipError_t mlp_forward(const void *state, int64_t b, const float *X, float *y, void *scratch,
                       hipStream_t st) {
  if (b <= 0) return hipSuccess;
  const char *s = static_cast<const char *>(state);
  char *w = static_cast<char *>(scratch);
  const int64_t bp = (b + 31) / 32 * 32;
  const Scratch L = scratch_layout(bp);
  const float *th = reinterpret_cast<const float *>(s + sTheta);
  hipLaunchKernelGGL(k_pack_x, dim3(blocks(bp * kIn, 256)), dim3(256), 0, st, X, b, bp,
                     reinterpret_cast<__bf16 *>(w + L.xh), reinterpret_cast<__bf16 *>(w + L.xht));
  MmArgs m1{};
  m1.A = reinterpret_cast<const __bf16 *>(w + L.xh);
  m1.Bt = reinterpret_cast<const __bf16 *>(s + sW1h);
  m1.M = bp;
  m1.N = kH;
  m1.K = kIn;
  m1.mode = 1;
  m1.Cf = reinterpret_cast<float *>(w + L.h1);
  m1.bias = th + oB1;
  m1.Ch = reinterpret_cast<__bf16 *>(w + L.h1h);
  m1.Cht = reinterpret_cast<__bf16 *>(w + L.h1ht);
  hipLaunchKernelGGL(k_mm_bf16, dim3(blocks((bp / 32) * (kH / 32), 4)), dim3(256), 0, st, m1);
  MmArgs m2 = m1;
  m2.A = reinterpret_cast<const __bf16 *>(w + L.h1h);
  m2.Bt = reinterpret_cast<const __bf16 *>(s + sW2h);
  m2.K = kH;
  m2.Cf = reinterpret_cast<float *>(w + L.h2);
  m2.bias = th + oB2;
  m2.Ch = reinterpret_cast<__bf16 *>(w + L.h2h);
  m2.Cht = reinterpret_cast<__bf16 *>(w + L.h2ht);
  hipLaunchKernelGGL(k_mm_bf16, dim3(blocks((bp / 32) * (kH / 32), 4)), dim3(256), 0, st, m2);
  hipLaunchKernelGGL(k_head_fwd, dim3(blocks(b, 256)), dim3(256), 0, st,
                     reinterpret_cast<const float *>(w + L.h2), th,
                     reinterpret_cast<const __bf16 *>(s + sW3h), b, y);
  return hipGetLastError();
}

hipError_t mlp_backward(void *state, int64_t b, const float *y, const float *target, float under,
                        float *loss, void *scratch, hipStream_t st) {
  if (b <= 0) return hipSuccess;
  char *s = static_cast<char *>(state);
  char *w = static_cast<char *>(scratch);
  const int64_t bp = (b + 31) / 32 * 32;
  const Scratch L = scratch_layout(bp);
  float *g = reinterpret_cast<float *>(s + sG);
  hipLaunchKernelGGL(k_zero_f32, dim3(blocks(kP, 256)), dim3(256), 0, st, g, kP);
  if (loss) hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(256), 0, st, loss, (int64_t)1);
  hipLaunchKernelGGL(k_head_bwd, dim3(blocks(bp, 256)), dim3(256), 0, st,
                     reinterpret_cast<const float *>(w + L.h2), y, target,
                     reinterpret_cast<const __bf16 *>(s + sW3h), b, bp, under, g, loss,
                     reinterpret_cast<__bf16 *>(w + L.dh2h), reinterpret_cast<__bf16 *>(w + L.dh2ht));
  // dW2 = dH2^T H1  (128 x 128, contraction over the batch)
  MmArgs a{};
  a.A = reinterpret_cast<const __bf16 *>(w + L.dh2ht);
  a.Bt = reinterpret_cast<const __bf16 *>(w + L.h1ht);
  a.M = kH;
  a.N = kH;
  a.K = bp;
  a.mode = 0;
  a.Cf = g + oW2;
  hipLaunchKernelGGL(k_mm_bf16, dim3(blocks((kH / 32) * (kH / 32), 4)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(128), 0, st,
                     reinterpret_cast<const __bf16 *>(w + L.dh2h), bp, kH, g + oB2);
  // dH1 = (dH2 W2) * [H1 > 0]   (bp x 128)
  MmArgs d{};
  d.A = reinterpret_cast<const __bf16 *>(w + L.dh2h);
  d.Bt = reinterpret_cast<const __bf16 *>(s + sW2th);
  d.M = bp;
  d.N = kH;
  d.K = kH;
  d.mode = 2;
  d.mask = reinterpret_cast<const float *>(w + L.h1);
  d.Ch = reinterpret_cast<__bf16 *>(w + L.dh1h);
  d.Cht = reinterpret_cast<__bf16 *>(w + L.dh1ht);
  hipLaunchKernelGGL(k_mm_bf16, dim3(blocks((bp / 32) * (kH / 32), 4)), dim3(256), 0, st, d);
  // dW1 = dH1^T X  (128 x 64)
  MmArgs e{};
  e.A = reinterpret_cast<const __bf16 *>(w + L.dh1ht);
  e.Bt = reinterpret_cast<const __bf16 *>(w + L.xht);
  e.M = kH;
  e.N = kIn;
  e.K = bp;
  e.mode = 0;
  e.Cf = g + oW1;
  hipLaunchKernelGGL(k_mm_bf16, dim3(blocks((kH / 32) * (kIn / 32), 4)), dim3(256), 0, st, e);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(128), 0, st,
                     reinterpret_cast<const __bf16 *>(w + L.dh1h), bp, kH, g + oB1);
  return hipGetLastError();
}

hipError_t mlp_adam(void *state, float lr, float b1, float b2, float eps, int64_t step,
                    hipStream_t st) {
  const float c1 = 1.0f - powf(b1, (float)step);
  const float c2 = 1.0f - powf(b2, (float)step);
  char *s = static_cast<char *>(state);
  hipLaunchKernelGGL(k_adam, dim3(blocks(kP, 256)), dim3(256), 0, st, s, lr, b1, b2, eps, c1, c2);
  hipLaunchKernelGGL(k_refresh_bf16, dim3(blocks(kH * kH, 256)), dim3(256), 0, st, s);
  return hipGetLastError();
}

}  // namespace oz
