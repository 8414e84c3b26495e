// Ozaki-II emulation of FP64 and complex-FP64 GEMM (Section 2.2 of the
// paper): both operands are scaled to integer matrices, each integer product
// is formed modulo N pairwise-coprime moduli as N exact INT8 x INT8 -> INT32
// matrix products, and the Chinese remainder theorem rebuilds the exact
// integer product, which is rounded once to FP64 and scaled back. Section 3
// runs it with 10..18 moduli.
//
// Rules of this library (listed with the C ABI in include/ozaki.h):
//   moduli     the N largest pairwise-coprime integers <= 256, taken greedily
//              from 256 downwards; a residue is the representative of x mod m
//              in [-floor(m/2), ceil(m/2) - 1], which fits INT8.
//   integers   A'_il = trunc(a_il 2^(beta - e_i)), B'_lj = trunc(b_lj 2^(beta -
//              f_j)), with e_i, f_j the frexp exponents of the row/column
//              maxima (the exponent scan of the Ozaki-I path) and beta =
//              min(63, floor((floor(log2 M) - 1 - ceil(log2 K')) / 2)) for
//              M = m_1 ... m_N; |A'B'| < K' 2^(2 beta) <= M/2.
//   products   C_k = (A' mod m_k)(B' mod m_k) in INT32: exact for K' <= 2^17
//              (|r| <= 127 for the odd moduli); for m = 256 the INT32
//              wrap-around keeps the value mod 256.
//   rebuild    the unique c in [-M/2, M/2) with c = C_k mod m_k (mixed-radix
//              digits, balanced), then P = RN(c) 2^(e_i + f_j - 2 beta) and
//              alpha/beta, non-finite rows/columns as NaN, exactly as the
//              Ozaki-I epilogue.
// Complex data is one real product with the contraction interleaved (K' = 2k):
// A' rows (Re, Im), B' rows 2j = (Re, -Im) and 2j+1 = (Im, Re) of column j.
#include "ozaki_internal.hpp"

namespace oz {
namespace crt {

// ---------------------------------------------------------------- constants
constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

struct Tables {
  int m[kModMax];             // the moduli, greedy from 256 downwards
  int pm[kModMax][kModMax];   // pm[j][q] = (m_0 ... m_{j-1}) mod m_q
  int inv[kModMax];           // inverse of (m_0 ... m_{k-1}) mod m_k
  int pw[kModMax][4];         // 2^(16 t) mod m_k
};

constexpr Tables make_tables() {
  Tables t{};
  int n = 0;
  for (int c = 256; n < kModMax; --c) {
    bool ok = true;
    for (int j = 0; j < n; ++j)
      if (gcd_c(c, t.m[j]) != 1) ok = false;
    if (ok) t.m[n++] = c;
  }
  for (int q = 0; q < kModMax; ++q) {
    int p = 1 % t.m[q];
    for (int j = 0; j < kModMax; ++j) {
      t.pm[j][q] = p;  // product of the moduli before j, mod m_q
      p = (p * t.m[j]) % t.m[q];
    }
  }
  for (int k = 0; k < kModMax; ++k) {
    const int a = t.pm[k][k];
    int x = 1;
    while ((a * x) % t.m[k] != 1 % t.m[k]) ++x;
    t.inv[k] = x % t.m[k];
    int w = 1;
    for (int s = 0; s < 4; ++s) {
      t.pw[k][s] = w % t.m[k];
      for (int b = 0; b < 16; ++b) w = (w * 2) % t.m[k];
    }
  }
  return t;
}

constexpr Tables kT = make_tables();
static_assert(kT.m[0] == 256 && kT.m[1] == 255 && kT.m[11] == 217 && kT.m[19] == 173,
              "greedy coprime moduli");

// x mod m in [0, m) for a 32-bit value. m = 256 reads the low byte, which is
// also right for INT32 sums that wrapped around.
template <int K>
__device__ __forceinline__ int mod_pos(int x) {
  constexpr int m = kT.m[K];
  if constexpr (m == 256) {
    return x & 255;
  } else {
    int r = x % m;
    return r < 0 ? r + m : r;
  }
}

// Balanced representative of r in [0, m).
template <int K>
__device__ __forceinline__ int balance(int r) {
  constexpr int m = kT.m[K];
  return r >= (m + 1) / 2 ? r - m : r;
}

// ---------------------------------------------------------------- residues
// Residue tile: 64 rows of X' x 64 contraction entries. Rows of X' are view
// rows, except for complex B where X' rows 2j and 2j+1 both come from view
// row j (32 view rows per tile).
template <bool CPLX, bool SIDEB>
struct ResTile {
  static constexpr int TR = (CPLX && SIDEB) ? 32 : 64;  // view rows
  static constexpr int TL = CPLX ? 32 : 64;              // contraction elements
  static constexpr int EW = CPLX ? 2 : 1;                // doubles per element
  static constexpr int PITCH = TL * EW + 1;              // doubles per LDS row
};
constexpr int kResTileDoubles = 64 * (64 + 1);

// |x| 2^(beta - e) truncated, as an unsigned integer (< 2^63), and the sign.
__device__ __forceinline__ uint64_t to_int(double x, int e, int beta, bool &neg) {
  const Sig s = decompose(x, e);
  neg = s.neg;
  const int sh = s.sh0 + beta;
  if (sh >= 0) return s.m << sh;  // |x| < 2^e: the result stays below 2^beta
  return sh > -64 ? (s.m >> (-sh)) : 0ull;
}

// Balanced residue of +-u modulo m_K from the 16-bit pieces of u.
template <int K>
__device__ __forceinline__ int residue(const uint32_t (&a)[4], bool neg) {
  constexpr int m = kT.m[K];
  uint32_t t = a[0];
  if constexpr (m != 256)
    t += a[1] * (uint32_t)kT.pw[K][1] + a[2] * (uint32_t)kT.pw[K][2] +
         a[3] * (uint32_t)kT.pw[K][3];  // < 2^16 (1 + 3 * 255) < 2^26
  int r = (int)(t % (uint32_t)m);
  if (neg && r != 0) r = m - r;
  return balance<K>(r);
}

template <int N, int K>
__device__ __forceinline__ void store_residues(const uint32_t (&a)[16][4], const bool (&neg)[16],
                                               int8_t *dst, int64_t plane) {
  if constexpr (K < N) {
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t word = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        word |= ((uint32_t)residue<K>(a[4 * q + b], neg[4 * q + b]) & 0xffu) << (8 * b);
      w[q] = word;
    }
    *reinterpret_cast<uint4 *>(dst + (int64_t)K * plane) = make_uint4(w[0], w[1], w[2], w[3]);
    store_residues<N, K + 1>(a, neg, dst, plane);
  }
}

// One block: X' rows [64 bx, 64 bx + 64) x contraction entries [64 by, 64 by
// + 64). The tile is first copied into LDS with consecutive threads on the
// unit-stride direction of the view; thread t then converts the 16 entries
// [16 (t % 4), +16) of X' row 64 bx + t / 4 and writes their N residues, one
// 16-byte store per modulus into plane k (row-major, `ldx` bytes per row).
template <bool CPLX, bool SIDEB, int N>
__global__ void __launch_bounds__(256) k_residues(View v, const int *code, int beta, int8_t *out,
                                                  int64_t ldx, int64_t plane) {
  using T = ResTile<CPLX, SIDEB>;
  __shared__ double tile[kResTileDoubles];
  const int64_t bx = blockIdx.x, by = blockIdx.y;
  const int64_t r0 = bx * T::TR, l0 = by * T::TL;
  const bool rows_fast = v.sr == 1 && v.sl != 1;
  for (int c = threadIdx.x; c < T::TR * T::TL; c += 256) {
    const int rr = rows_fast ? c % T::TR : c / T::TL;
    const int ll = rows_fast ? c / T::TR : c % T::TL;
    const int64_t r = r0 + rr, l = l0 + ll;
    const bool in = r < v.R && l < v.L;
    if constexpr (CPLX) {
      double2 z = make_double2(0.0, 0.0);
      if (in) z = reinterpret_cast<const double2 *>(v.base)[r * v.sr + l * v.sl];
      tile[rr * T::PITCH + 2 * ll] = z.x;
      tile[rr * T::PITCH + 2 * ll + 1] = v.conj ? -z.y : z.y;
    } else {
      tile[rr * T::PITCH + ll] = in ? reinterpret_cast<const double *>(v.base)[r * v.sr + l * v.sl] : 0.0;
    }
  }
  __syncthreads();

  const int tid = threadIdx.x;
  const int orow = tid >> 2;                    // X' row within the tile
  const int kq0 = (tid & 3) * 16;               // first contraction entry within the tile
  const int64_t rp = bx * 64 + orow;
  const int64_t rows = (CPLX && SIDEB) ? 2 * v.R : v.R;
  if (rp >= rows) return;
  const int trow = (CPLX && SIDEB) ? (orow >> 1) : orow;  // LDS row
  const int64_t vr = (CPLX && SIDEB) ? (rp >> 1) : rp;    // view row
  const int c = code[vr];
  const bool live = !code_bad(c);
  const int e = code_exp(c);

  uint32_t a[16][4];
  bool neg[16];
#pragma unroll
  for (int x = 0; x < 16; ++x) {
    double val = 0.0;
    if (live) {
      if constexpr (CPLX && SIDEB) {
        const int ll = (kq0 + x) >> 1;            // element of column j
        const double re = tile[trow * T::PITCH + 2 * ll];
        const double im = tile[trow * T::PITCH + 2 * ll + 1];
        if ((rp & 1) == 0)
          val = (x & 1) ? -im : re;               // row 2j: (Re, -Im)
        else
          val = (x & 1) ? re : im;                // row 2j+1: (Im, Re)
      } else {
        val = tile[trow * T::PITCH + kq0 + x];    // real, or (Re, Im) interleaved
      }
    }
    const uint64_t u = to_int(val, e, beta, neg[x]);
    a[x][0] = (uint32_t)(u & 0xffffu);
    a[x][1] = (uint32_t)((u >> 16) & 0xffffu);
    a[x][2] = (uint32_t)((u >> 32) & 0xffffu);
    a[x][3] = (uint32_t)(u >> 48);
  }
  int8_t *dst = out + rp * ldx + by * 64 + kq0;
  store_residues<N, 0>(a, neg, dst, plane);
}

// ---------------------------------------------------------------- reconstruction
// Two's-complement 192-bit integer (w0 least significant).
struct I192 {
  uint64_t w0, w1, w2;
};

// x <- x * mul + d for 0 < mul <= 256 and a small signed d.
__device__ __forceinline__ void mul_add(I192 &x, uint64_t mul, int d) {
  const uint64_t lo0 = x.w0 * mul, hi0 = __umul64hi(x.w0, mul);
  const uint64_t lo1 = x.w1 * mul, hi1 = __umul64hi(x.w1, mul);
  const uint64_t lo2 = x.w2 * mul;
  uint64_t r1 = lo1 + hi0;
  uint64_t r2 = lo2 + hi1 + (r1 < lo1 ? 1u : 0u);
  const uint64_t dd = (uint64_t)(int64_t)d, ext = d < 0 ? ~0ull : 0ull;
  const uint64_t r0 = lo0 + dd;
  const uint64_t c0 = r0 < lo0 ? 1u : 0u;
  const uint64_t s1 = r1 + ext;
  const uint64_t c1 = s1 < r1 ? 1u : 0u;
  const uint64_t t1 = s1 + c0;
  const uint64_t c2 = t1 < s1 ? 1u : 0u;
  x.w0 = r0;
  x.w1 = t1;
  x.w2 = r2 + ext + c1 + c2;
}

// Round-to-nearest-even FP64 value of a 192-bit integer (its magnitude stays
// below 2^160, so the result is finite and exact scaling applies).
__device__ __forceinline__ double to_double_rn(I192 x) {
  const bool neg = (int64_t)x.w2 < 0;
  if (neg) {
    x.w0 = ~x.w0;
    x.w1 = ~x.w1;
    x.w2 = ~x.w2;
    x.w0 += 1;
    const uint64_t c0 = x.w0 == 0 ? 1u : 0u;
    x.w1 += c0;
    x.w2 += (c0 && x.w1 == 0) ? 1u : 0u;
  }
  int h;  // index of the highest set bit
  if (x.w2 != 0)
    h = 128 + 63 - __clzll((long long)x.w2);
  else if (x.w1 != 0)
    h = 64 + 63 - __clzll((long long)x.w1);
  else if (x.w0 != 0)
    h = 63 - __clzll((long long)x.w0);
  else
    return 0.0;
  double r;
  if (h <= 52) {
    r = (double)x.w0;  // exact
  } else {
    // top = bits [h - 63, h] (h >= 63) or x << (63 - h); sticky = lower bits
    const int sh = h - 63;
    uint64_t top;
    bool sticky = false;
    if (sh <= 0) {
      top = x.w0 << (-sh);
    } else {
      const int q = sh >> 6, b = sh & 63;
      const uint64_t w[4] = {x.w0, x.w1, x.w2, 0ull};
      top = b ? ((w[q] >> b) | (w[q + 1] << (64 - b))) : w[q];
      for (int t = 0; t < q; ++t) sticky |= w[t] != 0;
      if (b) sticky |= (w[q] << (64 - b)) != 0;
    }
    uint64_t mant = top >> 11;  // 53 bits
    const bool rbit = (top >> 10) & 1u;
    sticky |= (top & 0x3ffu) != 0;
    if (rbit && (sticky || (mant & 1u))) ++mant;  // may carry to 2^53: still exact
    r = ldexp((double)mant, sh + 11);
  }
  return neg ? -r : r;
}

// Mixed-radix digits of c (Garner, balanced digits): d_K = (C_K - sum_{j<K}
// d_j P_j) P_K^-1 mod m_K with P_j = m_0 ... m_{j-1}. acc[q] carries
// sum_{j<K} d_j (P_j mod m_q) for the moduli still to come; its magnitude
// stays below 20 * 128 * 256 < 2^20, so no reduction is needed on the way.
template <int N, int K>
__device__ __forceinline__ void digits(const int (&Ck)[N], int (&acc)[N], int (&d)[N]) {
  if constexpr (K < N) {
    constexpr int m = kT.m[K];
    const int t = mod_pos<K>(mod_pos<K>(Ck[K]) - acc[K]);
    const int dk = balance<K>((t * kT.inv[K]) % m);
    d[K] = dk;
#pragma unroll
    for (int q = K + 1; q < N; ++q) acc[q] += dk * kT.pm[K][q];
    digits<N, K + 1>(Ck, acc, d);
  }
}

// The integer c in [-M/2, M/2) with c = C_k mod m_k for k < N:
// c = d_0 + m_0 (d_1 + m_1 (d_2 + ...)) evaluated in 192-bit arithmetic.
template <int N>
__device__ __forceinline__ I192 reconstruct(const int (&Ck)[N]) {
  int acc[N], d[N];
#pragma unroll
  for (int q = 0; q < N; ++q) acc[q] = 0;
  digits<N, 0>(Ck, acc, d);
  const uint64_t ext = d[N - 1] < 0 ? ~0ull : 0ull;
  I192 x{(uint64_t)(int64_t)d[N - 1], ext, ext};
#pragma unroll
  for (int k = N - 2; k >= 0; --k) mul_add(x, (uint64_t)kT.m[k], d[k]);
  return x;
}

// One output entry (i, j): rebuild the exact integer(s) from the N INT32
// planes, round to FP64, scale by 2^(e_i + f_j - 2 beta) and apply
// alpha/beta (no fused multiply-adds); non-finite rows/columns give NaN.
// Consecutive threads take consecutive rows i (coalesced plane reads and
// C writes).
template <bool CPLX, int N>
__global__ void __launch_bounds__(256) k_crt(CrtArgs a) {
  const int64_t nbi = (a.m + 255) >> 8;
  const int64_t j = (int64_t)blockIdx.x / nbi;
  const int64_t i = ((int64_t)blockIdx.x % nbi) * 256 + threadIdx.x;
  if (i >= a.m) return;
  const int ca = a.codeA[i], cb = a.codeB[j];
  const bool bad = code_bad(ca) || code_bad(cb);
  const int sc = code_exp(ca) + code_exp(cb) - 2 * a.beta;
  if constexpr (CPLX) {
    double2 *cp = reinterpret_cast<double2 *>(a.C) + i + j * a.ldc;
    if (bad) {
      *cp = make_double2(qnan(), qnan());
      return;
    }
    double p[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int32_t *src = a.Cint + i + (2 * j + h) * a.m;
      int Ck[N];
#pragma unroll
      for (int k = 0; k < N; ++k) Ck[k] = src[k * a.plane];
      p[h] = ldexp(to_double_rn(reconstruct<N>(Ck)), sc);
    }
    double re = sub_rn(mul_rn(a.ar, p[0]), mul_rn(a.ai, p[1]));
    double im = add_rn(mul_rn(a.ar, p[1]), mul_rn(a.ai, p[0]));
    if (!a.beta_zero) {
      const double2 z = *cp;
      re = add_rn(re, sub_rn(mul_rn(a.br, z.x), mul_rn(a.bi, z.y)));
      im = add_rn(im, add_rn(mul_rn(a.br, z.y), mul_rn(a.bi, z.x)));
    }
    *cp = make_double2(re, im);
  } else {
    double *cp = reinterpret_cast<double *>(a.C) + i + j * a.ldc;
    if (bad) {
      *cp = qnan();
      return;
    }
    const int32_t *src = a.Cint + i + j * a.m;
    int Ck[N];
#pragma unroll
    for (int k = 0; k < N; ++k) Ck[k] = src[k * a.plane];
    const double p = ldexp(to_double_rn(reconstruct<N>(Ck)), sc);
    double out = mul_rn(a.ar, p);
    if (!a.beta_zero) out = add_rn(out, mul_rn(a.br, *cp));
    *cp = out;
  }
}

}  // namespace crt

// ---------------------------------------------------------------- host side
int crt_modulus(int k) { return (k >= 0 && k < kModMax) ? crt::kT.m[k] : 0; }

int crt_log2_floor(int n) {
  if (n < 1 || n > kModMax) return -1;
  uint32_t w[6] = {1, 0, 0, 0, 0, 0};  // little-endian 32-bit limbs of the product
  for (int k = 0; k < n; ++k) {
    uint64_t carry = 0;
    for (int t = 0; t < 6; ++t) {
      const uint64_t v = (uint64_t)w[t] * (uint64_t)crt::kT.m[k] + carry;
      w[t] = (uint32_t)v;
      carry = v >> 32;
    }
  }
  for (int t = 5; t >= 0; --t)
    if (w[t] != 0) return 32 * t + 31 - __builtin_clz(w[t]);
  return -1;
}

int crt_beta(int n, int64_t kprime) {
  const int lm = crt_log2_floor(n);
  if (lm < 0) return 0;
  int lk = 0;
  while (lk < 62 && ((int64_t)1 << lk) < kprime) ++lk;
  const int num = lm - 1 - lk;
  const int b = num >= 0 ? num / 2 : -((-num + 1) / 2);  // floor division
  return b > 63 ? 63 : b;
}

namespace {
template <bool CPLX, bool SIDEB>
hipError_t residues_n(const View &v, const int *code, int n, int beta, int8_t *out, int64_t ldx,
                      int64_t plane, dim3 grid, hipStream_t st) {
  switch (n) {
#define OZ_RES(N)                                                                                  \
  case N:                                                                                          \
    hipLaunchKernelGGL((crt::k_residues<CPLX, SIDEB, N>), grid, dim3(256), 0, st, v, code, beta,  \
                       out, ldx, plane);                                                           \
    break;
    OZ_RES(2) OZ_RES(3) OZ_RES(4) OZ_RES(5) OZ_RES(6) OZ_RES(7) OZ_RES(8) OZ_RES(9) OZ_RES(10)
    OZ_RES(11) OZ_RES(12) OZ_RES(13) OZ_RES(14) OZ_RES(15) OZ_RES(16) OZ_RES(17) OZ_RES(18)
    OZ_RES(19) OZ_RES(20)
#undef OZ_RES
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool CPLX>
hipError_t crt_n(int n, const CrtArgs &a, dim3 grid, hipStream_t st) {
  switch (n) {
#define OZ_CRT(N)                                                                     \
  case N:                                                                             \
    hipLaunchKernelGGL((crt::k_crt<CPLX, N>), grid, dim3(256), 0, st, a);             \
    break;
    OZ_CRT(2) OZ_CRT(3) OZ_CRT(4) OZ_CRT(5) OZ_CRT(6) OZ_CRT(7) OZ_CRT(8) OZ_CRT(9) OZ_CRT(10)
    OZ_CRT(11) OZ_CRT(12) OZ_CRT(13) OZ_CRT(14) OZ_CRT(15) OZ_CRT(16) OZ_CRT(17) OZ_CRT(18)
    OZ_CRT(19) OZ_CRT(20)
#undef OZ_CRT
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_residues(const View &v, bool cplx, bool side_b, const int *code, int n, int beta,
                           int8_t *out, int64_t ldx, int64_t plane, hipStream_t st) {
  const int64_t rows = (cplx && side_b) ? 2 * v.R : v.R;
  if (rows <= 0 || ldx <= 0 || ldx % 64 != 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((rows + 63) / 64), (unsigned)(ldx / 64));
  if (cplx)
    return side_b ? residues_n<true, true>(v, code, n, beta, out, ldx, plane, grid, st)
                  : residues_n<true, false>(v, code, n, beta, out, ldx, plane, grid, st);
  return residues_n<false, false>(v, code, n, beta, out, ldx, plane, grid, st);
}

hipError_t launch_crt(int n, bool cplx, const CrtArgs &a, hipStream_t st) {
  if (a.m <= 0 || a.n <= 0) return hipSuccess;
  const int64_t blocks = ((a.m + 255) >> 8) * a.n;
  if (blocks > 0x7fffffffll) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  return cplx ? crt_n<true>(n, a, grid, st) : crt_n<false>(n, a, grid, st);
}

}  // namespace oz
