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
constexpr int kLimbs = 11;  // 16-bit limbs of the products P_k (< 2^160)

struct Tables {
  int m[kModMax];            // the moduli, greedy from 256 downwards
  int inv[kModMax];          // (P_k)^-1 mod m_k, P_k = m_0 ... m_{k-1} (balanced)
  int g[kModMax][kModMax];   // g[j][q] = P_j (P_q)^-1 mod m_q for j < q (balanced)
  int ng[(kModMax + 3) / 4][kModMax];  // -g[4 h + b][q] as bytes b of a word (0 for 4 h + b >= q)
  int pw[kModMax][5];        // 2^(13 t) mod m_k (balanced)
  int c13[kModMax][3];       // 2^(13 t) (P_k)^-1 mod m_k (balanced)
  int P[kModMax][kLimbs];    // 16-bit limbs of P_k
  int nl[kModMax];           // nonzero limbs of P_k
  int nlM[kModMax + 1];      // limbs of M_n = P_n plus a sign limb
};

constexpr int bal_c(int r, int m) {
  r %= m;
  if (r < 0) r += m;
  return r >= (m + 1) / 2 ? r - m : r;
}

constexpr Tables make_tables() {
  Tables t{};
  int n = 0;
  for (int c = 256; n < kModMax; --c) {
    bool ok = true;
    for (int j = 0; j < n; ++j)
      if (gcd_c(c, t.m[j]) != 1) ok = false;
    if (ok) t.m[n++] = c;
  }
  int pmod[kModMax][kModMax] = {};  // P_j mod m_q
  for (int q = 0; q < kModMax; ++q) {
    int p = 1 % t.m[q];
    for (int j = 0; j < kModMax; ++j) {
      pmod[j][q] = p;
      p = (p * t.m[j]) % t.m[q];
    }
  }
  for (int k = 0; k < kModMax; ++k) {
    const int mk = t.m[k];
    int x = 1;
    while ((pmod[k][k] * x) % mk != 1 % mk) ++x;
    t.inv[k] = bal_c(x, mk);
    for (int j = 0; j < k; ++j) t.g[j][k] = bal_c(pmod[j][k] * x, mk);
    for (int h = 0; h < (kModMax + 3) / 4; ++h) {
      unsigned w = 0;
      for (int b = 0; b < 4; ++b)
        if (4 * h + b < k) w |= (unsigned)(-t.g[4 * h + b][k] & 0xff) << (8 * b);
      t.ng[h][k] = (int)w;
    }
    int w = 1;
    for (int s = 0; s < 5; ++s) {
      t.pw[k][s] = bal_c(w, mk);
      if (s < 3) t.c13[k][s] = bal_c(w * x, mk);
      for (int b = 0; b < 13; ++b) w = (w * 2) % mk;
    }
  }
  int limb[kLimbs] = {1};
  for (int k = 0; k <= kModMax; ++k) {
    int top = 0;
    for (int l = 0; l < kLimbs; ++l)
      if (limb[l] != 0) top = l + 1;
    if (k < kModMax) {
      for (int l = 0; l < kLimbs; ++l) t.P[k][l] = limb[l];
      t.nl[k] = top;
    }
    // limbs of M_k (bits up to 16 top) plus one more for the sign of values in [-M/2, M/2)
    t.nlM[k] = top + 1 > kLimbs ? kLimbs : top + 1;
    if (k == kModMax) break;
    int carry = 0;
    for (int l = 0; l < kLimbs; ++l) {
      const int v = limb[l] * t.m[k] + carry;
      limb[l] = v & 0xffff;
      carry = v >> 16;
    }
  }
  return t;
}

constexpr Tables kT = make_tables();
static_assert(kT.m[0] == 256 && kT.m[1] == 255 && kT.m[11] == 217 && kT.m[19] == 173,
              "greedy coprime moduli");
static_assert(kT.nlM[kModMax] <= kLimbs, "limb count of the largest modulus product");

// Balanced residue of t modulo an odd m_K for |t| < 2^22: q = rint(t / m)
// computed in FP32 is the exact nearest quotient. t converts exactly, the
// quotient carries a relative error below 2^-23 (below 1/(2m) in absolute
// terms for |t| < 2^22), while t/m stays at least 1/(2m) away from every
// half-integer because m is odd. So r = t - q m is the balanced residue in
// [-(m-1)/2, (m-1)/2] without a correction step; every operation is a
// full-rate FP32 or 24-bit integer instruction.
template <int K>
__device__ __forceinline__ int bal_mod(int t) {
  constexpr int m = kT.m[K];
  static_assert(m % 2 == 1, "odd moduli only");
  constexpr float rm = 1.0f / (float)m;
  const int q = (int)__builtin_rintf((float)t * rm);
  return t - __mul24(q, m);
}

// ---------------------------------------------------------------- residues
// Residue tile: 16 view rows x 128 contraction entries of X' (64 complex
// elements); for complex B the 16 view rows (columns j) give the 32 X' rows
// 2j = (Re, -Im) and 2j+1 = (Im, Re). A thread converts 8 consecutive entries
// of one row, so the 16 threads of a row write its 128 residue bytes of one
// modulus as one full 128-byte line. In LDS entry e of a row sits at
// e + e / 8 (one pad double per 8), which spreads the 16 threads of a row
// over distinct banks.
constexpr int kResRows = 16;
constexpr int kResEntries = 128;
constexpr int kResPitch = kResEntries + kResEntries / 8 + 1;  // doubles per LDS row
constexpr int kResTileDoubles = kResRows * kResPitch;
__device__ __forceinline__ int res_slot(int e) { return e + (e >> 3); }

// trunc(x 2^(beta - e)) as five signed 13-bit pieces: x' = sum_t a_t 2^(13 t)
// with every a_t carrying the sign of x (|x'| < 2^63, so a_4 < 2^11).
constexpr int kPieces = 5;
__device__ __forceinline__ void to_pieces(double x, int e, int beta, int (&a)[kPieces]) {
  const Sig s = decompose(x, e);
  const int sh = s.sh0 + beta;
  uint64_t u;
  if (sh >= 0)
    u = s.m << sh;  // |x| < 2^e: the result stays below 2^beta
  else
    u = sh > -64 ? (s.m >> (-sh)) : 0ull;
#pragma unroll
  for (int t = 0; t < kPieces; ++t) {
    const int v = (int)((u >> (13 * t)) & 0x1fffu);
    a[t] = s.neg ? -v : v;
  }
}

// Balanced residue of x' modulo m_K from its signed pieces:
// x' = sum a_t 2^(13 t) = sum a_t pw_t (mod m) with |pw_t| <= 127, so the sum
// stays below 8191 * (1 + 4 * 127) < 2^22 and bal_mod is exact. For m = 256
// the residue is the low byte of x' in two's complement, which is the low
// byte of a_0 (2^13 = 0 mod 256).
template <int K>
__device__ __forceinline__ int residue(const int (&a)[kPieces]) {
  if constexpr (kT.m[K] == 256) {
    return a[0];  // only its low byte is stored
  } else {
    int t = a[0];
#pragma unroll
    for (int p = 1; p < kPieces; ++p) t += __mul24(a[p], kT.pw[K][p]);
    return bal_mod<K>(t);
  }
}

__device__ __forceinline__ uint32_t pack4(int r0, int r1, int r2, int r3) {
  return (uint32_t)(r0 & 0xff) | ((uint32_t)(r1 & 0xff) << 8) | ((uint32_t)(r2 & 0xff) << 16) |
         ((uint32_t)(r3 & 0xff) << 24);
}

// Residues of 16 consecutive contraction entries of one X' row, one 16-byte
// store per modulus.
template <int N, int K>
__device__ __forceinline__ void store_residues(const int (&a)[8][kPieces], int8_t *dst, int64_t plane) {
  if constexpr (K < N) {
    int r[8];
#pragma unroll
    for (int x = 0; x < 8; ++x) r[x] = residue<K>(a[x]);
    *reinterpret_cast<uint2 *>(dst + (int64_t)K * plane) =
        make_uint2(pack4(r[0], r[1], r[2], r[3]), pack4(r[4], r[5], r[6], r[7]));
    store_residues<N, K + 1>(a, dst, plane);
  }
}

// Complex B: the residues of 4 elements (Re, Im) give both X' rows: row 2j
// holds (Re, -Im) and row 2j+1 holds (Im, Re) along the contraction. The
// residue of -x is the negated residue (odd moduli: the balanced range is
// symmetric; 256: bytes negate modulo 256).
template <int N, int K>
__device__ __forceinline__ void store_residues_b(const int (&a)[8][kPieces], int8_t *dst0,
                                                 int8_t *dst1, int64_t plane) {
  if constexpr (K < N) {
    int r[8];
#pragma unroll
    for (int x = 0; x < 8; ++x) r[x] = residue<K>(a[x]);  // r[2e] = Re, r[2e+1] = Im
    *reinterpret_cast<uint2 *>(dst0 + (int64_t)K * plane) =
        make_uint2(pack4(r[0], -r[1], r[2], -r[3]), pack4(r[4], -r[5], r[6], -r[7]));
    *reinterpret_cast<uint2 *>(dst1 + (int64_t)K * plane) =
        make_uint2(pack4(r[1], r[0], r[3], r[2]), pack4(r[5], r[4], r[7], r[6]));
    store_residues_b<N, K + 1>(a, dst0, dst1, plane);
  }
}

// One block: view rows [16 bx, 16 bx + 16) x contraction entries [128 by,
// 128 by + 128) of X'. The tile is first copied into LDS with consecutive
// threads on the unit-stride direction of the view; thread t then converts
// the 8 entries [8 (t % 16), +8) of view row 16 bx + t / 16 and writes their
// N residues into plane k (row-major, `ldx` bytes per X' row).
template <bool CPLX, bool SIDEB, int N>
__global__ void __launch_bounds__(256) k_residues(View v, const int *code, int beta, int8_t *out,
                                                  int64_t ldx, int64_t plane) {
  constexpr int TL = CPLX ? kResEntries / 2 : kResEntries;  // view elements per tile row
  __shared__ double tile[kResTileDoubles];
  const int64_t bx = blockIdx.x, by = blockIdx.y;
  const int64_t r0 = bx * kResRows, l0 = by * TL;
  const bool rows_fast = v.sr == 1 && v.sl != 1;
  for (int c = threadIdx.x; c < kResRows * TL; c += 256) {
    const int rr = rows_fast ? c % kResRows : c / TL;
    const int ll = rows_fast ? c / kResRows : c % TL;
    const int64_t r = r0 + rr, l = l0 + ll;
    const bool in = r < v.R && l < v.L;
    if constexpr (CPLX) {
      double2 z = make_double2(0.0, 0.0);
      if (in) z = reinterpret_cast<const double2 *>(v.base)[r * v.sr + l * v.sl];
      tile[rr * kResPitch + res_slot(2 * ll)] = z.x;
      tile[rr * kResPitch + res_slot(2 * ll + 1)] = v.conj ? -z.y : z.y;
    } else {
      tile[rr * kResPitch + res_slot(ll)] =
          in ? reinterpret_cast<const double *>(v.base)[r * v.sr + l * v.sl] : 0.0;
    }
  }
  __syncthreads();

  const int tid = threadIdx.x;
  const int trow = tid >> 4;                    // view row within the tile
  const int kq0 = (tid & 15) * 8;               // first contraction entry within the tile
  const int64_t vr = bx * kResRows + trow;
  if (vr >= v.R) return;
  const int c = code[vr];
  const bool live = !code_bad(c);
  const int e = code_exp(c);

  int a[8][kPieces];
#pragma unroll
  for (int x = 0; x < 8; ++x)
    to_pieces(live ? tile[trow * kResPitch + res_slot(kq0 + x)] : 0.0, e, beta, a[x]);
  if constexpr (CPLX && SIDEB) {
    int8_t *dst0 = out + (2 * vr) * ldx + by * kResEntries + kq0;
    store_residues_b<N, 0>(a, dst0, dst0 + ldx, plane);
  } else {
    store_residues<N, 0>(a, out + vr * ldx + by * kResEntries + kq0, plane);
  }
}

// ---------------------------------------------------------------- reconstruction
// Two's-complement 192-bit integer (w0 least significant).
struct I192 {
  uint64_t w0, w1, w2;
};

// Round-to-nearest-even FP64 value of a 192-bit integer (its magnitude stays
// below 2^160, so the result is finite and the final scaling exact).
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
    } else if (sh < 64) {
      top = sh ? ((x.w0 >> sh) | (x.w1 << (64 - sh))) : x.w0;
      sticky = (x.w0 << (64 - sh)) != 0;
    } else {
      const int b = sh - 64;
      top = b ? ((x.w1 >> b) | (x.w2 << (64 - b))) : x.w1;
      sticky = x.w0 != 0 || (b && (x.w1 << (64 - b)) != 0);
    }
    uint64_t mant = top >> 11;  // 53 bits
    const bool rbit = (top >> 10) & 1u;
    sticky |= (top & 0x3ffu) != 0;
    if (rbit && (sticky || (mant & 1u))) ++mant;  // may carry to 2^53: still exact
    r = ldexp((double)mant, sh + 11);
  }
  return neg ? -r : r;
}

// Mixed-radix digits of c (Garner, balanced digits):
// d_K = (C_K - sum_{j<K} d_j P_j) P_K^-1 mod m_K. With C_K split into 13-bit
// pieces c_0 + c_1 2^13 + c_2 2^26 (c_2 signed, |c_2| <= 32),
// t = sum_p c_p (2^(13 p) P_K^-1) - sum_j d_j (P_j P_K^-1) is congruent to d_K
// and below 2 * 8191 * 127 + 32 * 127 + 20 * 128 * 127 < 2^22 in magnitude
// (balanced constants), so one exact bal_mod gives the digit. The digits are
// kept as bytes of W (d_j in byte j % 4 of W[j / 4]), so the sum over the
// earlier digits is one 4-way INT8 dot product per word.
template <int N, int K>
__device__ __forceinline__ void digits(const int (&Ck)[N], int (&W)[(N + 3) / 4], int (&d)[N]) {
  if constexpr (K < N) {
    int dk;
    if constexpr (K == 0) {
      dk = (int)(int8_t)(Ck[0] & 0xff);  // m_0 = 256: INT32 wrap-around keeps the low byte
      W[0] = Ck[0] & 0xff;
    } else {
      const int c0 = Ck[K] & 0x1fff, c1 = (Ck[K] >> 13) & 0x1fff, c2 = Ck[K] >> 26;
      int t = c0 * kT.c13[K][0] + __mul24(c1, kT.c13[K][1]) + __mul24(c2, kT.c13[K][2]);
#pragma unroll
      for (int h = 0; h <= (K - 1) / 4; ++h) t = __builtin_amdgcn_sdot4(W[h], kT.ng[h][K], t, false);
      dk = bal_mod<K>(t);
      if constexpr ((K & 3) == 0)
        W[K >> 2] = dk & 0xff;
      else
        W[K >> 2] |= (dk & 0xff) << (8 * (K & 3));
    }
    d[K] = dk;
    digits<N, K + 1>(Ck, W, d);
  }
}

// The integer c in [-M/2, M/2) with c = C_k mod m_k for k < N:
// c = sum_k d_k P_k accumulated in 16-bit limbs (|partial| < 2^28), one carry
// pass, then packed into a 192-bit two's-complement integer.
template <int N>
__device__ __forceinline__ I192 reconstruct(const int (&Ck)[N]) {
  constexpr int NL = kT.nlM[N];
  int W[(N + 3) / 4], d[N];
  digits<N, 0>(Ck, W, d);
  int L[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) L[l] = 0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
#pragma unroll
    for (int l = 0; l < kT.nl[k]; ++l) L[l] += __mul24(d[k], kT.P[k][l]);
  }
#pragma unroll
  for (int l = 0; l + 1 < NL; ++l) {
    L[l + 1] += L[l] >> 16;
    L[l] &= 0xffff;
  }
  uint64_t w[3] = {0ull, 0ull, 0ull};
#pragma unroll
  for (int l = 0; l + 1 < NL; ++l) w[l >> 2] |= (uint64_t)(uint32_t)L[l] << (16 * (l & 3));
  constexpr int lt = NL - 1;
  const int64_t top = (int64_t)L[lt];
  w[lt >> 2] |= (uint64_t)top << (16 * (lt & 3));
#pragma unroll
  for (int q = (lt >> 2) + 1; q < 3; ++q) w[q] = top < 0 ? ~0ull : 0ull;
  return I192{w[0], w[1], w[2]};
}

// One output entry (i, j): rebuild the exact integer(s) from the N INT32
// planes, round to FP64, scale by 2^(e_i + f_j - 2 beta) and apply
// alpha/beta (no fused multiply-adds); non-finite rows/columns give NaN.
// Consecutive threads take consecutive rows i (coalesced plane reads and
// C writes).
template <bool CPLX, int N>
__global__ void __launch_bounds__(256) k_crt(CrtArgs a) {
  const uint32_t nbi = (uint32_t)((a.m + 255) >> 8);
  const int64_t j = blockIdx.x / nbi;
  const int64_t i = (int64_t)(blockIdx.x % nbi) * 256 + threadIdx.x;
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
  if (v.R <= 0 || ldx <= 0 || ldx % crt::kResEntries != 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((v.R + crt::kResRows - 1) / crt::kResRows),
                  (unsigned)(ldx / crt::kResEntries));
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
