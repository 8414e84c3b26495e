// Chinese-remainder pieces shared by the Ozaki-II kernels of libozaki
// (gfx950): the moduli and their constant tables, an exact balanced
// reduction on full-rate units, Garner's mixed-radix digits taken one modulus
// at a time, and the correctly rounded conversion of the rebuilt integer.
#pragma once

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

// Garner's mixed-radix digit of modulus K (balanced):
// d_K = (C_K - sum_{j<K} d_j P_j) P_K^-1 mod m_K, from the INT32 product C_K
// modulo m_K and the earlier digits, kept as bytes of W (d_j in byte j % 4 of
// W[j / 4]). With C_K split into 13-bit pieces c_0 + c_1 2^13 + c_2 2^26 (c_2
// signed, |c_2| <= 32), t = sum_p c_p (2^(13 p) P_K^-1) - sum_j d_j (P_j
// P_K^-1) is congruent to d_K and below 2 * 8191 * 127 + 32 * 127 + 20 * 128 *
// 127 < 2^22 in magnitude (balanced constants), so one exact bal_mod gives the
// digit; the sum over the earlier digits is one 4-way INT8 dot product per
// word. m_0 = 256: the INT32 wrap-around keeps C_0 mod 2^32, whose low byte is
// the digit.
template <int K, int NW>
__device__ __forceinline__ void digit_step(int ck, int (&W)[NW]) {
  static_assert(K / 4 < NW, "digit word");
  if constexpr (K == 0) {
    W[0] = ck & 0xff;
  } else {
    const int c0 = ck & 0x1fff, c1 = (ck >> 13) & 0x1fff, c2 = ck >> 26;
    int t = c0 * kT.c13[K][0] + __mul24(c1, kT.c13[K][1]) + __mul24(c2, kT.c13[K][2]);
#pragma unroll
    for (int h = 0; h <= (K - 1) / 4; ++h) t = __builtin_amdgcn_sdot4(W[h], kT.ng[h][K], t, false);
    const int dk = bal_mod<K>(t);
    if constexpr ((K & 3) == 0)
      W[K >> 2] = dk & 0xff;
    else
      W[K >> 2] |= (dk & 0xff) << (8 * (K & 3));
  }
}

// The integer c in [-M/2, M/2) with digits d_0..d_{N-1} (bytes of W):
// c = sum_k d_k P_k accumulated in 16-bit limbs (|partial| < 2^28), one carry
// pass, then packed into a 192-bit two's-complement integer.
template <int N, int NW>
__device__ __forceinline__ I192 combine(const int (&W)[NW]) {
  constexpr int NL = kT.nlM[N];
  int L[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) L[l] = 0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int dk = (int)(int8_t)((W[k >> 2] >> (8 * (k & 3))) & 0xff);
#pragma unroll
    for (int l = 0; l < kT.nl[k]; ++l) L[l] += __mul24(dk, kT.P[k][l]);
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

}  // namespace crt
}  // namespace oz
