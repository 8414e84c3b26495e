// Shared definitions of the HIP kernels and the host runtime of libozaki.
//
// Exponent codes, the trunc-7 digit extraction and the packed slice layout
// used by every kernel. The arithmetic follows the Ozaki-I description in
// Section 2.2 of the paper (exponent alignment, slicing by significant bits);
// the exact rules are listed in include/ozaki.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oz {

constexpr int kDigitBits = 7;          // bits per slice
constexpr int kSMax = 12;              // largest slice count
constexpr int kCodeBias = 2048;        // exponent code = e + bias (zero -> 0)
constexpr int kCodeBad = 0x7fff0000;   // row/column holds Inf or NaN
constexpr int64_t kRowPad = 128;       // packed operand rows are padded to this
constexpr int64_t kKPad = 64;          // packed contraction length padded to this
constexpr int kFragBytes = 1024;       // one packed 32 x 32 int8 fragment

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));

inline int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// ---------------------------------------------------------------- exponents
// Code of one FP64 value: 0 for +-0, kCodeBad for Inf/NaN, otherwise
// e + kCodeBias where e is the frexp exponent (|v| in [2^(e-1), 2^e)).
// The frexp exponent of a row maximum is the maximum of the entries' codes.
// Written with selects, not branches: a scan issues its loads back to back
// only when nothing between them depends on a loaded value.
__device__ __forceinline__ int expo_code(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v) & 0x7fffffffffffffffull;
  const uint32_t E = (uint32_t)(b >> 52);
  // subnormal: value = b * 2^-1074 with its top set bit at position h (b | 1
  // keeps the count defined for b = 0, whose code is 0 anyway)
  const int h = 63 - __clzll((long long)(b | 1));
  const int e = E == 0 ? h - 1073 : (int)E - 1022;
  const int c = b == 0 ? 0 : e + kCodeBias;
  return E == 0x7ffu ? kCodeBad : c;
}

__host__ __device__ __forceinline__ bool code_bad(int c) { return c >= kCodeBad; }
__host__ __device__ __forceinline__ int code_exp(int c) {
  return (c == 0 || c >= kCodeBad) ? 0 : c - kCodeBias;
}

// ---------------------------------------------------------------- digits
// |v| * 2^-e = m * 2^sh0 with m the integer significand (hidden bit added for
// normal numbers). Digit p is floor(|x| 2^(7p)) mod 128 = floor(m 2^(sh0+7p))
// mod 128, with the sign of v. This is the integer form of repeated
// truncation: the p-th 7-bit group of |x| below the binary point.
struct Sig {
  uint64_t m;
  int sh0;
  bool neg;
};

__device__ __forceinline__ Sig decompose(double v, int e) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t E = (uint32_t)(b >> 52) & 0x7ffu;
  const uint64_t f = b & 0x000fffffffffffffull;
  Sig s;
  s.neg = (b >> 63) != 0;
  s.m = E ? (f | 0x0010000000000000ull) : f;
  const int lsb = E ? (int)E - 1075 : -1074;
  s.sh0 = lsb - e;
  return s;
}

__device__ __forceinline__ int digit(const Sig &x, int p) {
  const int sh = x.sh0 + kDigitBits * p;
  uint32_t d;
  if (sh >= 0) {
    d = (sh < kDigitBits) ? ((uint32_t)(x.m << sh) & 127u) : 0u;
  } else {
    const int rs = -sh;
    d = (rs < 64) ? ((uint32_t)(x.m >> rs) & 127u) : 0u;
  }
  return x.neg ? -(int)d : (int)d;
}

// ---------------------------------------------------------------- packed layout
// A packed operand X' (R' rows, K' contraction entries, both zero padded) is a
// sequence of 1 KiB fragments indexed [p][rb][kb] (slice, 32-row block,
// 32-entry contraction block). Inside a fragment byte (h*32 + r)*16 + b holds
// row 32*rb + r, contraction index 32*kb + 16*h + b: exactly the 16 bytes that
// lane (h*32 + r) of a 64-lane wave feeds to a 32x32x32 INT8 MFMA. A wave
// therefore moves a fragment with one contiguous 16-byte access per lane.
__host__ __device__ __forceinline__ int64_t frag_offset(int p, int64_t row, int64_t kk,
                                                        int64_t nrb, int64_t nkb) {
  const int64_t rb = row >> 5, kb = kk >> 5;
  const int64_t ri = row & 31, ki = kk & 31;
  return (((int64_t)p * nrb + rb) * nkb + kb) * kFragBytes + (((ki >> 4) * 32 + ri) * 16) +
         (ki & 15);
}

// ---------------------------------------------------------------- operand view
// Logical matrix X(r, l) (r < R, l < L) at element offset r*sr + l*sl from base.
// For op(A): r = row i, l = contraction index. For op(B): r = column j.
struct View {
  const void *base;
  int64_t R, L, sr, sl;
  bool conj;  // complex conjugate (trans 'C')
};

// FP64 helpers that are never contracted into fused multiply-adds.
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ double sub_rn(double a, double b) { return __dsub_rn(a, b); }

__device__ __forceinline__ double qnan() { return __longlong_as_double(0x7ff8000000000000ll); }

}  // namespace oz
