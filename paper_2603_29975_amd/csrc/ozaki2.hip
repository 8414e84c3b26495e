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
#include "ozaki2_crt.hpp"

namespace oz {
namespace crt {

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
// N residues into plane k of the packed fragment layout (nrb 32-row blocks x
// nkb 32-entry contraction blocks per plane, `plane` bytes apart), where 8
// consecutive entries of a row are 8 consecutive bytes. View rows beyond
// v.R (up to the padded row count the grid covers) get zero residues.
template <bool CPLX, bool SIDEB, int N>
__global__ void __launch_bounds__(256) k_residues(View v, const int *code, int beta, int8_t *out,
                                                  int64_t nrb, int64_t nkb, int64_t plane) {
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
  const int c = vr < v.R ? code[vr] : 0;
  const bool live = vr < v.R && !code_bad(c);
  const int e = code_exp(c);

  int a[8][kPieces];
#pragma unroll
  for (int x = 0; x < 8; ++x)
    to_pieces(live ? tile[trow * kResPitch + res_slot(kq0 + x)] : 0.0, e, beta, a[x]);
  const int64_t kk = by * kResEntries + kq0;
  if constexpr (CPLX && SIDEB) {
    store_residues_b<N, 0>(a, out + frag_offset(0, 2 * vr, kk, nrb, nkb),
                           out + frag_offset(0, 2 * vr + 1, kk, nrb, nkb), plane);
  } else {
    store_residues<N, 0>(a, out + frag_offset(0, vr, kk, nrb, nkb), plane);
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
hipError_t residues_n(const View &v, const int *code, int n, int beta, int8_t *out, int64_t nrb,
                      int64_t nkb, int64_t plane, dim3 grid, hipStream_t st) {
  switch (n) {
#define OZ_RES(N)                                                                                  \
  case N:                                                                                          \
    hipLaunchKernelGGL((crt::k_residues<CPLX, SIDEB, N>), grid, dim3(256), 0, st, v, code, beta,  \
                       out, nrb, nkb, plane);                                                      \
    break;
    OZ_RES(2) OZ_RES(3) OZ_RES(4) OZ_RES(5) OZ_RES(6) OZ_RES(7) OZ_RES(8) OZ_RES(9) OZ_RES(10)
    OZ_RES(11) OZ_RES(12) OZ_RES(13) OZ_RES(14) OZ_RES(15) OZ_RES(16) OZ_RES(17) OZ_RES(18)
    OZ_RES(19) OZ_RES(20)
#undef OZ_RES
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_residues(const View &v, bool cplx, bool side_b, const int *code, int n, int beta,
                           int8_t *out, int64_t nrb, int64_t nkb, hipStream_t st) {
  // 128 contraction entries (four blocks) per workgroup; view rows up to the
  // padded X' rows (complex B: two X' rows per view row)
  if (v.R <= 0 || nrb <= 0 || nkb <= 0 || nkb % 4 != 0) return hipErrorInvalidValue;
  const int64_t view_rows = (cplx && side_b) ? nrb * 16 : nrb * 32;
  if (view_rows < v.R) return hipErrorInvalidValue;
  const int64_t plane = nrb * nkb * kFragBytes;
  const dim3 grid((unsigned)(view_rows / crt::kResRows), (unsigned)(nkb / 4));
  if (cplx)
    return side_b ? residues_n<true, true>(v, code, n, beta, out, nrb, nkb, plane, grid, st)
                  : residues_n<true, false>(v, code, n, beta, out, nrb, nkb, plane, grid, st);
  return residues_n<false, false>(v, code, n, beta, out, nrb, nkb, plane, grid, st);
}


}  // namespace oz
