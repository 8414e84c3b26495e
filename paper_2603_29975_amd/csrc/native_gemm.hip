// Native FP64 GEMM on the gfx950 FP64 matrix cores (v_mfma_f64_16x16x4_f64).
//
// The comparator of the emulation: the paper's ground truth and speed
// baseline is native FP64 GEMM (Section 3.2). Same output orientation as the
// emulated kernel: MFMA rows are the output column side j' (the real- and
// imaginary-part rows of each column for complex data), MFMA columns are
// output rows i, so stores are contiguous in column-major C.
//
// Complex data is computed as one real GEMM over a contraction of length 2k:
// A'(i, 2l) = Re a_il, A'(i, 2l+1) = Im a_il; for column j of op(B) one B' row
// holds (Re b_lj, -Im b_lj) and another (Im b_lj, Re b_lj) at contraction
// positions (2l, 2l+1). The first row times A' gives Re (AB)_ij, the second
// Im (AB)_ij: four real products per complex product, as a plain ZGEMM does.
// Within each 16-row MFMA block, rows 0..7 are the real-part rows of 8
// consecutive columns j and rows 8..15 their imaginary-part rows. The FP64
// MFMA leaves D[l/16 + 4r][l%16] in lane l, register r, so registers r and
// r + 2 of a lane hold Re and Im of the same C entry.
//
// Tiles: 256 threads = 2 x 2 waves, wave tile 64 (j') x 64 (i) = 4 x 4 MFMA
// blocks of 16 x 16, contraction 16 per stage, LDS double buffered with a
// register prefetch of the next stage. Operands are gathered from their BLAS
// layout into LDS with the unit-stride dimension on consecutive lanes. The
// launch bounds ask for two workgroups per CU (<= 256 registers per wave):
// left free, the compiler takes 334 (accumulators in AGPRs), which allows one
// wave per SIMD and exposes every LDS and barrier wait (16384^3 complex: 26.6
// TFLOP/s at one wave per SIMD, 43.1 at two). The prefetch loads are
// unconditional (an element outside the matrix reads element (0, 0) and is
// replaced by zero when stored to LDS), so they stay in flight under the
// stage's MFMAs: with a bounds test around each load the compiler waited for
// every load before the MFMAs (43.1 -> 64.3 TFLOP/s at 16384^3).
#include "ozaki_internal.hpp"

namespace oz {

namespace {

constexpr int NBJ = 128;   // j' per workgroup tile
constexpr int NBI = 128;   // i per workgroup tile
constexpr int NBK = 16;    // contraction (real entries) per stage
constexpr int LDJ = NBJ + 1;  // padded LDS row length (doubles)
constexpr int LDI = NBI + 1;
constexpr int NTH = 256;

template <bool CPLX>
struct Loader {
  // Elements of the P (B') and Q (A') tiles a thread fetches per stage.
  static constexpr int PCNT = CPLX ? (NBJ / 2) * (NBK / 2) / NTH : NBJ * NBK / NTH;
  static constexpr int QCNT = CPLX ? NBI * (NBK / 2) / NTH : NBI * NBK / NTH;
  using T = typename std::conditional<CPLX, double2, double>::type;
};

// Raw element (r, l) of the view, or element (0, 0) when (r, l) lies outside
// it (ok = false; the caller substitutes zero). The load is unconditional, so
// the loads of a stage go out together and nothing waits for them before the
// stage's MFMAs; the conjugation is applied where the element is stored.
template <bool CPLX>
__device__ __forceinline__ typename Loader<CPLX>::T load_raw(const View &v, int64_t r, int64_t l,
                                                             bool &ok) {
  using T = typename Loader<CPLX>::T;
  ok = r < v.R && l < v.L;
  const int64_t off = ok ? r * v.sr + l * v.sl : 0;
  return reinterpret_cast<const T *>(v.base)[off];
}

template <bool CPLX>
__global__ void __launch_bounds__(NTH, 2) k_native(NativeArgs a) {
  using LD = Loader<CPLX>;
  using T = typename LD::T;
  __shared__ double ldsP[2][NBK * LDJ];
  __shared__ double ldsQ[2][NBK * LDI];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wj = wave & 1, wi = wave >> 1;

  const int64_t nprime = CPLX ? 2 * a.n : a.n;
  const int64_t nti = (a.m + NBI - 1) / NBI;
  const int64_t tj = blockIdx.x / nti;
  const int64_t ti = blockIdx.x % nti;
  const int64_t j0 = tj * NBJ;  // first j' of the tile
  const int64_t i0 = ti * NBI;
  const int64_t kreal = CPLX ? 2 * a.k : a.k;
  const int64_t nst = (kreal + NBK - 1) / NBK;

  // Tile geometry in source elements.
  constexpr int PR = CPLX ? NBJ / 2 : NBJ;  // source rows (columns j of op(B))
  constexpr int PL = CPLX ? NBK / 2 : NBK;  // source contraction entries
  constexpr int QR = NBI;
  constexpr int QL = PL;
  const bool p_rows_fast = a.B.sr == 1;
  const bool q_rows_fast = a.A.sr == 1;
  const int64_t pr0 = CPLX ? j0 / 2 : j0;

  T pbuf[LD::PCNT];
  T qbuf[LD::QCNT];
  bool pok[LD::PCNT], qok[LD::QCNT];
  const bool pconj = CPLX && a.B.conj, qconj = CPLX && a.A.conj;

  auto fetch = [&](int64_t st) {
    const int64_t l0 = st * PL;
#pragma unroll
    for (int x = 0; x < LD::PCNT; ++x) {
      const int e = tid + x * NTH;
      const int rl = p_rows_fast ? e % PR : e / PL;
      const int ll = p_rows_fast ? e / PR : e % PL;
      pbuf[x] = load_raw<CPLX>(a.B, pr0 + rl, l0 + ll, pok[x]);
    }
#pragma unroll
    for (int x = 0; x < LD::QCNT; ++x) {
      const int e = tid + x * NTH;
      const int rl = q_rows_fast ? e % QR : e / QL;
      const int ll = q_rows_fast ? e / QR : e % QL;
      qbuf[x] = load_raw<CPLX>(a.A, i0 + rl, l0 + ll, qok[x]);
    }
  };
  auto deposit = [&](int buf) {
    double *P = ldsP[buf];
    double *Q = ldsQ[buf];
#pragma unroll
    for (int x = 0; x < LD::PCNT; ++x) {
      const int e = tid + x * NTH;
      const int rl = p_rows_fast ? e % PR : e / PL;
      const int ll = p_rows_fast ? e / PR : e % PL;
      if constexpr (CPLX) {
        double2 z = pok[x] ? pbuf[x] : make_double2(0.0, 0.0);
        if (pconj) z.y = -z.y;
        const int rre = 16 * (rl >> 3) + (rl & 7);  // real-part row of column rl
        const int rim = rre + 8;                    // imaginary-part row
        P[(2 * ll) * LDJ + rre] = z.x;
        P[(2 * ll + 1) * LDJ + rre] = -z.y;
        P[(2 * ll) * LDJ + rim] = z.y;
        P[(2 * ll + 1) * LDJ + rim] = z.x;
      } else {
        P[ll * LDJ + rl] = pok[x] ? pbuf[x] : 0.0;
      }
    }
#pragma unroll
    for (int x = 0; x < LD::QCNT; ++x) {
      const int e = tid + x * NTH;
      const int rl = q_rows_fast ? e % QR : e / QL;
      const int ll = q_rows_fast ? e / QR : e % QL;
      if constexpr (CPLX) {
        double2 z = qok[x] ? qbuf[x] : make_double2(0.0, 0.0);
        if (qconj) z.y = -z.y;
        Q[(2 * ll) * LDI + rl] = z.x;
        Q[(2 * ll + 1) * LDI + rl] = z.y;
      } else {
        Q[ll * LDI + rl] = qok[x] ? qbuf[x] : 0.0;
      }
    }
  };

  v4d acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};

  fetch(0);
  deposit(0);
  __syncthreads();

  const int krow = lane >> 4;   // contraction row within a 4-step
  const int col = lane & 15;
  for (int64_t st = 0; st < nst; ++st) {
    const int buf = (int)(st & 1);
    if (st + 1 < nst) fetch(st + 1);
    const double *P = ldsP[buf];
    const double *Q = ldsQ[buf];
#pragma unroll
    for (int kk = 0; kk < NBK; kk += 4) {
      double pa[4], qb[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) pa[x] = P[(kk + krow) * LDJ + wj * 64 + x * 16 + col];
#pragma unroll
      for (int y = 0; y < 4; ++y) qb[y] = Q[(kk + krow) * LDI + wi * 64 + y * 16 + col];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[x], qb[y], acc[x][y], 0, 0, 0);
    }
    if (st + 1 < nst) deposit(buf ^ 1);
    __syncthreads();
  }

  // Epilogue: lane l holds rows l/16 + 4r (r = 0..3) of column l%16 of each
  // 16 x 16 block.
#pragma unroll
  for (int y = 0; y < 4; ++y) {
    const int64_t i = i0 + wi * 64 + y * 16 + col;
    if (i >= a.m) continue;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int64_t rb = j0 + wj * 64 + x * 16;  // first j' of the block
      if constexpr (CPLX) {
        double2 *C = reinterpret_cast<double2 *>(a.C);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const int64_t j = rb / 2 + krow + 4 * r;
          if (j >= a.n) continue;
          double2 *cp = C + i + j * a.ldc;
          const double pr = acc[x][y][r], pi = acc[x][y][r + 2];
          double re = sub_rn(mul_rn(a.ar, pr), mul_rn(a.ai, pi));
          double im = add_rn(mul_rn(a.ar, pi), mul_rn(a.ai, pr));
          if (!a.beta_zero) {
            const double2 z = *cp;
            re = add_rn(re, sub_rn(mul_rn(a.br, z.x), mul_rn(a.bi, z.y)));
            im = add_rn(im, add_rn(mul_rn(a.br, z.y), mul_rn(a.bi, z.x)));
          }
          *cp = make_double2(re, im);
        }
      } else {
        double *C = reinterpret_cast<double *>(a.C);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t j = rb + krow + 4 * r;
          if (j >= nprime) continue;
          double *cp = C + i + j * a.ldc;
          double out = mul_rn(a.ar, acc[x][y][r]);
          if (!a.beta_zero) out = add_rn(out, mul_rn(a.br, *cp));
          *cp = out;
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_native(const NativeArgs &a, hipStream_t st) {
  const int64_t nprime = a.cplx ? 2 * a.n : a.n;
  const int64_t tiles = ((nprime + NBJ - 1) / NBJ) * ((a.m + NBI - 1) / NBI);
  if (tiles <= 0) return hipSuccess;
  if (tiles > 0x7fffffffll) return hipErrorInvalidValue;
  if (a.cplx)
    hipLaunchKernelGGL(k_native<true>, dim3((unsigned)tiles), dim3(NTH), 0, st, a);
  else
    hipLaunchKernelGGL(k_native<false>, dim3((unsigned)tiles), dim3(NTH), 0, st, a);
  return hipGetLastError();
}

}  // namespace oz
