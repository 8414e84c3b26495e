// Fused slice-pair INT8 GEMM and FP64 recombination of libozaki (gfx950).
//
// Steps "low-precision matrix multiplications on the slices" and "accumulate
// in higher precision" of the Ozaki-I scheme (Section 2.2 of the paper).
//
// Output orientation: the MFMA row index is the output column side j' and the
// MFMA column index (lane % 32) is the output row i, so the 32 lanes of a
// half-wave hold 32 consecutive rows of one column of C and every store of the
// epilogue is a contiguous run in column-major C. For complex data j' = 2j + c
// (c = 0 real, 1 imaginary part of column j), so a lane holds Re and Im of one
// C entry in neighbouring accumulator registers and writes 16 bytes.
//
// Work per workgroup tile (BJ = 32*WJ columns j', BI = 32*WI rows i), per wave
// one 32 x 32 block with one INT32 accumulator set per diagonal t = 2..S+1:
//   for each 32-wide contraction block:
//     for p = 1..S, q = 1..S+1-p:  acc[p+q-2] += SB'_q(32x32) * SA'_p(32x32)^T
// using v_mfma_i32_32x32x32_i8 (exact INT8 x INT8 -> INT32). Slices are
// staged through LDS (double buffered, one barrier per contraction block);
// every global and LDS access is one contiguous 16-byte run per lane thanks to
// the packed fragment layout. The triangle of pairs gives natural operand
// reuse: each fragment feeds (S+1)/2 MFMAs on average.
//
// INT32 range: a diagonal of S pairs over 32*kb contraction entries is bounded
// by S * 32 * kb * 127^2; the contraction is cut into chunks that keep it
// below 2^31 and each chunk is carried exactly into int64 workgroup-private
// memory. The FP64 epilogue converts every S_t exactly (|S_t| < 2^53) and adds
// them largest weight first, one rounding per addition, then scales by
// 2^(e_i + f_j) and applies alpha/beta without fused multiply-adds.
#include "ozaki_internal.hpp"

namespace oz {

namespace {

template <int S, int WJ, int WI>
struct Cfg {
  static constexpr int NW = WJ * WI;
  static constexpr int NT = 64 * NW;
  static constexpr int BJ = 32 * WJ;
  static constexpr int BI = 32 * WI;
  static constexpr int NFP = S * WJ;  // B' fragments per contraction block
  static constexpr int NFQ = S * WI;  // A' fragments per contraction block
  static constexpr int NF = NFP + NFQ;
  static constexpr int NFW = (NF + NW - 1) / NW;  // fragments loaded per wave
  static constexpr int STAGE = NF * kFragBytes;
  static constexpr int LDS = 2 * STAGE;
};

// Contraction blocks of 32 a chunk may hold: S * 32 * kb * 127^2 <= 2^31 - 1.
__host__ __device__ constexpr int64_t chunk_blocks(int S) {
  return (int64_t)(2147483647ll / ((int64_t)S * 32 * 127 * 127));
}

template <int S, int WJ, int WI, bool RAW, bool CHUNKED>
__global__ void __launch_bounds__(64 * WJ * WI) k_ozgemm(GemmArgs a) {
  using C_ = Cfg<S, WJ, WI>;
  __shared__ __attribute__((aligned(16))) int8_t lds[C_::LDS];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wj = wave % WJ;
  const int wi = wave / WJ;

  const int64_t ntj = (a.nprime + C_::BJ - 1) / C_::BJ;
  const int64_t nti = (a.m + C_::BI - 1) / C_::BI;
  const int64_t ntiles = ntj * nti;
  const int64_t nkb = a.nkb;
  constexpr bool chunked = CHUNKED;

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t tj = tile / nti;
    const int64_t ti = tile % nti;

    // Global source of fragment f of contraction block kb (per lane).
    auto frag_src = [&](int f, int64_t kb) -> const int8_t * {
      if (f < C_::NFP) {
        const int p = f / WJ, rb = f % WJ;
        return a.SP + (((int64_t)p * a.nrbP + tj * WJ + rb) * nkb + kb) * kFragBytes + lane * 16;
      }
      const int g = f - C_::NFP;
      const int p = g / WI, rb = g % WI;
      return a.SQ + (((int64_t)p * a.nrbQ + ti * WI + rb) * nkb + kb) * kFragBytes + lane * 16;
    };

    v4i stage[C_::NFW];
    auto load_stage = [&](int64_t kb) {
#pragma unroll
      for (int x = 0; x < C_::NFW; ++x) {
        const int f = wave + x * C_::NW;
        if (f < C_::NF) stage[x] = *reinterpret_cast<const v4i *>(frag_src(f, kb));
      }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
      for (int x = 0; x < C_::NFW; ++x) {
        const int f = wave + x * C_::NW;
        if (f < C_::NF)
          *reinterpret_cast<v4i *>(lds + buf * C_::STAGE + f * kFragBytes + lane * 16) = stage[x];
      }
    };

    v16i acc[S];
#pragma unroll
    for (int t = 0; t < S; ++t) acc[t] = v16i{0};

    // Exact int64 carry of the INT32 accumulators (chunked contraction only).
    // All carry traffic uses device-scope atomics, so it goes to L2 and never
    // meets a stale line in the non-coherent vector L1.
    int64_t *ws = a.flush_ws + ((int64_t)blockIdx.x * C_::NW + wave) * (int64_t)S * 1024;
    auto carry = [&](bool first) {
#pragma unroll
      for (int t = 0; t < S; ++t) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          int64_t *p = ws + (t * 16 + r) * 64 + lane;
          if (first)
            __hip_atomic_store(p, (int64_t)acc[t][r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          else
            __hip_atomic_fetch_add(p, (int64_t)acc[t][r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        acc[t] = v16i{0};
      }
    };

    load_stage(0);
    store_stage(0);
    __syncthreads();

    int64_t next_flush = a.kb_chunk;

    for (int64_t kb = 0; kb < nkb; ++kb) {
      const int buf = (int)(kb & 1);
      if (kb + 1 < nkb) load_stage(kb + 1);

      const int8_t *L = lds + buf * C_::STAGE;
      v4i pf[S];
#pragma unroll
      for (int q = 0; q < S; ++q)
        pf[q] = *reinterpret_cast<const v4i *>(L + (q * WJ + wj) * kFragBytes + lane * 16);
#pragma unroll
      for (int p = 0; p < S; ++p) {
        const v4i qf =
            *reinterpret_cast<const v4i *>(L + (C_::NFP + p * WI + wi) * kFragBytes + lane * 16);
#pragma unroll
        for (int q = 0; q < S - p; ++q)
          acc[p + q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(pf[q], qf, acc[p + q], 0, 0, 0);
      }

      if (kb + 1 < nkb) store_stage(buf ^ 1);

      if constexpr (chunked) {
      if (kb + 1 == next_flush && kb + 1 < nkb) {
        carry(next_flush == a.kb_chunk);
        next_flush += a.kb_chunk;
      }
      }
      __syncthreads();
    }

    if constexpr (chunked) carry(false);

    // ------------------------------------------------------------ epilogue
    const int64_t i = ti * C_::BI + wi * 32 + (lane & 31);
    const int64_t jbase = tj * C_::BJ + wj * 32 + 4 * (lane >> 5);
    const bool row_ok = i < a.m;
    const int codeA = row_ok ? a.codeA[i] : 0;

    auto total = [&](int t, int r) -> int64_t {
      if constexpr (chunked)
        return __hip_atomic_load(ws + (t * 16 + r) * 64 + lane, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      return (int64_t)acc[t][r];
    };

    if constexpr (RAW) {
      // Debug output of the exact diagonals.
      if (row_ok) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t jp = jbase + 8 * (r >> 2) + (r & 3);
          if (jp >= a.nprime) continue;
#pragma unroll
          for (int t = 0; t < S; ++t) {
            const int64_t v = total(t, r);
            if (a.cplx) {
              const int64_t n = a.nprime >> 1;
              a.raw[(((int64_t)t * n + (jp >> 1)) * a.m + i) * 2 + (jp & 1)] = v;
            } else {
              a.raw[((int64_t)t * a.nprime + jp) * a.m + i] = v;
            }
          }
        }
      }
      continue;
    }

    double val[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      double acc64 = 0.0;
#pragma unroll
      for (int t = 0; t < S; ++t)
        acc64 = add_rn(acc64, ldexp((double)total(t, r), -kDigitBits * (t + 2)));
      val[r] = acc64;
    }
    if (!row_ok) continue;
    const int ea = code_exp(codeA);
    const bool bad_i = code_bad(codeA);

    if (a.cplx) {
      double2 *C = reinterpret_cast<double2 *>(a.C);
      const int64_t n = a.nprime >> 1;
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const int64_t jp = jbase + 8 * (r >> 2) + (r & 3);
        const int64_t j = jp >> 1;
        if (j >= n) continue;
        const int cb = a.codeB[j];
        double2 *cp = C + i + j * a.ldc;
        if (bad_i || code_bad(cb)) {
          *cp = make_double2(qnan(), qnan());
          continue;
        }
        const int sc = ea + code_exp(cb);
        const double pr = ldexp(val[r], sc);
        const double pi = ldexp(val[r + 1], sc);
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
      for (int r = 0; r < 16; ++r) {
        const int64_t j = jbase + 8 * (r >> 2) + (r & 3);
        if (j >= a.nprime) continue;
        const int cb = a.codeB[j];
        double *cp = C + i + j * a.ldc;
        if (bad_i || code_bad(cb)) {
          *cp = qnan();
          continue;
        }
        const double p = ldexp(val[r], ea + code_exp(cb));
        double out = mul_rn(a.ar, p);
        if (!a.beta_zero) out = add_rn(out, mul_rn(a.br, *cp));
        *cp = out;
      }
    }
  }
}

template <int S, int WJ, int WI>
hipError_t launch_cfg(const GemmArgs &a, int num_cu, hipStream_t st) {
  using C_ = Cfg<S, WJ, WI>;
  const int64_t ntiles = ((a.nprime + C_::BJ - 1) / C_::BJ) * ((a.m + C_::BI - 1) / C_::BI);
  // one workgroup per CU is resident (LDS and registers); persistent grid
  const int64_t grid = std::min<int64_t>(ntiles, (int64_t)num_cu);
  if (grid <= 0) return hipSuccess;
  const dim3 g((unsigned)grid), b(C_::NT);
  const bool chunked = a.nkb > a.kb_chunk;
  if (a.raw != nullptr) {
    if (chunked)
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, true, true>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, true, false>), g, b, 0, st, a);
  } else {
    if (chunked)
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, false, true>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, false, false>), g, b, 0, st, a);
  }
  return hipGetLastError();
}

// Tile shape per slice count: 8 waves of 32x32 (128 j' x 64 i) while the
// per-diagonal accumulators fit next to the operand registers (256 per lane
// at two waves per SIMD); 4 waves with a 512-register budget beyond that.
template <int S>
hipError_t launch_s(const GemmArgs &a, int num_cu, hipStream_t st) {
  if constexpr (S <= 9)
    return launch_cfg<S, 4, 2>(a, num_cu, st);
  else
    return launch_cfg<S, 2, 2>(a, num_cu, st);
}

constexpr int wave_count(int S) { return S <= 9 ? 8 : 4; }

}  // namespace

int64_t kb_chunk_for(int S) { return chunk_blocks(S); }

size_t gemm_flush_bytes(int S, int64_t m, int64_t nprime, int num_cu) {
  (void)m;
  (void)nprime;
  return (size_t)num_cu * wave_count(S) * (size_t)S * 1024 * sizeof(int64_t);
}

hipError_t launch_ozgemm(int S, const GemmArgs &a, int num_cu, hipStream_t st) {
  switch (S) {
    case 1: return launch_s<1>(a, num_cu, st);
    case 2: return launch_s<2>(a, num_cu, st);
    case 3: return launch_s<3>(a, num_cu, st);
    case 4: return launch_s<4>(a, num_cu, st);
    case 5: return launch_s<5>(a, num_cu, st);
    case 6: return launch_s<6>(a, num_cu, st);
    case 7: return launch_s<7>(a, num_cu, st);
    case 8: return launch_s<8>(a, num_cu, st);
    case 9: return launch_s<9>(a, num_cu, st);
    case 10: return launch_s<10>(a, num_cu, st);
    case 11: return launch_s<11>(a, num_cu, st);
    case 12: return launch_s<12>(a, num_cu, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace oz
