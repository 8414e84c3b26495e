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
// using v_mfma_i32_32x32x32_i8 (exact INT8 x INT8 -> INT32). Slice fragments
// move from global memory straight into an NBUF-stage LDS ring with
// global_load_lds_dwordx4 (one 1 KiB fragment per wave instruction, no staging
// registers), issued NBUF-1 contraction blocks ahead of their use. Waits are
// explicit (vmcnt for this wave's own copies, then s_barrier), because the
// generic workgroup barrier would drain every copy in flight. The packed
// fragment layout makes every global and LDS access one contiguous 16-byte
// run per lane and the LDS reads conflict free. The triangle of pairs gives
// natural operand reuse: each fragment feeds (S+1)/2 MFMAs on average.
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

template <int S, int WJ, int WI, int IB, int NBUF>
struct Cfg {
  static constexpr int NW = WJ * WI;
  static constexpr int NT = 64 * NW;
  static constexpr int BJ = 32 * WJ;
  static constexpr int BI = 32 * WI * IB;
  static constexpr int NQB = WI * IB;  // 32-row blocks of A' per tile
  static constexpr int NFP = S * WJ;   // B' fragments per contraction block
  static constexpr int NFQ = S * NQB;  // A' fragments per contraction block
  static constexpr int NF = NFP + NFQ;
  static constexpr int NFW = (NF + NW - 1) / NW;  // copies issued per wave (at most)
  static constexpr int MINW = NF / NW;            // copies issued per wave (at least)
  static constexpr int STAGE = NF * kFragBytes;
  static constexpr int LDS = NBUF * STAGE;
  static_assert(LDS <= 160 * 1024, "LDS ring too large");
  static_assert(MINW < 64, "vmcnt immediate (6 bits)");
};

// Wait until at most N vector-memory operations of this wave are in flight.
// Inline assembly with a memory clobber: the compiler neither moves memory
// accesses across it nor adds a drain of the LDS copies still in flight.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
__device__ __forceinline__ void barrier_only() { asm volatile("s_barrier" ::: "memory"); }

// Contraction blocks of 32 a chunk may hold: S * 32 * kb * 127^2 <= 2^31 - 1.
__host__ __device__ constexpr int64_t chunk_blocks(int S) {
  return (int64_t)(2147483647ll / ((int64_t)S * 32 * 127 * 127));
}

template <int S, int WJ, int WI, int IB, int NBUF, bool RAW, bool CHUNKED, bool GROUPED>
__global__ void __launch_bounds__(64 * WJ * WI) k_ozgemm(GemmArgs G) {
  using C_ = Cfg<S, WJ, WI, IB, NBUF>;
  __shared__ __attribute__((aligned(16))) int8_t lds[C_::LDS];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wj = wave % WJ;
  const int wi = wave / WJ;

  constexpr bool chunked = CHUNKED;
  const int64_t ntiles =
      GROUPED ? G.ntiles
              : ((G.one.nprime + C_::BJ - 1) / C_::BJ) * ((G.one.m + C_::BI - 1) / C_::BI);

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    // The problem this tile belongs to (uniform across the workgroup, so the
    // descriptor is fetched with scalar loads).
    const GemmProblem a = GROUPED ? G.probs[G.tile_prob[tile]] : G.one;
    const int64_t local = GROUPED ? (int64_t)G.tile_local[tile] : tile;
    const int64_t nti = (a.m + C_::BI - 1) / C_::BI;
    const int64_t tj = local / nti;
    const int64_t ti = local % nti;
    const int64_t nkb = a.nkb;

    // Copy of contraction block kb into LDS stage `buf`: fragment f lands at
    // stage offset f KiB (B' fragments first, then A' fragments).
    auto issue = [&](int64_t kb, int buf) {
#pragma unroll
      for (int x = 0; x < C_::NFW; ++x) {
        const int f = wave + x * C_::NW;
        if (f >= C_::NF) break;
        const int8_t *src;
        if (f < C_::NFP) {
          const int p = f / WJ, rb = f % WJ;
          src = a.SP + (((int64_t)p * a.nrbP + tj * WJ + rb) * nkb + kb) * kFragBytes;
        } else {
          const int g = f - C_::NFP;
          const int p = g / C_::NQB, rb = g % C_::NQB;
          src = a.SQ + (((int64_t)p * a.nrbQ + ti * C_::NQB + rb) * nkb + kb) * kFragBytes;
        }
        __builtin_amdgcn_global_load_lds(
            (const void *)(src + lane * 16),
            (__attribute__((address_space(3))) void *)(lds + buf * C_::STAGE + f * kFragBytes), 16,
            0, 0);
      }
    };

    v16i acc[IB][S];
#pragma unroll
    for (int ib = 0; ib < IB; ++ib)
#pragma unroll
      for (int t = 0; t < S; ++t) acc[ib][t] = v16i{0};

    // Exact int64 carry of the INT32 accumulators (chunked contraction only).
    // All carry traffic uses device-scope atomics, so it goes to L2 and never
    // meets a stale line in the non-coherent vector L1.
    int64_t *ws = G.flush_ws + ((int64_t)blockIdx.x * C_::NW + wave) * (int64_t)IB * S * 1024;
    auto carry = [&](bool first) {
#pragma unroll
      for (int ib = 0; ib < IB; ++ib)
#pragma unroll
      for (int t = 0; t < S; ++t) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          int64_t *p = ws + ((ib * S + t) * 16 + r) * 64 + lane;
          if (first)
            __hip_atomic_store(p, (int64_t)acc[ib][t][r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          else
            __hip_atomic_fetch_add(p, (int64_t)acc[ib][t][r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        acc[ib][t] = v16i{0};
      }
    };

    constexpr int D = NBUF - 1;  // prefetch distance in contraction blocks
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (d < nkb) issue(d, d);

    int64_t next_flush = G.kb_chunk;
    bool carried = false;
    int buf = 0;
    for (int64_t kb = 0; kb < nkb; ++kb) {
      // This wave's copies of block kb are complete when at most the copies
      // of the (up to D-1) younger blocks are in flight; the barrier then
      // makes every wave's copies visible and retires the reads of the stage
      // about to be refilled.
      if constexpr (D >= 2) {
        if (kb + 1 < nkb)
          wait_vmcnt<C_::MINW>();
        else
          wait_vmcnt<0>();
      } else {
        wait_vmcnt<0>();
      }
      barrier_only();
      if (kb + D < nkb) {
        int nb = buf + D;
        if (nb >= NBUF) nb -= NBUF;
        issue(kb + D, nb);
      }
      const int8_t *L = lds + buf * C_::STAGE;
      v4i pf[S];
#pragma unroll
      for (int q = 0; q < S; ++q)
        pf[q] = *reinterpret_cast<const v4i *>(L + (q * WJ + wj) * kFragBytes + lane * 16);
#pragma unroll
      for (int p = 0; p < S; ++p) {
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) {
          const v4i qf = *reinterpret_cast<const v4i *>(
              L + (C_::NFP + p * C_::NQB + wi * IB + ib) * kFragBytes + lane * 16);
#pragma unroll
          for (int q = 0; q < S - p; ++q)
            acc[ib][p + q] =
                __builtin_amdgcn_mfma_i32_32x32x32_i8(pf[q], qf, acc[ib][p + q], 0, 0, 0);
        }
      }
      if constexpr (chunked) {
        if (kb + 1 == next_flush && kb + 1 < nkb) {
          carry(!carried);
          carried = true;
          next_flush += G.kb_chunk;
          wait_vmcnt<0>();  // keep the in-order vmcnt accounting to LDS copies only
        }
      }
      buf = buf + 1 == NBUF ? 0 : buf + 1;
    }
    // every wave is done reading the ring before the next tile refills it
    barrier_only();

    if constexpr (chunked) carry(!carried);

    // ------------------------------------------------------------ epilogue
    auto epilogue = [&](int ib) {
      const int64_t i = ti * C_::BI + (wi * IB + ib) * 32 + (lane & 31);
      const int64_t jbase = tj * C_::BJ + wj * 32 + 4 * (lane >> 5);
      const bool row_ok = i < a.m;
      const int codeA = row_ok ? a.codeA[i] : 0;

      auto total = [&](int t, int r) -> int64_t {
        if constexpr (chunked)
          return __hip_atomic_load(ws + ((ib * S + t) * 16 + r) * 64 + lane, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        return (int64_t)acc[ib][t][r];
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
        return;
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
      if (!row_ok) return;
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
    };
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) epilogue(ib);
  }
}

template <int S, int WJ, int WI, int IB, int NBUF>
hipError_t launch_cfg(const GemmArgs &a, int num_cu, hipStream_t st) {
  using C_ = Cfg<S, WJ, WI, IB, NBUF>;
  const bool grouped = a.probs != nullptr;
  const int64_t ntiles =
      grouped ? a.ntiles
              : ((a.one.nprime + C_::BJ - 1) / C_::BJ) * ((a.one.m + C_::BI - 1) / C_::BI);
  // one workgroup per CU is resident (LDS ring); persistent grid
  const int64_t grid = std::min<int64_t>(ntiles, (int64_t)num_cu);
  if (grid <= 0) return hipSuccess;
  const dim3 g((unsigned)grid), b(C_::NT);
  if (grouped) {
    if (a.chunked)
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, IB, NBUF, false, true, true>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, IB, NBUF, false, false, true>), g, b, 0, st, a);
  } else if (a.one.raw != nullptr) {
    if (a.chunked)
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, IB, NBUF, true, true, false>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, IB, NBUF, true, false, false>), g, b, 0, st, a);
  } else {
    if (a.chunked)
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, IB, NBUF, false, true, false>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, IB, NBUF, false, false, false>), g, b, 0, st, a);
  }
  return hipGetLastError();
}

// Tile configurations. All use 32 x 32 x 32 INT8 MFMA blocks and one INT32
// accumulator set per diagonal.
//   0: 8 waves (4 along j', 2 along i), one 32 x 32 block each, two waves per
//      SIMD; workgroup tile 128 j' x 64 i.
//   1: 4 waves along j', two 32 x 32 blocks along i each (the B' fragments of
//      a wave feed both), one wave per SIMD; workgroup tile 128 j' x 64 i.
//   2: 2 x 2 waves with two blocks along i each; workgroup tile 64 j' x 128 i.
// The LDS ring holds three contraction blocks when it fits in 160 KiB, two
// otherwise.
constexpr int kNumCfg = 1;

template <int S, int CFG>
struct Pick;
template <int S>
struct Pick<S, 0> {
  static constexpr int WJ = 4, WI = 2, IB = 1;
};
template <int S>
struct Pick<S, 1> {
  static constexpr int WJ = 4, WI = 1, IB = 2;
};
template <int S>
struct Pick<S, 2> {
  static constexpr int WJ = 2, WI = 2, IB = 2;
};

template <int S, int CFG>
constexpr int nbuf_for() {
  using P = Pick<S, CFG>;
  return S * (P::WJ + P::WI * P::IB) * kFragBytes * 3 <= 160 * 1024 ? 3 : 2;
}

template <int S, int CFG>
hipError_t launch_pick(const GemmArgs &a, int num_cu, hipStream_t st) {
  using P = Pick<S, CFG>;
  return launch_cfg<S, P::WJ, P::WI, P::IB, nbuf_for<S, CFG>()>(a, num_cu, st);
}

template <int S>
hipError_t launch_s(int cfg, const GemmArgs &a, int num_cu, hipStream_t st) {
  (void)cfg;
  return launch_pick<S, 0>(a, num_cu, st);
}

template <int S>
size_t flush_bytes_s(int cfg, int num_cu) {
  (void)cfg;
  const int per = Pick<S, 0>::WJ * Pick<S, 0>::WI * Pick<S, 0>::IB;
  return (size_t)num_cu * per * (size_t)S * 1024 * sizeof(int64_t);
}

}  // namespace

int64_t kb_chunk_for(int S) { return chunk_blocks(S); }

int gemm_num_configs() { return kNumCfg; }

size_t gemm_flush_bytes(int S, int cfg, int num_cu) {
  // the largest per-workgroup carry space over the configurations, so that a
  // plan is valid whichever configuration runs
  (void)cfg;
  size_t mx = 0;
  for (int c = 0; c < kNumCfg; ++c) {
    size_t b = 0;
    switch (S) {
#define OZ_CASE(N) \
  case N: b = flush_bytes_s<N>(c, num_cu); break;
      OZ_CASE(1) OZ_CASE(2) OZ_CASE(3) OZ_CASE(4) OZ_CASE(5) OZ_CASE(6)
      OZ_CASE(7) OZ_CASE(8) OZ_CASE(9) OZ_CASE(10) OZ_CASE(11) OZ_CASE(12)
#undef OZ_CASE
      default: break;
    }
    mx = std::max(mx, b);
  }
  return mx;
}

int64_t gemm_tiles(int S, int cfg, int64_t m, int64_t nprime) {
  (void)S;
  (void)cfg;
  using P = Pick<1, 0>;
  const int64_t BJ = 32 * P::WJ, BI = 32 * P::WI * P::IB;
  return ((nprime + BJ - 1) / BJ) * ((m + BI - 1) / BI);
}

hipError_t launch_ozgemm_grouped(int S, int cfg, const GemmArgs &a, int num_cu, hipStream_t st) {
  return launch_ozgemm(S, cfg, a, num_cu, st);
}

hipError_t launch_ozgemm(int S, int cfg, const GemmArgs &a, int num_cu, hipStream_t st) {
  switch (S) {
#define OZ_CASE(N) \
  case N: return launch_s<N>(cfg, a, num_cu, st);
    OZ_CASE(1) OZ_CASE(2) OZ_CASE(3) OZ_CASE(4) OZ_CASE(5) OZ_CASE(6)
    OZ_CASE(7) OZ_CASE(8) OZ_CASE(9) OZ_CASE(10) OZ_CASE(11) OZ_CASE(12)
#undef OZ_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace oz
