// Fused Ozaki-II product of libozaki (gfx950): the N modular INT8 products of
// an output tile and the Chinese-remainder rebuild in one kernel.
//
// Section 2.2 of the paper: the integer operands are multiplied modulo
// several pairwise-coprime moduli on the integer matrix cores, and the Chinese
// remainder theorem gives back the exact integer product. Here every modular
// product of a tile is reduced, as soon as its contraction is complete, to its
// Garner mixed-radix digit (one byte per output entry and modulus, kept in
// registers), so the INT32 products never leave the chip; after the last
// modulus the digits are combined into the exact integer, rounded once to
// FP64, scaled by 2^(e_i + f_j - 2 beta) and alpha/beta is applied with the
// rounding order of the Ozaki-I epilogue.
//
// Work per workgroup tile (BJ = 128 output "rows" j' of B', BI = 32 * 2 * IB
// rows i of A'): 8 waves, 4 along j' x 2 along i, each wave one 32-row block
// of B' and IB 32-row blocks of A'. The contraction of modulus k runs over the
// nkb 32-entry blocks of its residue planes in steps of KS blocks; the walk
// over (k, step) is one flat sequence, so the LDS ring keeps prefetching
// across modulus boundaries. Each block: one v_mfma_i32_32x32x32_i8 per A'
// block. Residue fragments move from global memory straight into an
// NBUF-stage LDS ring (direct-to-LDS copies, one 1 KiB fragment per wave
// instruction) in the packed layout of the slices, so every access is one
// contiguous 16-byte run per lane. A plain product gives each fragment only
// IB MFMAs, so a stage holds KS blocks and the ring runs (NBUF - 1) KS blocks
// ahead to cover the memory latency.
//
// INT32 range: odd moduli have residues |r| <= 127 and K' <= 2^17 keeps every
// sum exact; for m = 256 the accumulator wraps modulo 2^32, which keeps the
// value modulo 256 (all the digit of that modulus reads).
#include <type_traits>

#include "ozaki2_crt.hpp"
#include "ozaki_gemm_tile.hpp"

namespace oz {

namespace {

constexpr int kWJ = 4;  // waves along j'
constexpr int kWI = 2;  // waves along i
constexpr int kNW = kWJ * kWI;
constexpr int kStep = 4;  // contraction blocks per ring stage (nkb is a multiple of 4)
constexpr int kRing = 4;  // ring stages: (4 + 2 IB) x 4 KiB each

// Wait until at most y steps of KS copies each are in flight (y <= Y).
template <int Y, int KS>
__device__ __forceinline__ void wait_steps(int y) {
  if constexpr (Y == 0) {
    tile::wait_vmcnt<0>();
  } else {
    if (y == Y)
      tile::wait_vmcnt<Y * KS>();
    else
      wait_steps<Y - 1, KS>(y);
  }
}

// Garner digit of modulus k for every accumulator entry of the wave's blocks.
template <int N, int IB, int NWD, int K>
__device__ __forceinline__ void digits_at(int k, const v16i (&acc)[IB], int (&W)[IB][16][NWD]) {
  if constexpr (K < N) {
    if (k == K) {
#pragma unroll
      for (int ib = 0; ib < IB; ++ib)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          crt::digit_step<K, NWD>(acc[ib][r], W[ib][r]);
          // one entry at a time: interleaving all 16 IB of them needs more
          // registers than the digits leave
          __builtin_amdgcn_sched_barrier(0);
        }
      return;
    }
    digits_at<N, IB, NWD, K + 1>(k, acc, W);
  }
}

template <int N, int IB, int NBUF, int KS>
__global__ void __launch_bounds__(64 * kNW, 1) k_oz2gemm(Oz2Args G) {
  constexpr int NQB = kWI * IB;    // A' row blocks per tile
  constexpr int NF = kWJ + NQB;    // fragments per (modulus, contraction block)
  constexpr int BJ = 32 * kWJ;
  constexpr int BI = 32 * NQB;
  constexpr int STAGE = NF * KS * kFragBytes;  // fragment f, block x at (f KS + x) KiB
  constexpr int NWD = (N + 3) / 4;  // digit words per output entry
  constexpr int D = NBUF - 1;       // prefetch distance in steps
  static_assert(NF <= kNW, "one fragment row per wave");
  static_assert(D >= 1 && (D - 1) * KS < 64, "vmcnt immediate (6 bits)");
  static_assert(NBUF * STAGE <= 160 * 1024, "LDS ring");
  __shared__ __attribute__((aligned(16))) int8_t lds[NBUF * STAGE];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform
  const int wj = wave % kWJ;
  const int wi = wave / kWJ;
  const int64_t nkb = G.nkb;           // a multiple of KS
  const int64_t nst = nkb / KS;        // steps per modulus
  const int64_t T = (int64_t)N * nst;  // steps per tile
  const int64_t planeA = G.nrbQ * nkb * kFragBytes;
  const int64_t planeB = G.nrbP * nkb * kFragBytes;
  const int64_t ntiles = ((G.nprime + BJ - 1) / BJ) * ((G.m + BI - 1) / BI);

  for (int64_t tn = blockIdx.x; tn < ntiles; tn += gridDim.x) {
    int64_t tj, ti;
    tile::tile_coords(tn, 1, G.m, G.nprime, BJ, BI, tj, ti);
    // this wave's fragment of every step: B' row block (wave < 4) or A' row
    // block; step (k, kb) is at plane k, contraction block kb
    const int8_t *src = nullptr;
    int64_t plane = 0;
    if (wave < kWJ) {
      src = G.RB + (tj * kWJ + wave) * nkb * kFragBytes;
      plane = planeB;
    } else if (wave < NF) {
      src = G.RA + (ti * NQB + (wave - kWJ)) * nkb * kFragBytes;
      plane = planeA;
    }
    src += lane * 16;
    // issue pointer: the next step to copy, as (modulus, first block)
    int64_t ik = 0, ikb = 0;
    auto issue = [&](int buf) {
      if (wave < NF) {
#pragma unroll
        for (int x = 0; x < KS; ++x)
          tile::copy_frag(src + ik * plane + (ikb + x) * kFragBytes,
                          lds + buf * STAGE + (wave * KS + x) * kFragBytes);
      }
      ikb += KS;
      if (ikb == nkb) {
        ikb = 0;
        ++ik;
      }
    };

    v16i acc[IB];
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) acc[ib] = v16i{0};
    int W[IB][16][NWD];
#pragma unroll
    for (int ib = 0; ib < IB; ++ib)
#pragma unroll
      for (int r = 0; r < 16; ++r)
#pragma unroll
        for (int w = 0; w < NWD; ++w) W[ib][r][w] = 0;

#pragma unroll
    for (int d = 0; d < D; ++d)
      if (d < T) issue(d);

    int buf = 0;
    int k = 0;
    int64_t st = 0;
    for (int64_t it = 0; it < T; ++it) {
      // This wave's copies of step `it` have landed once at most the copies
      // of the younger steps already issued are in flight (KS per step); the
      // barrier then makes every wave's copies visible and retires the reads
      // of the stage about to be refilled.
      const int64_t younger = T - 1 - it;
      wait_steps<D - 1, KS>(younger < D - 1 ? (int)younger : D - 1);
      tile::barrier_only();
      if (it + D < T) {
        int nb = buf + D;
        if (nb >= NBUF) nb -= NBUF;
        issue(nb);
      }
      const int8_t *L = lds + buf * STAGE + lane * 16;
#pragma unroll
      for (int x = 0; x < KS; ++x) {
        const v4i pf = *reinterpret_cast<const v4i *>(L + (wj * KS + x) * kFragBytes);
        v4i qf[IB];
#pragma unroll
        for (int ib = 0; ib < IB; ++ib)
          qf[ib] = *reinterpret_cast<const v4i *>(L + ((kWJ + wi * IB + ib) * KS + x) * kFragBytes);
#pragma unroll
        for (int ib = 0; ib < IB; ++ib)
          acc[ib] = __builtin_amdgcn_mfma_i32_32x32x32_i8(pf, qf[ib], acc[ib], 0, 0, 0);
      }
      if (++st == nst) {
        digits_at<N, IB, NWD, 0>(k, acc, W);
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) acc[ib] = v16i{0};
        st = 0;
        ++k;
      }
      buf = buf + 1 == NBUF ? 0 : buf + 1;
    }
    // every wave is done reading the ring before the next tile refills it
    tile::barrier_only();

    // ------------------------------------------------------------ epilogue
    // Lane register r of block ib holds output row i and column side
    // j' = jbase + 8 (r / 4) + r % 4 (complex: r, r + 1 are Re, Im of column
    // j = j' / 2).
    const int64_t jbase = tj * BJ + wj * 32 + 4 * (lane >> 5);
    // one call per A' block with a compile-time block index: as a loop the
    // compiler kept it rolled and the digit array went to scratch memory
    auto epilogue = [&](auto ibc) {
      constexpr int ib = decltype(ibc)::value;
      const int64_t i = ti * BI + (wi * IB + ib) * 32 + (lane & 31);
      if (i >= G.m) return;
      const int ca = G.codeA[i];
      const bool bad_i = code_bad(ca);
      const int ea = code_exp(ca) - 2 * G.beta;
      if (G.cplx) {
        double2 *C = reinterpret_cast<double2 *>(G.C);
        const int64_t n = G.nprime >> 1;
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
          const int64_t jp = jbase + 8 * (r >> 2) + (r & 3);
          const int64_t j = jp >> 1;
          if (j >= n) continue;
          const int cb = G.codeB[j];
          double2 *cp = C + i + j * G.ldc;
          if (bad_i || code_bad(cb)) {
            *cp = make_double2(qnan(), qnan());
            continue;
          }
          const int sc = ea + code_exp(cb);
          const double pr = ldexp(crt::to_double_rn(crt::combine<N, NWD>(W[ib][r])), sc);
          const double pi = ldexp(crt::to_double_rn(crt::combine<N, NWD>(W[ib][r + 1])), sc);
          double re = sub_rn(mul_rn(G.ar, pr), mul_rn(G.ai, pi));
          double im = add_rn(mul_rn(G.ar, pi), mul_rn(G.ai, pr));
          if (!G.beta_zero) {
            const double2 z = *cp;
            re = add_rn(re, sub_rn(mul_rn(G.br, z.x), mul_rn(G.bi, z.y)));
            im = add_rn(im, add_rn(mul_rn(G.br, z.y), mul_rn(G.bi, z.x)));
          }
          *cp = make_double2(re, im);
          __builtin_amdgcn_sched_barrier(0);  // one entry at a time, as in digits_at
        }
      } else {
        double *C = reinterpret_cast<double *>(G.C);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t j = jbase + 8 * (r >> 2) + (r & 3);
          if (j >= G.nprime) continue;
          const int cb = G.codeB[j];
          double *cp = C + i + j * G.ldc;
          if (bad_i || code_bad(cb)) {
            *cp = qnan();
            continue;
          }
          const double p =
              ldexp(crt::to_double_rn(crt::combine<N, NWD>(W[ib][r])), ea + code_exp(cb));
          double out = mul_rn(G.ar, p);
          if (!G.beta_zero) out = add_rn(out, mul_rn(G.br, *cp));
          *cp = out;
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    };
    epilogue(std::integral_constant<int, 0>{});
    if constexpr (IB > 1) epilogue(std::integral_constant<int, 1>{});
  }
}

template <int N, int IB, int NBUF, int KS>
hipError_t launch_v(const Oz2Args &a, int num_cu, hipStream_t st) {
  constexpr int BJ = 32 * kWJ, BI = 32 * kWI * IB;
  const int64_t ntiles = ((a.nprime + BJ - 1) / BJ) * ((a.m + BI - 1) / BI);
  const int64_t grid = std::min<int64_t>(ntiles, num_cu);
  if (grid <= 0) return hipSuccess;
  if (a.nkb % KS != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_oz2gemm<N, IB, NBUF, KS>), dim3((unsigned)grid), dim3(64 * kNW), 0, st, a);
  return hipGetLastError();
}

template <int N>
hipError_t launch_n(const Oz2Args &a, int num_cu, hipStream_t st) {
  // two A' blocks per wave while the digits of 2 x 16 entries fit the
  // registers (N <= 16: 4 words per entry), else one. Measured at 2048^3
  // complex (GEMM per launch): 13 moduli 0.687 ms with two blocks, 0.824 with
  // one; 15 moduli 0.762 against 0.958; at 14 moduli the compiler spills 79
  // registers in the main loop with two blocks (1.010 ms) and one block is
  // faster (0.900 ms). A five-stage ring (160 KiB) and an eight-stage ring of
  // two-block stages were no faster at 13 moduli.
  constexpr int IB = (N <= 16 && N != 14) ? 2 : 1;
  return launch_v<N, IB, kRing, kStep>(a, num_cu, st);
}

}  // namespace

hipError_t launch_oz2gemm(int n, const Oz2Args &a, int num_cu, hipStream_t st) {
  if (a.m <= 0 || a.nprime <= 0) return hipSuccess;
  if (a.nkb <= 0 || a.nkb % kStep != 0 || a.nrbQ * 32 < round_up(a.m, kRowPad) ||
      a.nrbP * 32 < round_up(a.nprime, kRowPad))
    return hipErrorInvalidValue;
  switch (n) {
#define OZ_N(N) \
  case N: return launch_n<N>(a, num_cu, st);
    OZ_N(2) OZ_N(3) OZ_N(4) OZ_N(5) OZ_N(6) OZ_N(7) OZ_N(8) OZ_N(9) OZ_N(10) OZ_N(11)
    OZ_N(12) OZ_N(13) OZ_N(14) OZ_N(15) OZ_N(16) OZ_N(17) OZ_N(18) OZ_N(19) OZ_N(20)
#undef OZ_N
    default: return hipErrorInvalidValue;
  }
}

}  // namespace oz
