// Fused slice-pair INT8 GEMM and FP64 recombination, one wave per SIMD
// (gfx950): the large-register form of the kernel in ozaki_gemm.hip.
//
// Same arithmetic, packed operands, LDS ring of global_load_lds copies and
// epilogue (Section 2.2 of the paper: low-precision products of the slices,
// accumulated exactly and recombined in FP64). What differs is the wave shape:
//   - 4 waves per workgroup, one per SIMD, so a wave may hold up to 512
//     registers (architectural VGPRs plus accumulation registers);
//   - each wave owns two 32 x 32 output blocks along j' (64 j' x 32 i), so one
//     A' fragment read from LDS feeds twice as many MFMAs and the LDS read
//     traffic per MFMA drops by a quarter (3S instead of 4S fragment reads per
//     2 S(S+1)/2 MFMAs);
//   - the fragments of contraction block kb+1 are read from LDS into a second
//     register set while the MFMAs of block kb run, so the matrix pipe does
//     not wait for LDS after each barrier. With fragments in registers, the
//     LDS stage of block kb is free as soon as its reads have returned, so the
//     copies run NBUF blocks ahead (the full ring) instead of NBUF - 1.
// Workgroup tile: 128 j' x 64 i (2 waves along j', 2 along i), as the default
// configuration of the 8-wave kernel, so plans and tile counts are shared.
// Registers: 2 S 16 accumulators + 2 x 3S x 4 fragment registers, which fits
// 512 for S <= 8. Contractions long enough to need the int64 carry (more than
// chunk_blocks(S) blocks of 32) run on the 8-wave kernel instead.
#include "ozaki_gemm_tile.hpp"

namespace oz {

namespace {

using tile::barrier_only;
using tile::wait_lgkm0;
using tile::wait_vmcnt;

constexpr int kW1MaxS = 8;

template <int S, int NBUF>
struct CfgW1 {
  static constexpr int WJ = 2, WI = 2, JB = 2;  // waves along j', i; blocks per wave along j'
  static constexpr int NW = WJ * WI;
  static constexpr int NT = 64 * NW;
  static constexpr int NJB = WJ * JB;          // 32-row blocks of B' per tile
  static constexpr int BJ = 32 * NJB;
  static constexpr int BI = 32 * WI;
  static constexpr int NFP = S * NJB;          // B' fragments per contraction block
  static constexpr int NFQ = S * WI;           // A' fragments per contraction block
  static constexpr int NF = NFP + NFQ;
  static constexpr int NFW = (NF + NW - 1) / NW;
  static constexpr int MINW = NF / NW;
  static constexpr int STAGE = NF * kFragBytes;
  static constexpr int LDS = NBUF * STAGE;
  static_assert(LDS <= 160 * 1024, "LDS ring too large");
  static_assert(MINW * (NBUF - 1) < 64, "vmcnt immediate (6 bits)");
};

// Wait until the copies of all but the `younger` most recently issued
// contraction blocks of this wave have landed (MINW copies per block is the
// least any wave issues, so the wait is never short).
template <int MINW, int NBUF>
__device__ __forceinline__ void wait_blocks(int younger) {
  static_assert(NBUF <= 4, "ring depth");
  if (NBUF >= 4 && younger >= 3) {
    wait_vmcnt<MINW * 3 < 64 ? MINW * 3 : 0>();
  } else if (NBUF >= 3 && younger >= 2) {
    wait_vmcnt<MINW * 2 < 64 ? MINW * 2 : 0>();
  } else if (younger >= 1) {
    wait_vmcnt<MINW>();
  } else {
    wait_vmcnt<0>();
  }
}

template <int S>
struct Frags {
  v4i b[2][S];  // B' fragments of the wave's two j' blocks, slice q
  v4i a[S];     // A' fragments of the wave's i block, slice p
};

template <int S, int NBUF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_ozgemm_w1(GemmArgs G) {
  using C_ = CfgW1<S, NBUF>;
  __shared__ __attribute__((aligned(16))) int8_t lds[C_::LDS];
  // Naming an accumulation register keeps the compiler from concluding that
  // the kernel needs none; the MFMAs are then selected with their
  // accumulators in AGPRs, which doubles the registers a wave can use.
  asm volatile("" ::: "a0");

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int wj = wave % C_::WJ;
  const int wi = wave / C_::WJ;

  const GemmProblem &a = G.one;
  const int64_t nkb = a.nkb;
  const int64_t ntiles = ((a.nprime + C_::BJ - 1) / C_::BJ) * ((a.m + C_::BI - 1) / C_::BI);

  for (int64_t tn = blockIdx.x; tn < ntiles; tn += gridDim.x) {
    int64_t tj, ti;
    tile::tile_coords(tn, G.order, a.m, a.nprime, C_::BJ, C_::BI, tj, ti);

    // Copy of contraction block kb into LDS stage `buf` (B' fragments first).
    auto issue = [&](int64_t kb, int buf) {
#pragma unroll
      for (int x = 0; x < C_::NFW; ++x) {
        const int f = wave + x * C_::NW;
        if (f >= C_::NF) break;
        const int8_t *src;
        if (f < C_::NFP) {
          const int p = f / C_::NJB, rb = f % C_::NJB;
          src = a.SP + (((int64_t)p * a.nrbP + tj * C_::NJB + rb) * nkb + kb) * kFragBytes;
        } else {
          const int g = f - C_::NFP;
          const int p = g / C_::WI, rb = g % C_::WI;
          src = a.SQ + (((int64_t)p * a.nrbQ + ti * C_::WI + rb) * nkb + kb) * kFragBytes;
        }
        tile::copy_frag(src + lane * 16, lds + buf * C_::STAGE + f * kFragBytes);
      }
    };
    auto read = [&](int buf, Frags<S> &F) {
      const int8_t *L = lds + buf * C_::STAGE + lane * 16;
#pragma unroll
      for (int p = 0; p < S; ++p) {
        F.a[p] = *reinterpret_cast<const v4i *>(L + (C_::NFP + p * C_::WI + wi) * kFragBytes);
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
          F.b[jb][p] =
              *reinterpret_cast<const v4i *>(L + (p * C_::NJB + wj * 2 + jb) * kFragBytes);
      }
    };

    v16i acc[2][S];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int t = 0; t < S; ++t) acc[jb][t] = v16i{0};

    auto compute = [&](const Frags<S> &F) {
#pragma unroll
      for (int p = 0; p < S; ++p)
#pragma unroll
        for (int q = 0; q < S - p; ++q)
#pragma unroll
          for (int jb = 0; jb < 2; ++jb)
            acc[jb][p + q] =
                __builtin_amdgcn_mfma_i32_32x32x32_i8(F.b[jb][q], F.a[p], acc[jb][p + q], 0, 0, 0);
    };

    // One contraction block: Fc holds block kb (its LDS reads may still be
    // in flight), Fn receives block kb + 1.
    auto step = [&](int64_t kb, const Frags<S> &Fc, Frags<S> &Fn) {
      if (kb + 1 < nkb) {
        // Blocks issued so far: up to min(kb + NBUF - 1, nkb - 1); this
        // wave's copies of kb + 1 must have landed, the younger ones may fly.
        const int64_t youngest = kb + NBUF - 1 < nkb - 1 ? kb + NBUF - 1 : nkb - 1;
        wait_blocks<C_::MINW, NBUF>((int)(youngest - (kb + 1)));
        wait_lgkm0();     // Fc is in registers: the stage of block kb is free
        barrier_only();   // every wave's copies of kb + 1 visible, reads of kb done
        if (kb + NBUF < nkb) issue(kb + NBUF, (int)(kb % NBUF));
        read((int)((kb + 1) % NBUF), Fn);
      }
      compute(Fc);
    };

    Frags<S> F0, F1;
    const int pro = nkb < NBUF ? (int)nkb : NBUF;
#pragma unroll
    for (int d = 0; d < NBUF; ++d)
      if (d < pro) issue(d, d);
    wait_blocks<C_::MINW, NBUF>(pro - 1);
    barrier_only();
    read(0, F0);
    for (int64_t kb = 0; kb < nkb; ++kb) {
      step(kb, F0, F1);
      F0 = F1;  // register renaming; the copy overlaps the MFMAs in flight
    }
    // every wave's reads of the ring are done before the next tile refills it
    wait_lgkm0();
    barrier_only();

    const int64_t i = ti * C_::BI + wi * 32 + (lane & 31);
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
      tile::store_block<S, false, false>(a, acc[jb], nullptr, lane, i,
                                           tj * C_::BJ + (wj * 2 + jb) * 32 + 4 * (lane >> 5));
  }
}

template <int S>
constexpr int w1_nbuf() {
  return CfgW1<S, 3>::STAGE * 3 <= 160 * 1024 ? 3 : 2;
}

template <int S>
hipError_t launch_w1_s(const GemmArgs &a, int num_cu, hipStream_t st) {
  constexpr int NBUF = w1_nbuf<S>();
  using C_ = CfgW1<S, NBUF>;
  const int64_t ntiles =
      ((a.one.nprime + C_::BJ - 1) / C_::BJ) * ((a.one.m + C_::BI - 1) / C_::BI);
  const int64_t grid = std::min<int64_t>(ntiles, (int64_t)num_cu);
  if (grid <= 0) return hipSuccess;
  const dim3 g((unsigned)grid), b(C_::NT);
  hipLaunchKernelGGL((k_ozgemm_w1<S, NBUF>), g, b, 0, st, a);
  return hipGetLastError();
}

}  // namespace

int gemm_w1_max_slices() { return kW1MaxS; }

int64_t gemm_w1_tile_j() { return CfgW1<1, 2>::BJ; }
int64_t gemm_w1_tile_i() { return CfgW1<1, 2>::BI; }

hipError_t launch_ozgemm_w1(int S, const GemmArgs &a, int num_cu, hipStream_t st) {
  if (a.probs != nullptr || a.one.raw != nullptr || a.chunked) return hipErrorInvalidValue;
  switch (S) {
#define OZ_CASE(N) \
  case N: return launch_w1_s<N>(a, num_cu, st);
    OZ_CASE(1) OZ_CASE(2) OZ_CASE(3) OZ_CASE(4) OZ_CASE(5) OZ_CASE(6) OZ_CASE(7) OZ_CASE(8)
#undef OZ_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace oz
