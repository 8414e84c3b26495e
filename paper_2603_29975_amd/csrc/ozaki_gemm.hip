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
// by S * 32 * kb * 127^2. Past that bound a single product with one A' block
// per wave splits each diagonal's pairs over two INT32 sets (p below or from
// ceil(S/2)), which doubles the reach; beyond that, or with two A' blocks per
// wave, the contraction is cut into chunks that keep each sum below 2^31 and
// each chunk is carried exactly into int64 workgroup-private memory. The FP64 epilogue converts every S_t exactly (|S_t| < 2^53) and adds
// them largest weight first, one rounding per addition, then scales by
// 2^(e_i + f_j) and applies alpha/beta without fused multiply-adds.
#include "ozaki_gemm_tile.hpp"

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

using tile::barrier_only;
using tile::chunk_blocks;
using tile::wait_vmcnt;

template <int S, int WJ, int WI, int IB, int NBUF, bool RAW, bool CHUNKED, bool GROUPED,
          bool EARLY, bool SPLIT = false>
__global__ void __launch_bounds__(64 * WJ * WI, 512 / (64 * WJ * WI)) k_ozgemm(GemmArgs G) {
  using C_ = Cfg<S, WJ, WI, IB, NBUF>;
  static_assert(!(SPLIT && (CHUNKED || RAW)), "split accumulation replaces the carry");
  constexpr int PM = tile::split_pm(S);
  constexpr int XN = SPLIT ? tile::split_extra(S) : 0;
  __shared__ __attribute__((aligned(16))) int8_t lds[C_::LDS];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform
  const int wj = wave % WJ;
  const int wi = wave / WJ;

  constexpr bool chunked = CHUNKED;
  const int64_t ntiles =
      GROUPED ? G.ntiles
              : ((G.one.nprime + C_::BJ - 1) / C_::BJ) * ((G.one.m + C_::BI - 1) / C_::BI);

  for (int64_t tn = blockIdx.x; tn < ntiles; tn += gridDim.x) {
    // The problem this tile belongs to (uniform across the workgroup, so the
    // descriptor is fetched with scalar loads).
    const GemmProblem a = GROUPED ? G.probs[G.tile_prob[tn]] : G.one;
    int64_t local = GROUPED ? (int64_t)G.tile_local[tn] : tn;
    if (!GROUPED && G.order == 3) local = tile::xcd_major(tn, ntiles);
    int64_t tj, ti;
    tile::tile_coords(local, G.order, a.m, a.nprime, C_::BJ, C_::BI, tj, ti);
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
        tile::copy_frag(src + lane * 16, lds + buf * C_::STAGE + f * kFragBytes);
      }
    };

    v16i acc[IB][S];
    v16i accx[IB][XN > 0 ? XN : 1];
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) {
#pragma unroll
      for (int t = 0; t < S; ++t) acc[ib][t] = v16i{0};
#pragma unroll
      for (int t = 0; t < XN; ++t) accx[ib][t] = v16i{0};
    }

    // Exact int64 carry of the INT32 accumulators (chunked contraction only).
    int64_t *ws = G.flush_ws + ((int64_t)blockIdx.x * C_::NW + wave) * (int64_t)IB * S * 1024;
    auto carry = [&](bool first) {
#pragma unroll
      for (int ib = 0; ib < IB; ++ib) tile::carry_block<S>(acc[ib], ws + ib * S * 1024, lane, first);
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
      // One MFMA of slice pair (p, q) into the set of diagonal p + q.
      auto mfma = [&](int p, int q, int ib, const v4i &pq, const v4i &qp) {
        if (XN > 0 && p >= PM)  // the second set of diagonal p + q
          accx[ib][p + q - PM] =
              __builtin_amdgcn_mfma_i32_32x32x32_i8(pq, qp, accx[ib][p + q - PM], 0, 0, 0);
        else
          acc[ib][p + q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(pq, qp, acc[ib][p + q], 0, 0, 0);
      };
      auto read_q = [&](int p, int ib) {
        return *reinterpret_cast<const v4i *>(L + (C_::NFP + p * C_::NQB + wi * IB + ib) * kFragBytes +
                                              lane * 16);
      };
      if constexpr (!EARLY) {
        // Left to itself the compiler reads each A' fragment just before its
        // MFMAs (with two A' blocks per wave, into one register set: the
        // fragments of every slice do not fit next to the 2 S accumulator
        // sets) and waits out every LDS latency. Here the A' reads of slice
        // p + 1 go out before the MFMAs of slice p (two register sets), the
        // order pinned by scheduling barriers.
        v4i pf[S], qa[IB], qb[IB];
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) qa[ib] = read_q(0, ib);
        pf[S - 1] = *reinterpret_cast<const v4i *>(L + ((S - 1) * WJ + wj) * kFragBytes + lane * 16);
#pragma unroll
        for (int q = 0; q < S - 1; ++q)
          pf[q] = *reinterpret_cast<const v4i *>(L + (q * WJ + wj) * kFragBytes + lane * 16);
#pragma unroll
        for (int p = 0; p < S; ++p) {
          if (p + 1 < S) {
#pragma unroll
            for (int ib = 0; ib < IB; ++ib) qb[ib] = read_q(p + 1, ib);
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int ib = 0; ib < IB; ++ib)
#pragma unroll
            for (int q = 0; q < S - p; ++q) mfma(p, q, ib, pf[q], qa[ib]);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int ib = 0; ib < IB; ++ib) qa[ib] = qb[ib];
        }
      } else {
        // All fragment reads of the block are issued up front, A' of slice 1
        // first; a wave's LDS reads return in order, so each MFMA waits only
        // for the reads it needs and the later ones arrive under the earlier
        // MFMAs.
        v4i qf[S][IB];
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) qf[0][ib] = read_q(0, ib);
        // The compiler starts each block with the MFMA of the longest
        // accumulation chain (slice pair 1, S), so B' slice S is read second.
        v4i pf[S];
        pf[S - 1] = *reinterpret_cast<const v4i *>(L + ((S - 1) * WJ + wj) * kFragBytes + lane * 16);
#pragma unroll
        for (int q = 0; q < S - 1; ++q)
          pf[q] = *reinterpret_cast<const v4i *>(L + (q * WJ + wj) * kFragBytes + lane * 16);
#pragma unroll
        for (int p = 1; p < S; ++p)
#pragma unroll
          for (int ib = 0; ib < IB; ++ib) qf[p][ib] = read_q(p, ib);
        // EARLY keeps the reads above the MFMAs (the scheduler would otherwise
        // sink each A' read to just before its first use and expose its
        // latency); for large S the registers of all fragments would not fit
        if constexpr (EARLY && S * (1 + IB) <= 18) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int p = 0; p < S; ++p)
#pragma unroll
          for (int ib = 0; ib < IB; ++ib)
#pragma unroll
            for (int q = 0; q < S - p; ++q) mfma(p, q, ib, pf[q], qf[p][ib]);
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
#pragma unroll
    for (int ib = 0; ib < IB; ++ib)
      tile::store_block<S, CHUNKED, RAW, XN>(a, acc[ib], ws + ib * S * 1024, lane,
                                             ti * C_::BI + (wi * IB + ib) * 32 + (lane & 31),
                                             tj * C_::BJ + wj * 32 + 4 * (lane >> 5), accx[ib]);
  }
}

template <int S, int WJ, int WI, int IB, int NBUF, bool WITH_RAW, bool EARLY = false>
hipError_t launch_cfg(const GemmArgs &a, int num_cu, hipStream_t st) {
  using C_ = Cfg<S, WJ, WI, IB, NBUF>;
  const bool grouped = a.probs != nullptr;
  const int64_t ntiles =
      grouped ? a.ntiles
              : ((a.one.nprime + C_::BJ - 1) / C_::BJ) * ((a.one.m + C_::BI - 1) / C_::BI);
  // persistent grid: 8 waves per CU, i.e. one workgroup of 8 waves or two of 4
  // (whose barriers are independent, so one's MFMAs fill the other's waits)
  const int64_t per_cu = C_::NW >= 8 ? 1 : 8 / C_::NW;
  int64_t grid = std::min<int64_t>(ntiles, per_cu * num_cu);
  if (a.max_groups > 0) grid = std::min<int64_t>(grid, a.max_groups);
  if (grid <= 0) return hipSuccess;
  const dim3 g((unsigned)grid), b(C_::NT);
  if (grouped) {
    if (a.chunked)
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, IB, NBUF, false, true, true, EARLY>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, IB, NBUF, false, false, true, EARLY>), g, b, 0, st, a);
  } else if (a.one.raw != nullptr) {
    if constexpr (WITH_RAW) {
      if (a.chunked)
        hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, IB, NBUF, true, true, false, EARLY>), g, b, 0, st, a);
      else
        hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, IB, NBUF, true, false, false, EARLY>), g, b, 0, st, a);
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    // a contraction each of whose diagonals fits two INT32 sets takes the
    // split accumulation where its extra sets fit the registers (one A' block
    // per wave, S <= 7; two blocks' extra sets, or S >= 8, spill)
    bool split = false;
    if constexpr (IB == 1 && S >= 2 && S <= 7) {
      if (a.chunked && a.split) {
        hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, IB, NBUF, false, false, false, EARLY, true>), g, b,
                           0, st, a);
        split = true;
      }
    }
    if (split)
      ;
    else if (a.chunked)
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, IB, NBUF, false, true, false, EARLY>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_ozgemm<S, WJ, WI, IB, NBUF, false, false, false, EARLY>), g, b, 0, st, a);
  }
  return hipGetLastError();
}

// Tile configurations (the autotuner's candidates). All use 32 x 32 x 32 INT8
// MFMA blocks, one INT32 accumulator set per diagonal and 8 waves (two per
// SIMD), one 32 x 32 output block per wave:
//   0: 4 waves along j' x 2 along i (workgroup tile 128 j' x 64 i), LDS ring of
//      three contraction blocks where it fits in 160 KiB (S <= 8), else two
//   1: 2 along j' x 4 along i (64 j' x 128 i), same ring
//   2: as 0 with a ring of two blocks (prefetch distance one)
//   3: as 2 with every fragment read of a block issued before its MFMAs
//   4: 4 waves (2 x 2), tile 64 j' x 64 i, ring of two, two workgroups per CU
//   5: as 4 with the reads of 3 (4 and 5 fall back to 2 for S >= 11)
//   6: as 2 with two 32-row blocks of A' per wave (tile 128 j' x 128 i): each
//      B' fragment feeds two MFMAs; S <= 6 only (else configuration 2)
// A tuning id below 14 is 2 * configuration + tile order (0: consecutive
// tiles walk down the rows i, 1: along the columns j'); ids 14 .. 20 are
// configurations 0 .. 6 with the grouped tile order 2, ids 21 .. 27 with the
// XCD-aware order 3 (see tile_coords and xcd_major).
constexpr int kNumCfg = 7;
constexpr int id_cfg(int id) { return id < 2 * kNumCfg ? id >> 1 : (id - 2 * kNumCfg) % kNumCfg; }
constexpr int id_order(int id) { return id < 2 * kNumCfg ? (id & 1) : 2 + (id - 2 * kNumCfg) / kNumCfg; }

template <int CFG>
struct Pick;
template <>
struct Pick<0> {
  static constexpr int WJ = 4, WI = 2, IB = 1, RING = 3;
};
template <>
struct Pick<1> {
  static constexpr int WJ = 2, WI = 4, IB = 1, RING = 3;
};
template <>
struct Pick<2> {
  static constexpr int WJ = 4, WI = 2, IB = 1, RING = 2;
};
template <>
struct Pick<3> {  // two 32-row blocks of A' per wave (S <= 6: the accumulators fit)
  static constexpr int WJ = 4, WI = 2, IB = 2, RING = 2;
};

template <int S, int CFG>
constexpr int nbuf_for() {
  using P = Pick<CFG>;
  return (P::RING == 3 && S * (P::WJ + P::WI * P::IB) * kFragBytes * 3 <= 160 * 1024) ? 3 : 2;
}

template <int S, int CFG>
hipError_t launch_pick(const GemmArgs &a, int num_cu, hipStream_t st) {
  using P = Pick<CFG>;
  return launch_cfg<S, P::WJ, P::WI, P::IB, nbuf_for<S, CFG>(), CFG == 0>(a, num_cu, st);
}

template <int S>
hipError_t launch_s(int cfg, const GemmArgs &a, int num_cu, hipStream_t st) {
  switch (cfg) {
    case 1: return launch_pick<S, 1>(a, num_cu, st);
    case 2: return launch_pick<S, 2>(a, num_cu, st);
    case 3: return launch_cfg<S, 4, 2, 1, 2, false, true>(a, num_cu, st);
    case 4:
    case 5:
      // two four-wave workgroups per CU need <= 256 registers per wave, which
      // the accumulators of S >= 11 exceed: configuration 2 there
      if constexpr (S <= 10) {
        if (cfg == 4) return launch_cfg<S, 2, 2, 1, 2, false, false>(a, num_cu, st);
        return launch_cfg<S, 2, 2, 1, 2, false, true>(a, num_cu, st);
      } else {
        return launch_pick<S, 2>(a, num_cu, st);
      }
    case 6:
      if constexpr (S <= 6)
        return launch_pick<S, 3>(a, num_cu, st);
      else
        return launch_pick<S, 2>(a, num_cu, st);
    default: return launch_pick<S, 0>(a, num_cu, st);
  }
}

template <int CFG>
constexpr int waves_of() {
  return Pick<CFG>::WJ * Pick<CFG>::WI * Pick<CFG>::IB;
}

}  // namespace

int64_t kb_chunk_for(int S, bool b8) { return chunk_blocks(S, b8 ? 128 : 127); }
int64_t kb_split_for(int S, bool b8) { return chunk_blocks(tile::split_pm(S), b8 ? 128 : 127); }

int gemm_num_configs() { return 4 * kNumCfg; }

size_t gemm_flush_bytes(int S, int cfg, int num_cu) {
  // the largest per-workgroup carry space over the configurations, so that a
  // plan is valid whichever configuration runs
  (void)cfg;
  const int waves =
      std::max(std::max(waves_of<0>(), waves_of<1>()), std::max(waves_of<2>(), waves_of<3>()));
  return (size_t)num_cu * waves * (size_t)S * 1024 * sizeof(int64_t);
}

int64_t gemm_tiles(int S, int cfg, int64_t m, int64_t nprime) {
  int64_t BJ, BI;
  switch (id_cfg(cfg)) {
    case 1: BJ = 32 * Pick<1>::WJ; BI = 32 * Pick<1>::WI * Pick<1>::IB; break;
    case 2: BJ = 32 * Pick<2>::WJ; BI = 32 * Pick<2>::WI * Pick<2>::IB; break;
    case 3: BJ = 32 * Pick<2>::WJ; BI = 32 * Pick<2>::WI * Pick<2>::IB; break;
    case 4:
    case 5:
      if (S <= 10) {
        BJ = 64;
        BI = 64;
      } else {  // launched as configuration 2
        BJ = 32 * Pick<2>::WJ;
        BI = 32 * Pick<2>::WI * Pick<2>::IB;
      }
      break;
    case 6:
      if (S <= 6) {
        BJ = 32 * Pick<3>::WJ;
        BI = 32 * Pick<3>::WI * Pick<3>::IB;
      } else {  // launched as configuration 2
        BJ = 32 * Pick<2>::WJ;
        BI = 32 * Pick<2>::WI * Pick<2>::IB;
      }
      break;
    default: BJ = 32 * Pick<0>::WJ; BI = 32 * Pick<0>::WI * Pick<0>::IB; break;
  }
  return ((nprime + BJ - 1) / BJ) * ((m + BI - 1) / BI);
}

hipError_t launch_ozgemm_grouped(int S, int cfg, const GemmArgs &a, int num_cu, hipStream_t st) {
  return launch_ozgemm(S, cfg, a, num_cu, st);
}

hipError_t launch_ozgemm(int S, int tune_id, const GemmArgs &a0, int num_cu, hipStream_t st) {
  GemmArgs a = a0;
  a.order = id_order(tune_id);
  const int cfg = id_cfg(tune_id);
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
