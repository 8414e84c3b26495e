// Pieces shared by the fused slice GEMM kernels of libozaki (gfx950): explicit
// wait/barrier primitives, the INT32 chunk bound, the int64 carry of a 32 x 32
// accumulator block and the FP64 recombination epilogue of one block.
//
// Accumulator layout of v_mfma_i32_32x32x32_i8 as used here: the MFMA row
// index is the output column side j', the MFMA column index (lane % 32) is the
// output row i. Register r of a lane holds j' = jbase + 8 (r / 4) + r % 4 with
// jbase = 32 * block + 4 * (lane / 32).
#pragma once

#include "ozaki_internal.hpp"

namespace oz {
namespace tile {

// Wait until at most N vector-memory operations of this wave are in flight.
// Inline assembly with a memory clobber: the compiler neither moves memory
// accesses across it nor adds a drain of the LDS copies still in flight.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
// Wait until this wave's LDS reads have returned.
__device__ __forceinline__ void wait_lgkm0() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void barrier_only() { asm volatile("s_barrier" ::: "memory"); }

// One 1 KiB slice fragment from global memory straight into LDS: lane l
// copies the 16 bytes at src_lane (its own part of the fragment) to LDS
// address lds_wave + 16 l. Inline assembly rather than the compiler's builtin
// for the same instruction: with the builtin in a loop the compiler waits for
// every outstanding LDS read (lgkmcnt(0)) before each fragment's first use,
// which serialises the fragment reads with the MFMAs; with the copy hidden
// from it, it waits for exactly the reads each MFMA needs. The copy counts in
// vmcnt, which the kernels wait on explicitly (wait_vmcnt); the LDS base goes
// through M0, set in the same statement.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void copy_frag(const int8_t *src_lane, const int8_t *lds_wave) {
  const uint32_t la = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) int8_t *)lds_wave;
  asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src_lane), "s"(la)
               : "memory", "m0");
}
#pragma clang diagnostic pop

// Contraction blocks of 32 a chunk may hold: S * 32 * kb * dmax^2 <= 2^31 - 1
// with dmax = 127 (trunc-7 digits) or 128 (8-bit balanced digits).
__host__ __device__ constexpr int64_t chunk_blocks(int S, int dmax = 127) {
  return (int64_t)(2147483647ll / ((int64_t)S * 32 * dmax * dmax));
}

// Exact int64 carry of one block's S INT32 accumulator sets into its carry
// space `ws` (S * 16 * 64 int64, lane-interleaved); the accumulators restart
// at zero. Device-scope atomics keep the traffic in L2, away from stale lines
// of the non-coherent vector L1.
// The lane's base address goes through an empty asm statement: the S x 16
// addresses are then formed here, one at a time, instead of being hoisted out
// of the contraction loop, where keeping them live costs 2 S x 16 registers
// and the compiler spills.
template <int S>
__device__ __forceinline__ void carry_block(v16i (&acc)[S], int64_t *ws, int lane, bool first) {
  int64_t *q = ws + lane;
  asm volatile("" : "+v"(q));
#pragma unroll
  for (int t = 0; t < S; ++t) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      int64_t *p = q + (t * 16 + r) * 64;
      if (first)
        __hip_atomic_store(p, (int64_t)acc[t][r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else
        __hip_atomic_fetch_add(p, (int64_t)acc[t][r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    acc[t] = v16i{0};
  }
}

// Split accumulation: diagonal t (t + 1 slice pairs) keeps the pairs with
// p < split_pm(S) in one INT32 set and the others (at most as many) in a
// second, so a contraction of up to chunk_blocks(split_pm(S)) blocks needs no
// int64 carry; the two sets add exactly in int64 in the epilogue.
__host__ __device__ constexpr int split_pm(int S) { return (S + 1) / 2; }
__host__ __device__ constexpr int split_extra(int S) { return S - split_pm(S); }

// Recombination and store of one 32 x 32 block: row i of the output, lane
// register r at column side j' = jbase + 8 (r / 4) + r % 4. Diagonal t + 2 of
// the block is acc[t] (plus accx[t - split_pm(S)] for t >= split_pm(S) when XN
// > 0; or, for a chunked contraction, the int64 total in the carry space
// `ws`). acc = RN(acc + S_t 2^(woff - wbits t)) for t = 2..S+1 (2^-7t for
// trunc-7 slices, 2^(4-8t) for 8-bit balanced ones), then ldexp(acc, e_i +
// f_j) and alpha/beta without fused multiply-adds; rows or columns flagged
// non-finite give NaN. RAW writes the exact diagonals instead.
template <int S, bool CHUNKED, bool RAW, int XN = 0>
__device__ __forceinline__ void store_block(const GemmProblem &a, const v16i (&acc)[S],
                                            const int64_t *ws, int lane, int64_t i,
                                            int64_t jbase, const v16i *accx = nullptr) {
  const bool row_ok = i < a.m;
  const int codeA = row_ok ? a.codeA[i] : 0;

  const int64_t *q = ws + lane;
  if constexpr (CHUNKED) asm volatile("" : "+v"(q));  // as in carry_block
  auto total = [&](int t, int r) -> int64_t {
    if constexpr (CHUNKED)
      return __hip_atomic_load(q + (t * 16 + r) * 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if constexpr (XN > 0) {
      if (t >= S - XN) return (int64_t)acc[t][r] + (int64_t)accx[t - (S - XN)][r];
    }
    return (int64_t)acc[t][r];
  };

  if constexpr (RAW) {
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
      acc64 = add_rn(acc64, ldexp((double)total(t, r), a.woff - a.wbits * (t + 2)));
    val[r] = acc64;
    // chunked: the S int64 totals of one entry at a time (issuing all 16 S
    // loads at once needs 32 S registers)
    if constexpr (CHUNKED) __builtin_amdgcn_sched_barrier(0);
  }
  if (!row_ok) return;
  const int ea = code_exp(codeA);
  const bool bad_i = code_bad(codeA);

  if (a.unscaled) {
    // the recombined sums as they are (NaN for non-finite rows/columns): a
    // later diagonal adds to them exactly as the loop above would have
    if (a.cplx) {
      double2 *C = reinterpret_cast<double2 *>(a.C);
      const int64_t n = a.nprime >> 1;
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const int64_t j = (jbase + 8 * (r >> 2) + (r & 3)) >> 1;
        if (j >= n) continue;
        const bool bad = bad_i || code_bad(a.codeB[j]);
        C[i + j * a.ldc] = bad ? make_double2(qnan(), qnan()) : make_double2(val[r], val[r + 1]);
      }
    } else {
      double *C = reinterpret_cast<double *>(a.C);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t j = jbase + 8 * (r >> 2) + (r & 3);
        if (j >= a.nprime) continue;
        C[i + j * a.ldc] = (bad_i || code_bad(a.codeB[j])) ? qnan() : val[r];
      }
    }
    return;
  }

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

// Order 3: workgroup w of a persistent grid runs on XCD w % 8 (workgroups are
// dealt to the 8 XCDs round-robin), and each XCD has its own L2. Within each
// full round of gridDim.x tiles, tile number tn is given to slot w of the
// round as xcd_major(tn): the tiles of one XCD's workgroups are consecutive
// in the grouped order (8 tile rows per group), so they share 8 A' stripes
// and few B' stripes in that XCD's L2 instead of every XCD fetching all the
// stripes of the round. A partial last round keeps the identity.
__device__ __forceinline__ int64_t xcd_major(int64_t tn, int64_t ntiles) {
  const int64_t G = gridDim.x;
  if ((G & 7) != 0) return tn;
  const int64_t r0 = tn - tn % G;
  if (r0 + G > ntiles) return tn;
  const int64_t w = tn - r0;
  return r0 + (w & 7) * (G >> 3) + (w >> 3);
}

// Output tile (tj, ti) of tile number `local` in a grid of tiles BJ x BI:
// order 0 walks down the rows i first, order 1 along the columns j' first,
// order 2 in groups of 16 tile rows, down the rows of a group first (the
// tiles in flight at once then share 16 A' stripes and few B' stripes, which
// keeps long contractions in the caches instead of streaming every B' stripe
// once per round); order 3 in groups of 8 tile rows (after xcd_major).
__device__ __forceinline__ void tile_coords(int64_t local, int order, int64_t m, int64_t nprime,
                                            int BJ, int BI, int64_t &tj, int64_t &ti) {
  const int64_t nti = (m + BI - 1) / BI;
  if (order == 0) {
    tj = local / nti;
    ti = local % nti;
  } else if (order == 1) {
    const int64_t ntj = (nprime + BJ - 1) / BJ;
    ti = local / ntj;
    tj = local % ntj;
  } else {
    const int64_t kGroup = order == 2 ? 16 : 8;
    const int64_t ntj = (nprime + BJ - 1) / BJ;
    const int64_t g = local / (kGroup * ntj), r = local - g * (kGroup * ntj);
    const int64_t gh = nti - g * kGroup < kGroup ? nti - g * kGroup : kGroup;
    ti = g * kGroup + r % gh;
    tj = r / gh;
  }
}

}  // namespace tile
}  // namespace oz
