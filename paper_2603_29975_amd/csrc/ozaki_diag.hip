// One more slice-pair diagonal on top of a stored recombination (gfx950).
//
// With trunc-7 slices the digits at s slices are a prefix of those at s + 1,
// so the product at s + 1 slices differs from the one at s only by the new
// diagonal S_d = sum_{p + q = d} SA_p SB_q, d = s + 2, and the recombination
// (largest weight first, one rounding per addition) continues from where it
// stopped: acc_{s+1} = RN(acc_s + S_d 2^-7d). The automatic slice mode raises a
// product whose residual probe misses the target this way instead of forming
// it again.
//
// Work: a tile table of 64 x 64 output tiles (j' x i) over the problems; each
// of the 4 waves owns one 32 x 32 block, loads its B' and A' fragments of
// every slice pair of the diagonal straight from the packed operands (one
// contiguous 16-byte run per lane) and accumulates with
// v_mfma_i32_32x32x32_i8; INT32 partial sums are carried into int64 before
// (d - 1) * 32 * kb * 127^2 could reach 2^31. Only problems flagged for a
// raise do any work (flag[id] == 1); the others' tiles return at once.
#include "ozaki_gemm_tile.hpp"

namespace oz {

namespace {

constexpr int kDiagTile = 64;

__global__ void __launch_bounds__(256) k_add_diagonal(const DiagTask *tasks, const int *tile_task,
                                                      const int *tile_local, const int *s,
                                                      const int *flag) {
  const DiagTask tk = tasks[tile_task[blockIdx.x]];
  if (flag[tk.id] != 1) return;
  const int d = s[tk.id] + 1;  // the new diagonal: slices 1..d-1 on each side
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int wj = wave & 1, wi = wave >> 1;
  const int64_t ntj = (tk.nprime + kDiagTile - 1) / kDiagTile;
  const int64_t local = tile_local[blockIdx.x];
  const int64_t tj = local % ntj, ti = local / ntj;
  const int64_t rbP = tj * 2 + wj, rbQ = ti * 2 + wi;
  const int64_t nkb = tk.nkb;
  const int64_t planeP = tk.nrbP * nkb * kFragBytes, planeQ = tk.nrbQ * nkb * kFragBytes;
  const int8_t *bp = tk.SP + rbP * nkb * kFragBytes + lane * 16;
  const int8_t *aq = tk.SQ + rbQ * nkb * kFragBytes + lane * 16;
  const int64_t chunk = tile::chunk_blocks(d - 1);

  int64_t tot[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) tot[r] = 0;
  v16i acc = v16i{0};
  int64_t next = chunk;
  for (int64_t kb = 0; kb < nkb; ++kb) {
    // four slice pairs per pass, their eight fragment loads issued together
    // (past the last pair: the last pair's fragments again, not used)
    for (int p0 = 1; p0 < d; p0 += 4) {
      v4i bf[4], af[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int p = p0 + x < d ? p0 + x : d - 1;
        bf[x] = *reinterpret_cast<const v4i *>(bp + (d - p - 1) * planeP + kb * kFragBytes);
        af[x] = *reinterpret_cast<const v4i *>(aq + (p - 1) * planeQ + kb * kFragBytes);
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
        if (p0 + x < d) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(bf[x], af[x], acc, 0, 0, 0);
    }
    if (kb + 1 == next || kb + 1 == nkb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) tot[r] += (int64_t)acc[r];
      acc = v16i{0};
      next += chunk;
    }
  }

  // lane register r: output row i, column side j' = jbase + 8 (r / 4) + r % 4
  const int64_t i = ti * kDiagTile + wi * 32 + (lane & 31);
  if (i >= tk.m) return;
  const int64_t jbase = tj * kDiagTile + wj * 32 + 4 * (lane >> 5);
  const int w = tk.woff - tk.wbits * d;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t jp = jbase + 8 * (r >> 2) + (r & 3);
    if (jp >= tk.nprime) continue;
    // complex: j' = 2 j + c is part c of column j
    double *pp = tk.cplx ? reinterpret_cast<double *>(tk.P) + 2 * (i + (jp >> 1) * tk.m) + (jp & 1)
                         : reinterpret_cast<double *>(tk.P) + i + jp * tk.m;
    *pp = add_rn(*pp, ldexp((double)tot[r], w));
  }
}

}  // namespace

int64_t diag_tiles(int64_t m, int64_t nprime) {
  return ((nprime + kDiagTile - 1) / kDiagTile) * ((m + kDiagTile - 1) / kDiagTile);
}

hipError_t launch_add_diagonal(const DiagTask *tasks, const int *tile_task, const int *tile_local,
                               int64_t ntiles, const int *s, const int *flag, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7fffffffll) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_add_diagonal, dim3((unsigned)ntiles), dim3(256), 0, st, tasks, tile_task,
                     tile_local, s, flag);
  return hipGetLastError();
}

}  // namespace oz
