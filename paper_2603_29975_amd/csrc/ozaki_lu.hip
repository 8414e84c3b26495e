// Blocked LU with partial pivoting and the inverse of a complex matrix: the
// kernels around the trailing-update GEMMs. The paper's solver inverts the
// multiple-scattering matrix by LU (Section 3.2: ZGEMM and ZTRSM take most of
// its time), so the emulated ZGEMM sits inside this factorization. Every
// complex operation is written out with separately rounded real operations
// (no fused multiply-adds) in a fixed order, so the CPU model repeats it bit
// for bit:
//   product   (ar br - ai bi, ar bi + ai br)
//   quotient  d = br br + bi bi, ((ar br + ai bi) / d, (ai br - ar bi) / d)
//   multiplier a_ic (1 / a_cc), the reciprocal (pr / d, (-pi) / d) with
//             d = pr pr + pi pi (the reference LAPACK's unblocked
//             factorization scales the column by the pivot's reciprocal too)
//   pivot     the first row of the largest |Re| + |Im| in the column (NaN
//             counts as the largest)
#include "ozaki_internal.hpp"

namespace oz {
namespace {

struct Z {
  double re, im;
};

__device__ __forceinline__ Z ld(const double2 *p) {
  const double2 v = *p;
  return Z{v.x, v.y};
}
__device__ __forceinline__ void st(double2 *p, Z z) { *p = make_double2(z.re, z.im); }

__device__ __forceinline__ Z zmul(Z a, Z b) {
  return Z{sub_rn(mul_rn(a.re, b.re), mul_rn(a.im, b.im)), add_rn(mul_rn(a.re, b.im), mul_rn(a.im, b.re))};
}
__device__ __forceinline__ Z zsub(Z a, Z b) { return Z{sub_rn(a.re, b.re), sub_rn(a.im, b.im)}; }
__device__ __forceinline__ Z zdiv(Z a, Z b) {
  const double d = add_rn(mul_rn(b.re, b.re), mul_rn(b.im, b.im));
  return Z{__ddiv_rn(add_rn(mul_rn(a.re, b.re), mul_rn(a.im, b.im)), d),
           __ddiv_rn(sub_rn(mul_rn(a.im, b.re), mul_rn(a.re, b.im)), d)};
}
__device__ __forceinline__ Z zrcp(Z b) {
  const double d = add_rn(mul_rn(b.re, b.re), mul_rn(b.im, b.im));
  return Z{__ddiv_rn(b.re, d), __ddiv_rn(-b.im, d)};
}
__device__ __forceinline__ double cabs1(Z a) { return add_rn(fabs(a.re), fabs(a.im)); }

// Pivot order: the larger |Re| + |Im| wins, a NaN counts as larger than any
// number, and equal values (or two NaNs) go to the lower row.
// Written without branches (bitwise on the comparisons), so a reduction
// over it stays straight-line code.
__device__ __forceinline__ bool beats(double v, int64_t i, double bv, int64_t bi) {
  const bool vn = v != v, bn = bv != bv, lower = i < bi;
  return (vn & !bn) | ((vn == bn) & ((vn & lower) | (v > bv) | ((v == bv) & lower)));
}

// Pivot of column c (rows c..n-1), then the swap of rows c and the pivot row
// over the panel columns [p0, p1). One workgroup of 256 threads, rows in
// batches of 8 per thread with their loads in flight together; the waves
// reduce with cross-lane shuffles and every thread reduces the 4 wave results
// itself. A pivot that is zero or NaN is recorded in *singular (the smallest
// such column). The panel's columns keep their unscaled entries below the
// diagonal until k_panel_scale turns them into multipliers at the end of the
// panel (column c is not updated after step c, only its rows exchanged, so
// the multipliers come out the same).
__global__ void __launch_bounds__(256) k_pivot_swap(double2 *A, int64_t lda, int64_t n, int64_t c,
                                                    int64_t p0, int64_t p1, int64_t *ipiv,
                                                    int64_t *singular) {
  constexpr int kB = 8;
  __shared__ double sv[4];
  __shared__ int64_t si[4];
  const int t = threadIdx.x;
  double best = -1.0;
  int64_t bi = n;
  for (int64_t i0 = c + t; i0 < n; i0 += 256 * kB) {
    Z v[kB];
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const int64_t i = i0 + 256 * j;
      if (i < n) v[j] = ld(A + i + c * lda);
    }
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const int64_t i = i0 + 256 * j;
      if (i < n) {
        const double a = cabs1(v[j]);
        if (beats(a, i, best, bi)) {  // rows of a thread in increasing order
          best = a;
          bi = i;
        }
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(best, o);
    const int64_t oi = __shfl_xor(bi, o);
    if (beats(ov, oi, best, bi)) {
      best = ov;
      bi = oi;
    }
  }
  if ((t & 63) == 0) {
    sv[t >> 6] = best;
    si[t >> 6] = bi;
  }
  __syncthreads();
  best = sv[0];
  bi = si[0];
#pragma unroll
  for (int w = 1; w < 4; ++w)
    if (beats(sv[w], si[w], best, bi)) {
      best = sv[w];
      bi = si[w];
    }
  // row c itself takes part, so bi is a row of [c, n) (any value or NaN beats -1)
  const int64_t piv = bi;
  if (t == 0) {
    ipiv[c] = piv;
    if (!(best > 0.0)) atomicMin(reinterpret_cast<unsigned long long *>(singular),
                                 (unsigned long long)c);
  }
  if (piv != c) {
    for (int64_t k0 = p0 + t; k0 < p1; k0 += 256 * 4) {
      Z x[4], y[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t k = k0 + 256 * j;
        if (k < p1) {
          x[j] = ld(A + c + k * lda);
          y[j] = ld(A + piv + k * lda);
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t k = k0 + 256 * j;
        if (k < p1) {
          st(A + c + k * lda, y[j]);
          st(A + piv + k * lda, x[j]);
        }
      }
    }
  }
}

// Panel update after the pivot of column c: a_ik -= (a_ic (1 / a_cc)) a_ck for
// rows i > c and panel columns c < k < p1, one thread per element (each
// computes its row's multiplier from the unscaled a_ic).
__global__ void __launch_bounds__(256) k_panel_update(double2 *A, int64_t lda, int64_t n, int64_t c) {
  const int64_t i = c + 1 + (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t k = c + 1 + blockIdx.y;
  if (i >= n) return;
  const Z l = zmul(ld(A + i + c * lda), zrcp(ld(A + c + c * lda)));
  st(A + i + k * lda, zsub(ld(A + i + k * lda), zmul(l, ld(A + c + k * lda))));
}

// End of the panel [p0, p1): the multipliers l_ic = a_ic (1 / a_cc) of every
// panel column c, rows i > c, in place (one thread per entry).
__global__ void __launch_bounds__(256) k_panel_scale(double2 *A, int64_t lda, int64_t n, int64_t p0) {
  const int64_t c = p0 + blockIdx.y;
  const int64_t i = p0 + 1 + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i <= c || i >= n) return;
  st(A + i + c * lda, zmul(ld(A + i + c * lda), zrcp(ld(A + c + c * lda))));
}

// Pivot order of the leaf as one key per candidate: the bits of |Re| + |Im|
// (a non-negative double, whose bit patterns order like its values) with
// every NaN mapped to one key above +inf, and the row below the leaf's first
// row as a 32-bit tie-break. The larger key wins, equal keys go to the lower
// row: the order `beats` defines, in two integer compares.
constexpr uint64_t kNaNKey = 0x7FF8000000000000ull;
constexpr uint32_t kNoRow = 0xFFFFFFFFu;
__device__ __forceinline__ uint64_t pivot_key(double v) {
  return v != v ? kNaNKey : (uint64_t)__double_as_longlong(v);
}
__device__ __forceinline__ bool key_beats(uint64_t k, uint32_t r, uint64_t bk, uint32_t br) {
  return (k > bk) | ((k == bk) & (r < br));
}

// One step of a wave's pivot reduction with a DPP lane pattern (VALU moves, no
// LDS round trip): each lane compares with the lane CTRL names.
template <int CTRL>
__device__ __forceinline__ void best_dpp(uint64_t &bk, uint32_t &br) {
  const int klo = (int)(uint32_t)bk, khi = (int)(uint32_t)(bk >> 32), r = (int)br;
  const uint32_t oklo = (uint32_t)__builtin_amdgcn_update_dpp(klo, klo, CTRL, 0xF, 0xF, false);
  const uint32_t okhi = (uint32_t)__builtin_amdgcn_update_dpp(khi, khi, CTRL, 0xF, 0xF, false);
  const uint32_t orow = (uint32_t)__builtin_amdgcn_update_dpp(r, r, CTRL, 0xF, 0xF, false);
  const uint64_t ok = ((uint64_t)okhi << 32) | oklo;
  const bool take = key_beats(ok, orow, bk, br);
  bk = take ? ok : bk;
  br = take ? orow : br;
}

// The wave's best (key, row) in every lane: within each 16-lane row by DPP
// (quad exchanges 1 and 2, then half-row and row mirrors), across rows by two
// shuffles. The order of comparisons does not matter: the (key, row) order is
// a strict total order.
__device__ __forceinline__ void wave_best(uint64_t &bk, uint32_t &br) {
  best_dpp<0xB1>(bk, br);   // quad_perm [1, 0, 3, 2]
  best_dpp<0x4E>(bk, br);   // quad_perm [2, 3, 0, 1]
  best_dpp<0x141>(bk, br);  // row_half_mirror
  best_dpp<0x140>(bk, br);  // row_mirror
#pragma unroll
  for (int o = 16; o < 64; o <<= 1) {
    const uint64_t ok = __shfl_xor(bk, o);
    const uint32_t orow = (uint32_t)__shfl_xor((int)br, o);
    const bool take = key_beats(ok, orow, bk, br);
    bk = take ? ok : bk;
    br = take ? orow : br;
  }
}

// A leaf of the panel: the columns [c0, c1) (at most L) over the rows [c0, n),
// factored by one workgroup with every entry in registers (thread t holds rows
// c0 + t + 512 j, j < RPT, of each leaf column), so the L dependent steps cost
// one barrier each instead of two kernel launches. Step c:
//   pivot: each wave reduces its rows (DPP, two shuffles); the lane holding the
//     wave's best row copies that row of the leaf to LDS (and lane c - c0,
//     which holds row c, copies row c); after the barrier every thread reduces
//     the 8 wave results itself and reads the pivot row from its wave's slot;
//   interchange of rows c and the pivot row within the leaf columns;
//   update a_ik -= l_ic a_ck of rows i > c, leaf columns k > c, with the
//     multiplier l_ic = a_ic (1 / a_cc), which replaces a_ic (every thread
//     forms the reciprocal itself).
// These are k_pivot_swap's, k_panel_update's and k_panel_scale's operations on
// the leaf columns (the multiplier is the same product whether taken at step
// c or at the end of the panel: column c is only permuted after step c), so
// the leaf ends bit for bit as it would under them; the other panel columns
// take the leaf's interchanges and updates in k_lu_trail. A
// leaf narrower than L carries zero columns up to L: they are updated like
// the others (straight-line code, no per-column tests) but never read by a
// pivot search and never stored. The LDS slots alternate between even and odd
// steps, so a thread one step ahead never overwrites a slot still being read.
// RPT is 4, 8 or 16 for leaves of 8, 4 or 2 columns (up to 2048, 4096 or 8192
// rows); a leaf of 8 columns over at most 1024 or 512 rows takes RPT 2 or 1.
constexpr int kLeafThreads = 512;

template <int RPT, int L>
__global__ void __launch_bounds__(kLeafThreads) k_lu_leaf(double2 *A, int64_t lda, int64_t n,
                                                          int64_t c0, int64_t c1, int64_t *ipiv,
                                                          int64_t *singular) {
  constexpr int NT = kLeafThreads, NW = NT / 64;
  __shared__ double2 srow[2][NW][L];
  __shared__ double2 sc[2][L];
  __shared__ uint64_t sk[2][NW];
  __shared__ uint32_t sr[2][NW];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int w = (int)(c1 - c0);
  // rows below the leaf's first row (the launch guarantees rows <= NT * RPT)
  const uint32_t rows = (uint32_t)(n - c0);
  Z x[RPT][L];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const uint32_t r = (uint32_t)(t + NT * j);
#pragma unroll
    for (int k = 0; k < L; ++k)
      x[j][k] = (r < rows && k < w) ? ld(A + c0 + r + (c0 + k) * lda) : Z{0.0, 0.0};
  }
  int64_t pivs[L];
  int first_zero = -1;
#pragma unroll
  for (int cc = 0; cc < L; ++cc) {
    if (cc >= w) break;
    const int b = cc & 1;
    uint64_t bk = 0;
    uint32_t br = kNoRow;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {  // a thread's rows in increasing order
      const uint32_t r = (uint32_t)(t + NT * j);
      const uint64_t k = pivot_key(cabs1(x[j][cc]));
      const bool take = (r >= (uint32_t)cc) & (r < rows) & key_beats(k, r, bk, br);
      bk = take ? k : bk;
      br = take ? r : br;
    }
    wave_best(bk, br);
    if (br != kNoRow && (int)(br & (NT - 1)) == t) {
      const int jb = (int)(br / NT);
#pragma unroll
      for (int j = 0; j < RPT; ++j)
        if (j == jb)
#pragma unroll
          for (int k = 0; k < L; ++k) srow[b][wave][k] = make_double2(x[j][k].re, x[j][k].im);
    }
    if (lane == 0) {
      sk[b][wave] = bk;
      sr[b][wave] = br;
    }
    if (t == cc)  // row c = c0 + cc is thread cc's first row
#pragma unroll
      for (int k = 0; k < L; ++k) sc[b][k] = make_double2(x[0][k].re, x[0][k].im);
    __syncthreads();
    uint64_t ck[NW];
    uint32_t cr[NW];
#pragma unroll
    for (int v = 0; v < NW; ++v) {  // all reads first, then the reduction
      ck[v] = sk[b][v];
      cr[v] = sr[b][v];
    }
    bk = ck[0];
    br = cr[0];
    int win = 0;
#pragma unroll
    for (int v = 1; v < NW; ++v) {
      const bool take = key_beats(ck[v], cr[v], bk, br);
      bk = take ? ck[v] : bk;
      br = take ? cr[v] : br;
      win = take ? v : win;
    }
    // row c takes part, so the pivot is a row of [c, n); the pivots go out
    // after the last step (a store in flight would hold up the next barrier).
    // A pivot of |Re| + |Im| = 0 or NaN makes the matrix singular.
    const int64_t piv = c0 + br;
    pivs[cc] = piv;
    if ((bk == 0 || bk == kNaNKey) && first_zero < 0) first_zero = cc;
    Z pr[L];  // the pivot row: row c after the interchange
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const double2 v = srow[b][win][k];
      pr[k] = Z{v.x, v.y};
    }
    if (br != (uint32_t)cc) {
      if (t == cc)
#pragma unroll
        for (int k = 0; k < L; ++k) x[0][k] = pr[k];
      if ((int)(br & (NT - 1)) == t) {
        const int jp = (int)(br / NT);
#pragma unroll
        for (int j = 0; j < RPT; ++j)
          if (j == jp)
#pragma unroll
            for (int k = 0; k < L; ++k) {
              const double2 v = sc[b][k];
              x[j][k] = Z{v.x, v.y};
            }
      }
    }
    const Z rc = zrcp(pr[cc]);
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const uint32_t r = (uint32_t)(t + NT * j);
      if (r > (uint32_t)cc && r < rows) {
        const Z l = zmul(x[j][cc], rc);
        x[j][cc] = l;  // the multiplier, final up to later interchanges
#pragma unroll
        for (int k = cc + 1; k < L; ++k) x[j][k] = zsub(x[j][k], zmul(l, pr[k]));
      }
    }
  }
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const uint32_t r = (uint32_t)(t + NT * j);
    if (r < rows)
#pragma unroll
      for (int k = 0; k < L; ++k)
        if (k < w) st(A + c0 + r + (c0 + k) * lda, x[j][k]);
  }
  if (t == 0) {
#pragma unroll
    for (int cc = 0; cc < L; ++cc)
      if (cc < w) ipiv[c0 + cc] = pivs[cc];
    if (first_zero >= 0)
      atomicMin(reinterpret_cast<unsigned long long *>(singular), (unsigned long long)(c0 + first_zero));
  }
}

// The other panel columns after the leaf [c0, c1) (w = c1 - c0 <= L), one
// workgroup per column k: k in [p0, c0) takes the leaf's interchanges only; k
// in [c1, p1) takes them and then the leaf's steps c = c0 .. c1-1 in order,
// a_ik -= l_ic a_ck for rows i > c with the multipliers the leaf stored, as
// k_pivot_swap and k_panel_update would have applied them one column at a
// time. Exchanging all rows first and updating afterwards gives the same
// entries: every row exchanged at step c is below every earlier pivot row, so
// both take each earlier step's update with the multiplier that moves with
// them. The interchanges touch at most 2 w rows ("slots": rows c0 .. c1-1,
// then each pivot row below c1 once); thread s < 2w finds which slot's entry
// ends in slot s by running the exchanges backwards on the slot index, so the
// exchange is one gather. Rows c0 .. c1-1 then form a chain of w dependent
// steps, run by the first w lanes of wave 0 with shuffles; each row below c1
// subtracts its w terms in the order of c.
constexpr int kTrailThreads = 512, kTrailRows = 4;

template <int L>
__global__ void __launch_bounds__(kTrailThreads) k_lu_trail(double2 *A, int64_t lda, int64_t n, int64_t c0,
                                                  int64_t c1, int64_t p0, const int64_t *ipiv) {
  __shared__ double2 lm[L][L];  // leaf multipliers l_rc, r > c
  __shared__ double2 u[L];
  const int t = threadIdx.x;
  const int w = (int)(c1 - c0);
  const int64_t b = blockIdx.x;
  const bool left = b < c0 - p0;
  const int64_t k = left ? p0 + b : c1 + (b - (c0 - p0));
  double2 *col = A + k * lda;
  // The interchanges touch at most 2 w <= 16 slots, so wave 0 alone works
  // out the slots and gathers (the slot logic is uniform scalar code: the
  // other waves would only queue on the CU's scalar unit behind it).
  int m = 0;
  Z val{0.0, 0.0};
  int64_t row = 0;
  if (t < 64) {
    // the w pivots (an entry outside [c, n) is no exchange)
    int64_t pv[L];
#pragma unroll
    for (int q = 0; q < L; ++q) {
      const int64_t p = q < w ? ipiv[c0 + q] : c0 + q;
      pv[q] = (p < c0 + q || p >= n) ? c0 + q : p;
    }
    if (!left && t < w * w) {
      const int r = t % w, q = t / w;
      if (r > q) lm[r][q] = A[c0 + r + (c0 + q) * lda];
    }
    // slot of each exchange's pivot row: p - c0 inside the leaf, else w + the
    // number of distinct pivot rows below c1 named before it first is. nw[e]:
    // exchange e names a row below c1 that no earlier exchange named (O(L^2)
    // compares in straight-line code).
    bool nw[L];
    m = w;
#pragma unroll
    for (int e = 0; e < L; ++e) {
      bool fresh = e < w && pv[e] >= c1;
#pragma unroll
      for (int f = 0; f < e; ++f) fresh = fresh && pv[f] != pv[e];
      nw[e] = fresh;
      m += fresh ? 1 : 0;
    }
    int ps[L];
#pragma unroll
    for (int q = 0; q < L; ++q) {
      int first = q;  // the first exchange naming pv[q]
#pragma unroll
      for (int e = q - 1; e >= 0; --e) first = pv[e] == pv[q] ? e : first;
      int rank = 0;
#pragma unroll
      for (int e = 0; e < q; ++e) rank += (nw[e] && e < first) ? 1 : 0;
      ps[q] = q < w ? (pv[q] < c1 ? (int)(pv[q] - c0) : w + rank) : q;
    }
    // thread t < m: the row of slot t and the slot whose entry ends there
    if (t < m) {
      if (t < w) {
        row = c0 + t;
      } else {
#pragma unroll
        for (int q = 0; q < L; ++q)
          if (q < w && ps[q] == t) row = pv[q];
      }
      int src = t;
#pragma unroll
      for (int q = L - 1; q >= 0; --q)
        if (q < w) src = src == q ? ps[q] : (src == ps[q] ? q : src);
      int64_t srow = c0 + src;
      if (src >= w)
#pragma unroll
        for (int q = 0; q < L; ++q)
          if (q < w && ps[q] == src) srow = pv[q];
      val = ld(col + srow);
    }
  }
  __syncthreads();  // every slot read before any is overwritten
  if (left) {
    if (t < m) st(col + row, val);
    return;
  }
  if (t >= w && t < m) st(col + row, val);
  if (t < 64) {
    Z xr = val;
#pragma unroll
    for (int q = 0; q < L; ++q) {
      if (q >= w) break;
      const double ure = __shfl(xr.re, q), uim = __shfl(xr.im, q);
      if (t > q && t < w) {
        const double2 l = lm[t][q];
        xr = zsub(xr, zmul(Z{l.x, l.y}, Z{ure, uim}));
      }
    }
    if (t < w) {
      u[t] = make_double2(xr.re, xr.im);
      st(col + c0 + t, xr);
    }
  }
  __syncthreads();
  // kTrailRows rows per thread per pass, every load of a pass issued before
  // any use (a row past n reads row n - 1 and stores nothing)
  for (int64_t i0 = c1 + t; i0 < n; i0 += kTrailRows * kTrailThreads) {
    Z a[kTrailRows][L], y[kTrailRows];
#pragma unroll
    for (int h = 0; h < kTrailRows; ++h) {
      const int64_t i = std::min<int64_t>(i0 + h * kTrailThreads, n - 1);
#pragma unroll
      for (int q = 0; q < L; ++q)
        if (q < w) a[h][q] = ld(A + i + (c0 + q) * lda);
      y[h] = ld(col + i);
    }
#pragma unroll
    for (int h = 0; h < kTrailRows; ++h) {
      const int64_t i = i0 + h * kTrailThreads;
#pragma unroll
      for (int q = 0; q < L; ++q)
        if (q < w) {
          const double2 uq = u[q];
          y[h] = zsub(y[h], zmul(a[h][q], Z{uq.x, uq.y}));
        }
      if (i < n) st(col + i, y[h]);
    }
  }
}

// The row interchanges ipiv[c0..c1) (rows c and ipiv[c] exchanged for c =
// c0, c0+1, ... in turn, ipiv[c] in [c, n)) as one gather: row dst[e] of the
// result is row src[e] of the input, for the w = c1 - c0 <= 1024 slots
// e = t (dst = c0 + t) and the slots e = w + t (dst = ipiv[c0 + t] when that
// row lies below c1 and no later interchange names it; dst = -1 otherwise).
// Derivation, with t' < t meaning an earlier interchange: row c0 + t is final
// after interchange t, when it takes what row ipiv[c0 + t] held just before.
// Let E(t) be what row c0 + t held just before interchange t: its own row if
// no earlier interchange named it, else E of the latest one that did (a chain
// of decreasing t, resolved by pointer jumping). Row x >= c0 + t holds, just
// before interchange t, E(t') for the latest t' < t with ipiv[c0 + t'] = x, or
// x itself if there is none. One workgroup of w threads rounded up to a
// wave, thread t for interchange t, each scanning the w pivots in LDS. An
// entry outside [c, n) counts as no interchange.
__global__ void __launch_bounds__(1024) k_swap_pairs(const int64_t *ipiv, int64_t c0, int64_t c1,
                                                     int64_t n, int64_t *dst, int64_t *src) {
  __shared__ int64_t piv[1024];
  __shared__ int nxt[1024];
  const int w = (int)(c1 - c0);
  const int t = threadIdx.x;
  int64_t pt = -1;
  if (t < w) {
    pt = ipiv[c0 + t];
    if (pt < c0 + t || pt >= n) pt = c0 + t;
    piv[t] = pt;
  }
  __syncthreads();
  int named_by = -1, prev_same = -1;
  bool last = true;
  if (t < w) {
    for (int u = 0; u < w; ++u) {
      const int64_t pu = piv[u];
      if (u < t) {
        if (pu == c0 + t) named_by = u;
        if (pu == pt) prev_same = u;
      } else if (u > t && pu == pt) {
        last = false;
      }
    }
  }
  nxt[t] = named_by >= 0 ? named_by : t;
  __syncthreads();
  for (int r = 1; r < w; r <<= 1) {  // a chain has fewer than w links
    const int v = nxt[nxt[t]];
    __syncthreads();
    nxt[t] = v;
    __syncthreads();
  }
  if (t < w) {
    dst[t] = c0 + t;
    src[t] = prev_same >= 0 ? c0 + nxt[prev_same] : pt;
    const bool below = pt >= c1 && last;
    dst[w + t] = below ? pt : -1;
    src[w + t] = below ? c0 + nxt[t] : -1;
  }
}

// Applies the gather of k_swap_pairs (2w <= 2048 slots) to the columns
// [q0, q1) and [q2, q3) of A, one workgroup per column: every thread reads its
// slots' source rows, waits for them, and after the barrier writes them.
__global__ void __launch_bounds__(256) k_apply_pairs(double2 *A, int64_t lda, int slots,
                                                     const int64_t *dst, const int64_t *src,
                                                     int64_t q0, int64_t q1, int64_t q2) {
  const int64_t b = blockIdx.x;
  const int64_t k = b < q1 - q0 ? q0 + b : q2 + (b - (q1 - q0));
  double2 *col = A + k * lda;
  double2 v[8];
  int64_t d[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int e = threadIdx.x + 256 * j;
    d[j] = -1;
    if (e < slots) {
      const int64_t de = dst[e], se = src[e];
      if (de >= 0 && de != se) {
        d[j] = de;
        v[j] = col[se];
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (d[j] >= 0) col[d[j]] = v[j];
}

// Lane l's value of v, read by every lane (l uniform): two v_readlane.
__device__ __forceinline__ double readlane_d(double v, int l) {
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// X <- T^-1 X for the nb x nb triangle T (at T, leading dimension ldt) on
// ncols columns of X, column-oriented. Unit lower (forward): for k = 0, 1,
// ..., x_k is final and every x_r with r > k takes x_r -= t_rk x_k. Non-unit
// upper (backward): for k = nb-1 down to 0, x_k = x_k / t_kk is final and
// every x_r with r < k takes x_r -= t_rk x_k. Each x_r thus subtracts its
// terms in the order of k (forward: increasing, backward: decreasing). One
// wave per CW columns of X: lane l holds x_r of each of them for the rows
// r = l + 64 j (j < R, nb <= 64 R), so a step needs no barrier: the final x_k
// comes from its lane by v_readlane and every lane updates its own rows. Each
// t_rk is loaded once per wave and used for all CW columns. Each lane loads
// its t_rk kPre steps ahead into a ring of registers (one load per row slot
// and step; rows past nb read row nb - 1, steps past the last read the last
// column), so the L2 latency of T is off the chain of steps. One column per
// wave measured fastest: with four, the waves were a quarter as many and each
// step four times longer (2048 KKR inverse: upper solves 53 -> 87 us).
constexpr int kTrsmCols = 1;

template <bool UPPER, int R>
__global__ void __launch_bounds__(256) k_trsm(const double2 *T, int64_t ldt, int nb, double2 *X,
                                              int64_t ldx, int64_t ncols) {
  constexpr int CW = kTrsmCols;
  constexpr int kPre = R <= 2 ? 8 : (R >= 16 ? 1 : 16 / R);
  const int lane = threadIdx.x & 63;
  const int64_t c0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * CW;
  if (c0 >= ncols) return;  // a whole wave
  Z xr[R][CW], dg[R];
  int rr[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int r = lane + 64 * j;
    rr[j] = r < nb ? r : nb - 1;
#pragma unroll
    for (int c = 0; c < CW; ++c)
      xr[j][c] = (r < nb && c0 + c < ncols) ? ld(X + (c0 + c) * ldx + r) : Z{0.0, 0.0};
    dg[j] = UPPER ? ld(T + rr[j] + (int64_t)rr[j] * ldt) : Z{1.0, 0.0};
  }
  const int steps = UPPER ? nb : nb - 1;
  auto col = [&](int s) { return UPPER ? nb - 1 - s : s; };
  if (steps > 0) {
    Z ring[kPre][R];
#pragma unroll
    for (int p = 0; p < kPre; ++p) {
      const int64_t kk = col(p < steps ? p : steps - 1);
#pragma unroll
      for (int j = 0; j < R; ++j) ring[p][j] = ld(T + rr[j] + kk * ldt);
      // slot order kept: the loop's waits count on slot 0 being the oldest
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int s0 = 0; s0 < steps; s0 += kPre) {
#pragma unroll
      for (int p = 0; p < kPre; ++p) {
        const int s = s0 + p;
        if (s < steps) {
          const int k = col(s);
          const int kl = k & 63, ks = k >> 6;
          if constexpr (UPPER) {
#pragma unroll
            for (int j = 0; j < R; ++j)
              if (j == ks && lane == kl)
#pragma unroll
                for (int c = 0; c < CW; ++c) xr[j][c] = zdiv(xr[j][c], dg[j]);
          }
          Z u[CW];
#pragma unroll
          for (int c = 0; c < CW; ++c) {
            Z cur = xr[0][c];
#pragma unroll
            for (int j = 1; j < R; ++j)
              if (j == ks) cur = xr[j][c];
            u[c] = Z{readlane_d(cur.re, kl), readlane_d(cur.im, kl)};
          }
#pragma unroll
          for (int j = 0; j < R; ++j) {
            const int r = lane + 64 * j;
            if (r < nb && (UPPER ? r < k : r > k))
#pragma unroll
              for (int c = 0; c < CW; ++c) xr[j][c] = zsub(xr[j][c], zmul(ring[p][j], u[c]));
          }
        }
        // the slot's next load goes out once its value is used; the scheduling
        // barrier keeps the compiler from hoisting it above the use, where the
        // in-order load counter would make this step wait for every newer
        // prefetch
        __builtin_amdgcn_sched_barrier(0);
        const int sn = s + kPre < steps ? s + kPre : steps - 1;
        const int64_t kk = col(sn);
#pragma unroll
        for (int j = 0; j < R; ++j) ring[p][j] = ld(T + rr[j] + kk * ldt);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j)
    if (lane + 64 * j < nb)
#pragma unroll
      for (int c = 0; c < CW; ++c)
        if (c0 + c < ncols) st(X + (c0 + c) * ldx + lane + 64 * j, xr[j][c]);
}

// X = identity (n x n, leading dimension ldx).
__global__ void __launch_bounds__(256) k_identity(double2 *X, int64_t ldx, int64_t n) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx % n, j = idx / n;
  X[i + j * ldx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
}

__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, st, p, v);
  return hipGetLastError();
}

hipError_t launch_lu_column(double2 *A, int64_t lda, int64_t n, int64_t c, int64_t p0, int64_t p1,
                            int64_t *ipiv, int64_t *singular, hipStream_t st) {
  hipLaunchKernelGGL(k_pivot_swap, dim3(1), dim3(256), 0, st, A, lda, n, c, p0, p1, ipiv, singular);
  if (c + 1 < n && c + 1 < p1)
    hipLaunchKernelGGL(k_panel_update, dim3(blocks(n - c - 1), (unsigned)(p1 - c - 1)), dim3(256), 0, st,
                       A, lda, n, c);
  return hipGetLastError();
}

static int lu_leaf_width(int64_t rows, int mode) {
  // the widest leaf whose rows fit in registers: 512 threads x RPT rows
  if (mode == kLuPanelColumns) return 0;
  if (mode == kLuPanelLeaf8 || mode == kLuPanelAuto) {
    if (rows <= 2048) return 8;
    if (mode == kLuPanelLeaf8) return 0;
  }
  if (mode == kLuPanelLeaf4 || mode == kLuPanelAuto) {
    if (rows <= 4096) return 4;
    if (mode == kLuPanelLeaf4) return 0;
  }
  return rows <= 8192 ? 2 : 0;
}

hipError_t launch_lu_panel(double2 *A, int64_t lda, int64_t n, int64_t p0, int64_t p1, int64_t *ipiv,
                           int64_t *singular, int mode, hipStream_t st) {
  // the rows below a column only shrink, so the columns taken one at a time
  // (rows that do not fit a leaf) are a prefix [p0, pc) of the panel
  int64_t c0 = p0, pc = p0;
  while (c0 < p1) {
    const int L = lu_leaf_width(n - c0, mode);
    if (L == 0) {
      const hipError_t e = launch_lu_column(A, lda, n, c0, p0, p1, ipiv, singular, st);
      if (e != hipSuccess) return e;
      pc = ++c0;
      continue;
    }
    const int64_t c1 = std::min(p1, c0 + L);
    const dim3 lb(kLeafThreads);
    switch (L) {
      case 8:
        if (n - c0 <= kLeafThreads)
          hipLaunchKernelGGL((k_lu_leaf<1, 8>), dim3(1), lb, 0, st, A, lda, n, c0, c1, ipiv, singular);
        else if (n - c0 <= 2 * kLeafThreads)
          hipLaunchKernelGGL((k_lu_leaf<2, 8>), dim3(1), lb, 0, st, A, lda, n, c0, c1, ipiv, singular);
        else
          hipLaunchKernelGGL((k_lu_leaf<4, 8>), dim3(1), lb, 0, st, A, lda, n, c0, c1, ipiv, singular);
        break;
      case 4: hipLaunchKernelGGL((k_lu_leaf<8, 4>), dim3(1), lb, 0, st, A, lda, n, c0, c1, ipiv, singular); break;
      default: hipLaunchKernelGGL((k_lu_leaf<16, 2>), dim3(1), lb, 0, st, A, lda, n, c0, c1, ipiv, singular); break;
    }
    const int64_t cols = (c0 - p0) + (p1 - c1);
    if (cols > 0) {
      const dim3 g((unsigned)cols), tb(kTrailThreads);
      switch (L) {
        case 8: hipLaunchKernelGGL(k_lu_trail<8>, g, tb, 0, st, A, lda, n, c0, c1, p0, ipiv); break;
        case 4: hipLaunchKernelGGL(k_lu_trail<4>, g, tb, 0, st, A, lda, n, c0, c1, p0, ipiv); break;
        default: hipLaunchKernelGGL(k_lu_trail<2>, g, tb, 0, st, A, lda, n, c0, c1, p0, ipiv); break;
      }
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    c0 = c1;
  }
  // the leaves stored their multipliers; the prefix's columns still hold the
  // unscaled entries
  return launch_lu_scale(A, lda, n, p0, pc, st);
}

hipError_t launch_lu_scale(double2 *A, int64_t lda, int64_t n, int64_t p0, int64_t p1, hipStream_t st) {
  if (p0 + 1 >= n || p1 <= p0) return hipSuccess;
  hipLaunchKernelGGL(k_panel_scale, dim3(blocks(n - p0 - 1), (unsigned)(p1 - p0)), dim3(256), 0, st, A,
                     lda, n, p0);
  return hipGetLastError();
}

hipError_t launch_swap_pairs(const int64_t *ipiv, int64_t c0, int64_t c1, int64_t n,
                             int64_t *pairs, hipStream_t st) {
  if (c1 <= c0) return hipSuccess;
  if (c1 - c0 > kLuMaxBlock) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_swap_pairs, dim3(1), dim3((unsigned)((c1 - c0 + 63) / 64 * 64)), 0, st, ipiv,
                     c0, c1, n, pairs,
                     pairs + 2 * kLuMaxBlock);
  return hipGetLastError();
}

hipError_t launch_apply_pairs(double2 *A, int64_t lda, int64_t w, const int64_t *pairs, int64_t q0,
                              int64_t q1, int64_t q2, int64_t q3, hipStream_t st) {
  const int64_t cols = std::max<int64_t>(0, q1 - q0) + std::max<int64_t>(0, q3 - q2);
  if (cols == 0 || w <= 0) return hipSuccess;
  if (w > kLuMaxBlock || cols > 0x7fffffffll) return hipErrorInvalidValue;
  if (q1 < q0) q1 = q0;
  hipLaunchKernelGGL(k_apply_pairs, dim3((unsigned)cols), dim3(256), 0, st, A, lda, (int)(2 * w),
                     pairs, pairs + 2 * kLuMaxBlock, q0, q1, q2);
  return hipGetLastError();
}

hipError_t launch_trsm(bool upper, const double2 *T, int64_t ldt, int64_t nb, double2 *X,
                       int64_t ldx, int64_t ncols, hipStream_t st) {
  if (ncols <= 0 || nb <= 0) return hipSuccess;
  const int64_t waves = (ncols + kTrsmCols - 1) / kTrsmCols;
  if (nb > kLuMaxBlock || (waves + 3) / 4 > 0x7fffffffll) return hipErrorInvalidValue;
  const dim3 g((unsigned)((waves + 3) / 4)), b(256);
  const int n = (int)nb;
#define OZ_TRSM(RR)                                                                            \
  if (upper)                                                                                   \
    hipLaunchKernelGGL((k_trsm<true, RR>), g, b, 0, st, T, ldt, n, X, ldx, ncols);            \
  else                                                                                         \
    hipLaunchKernelGGL((k_trsm<false, RR>), g, b, 0, st, T, ldt, n, X, ldx, ncols);
  if (nb <= 64) {
    OZ_TRSM(1)
  } else if (nb <= 128) {
    OZ_TRSM(2)
  } else if (nb <= 256) {
    OZ_TRSM(4)
  } else if (nb <= 512) {
    OZ_TRSM(8)
  } else {
    OZ_TRSM(16)
  }
#undef OZ_TRSM
  return hipGetLastError();
}

hipError_t launch_identity(double2 *X, int64_t ldx, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_identity, dim3(blocks(n * n)), dim3(256), 0, st, X, ldx, n);
  return hipGetLastError();
}

}  // namespace oz
