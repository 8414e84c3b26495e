// Exponent scan, slicing and small helper kernels of libozaki (gfx950).
//
// Steps "exponent alignment" and "split into slices by significant bits" of
// the Ozaki-I scheme (Section 2.2 of the paper). Both are HBM-bound: the scan
// reads each operand once, the split reads it again and writes S (real) or
// 2S (complex) bytes per element in the packed fragment layout.
#include "ozaki_internal.hpp"

namespace oz {

namespace {

__global__ void __launch_bounds__(256) k_fill_i32(int *p, int64_t n, int value) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = value;
}

// Pseudo-random INT8 digits in [-127, 127] (SplitMix64 finaliser of the byte
// index): stand-in slice data for timing the slice GEMM, whose power draw and
// clock depend on the operand bits.
// Grid-stride: the fills of large workspaces exceed the grid size limit.
__global__ void __launch_bounds__(256) k_fill_digits(int8_t *p, int64_t n, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    uint64_t z = seed + 0x9e3779b97f4a7c15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    p[i] = (int8_t)((int)(z % 255u) - 127);
  }
}

template <bool CPLX>
__device__ __forceinline__ int elem_code(const void *base, int64_t off) {
  if (CPLX) {
    const double2 z = reinterpret_cast<const double2 *>(base)[off];
    return max(expo_code(z.x), expo_code(z.y));
  }
  return expo_code(reinterpret_cast<const double *>(base)[off]);
}

// Rows are unit-stride in memory (sr == 1): 64 consecutive rows per block,
// four threads per row walking the contraction index; each warp-wide load is
// one contiguous run of 64 elements.
// `direct`: the block covers the whole contraction range, so the row code is
// stored instead of max-combined with other blocks.
template <bool CPLX>
__device__ __forceinline__ void scan_rowsfast_block(const View &v, int64_t rb, int64_t l0,
                                                    int64_t l1, int *code, bool direct) {
  const int tid = threadIdx.x;
  const int64_t r = rb * 64 + (tid & 63);
  int c = 0;
  if (r < v.R) {
    // eight loads in flight per pass (a block that covers a long contraction
    // alone is latency-bound), then four, then the remainder
    int64_t l = l0 + (tid >> 6);
    for (; l + 28 < l1; l += 32) {
      int a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = elem_code<CPLX>(v.base, r + (l + 4 * q) * v.sl);
      c = max(c, max(max(max(a[0], a[1]), max(a[2], a[3])), max(max(a[4], a[5]), max(a[6], a[7]))));
    }
    for (; l + 12 < l1; l += 16) {
      const int a0 = elem_code<CPLX>(v.base, r + l * v.sl);
      const int a1 = elem_code<CPLX>(v.base, r + (l + 4) * v.sl);
      const int a2 = elem_code<CPLX>(v.base, r + (l + 8) * v.sl);
      const int a3 = elem_code<CPLX>(v.base, r + (l + 12) * v.sl);
      c = max(c, max(max(a0, a1), max(a2, a3)));
    }
    for (; l < l1; l += 4) c = max(c, elem_code<CPLX>(v.base, r + l * v.sl));
  }
  __shared__ int red[256];
  red[tid] = c;
  __syncthreads();
  if (tid < 64) {
    c = max(max(red[tid], red[tid + 64]), max(red[tid + 128], red[tid + 192]));
    if (r < v.R) {
      if (direct)
        code[r] = c;
      else if (c > 0)
        atomicMax(code + r, c);
    }
  }
}

template <bool CPLX>
__global__ void __launch_bounds__(256) k_scan_rowsfast(View v, int64_t lchunk, int *code) {
  const int64_t l0 = (int64_t)blockIdx.y * lchunk;
  scan_rowsfast_block<CPLX>(v, blockIdx.x, l0, min(v.L, l0 + lchunk), code, false);
}

// Each row is unit-stride (sl == 1): one wave per row and contraction chunk,
// lanes read consecutive elements, a wave max-reduction gives the row code.
template <bool CPLX>
__device__ __forceinline__ void scan_rowcontig_block(const View &v, int64_t rb, int64_t l0,
                                                     int64_t l1, int *code, bool direct) {
  const int lane = threadIdx.x & 63;
  const int64_t r = rb * 4 + (threadIdx.x >> 6);
  if (r >= v.R) return;
  int c = 0;
  int64_t l = l0 + lane;
  for (; l + 192 < l1; l += 256) {  // four loads in flight per pass
    const int a0 = elem_code<CPLX>(v.base, r * v.sr + l);
    const int a1 = elem_code<CPLX>(v.base, r * v.sr + l + 64);
    const int a2 = elem_code<CPLX>(v.base, r * v.sr + l + 128);
    const int a3 = elem_code<CPLX>(v.base, r * v.sr + l + 192);
    c = max(c, max(max(a0, a1), max(a2, a3)));
  }
  for (; l < l1; l += 64) c = max(c, elem_code<CPLX>(v.base, r * v.sr + l));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c = max(c, __shfl_xor(c, off));
  if (lane == 0) {
    if (direct)
      code[r] = c;
    else if (c > 0)
      atomicMax(code + r, c);
  }
}

template <bool CPLX>
__global__ void __launch_bounds__(256) k_scan_rowcontig(View v, int64_t lchunk, int *code) {
  const int64_t l0 = (int64_t)blockIdx.y * lchunk;
  scan_rowcontig_block<CPLX>(v, blockIdx.x, l0, min(v.L, l0 + lchunk), code, false);
}

// One thread per (packed row, 16 consecutive packed contraction entries):
// reads the 16 source values (8 complex elements), splits each into S digits
// and writes one 16-byte run per slice into the packed fragment layout.
// Rows and entries beyond the operand are written as zero digits (padding).
// Per-byte negation of four packed digits in [0, 127]: bytes whose mask byte
// is 0xff become (-d) mod 256. (d ^ 0x7f) + 1 = 128 - d never carries out of
// its byte, and xor 0x80 then adds 128.
__device__ __forceinline__ uint32_t neg_bytes(uint32_t w, uint32_t mask) {
  return ((w ^ (mask & 0x7f7f7f7fu)) + (mask & 0x01010101u)) ^ (mask & 0x80808080u);
}

// floor(|x| 2^(7S)) for S <= 9 (at most 63 bits): the top 7S bits of |x|
// below the binary point as one integer, so digit p is bits
// [7(S-p), 7(S-p)+7) of it.
template <int S>
__device__ __forceinline__ uint64_t top_bits(const Sig &x) {
  const int sh = x.sh0 + kDigitBits * S;
  if (sh >= 0) return x.m << sh;  // sh <= 7S - 53 <= 10: no overflow
  return (sh > -64) ? (x.m >> (-sh)) : 0ull;
}

// trunc(|x| 2^NB) for NB <= 62 (|x| < 1 after the exponent shift, so the
// result stays below 2^NB).
template <int NB>
__device__ __forceinline__ uint64_t top_nbits(const Sig &x) {
  const int sh = x.sh0 + NB;
  if (sh >= 0) return x.m << sh;
  return (sh > -64) ? (x.m >> (-sh)) : 0ull;
}

// View rows and contraction entries (elements) covered by one split block.
template <bool CPLX, bool SIDEB>
struct SplitTile {
  static constexpr int TR = (CPLX && SIDEB) ? 32 : 64;  // view rows
  static constexpr int TL = CPLX ? 32 : 64;              // contraction elements
  static constexpr int EW = CPLX ? 2 : 1;                // doubles per element
  static constexpr int PITCH = (TL + 1) * EW;            // doubles per LDS row (padded)
};
constexpr int kSplitTileDoubles = 64 * 33 * 2;  // the largest tile (complex, 64 rows)

// When the contraction is the unit-stride direction (sl == 1) a thread's 16
// packed entries lie along one row in memory, and the lanes of a wave would
// read 64 different rows. The block then first copies its tile into LDS with
// consecutive threads on consecutive elements of a row (coalesced), and the
// threads take their values from there. Rows or elements outside the view
// are stored as zeros.
// Every load is issued before the first store to LDS (an element outside the
// view reads element (0, 0) and is stored as zero), so a thread's loads are in
// flight together.
template <bool CPLX, bool SIDEB>
__device__ __forceinline__ void load_split_tile(const View &v, int64_t bx, int64_t by, double *tile) {
  using T = SplitTile<CPLX, SIDEB>;
  using E = typename std::conditional<CPLX, double2, double>::type;
  constexpr int IT = T::TR * T::TL / 256;
  static_assert(T::TR * T::TL % 256 == 0, "whole passes");
  const int64_t r0 = bx * T::TR, l0 = by * T::TL;
  E val[IT];
  bool in[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int c = threadIdx.x + 256 * it;
    const int64_t r = r0 + c / T::TL, l = l0 + c % T::TL;
    in[it] = r < v.R && l < v.L;
    val[it] = reinterpret_cast<const E *>(v.base)[in[it] ? r * v.sr + l : 0];
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int c = threadIdx.x + 256 * it;
    const int rr = c / T::TL, ll = c % T::TL;
    if constexpr (CPLX)
      *reinterpret_cast<double2 *>(tile + rr * T::PITCH + ll * 2) =
          in[it] ? val[it] : make_double2(0.0, 0.0);
    else
      tile[rr * T::PITCH + ll] = in[it] ? val[it] : 0.0;
  }
  __syncthreads();
}

template <bool CPLX, bool SIDEB, int SC, bool TRP, bool B8>
__device__ __forceinline__ void split_block(const View &v, const int *code, int S, int8_t *out,
                                            int64_t nrb, int64_t nkb, int64_t bx, int64_t by,
                                            const double *tile) {
  const int tid = threadIdx.x;
  const int64_t rp = bx * 64 + (tid & 63);
  const int64_t kp0 = (by * 4 + (tid >> 6)) * 16;
  const int64_t Rrows = (CPLX && SIDEB) ? 2 * v.R : v.R;
  const int64_t r = (CPLX && SIDEB) ? (rp >> 1) : rp;
  const int cr = (CPLX && SIDEB) ? (int)(rp & 1) : 0;
  const int c = (rp < Rrows) ? code[r] : 0;
  const bool live = (rp < Rrows) && !code_bad(c);
  const int e = code_exp(c);

  Sig sg[16];
  if (CPLX) {
    const double2 *X = reinterpret_cast<const double2 *>(v.base);
    // every load of the thread is issued before any is used (an entry outside
    // the view reads element (0, 0), or its zero in the staged tile, and
    // counts as zero)
    double2 zs[8];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      const int64_t l = (kp0 >> 1) + x;
      if constexpr (TRP) {
        using T = SplitTile<CPLX, SIDEB>;
        zs[x] = *reinterpret_cast<const double2 *>(tile + (r - bx * T::TR) * T::PITCH +
                                                   (l - by * T::TL) * 2);
      } else {
        zs[x] = X[(live && l < v.L) ? r * v.sr + l * v.sl : 0];
      }
    }
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      const int64_t l = (kp0 >> 1) + x;
      const bool ok = live && l < v.L;
      const double re = ok ? zs[x].x : 0.0;
      const double im = ok ? (v.conj ? -zs[x].y : zs[x].y) : 0.0;
      double v0, v1;
      if (!SIDEB) {
        v0 = re;
        v1 = im;
      } else if (cr == 0) {
        v0 = re;
        v1 = -im;
      } else {
        v0 = im;
        v1 = re;
      }
      sg[2 * x] = decompose(v0, e);
      sg[2 * x + 1] = decompose(v1, e);
    }
  } else {
    const double *X = reinterpret_cast<const double *>(v.base);
    double vs[16];
#pragma unroll
    for (int x = 0; x < 16; ++x) {
      const int64_t l = kp0 + x;
      if constexpr (TRP) {
        using T = SplitTile<CPLX, SIDEB>;
        vs[x] = tile[(r - bx * T::TR) * T::PITCH + (l - by * T::TL)];
      } else {
        vs[x] = X[(live && l < v.L) ? r * v.sr + l * v.sl : 0];
      }
    }
#pragma unroll
    for (int x = 0; x < 16; ++x) {
      const int64_t l = kp0 + x;
      sg[x] = decompose((live && l < v.L) ? vs[x] : 0.0, e);
    }
  }

  if constexpr (B8) {
    // 8-bit balanced slices: X = trunc(x 2^(8S - 2)) with the sign of x, and
    // its balanced base-256 digits d_p in [-128, 127] (slice p holds the digit
    // of weight 256^(S - p)). With Y = X + 128 (256^S - 1) / 255, which lies in
    // [0, 256^S) because |X| < 2^(8S - 2), the plain base-256 bytes b_p of Y
    // are d_p + 128: the same digits as the recurrence d = ((X + 128) mod 256)
    // - 128, X <- (X - d) / 256, read off as bytes, with d_p = b_p - 128 being
    // b_p XOR 0x80 in two's complement. Every value is split as it stands, so
    // the -Im row of complex B gets the digits of -Im.
    static_assert(SC >= 1 && SC <= 8, "8-bit slices need 8S - 2 <= 62");
    constexpr uint64_t kBias = 0x8080808080808080ull >> (8 * (8 - SC));  // 128 (256^S - 1) / 255
    uint64_t Y[16];
#pragma unroll
    for (int x = 0; x < 16; ++x) {
      const uint64_t u = top_nbits<8 * SC - 2>(sg[x]);
      Y[x] = (sg[x].neg ? (0ull - u) : u) + kBias;  // mod 2^64; the true value is in [0, 256^S)
    }
#pragma unroll
    for (int p = SC; p >= 1; --p) {
      const int sh = 8 * (SC - p);
      uint32_t w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) word |= ((uint32_t)(Y[4 * q + b] >> sh) & 0xffu) << (8 * b);
        w[q] = word ^ 0x80808080u;
      }
      int8_t *dst = out + frag_offset(p - 1, rp, kp0, nrb, nkb);
      *reinterpret_cast<uint4 *>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  } else if constexpr (SC > 0) {
    // S known at compile time and 7S <= 63: one integer per value, digits by
    // constant shifts, signs applied four bytes at a time.
    uint64_t T[16];
    uint32_t neg[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t mk = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        T[4 * q + b] = top_bits<SC>(sg[4 * q + b]);
        mk |= (sg[4 * q + b].neg ? 0xffu : 0u) << (8 * b);
      }
      neg[q] = mk;
    }
#pragma unroll
    for (int p = 1; p <= SC; ++p) {
      uint32_t w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
          word |= ((uint32_t)(T[4 * q + b] >> (kDigitBits * (SC - p))) & 127u) << (8 * b);
        w[q] = neg_bytes(word, neg[q]);
      }
      int8_t *dst = out + frag_offset(p - 1, rp, kp0, nrb, nkb);
      *reinterpret_cast<uint4 *>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  } else {
    for (int p = 1; p <= S; ++p) {
      uint32_t w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) word |= ((uint32_t)digit(sg[4 * q + b], p) & 0xffu) << (8 * b);
        w[q] = word;
      }
      int8_t *dst = out + frag_offset(p - 1, rp, kp0, nrb, nkb);
      *reinterpret_cast<uint4 *>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
}

template <bool CPLX, bool SIDEB, bool TRP, bool B8>
__device__ __forceinline__ void split_s(const View &v, const int *code, int S, int8_t *out,
                                        int64_t nrb, int64_t nkb, int64_t bx, int64_t by,
                                        const double *tile) {
  if constexpr (B8) {
    // 1..8 slices (the host rejects more)
    switch (S) {
#define OZ_SPLIT(N) \
  case N: split_block<CPLX, SIDEB, N, TRP, true>(v, code, S, out, nrb, nkb, bx, by, tile); break;
      OZ_SPLIT(1) OZ_SPLIT(2) OZ_SPLIT(3) OZ_SPLIT(4) OZ_SPLIT(5) OZ_SPLIT(6) OZ_SPLIT(7)
      OZ_SPLIT(8)
#undef OZ_SPLIT
      default: break;
    }
  } else {
    switch (S) {
#define OZ_SPLIT(N) \
  case N: split_block<CPLX, SIDEB, N, TRP, false>(v, code, S, out, nrb, nkb, bx, by, tile); break;
      OZ_SPLIT(1) OZ_SPLIT(2) OZ_SPLIT(3) OZ_SPLIT(4) OZ_SPLIT(5) OZ_SPLIT(6) OZ_SPLIT(7)
      OZ_SPLIT(8) OZ_SPLIT(9)
#undef OZ_SPLIT
      default: split_block<CPLX, SIDEB, 0, TRP, false>(v, code, S, out, nrb, nkb, bx, by, tile); break;
    }
  }
}

// The LDS-staged form is taken when the contraction is unit-stride and the
// rows are not (the choice is uniform over the block) and the caller provides
// the LDS tile.
__host__ __device__ __forceinline__ bool split_staged(const View &v) {
  return v.sl == 1 && v.sr != 1;
}

template <bool CPLX, bool SIDEB, bool B8 = false>
__device__ __forceinline__ void split_dispatch(const View &v, const int *code, int S, int8_t *out,
                                               int64_t nrb, int64_t nkb, int64_t bx, int64_t by,
                                               double *tile) {
  if (tile != nullptr && split_staged(v)) {
    load_split_tile<CPLX, SIDEB>(v, bx, by, tile);
    split_s<CPLX, SIDEB, true, B8>(v, code, S, out, nrb, nkb, bx, by, tile);
  } else {
    split_s<CPLX, SIDEB, false, B8>(v, code, S, out, nrb, nkb, bx, by, nullptr);
  }
}

template <bool CPLX, bool SIDEB, bool STAGED, bool B8>
__global__ void __launch_bounds__(256) k_split(View v, const int *code, int S, int8_t *out,
                                               int64_t nrb, int64_t nkb) {
  if constexpr (STAGED) {
    __shared__ __attribute__((aligned(16))) double tile[kSplitTileDoubles];
    split_dispatch<CPLX, SIDEB, B8>(v, code, S, out, nrb, nkb, blockIdx.x, blockIdx.y, tile);
  } else {
    split_dispatch<CPLX, SIDEB, B8>(v, code, S, out, nrb, nkb, blockIdx.x, blockIdx.y, nullptr);
  }
}

// ---------------------------------------------------------------- batched
// Block b of a batched launch belongs to the task t with
// start[t] <= b < start[t + 1] (binary search, uniform per block).
__device__ __forceinline__ int find_task(const int64_t *start, int ntasks, int64_t b) {
  int lo = 0, hi = ntasks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// One task scans all rows of one operand view over the whole contraction.
__global__ void __launch_bounds__(256) k_scan_batched(const ScanTask *tasks, const int64_t *start,
                                                      int ntasks) {
  const int64_t b = blockIdx.x;
  const int t = find_task(start, ntasks, b);
  const ScanTask tk = tasks[t];
  const int64_t rb = b - start[t];
  if (tk.rows_fast) {
    if (tk.cplx)
      scan_rowsfast_block<true>(tk.v, rb, 0, tk.v.L, tk.code, true);
    else
      scan_rowsfast_block<false>(tk.v, rb, 0, tk.v.L, tk.code, true);
  } else {
    if (tk.cplx)
      scan_rowcontig_block<true>(tk.v, rb, 0, tk.v.L, tk.code, true);
    else
      scan_rowcontig_block<false>(tk.v, rb, 0, tk.v.L, tk.code, true);
  }
}

// One task splits one operand view into its packed buffer; its blocks cover
// nrb * 32 / 64 packed-row groups times nkb * 32 / 64 contraction groups.
__global__ void __launch_bounds__(256) k_split_batched(const SplitTask *tasks, const int64_t *start,
                                                       int ntasks) {
  const int64_t b = blockIdx.x;
  const int t = find_task(start, ntasks, b);
  const SplitTask tk = tasks[t];
  const int64_t local = b - start[t];
  const int64_t nbx = tk.nrb / 2;
  const int64_t bx = local % nbx, by = local / nbx;
  __shared__ __attribute__((aligned(16))) double tile[kSplitTileDoubles];
  if (tk.cplx) {
    if (tk.side_b)
      split_dispatch<true, true>(tk.v, tk.code, tk.S, tk.out, tk.nrb, tk.nkb, bx, by, tile);
    else
      split_dispatch<true, false>(tk.v, tk.code, tk.S, tk.out, tk.nrb, tk.nkb, bx, by, tile);
  } else {
    split_dispatch<false, false>(tk.v, tk.code, tk.S, tk.out, tk.nrb, tk.nkb, bx, by, tile);
  }
}

template <bool CPLX, bool SIDEB>
__global__ void __launch_bounds__(256) k_unpack(const int8_t *packed, int64_t R, int64_t L, int S,
                                                int64_t nrb, int64_t nkb, int8_t *digits) {
  const int cc = CPLX ? 2 : 1;
  const int64_t total = (int64_t)S * R * L * cc;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const int part = (int)(idx % cc);
  int64_t rest = idx / cc;
  const int64_t l = rest % L;
  rest /= L;
  const int64_t r = rest % R;
  const int p = (int)(rest / R);
  int val;
  if (!CPLX) {
    val = packed[frag_offset(p, r, l, nrb, nkb)];
  } else if (!SIDEB) {
    val = packed[frag_offset(p, r, 2 * l + part, nrb, nkb)];
  } else {
    // row 2j holds (Re, -Im), row 2j+1 (Im, Re): the Re and Im digits are the
    // even entries of the two rows
    val = packed[frag_offset(p, 2 * r + part, 2 * l, nrb, nkb)];
  }
  digits[idx] = (int8_t)val;
}

__global__ void __launch_bounds__(256) k_codes(const int *code, int64_t R, int32_t *exps,
                                               uint8_t *flags) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= R) return;
  const int c = code[r];
  exps[r] = code_exp(c);
  flags[r] = code_bad(c) ? 1 : 0;
}

template <bool CPLX>
__global__ void __launch_bounds__(256) k_scale(int64_t m, int64_t n, double br, double bi,
                                               int beta_zero, void *C, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t i = idx % m, j = idx / m;
  if (CPLX) {
    double2 *c = reinterpret_cast<double2 *>(C) + i + j * ldc;
    if (beta_zero) {
      *c = make_double2(0.0, 0.0);
    } else {
      const double2 z = *c;
      *c = make_double2(sub_rn(mul_rn(br, z.x), mul_rn(bi, z.y)), add_rn(mul_rn(br, z.y), mul_rn(bi, z.x)));
    }
  } else {
    double *c = reinterpret_cast<double *>(C) + i + j * ldc;
    *c = beta_zero ? 0.0 : mul_rn(br, *c);
  }
}

inline unsigned grid1(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_fill_i32(int *p, int64_t n, int value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid1(n)), dim3(256), 0, st, p, n, value);
  return hipGetLastError();
}

hipError_t launch_fill_digits(int8_t *p, int64_t n, uint64_t seed, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_digits, dim3((unsigned)std::min<int64_t>(grid1(n), 1 << 20)), dim3(256),
                     0, st, p, n, seed);
  return hipGetLastError();
}

hipError_t launch_scan(const View &v, bool cplx, int *code, hipStream_t st) {
  if (v.R <= 0 || v.L <= 0) return hipSuccess;
  const int64_t target = 2048;
  if (v.sr == 1 && !(v.sl == 1 && v.R < 64)) {
    const int64_t rb = (v.R + 63) / 64;
    int64_t ncol = std::max<int64_t>(1, std::min<int64_t>((v.L + 15) / 16, target / rb));
    const int64_t lchunk = (v.L + ncol - 1) / ncol;
    ncol = (v.L + lchunk - 1) / lchunk;
    dim3 g((unsigned)rb, (unsigned)ncol);
    if (cplx)
      hipLaunchKernelGGL(k_scan_rowsfast<true>, g, dim3(256), 0, st, v, lchunk, code);
    else
      hipLaunchKernelGGL(k_scan_rowsfast<false>, g, dim3(256), 0, st, v, lchunk, code);
  } else {
    // sl == 1 (each row contiguous). A general-stride operand never reaches
    // here: one of the two strides of a BLAS operand is always 1.
    const int64_t rb = (v.R + 3) / 4;
    int64_t ncol = std::max<int64_t>(1, std::min<int64_t>((v.L + 255) / 256, std::max<int64_t>(1, target / rb)));
    const int64_t lchunk = (v.L + ncol - 1) / ncol;
    ncol = (v.L + lchunk - 1) / lchunk;
    dim3 g((unsigned)rb, (unsigned)ncol);
    if (cplx)
      hipLaunchKernelGGL(k_scan_rowcontig<true>, g, dim3(256), 0, st, v, lchunk, code);
    else
      hipLaunchKernelGGL(k_scan_rowcontig<false>, g, dim3(256), 0, st, v, lchunk, code);
  }
  return hipGetLastError();
}

namespace {
template <bool B8>
void split_launch(const View &v, bool cplx, bool side_b, const int *code, int S, int8_t *out,
                  int64_t nrb, int64_t nkb, dim3 g, hipStream_t st) {
#define OZ_SPLIT_LAUNCH(C, B, T) \
  hipLaunchKernelGGL((k_split<C, B, T, B8>), g, dim3(256), 0, st, v, code, S, out, nrb, nkb)
  const bool staged = split_staged(v);
  if (cplx && side_b) {
    if (staged) OZ_SPLIT_LAUNCH(true, true, true); else OZ_SPLIT_LAUNCH(true, true, false);
  } else if (cplx) {
    if (staged) OZ_SPLIT_LAUNCH(true, false, true); else OZ_SPLIT_LAUNCH(true, false, false);
  } else {
    if (staged) OZ_SPLIT_LAUNCH(false, false, true); else OZ_SPLIT_LAUNCH(false, false, false);
  }
#undef OZ_SPLIT_LAUNCH
}
}  // namespace

hipError_t launch_split(const View &v, bool cplx, bool side_b, const int *code, int S, int8_t *out,
                        int64_t nrb, int64_t nkb, hipStream_t st, bool b8) {
  // nrb * 32 is a multiple of 64 (rows padded to 128) and nkb * 32 a multiple
  // of 64 (contraction padded to 64): the grid covers the buffer exactly.
  if (b8 && (S < 1 || S > kS8Max)) return hipErrorInvalidValue;
  dim3 g((unsigned)(nrb * 32 / 64), (unsigned)(nkb * 32 / 64));
  if (b8)
    split_launch<true>(v, cplx, side_b, code, S, out, nrb, nkb, g, st);
  else
    split_launch<false>(v, cplx, side_b, code, S, out, nrb, nkb, g, st);
  return hipGetLastError();
}

hipError_t launch_unpack(const int8_t *packed, bool cplx, bool side_b, int64_t R, int64_t L, int S,
                         int64_t nrb, int64_t nkb, int8_t *digits, hipStream_t st) {
  const int64_t total = (int64_t)S * R * L * (cplx ? 2 : 1);
  if (total <= 0) return hipSuccess;
  dim3 g(grid1(total));
  if (cplx) {
    if (side_b)
      hipLaunchKernelGGL((k_unpack<true, true>), g, dim3(256), 0, st, packed, R, L, S, nrb, nkb, digits);
    else
      hipLaunchKernelGGL((k_unpack<true, false>), g, dim3(256), 0, st, packed, R, L, S, nrb, nkb, digits);
  } else {
    hipLaunchKernelGGL((k_unpack<false, false>), g, dim3(256), 0, st, packed, R, L, S, nrb, nkb, digits);
  }
  return hipGetLastError();
}

hipError_t launch_codes_to_exps(const int *code, int64_t R, int32_t *exps, uint8_t *flags,
                                hipStream_t st) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_codes, dim3(grid1(R)), dim3(256), 0, st, code, R, exps, flags);
  return hipGetLastError();
}

int64_t scan_task_blocks(const ScanTask &t) {
  return t.rows_fast ? (t.v.R + 63) / 64 : (t.v.R + 3) / 4;
}

int64_t split_task_blocks(const SplitTask &t) { return (t.nrb / 2) * (t.nkb / 2); }

hipError_t launch_scan_batched(const ScanTask *tasks, const int64_t *start, int ntasks,
                               int64_t nblocks, hipStream_t st) {
  if (ntasks <= 0 || nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_batched, dim3((unsigned)nblocks), dim3(256), 0, st, tasks, start, ntasks);
  return hipGetLastError();
}

hipError_t launch_split_batched(const SplitTask *tasks, const int64_t *start, int ntasks,
                                int64_t nblocks, hipStream_t st) {
  if (ntasks <= 0 || nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_batched, dim3((unsigned)nblocks), dim3(256), 0, st, tasks, start, ntasks);
  return hipGetLastError();
}

hipError_t launch_scale(bool cplx, int64_t m, int64_t n, double br, double bi, bool beta_zero,
                        void *C, int64_t ldc, hipStream_t st) {
  if (m <= 0 || n <= 0) return hipSuccess;
  dim3 g(grid1(m * n));
  if (cplx)
    hipLaunchKernelGGL(k_scale<true>, g, dim3(256), 0, st, m, n, br, bi, (int)beta_zero, C, ldc);
  else
    hipLaunchKernelGGL(k_scale<false>, g, dim3(256), 0, st, m, n, br, bi, (int)beta_zero, C, ldc);
  return hipGetLastError();
}

}  // namespace oz
