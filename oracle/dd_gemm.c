/*
 * Double-double GEMM on the host: the accuracy reference of the oracle.
 *
 * TEST INFRASTRUCTURE ONLY. Built by oracle/build_dd.py with gcc; never linked
 * into the GPU library.
 *
 * Double-double arithmetic after Hida, Li and Bailey (2001), which the paper
 * cites for emulating higher precision with FP64 (Section 2.2): each product is
 * made exact with TwoProd (fma gives the rounding error of a*b exactly) and
 * added into a (hi, lo) pair with the accurate double-double addition built on
 * TwoSum. The result of a length-L dot product is within about L * 2^-104 of
 * sum |a_l b_l| of the exact value.
 *
 * Layouts: A is row-major (m x L), Bt is row-major (n x L) = op(B)^T, so both
 * inner loops are unit-stride. Complex data is passed as interleaved (re, im)
 * pairs and uses 2L real terms per component:
 *   Re = sum ar*br - ai*bi,   Im = sum ar*bi + ai*br.
 * This file must be compiled without fast-math and with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>

static inline void two_sum(double a, double b, double *s, double *e) {
  double x = a + b;
  double z = x - a;
  *e = (a - (x - z)) + (b - z);
  *s = x;
}

static inline void quick_two_sum(double a, double b, double *s, double *e) {
  double x = a + b;
  *e = b - (x - a);
  *s = x;
}

static inline void two_prod(double a, double b, double *p, double *e) {
  double x = a * b;
  *e = fma(a, b, -x);
  *p = x;
}

/* (hi, lo) += (bh, bl), accurate double-double addition. */
static inline void dd_add(double *hi, double *lo, double bh, double bl) {
  double s1, s2, t1, t2;
  two_sum(*hi, bh, &s1, &s2);
  two_sum(*lo, bl, &t1, &t2);
  s2 += t1;
  quick_two_sum(s1, s2, &s1, &s2);
  s2 += t2;
  quick_two_sum(s1, s2, hi, lo);
}

static inline void dd_mac(double *hi, double *lo, double a, double b) {
  double p, e;
  two_prod(a, b, &p, &e);
  dd_add(hi, lo, p, e);
}

static void entry_real(const double *a, const double *b, int64_t L, double *hi, double *lo) {
  double h = 0.0, l = 0.0;
  for (int64_t x = 0; x < L; ++x) dd_mac(&h, &l, a[x], b[x]);
  *hi = h;
  *lo = l;
}

static void entry_complex(const double *a, const double *b, int64_t L, double *out) {
  double rh = 0.0, rl = 0.0, ih = 0.0, il = 0.0;
  for (int64_t x = 0; x < L; ++x) {
    double ar = a[2 * x], ai = a[2 * x + 1], br = b[2 * x], bi = b[2 * x + 1];
    dd_mac(&rh, &rl, ar, br);
    dd_mac(&rh, &rl, -ai, bi);
    dd_mac(&ih, &il, ar, bi);
    dd_mac(&ih, &il, ai, br);
  }
  out[0] = rh; out[1] = rl; out[2] = ih; out[3] = il;
}

/* Full product: hi/lo are row-major m x n. */
void dd_gemm_real(int64_t m, int64_t n, int64_t L, const double *A, const double *Bt,
                  double *hi, double *lo) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j)
      entry_real(A + i * L, Bt + j * L, L, hi + i * n + j, lo + i * n + j);
}

/* out is row-major m x n x 4: (re_hi, re_lo, im_hi, im_lo). */
void dd_gemm_complex(int64_t m, int64_t n, int64_t L, const double *A, const double *Bt,
                     double *out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j)
      entry_complex(A + 2 * i * L, Bt + 2 * j * L, L, out + 4 * (i * n + j));
}

/* Selected entries (ri[x], cj[x]), x < cnt. */
void dd_entries_real(int64_t cnt, const int64_t *ri, const int64_t *cj, int64_t L,
                     const double *A, const double *Bt, double *hi, double *lo) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t x = 0; x < cnt; ++x)
    entry_real(A + ri[x] * L, Bt + cj[x] * L, L, hi + x, lo + x);
}

void dd_entries_complex(int64_t cnt, const int64_t *ri, const int64_t *cj, int64_t L,
                        const double *A, const double *Bt, double *out) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t x = 0; x < cnt; ++x)
    entry_complex(A + 2 * ri[x] * L, Bt + 2 * cj[x] * L, L, out + 4 * x);
}
