/*
 * ozaki.h - C ABI of the MI355X (gfx950) Ozaki-I and Ozaki-II FP64 /
 * complex-FP64 GEMM emulator (libozaki.so).
 *
 * The method is the Ozaki-I scheme as the paper describes it (Section 2.2,
 * GEMM Emulation on Integer Matrix Multiplication Unit): exponent alignment,
 * splitting of the FP64 inputs into low-precision slices, low-precision slice
 * products, accumulation in higher precision. The paper applies it to the
 * ZGEMM calls of the KKR/LSMS solver by intercepting standard BLAS calls
 * (Section 3.1), so the interface is BLAS-shaped. The precise rules the paper
 * leaves open are fixed as follows and are the same in every entry point:
 *
 *   exponents  e_i = frexp exponent of max_l max(|Re a_il|, |Im a_il|) over
 *              row i of op(A); f_j likewise over column j of op(B). Zero
 *              rows/columns take 0.
 *   slices     x = a * 2^-e_i, then s signed 7-bit digits (truncation toward
 *              zero): d_p = trunc(r * 2^7p), r -= d_p * 2^-7p. |d_p| <= 127.
 *   products   S_t = sum_{p+q=t} SA_p SB_q for t = 2..s+1, exact integers
 *              (INT8 x INT8 -> INT32 matrix cores, exact int64 carry when the
 *              INT32 range would be exceeded). Complex data: four real products
 *              per slice pair, Re = Ar Br - Ai Bi, Im = Ar Bi + Ai Br.
 *   recombine  acc = 0; acc = RN(acc + S_t * 2^-7t) for t = 2..s+1; then
 *              P_ij = acc * 2^(e_i + f_j).
 *   alpha/beta C = alpha P + beta C with every product and sum rounded on its
 *              own (complex: Re = (ar Pr - ai Pi) + (br Cr - bi Ci),
 *              Im = (ar Pi + ai Pr) + (br Ci + bi Cr)). beta == 0: C is not
 *              read. alpha == 0 or k == 0: C = beta C (untouched if beta == 1).
 *   non-finite every C_ij whose row of op(A) or column of op(B) holds Inf or NaN
 *              becomes NaN (a documented deviation from IEEE GEMM).
 *
 * Conventions for every entry point:
 *   - Matrices are column-major with BLAS leading dimensions. trans is one of
 *     'N', 'T', 'C' (case-insensitive); 'C' equals 'T' for real data.
 *   - A, B, C (and every array passed to the debug hooks) are DEVICE pointers
 *     owned by the caller; the library never frees them. Scratch memory comes
 *     from the workspace given to ozaki_set_workspace, or else from a
 *     grow-only device buffer the library allocates and frees in
 *     ozaki_finalize.
 *   - Work is enqueued on the stream given to ozaki_set_stream (default: the
 *     null stream) and is asynchronous: the call returns before the result is
 *     ready, the caller synchronises.
 *   - Return value: 0 on success; -i when argument i (1-based, reference-BLAS
 *     numbering) is invalid and nothing was launched; a positive OZAKI_ERR_*
 *     code on a runtime failure.
 *   - Calls are not thread safe: one host thread drives the library at a time.
 */
#ifndef OZAKI_H
#define OZAKI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Layout-compatible with C99 double _Complex and std::complex<double>. */
typedef struct {
  double re;
  double im;
} ozaki_z;

#define OZAKI_S_MAX 12 /* slices accepted: 1..OZAKI_S_MAX */

enum ozaki_status {
  OZAKI_OK = 0,
  OZAKI_ERR_HIP = 1,          /* a HIP runtime call or kernel launch failed */
  OZAKI_ERR_ALLOC = 2,        /* device workspace could not be obtained */
  OZAKI_ERR_WORKSPACE = 3,    /* the caller's workspace is too small */
  OZAKI_ERR_NO_DEVICE = 4,    /* no usable gfx950 device */
  OZAKI_ERR_INTERNAL = 5,
  OZAKI_ERR_NO_SELECTOR = 6,  /* automatic slice selection without a loaded selector */
  OZAKI_ERR_IO = 7,           /* tuning cache file missing, unwritable or malformed */
  OZAKI_ERR_SINGULAR = 8,     /* ozaki_zgetrf met an exactly zero pivot */
  OZAKI_ERR_TOO_LARGE = 9     /* ozaki_zgemm_noalloc: scratch beyond its fixed array */
};

/*
 * C <- alpha op(A) op(B) + beta C, FP64, emulated with `slices` INT8 slices.
 * op(A) is m x k, op(B) is k x n, C is m x n.
 * Argument numbers for errors: transa 1, transb 2, m 3, n 4, k 5, lda 8,
 * ldb 10, ldc 13, slices 14. lda >= max(1, rows of A as stored), likewise ldb,
 * ldc >= max(1, m). m, n, k >= 0.
 */
int ozaki_dgemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
                double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                double beta, double *C, int64_t ldc, int slices);

/* Complex FP64 (interleaved re, im) version of ozaki_dgemm; same numbering. */
int ozaki_zgemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
                ozaki_z alpha, const ozaki_z *A, int64_t lda, const ozaki_z *B, int64_t ldb,
                ozaki_z beta, ozaki_z *C, int64_t ldc, int slices);

/*
 * ozaki_zgemm without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. Same arguments, numbering, slice kind, tile table and
 * result (bit for bit) as ozaki_zgemm; the caller still owns A, B and C.
 *
 * Its scratch (exponent codes, packed slices, the int64 carry space of long
 * contractions) is one fixed device array of OZAKI_NOALLOC_SCRATCH_BYTES per
 * device, held from the library's load on that device until the process
 * ends; the call allocates and frees nothing, ignores ozaki_set_workspace and
 * records no phase timing. A product whose scratch would exceed the array
 * (ozaki_workspace_bytes('z', m, n, k, slices) > OZAKI_NOALLOC_SCRATCH_BYTES;
 * e.g. 1024^3 at s = 7 fits, 1536^3 does not) returns OZAKI_ERR_TOO_LARGE
 * with nothing launched. Every call on one device shares that array, which
 * keeps the last call's contents (each call rewrites what it reads): calls
 * that overlap on one device (other streams, other host threads) race.
 */
#define OZAKI_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int ozaki_zgemm_noalloc(char transa, char transb, int64_t m, int64_t n, int64_t k,
                        ozaki_z alpha, const ozaki_z *A, int64_t lda, const ozaki_z *B,
                        int64_t ldb, ozaki_z beta, ozaki_z *C, int64_t ldc, int slices);

/*
 * Slice kind of ozaki_dgemm / ozaki_zgemm (and of ozaki_workspace_bytes and
 * the debug hooks). Section 3.2 labels the Ozaki-I modes by 8s - 1 mantissa
 * bits, i.e. slices that use all 8 bits of an INT8; the default trunc-7
 * slices above keep 7. OZAKI_SPLIT_BAL8 selects 8-bit balanced slices:
 *   integer    X = trunc(a * 2^(8s - 2 - e_i)), |X| < 2^(8s - 2), s <= 8.
 *   digits     the balanced base-256 digits of X, each in [-128, 127]
 *              (d = ((X + 128) mod 256) - 128, X <- (X - d) / 256, least
 *              significant first); slice p holds the digit of 256^(s - p).
 *   products   the triangle p + q <= s + 1, as above; complex data splits the
 *              -Im b operand as it stands (its digits are not always the
 *              negated digits of Im b).
 *   recombine  acc = RN(acc + S_t * 2^(4 - 8t)) for t = 2..s+1, then
 *              P = acc * 2^(e_i + f_j); alpha/beta and non-finite as above.
 * 8s - 2 bits at s slices (trunc-7: 7s). With OZAKI_SPLIT_BAL8 the slice count
 * argument accepts 1..OZAKI_S8_MAX. The batched entry point always uses trunc-7
 * slices (its automatic mode raises s by adding diagonals, which needs the
 * prefix property of trunc-7 digits). The environment variable OZAKI_SPLIT=b8
 * sets the initial mode. ozaki_set_split returns -1 for an unknown mode.
 */
#define OZAKI_SPLIT_TRUNC7 0
#define OZAKI_SPLIT_BAL8 1
#define OZAKI_S8_MAX 8
int ozaki_set_split(int mode);
int ozaki_get_split(void);

/*
 * Ozaki-II emulation (Section 2.2: the inputs become integer matrices, their
 * products are taken modulo several pairwise-coprime moduli on the INT8
 * matrix cores and the Chinese remainder theorem rebuilds the result;
 * Section 3 uses 10..18 moduli). C <- alpha op(A) op(B) + beta C with
 * `moduli` moduli. Rules, on top of the exponents, alpha/beta and non-finite
 * rules above:
 *   moduli     the `moduli` largest pairwise-coprime integers <= 256, taken
 *              greedily from 256 downwards (256, 255, 253, 251, 247, 241,
 *              239, 233, 229, 227, 223, 217, 211, 199, 197, 193, 191, 181,
 *              179, 173); M is their product.
 *   integers   K' = k (real) or 2k (complex); beta = min(63, floor((floor(log2
 *              M) - 1 - ceil(log2 K')) / 2)); A'_il = trunc(a_il 2^(beta -
 *              e_i)), B'_lj = trunc(b_lj 2^(beta - f_j)) (Re and Im apart).
 *   products   A' mod m_q, B' mod m_q as balanced residues in [-floor(m_q/2),
 *              ceil(m_q/2) - 1]; one exact INT8 x INT8 -> INT32 product per
 *              modulus (complex data: one real product of A' rows (Re, Im)
 *              and B' rows (Re, -Im), (Im, Re) along the interleaved
 *              contraction).
 *   rebuild    c = the integer in [-M/2, M/2) congruent to every product mod
 *              m_q; it equals A'B' exactly. P_ij = RN(c) 2^(e_i + f_j - 2 beta)
 *              (one rounding), then alpha/beta.
 * Argument numbers as ozaki_dgemm, with moduli 14 (OZAKI2_MODULI_MIN ..
 * OZAKI2_MODULI_MAX, and -14 also when beta < 1: too few moduli for K').
 * K' above OZAKI2_K_MAX (exact INT32 sums) returns -5. The workspace holds
 * the residue planes (see ozaki2_workspace_bytes); the modular products and
 * the rebuild run in one fused kernel and never leave the chip.
 */
#define OZAKI2_MODULI_MIN 2
#define OZAKI2_MODULI_MAX 20
#define OZAKI2_K_MAX 131072
int ozaki2_dgemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
                 double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                 double beta, double *C, int64_t ldc, int moduli);
int ozaki2_zgemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
                 ozaki_z alpha, const ozaki_z *A, int64_t lda, const ozaki_z *B, int64_t ldb,
                 ozaki_z beta, ozaki_z *C, int64_t ldc, int moduli);
/* Host-side queries (no device work): the first `moduli` moduli into out[]
 * (host array); beta for `moduli` moduli and contraction length K' (0 when
 * beta < 1, negative for arguments out of range); workspace bytes of one
 * call (0 for invalid arguments or sizes the path rejects). */
int ozaki2_moduli(int moduli, int32_t *out);
int ozaki2_beta_bits(int moduli, int64_t kprime);
size_t ozaki2_workspace_bytes(char kind, int64_t m, int64_t n, int64_t k, int moduli);

/*
 * Blocked LU with partial pivoting and the inverse of an n x n complex matrix,
 * the step around the ZGEMM in the paper's solver (the multiple-scattering
 * matrix is inverted by LU; ZGEMM and ZTRSM dominate its run time, Section
 * 3.2). The trailing updates C -= A B are ZGEMMs through ozaki_zgemm with
 * `slices` slices of the current slice kind, or the native FP64 ZGEMM for
 * slices == 0. Every other step runs in its own kernels with each complex
 * operation written out as separately rounded real operations:
 *   product  (ar br - ai bi, ar bi + ai br)
 *   quotient d = br^2 + bi^2, ((ar br + ai bi) / d, (ai br - ar bi) / d)
 *   pivot    the first row of the largest |Re| + |Im| in the column (a NaN
 *            counts as the largest)
 * ozaki_zgetrf: A (device, column-major, lda >= n) is overwritten by L (unit
 *   lower, below the diagonal) and U, with P A = L U; ipiv (device, n int64)
 *   receives the 0-based pivot row of each column (rows c and ipiv[c]
 *   exchanged in order). Panels of nb columns (1 <= nb <= 1024): pivot, swap
 *   and rank-one update per column inside the panel, the interchanges applied
 *   to the other columns, U12 = L11^-1 A12 (forward substitution), then
 *   A22 -= L21 U12. Returns OZAKI_ERR_SINGULAR (factors complete) if a pivot
 *   is exactly zero or NaN. Synchronises with the stream before returning.
 *   The panel runs in leaves of up to 8 columns held in registers by one
 *   workgroup while at most 8192 rows lie below the leaf, else column by
 *   column; OZAKI_LU_PANEL=columns, leaf8, leaf4 or leaf2 in the environment
 *   (read at every call) forces a form. Every form gives the same factors and
 *   pivots bit for bit.
 * ozaki_zgetri: X (device, ldx >= n, not overlapping LU) = A^-1 from the
 *   factors: X = P I (an ipiv entry outside [c, n) counts as no exchange);
 *   block rows of nb top down X_i = L_ii^-1 X_i, X_below -=
 *   L_below,i X_i; then bottom up X_i = U_ii^-1 X_i, X_above -= U_above,i X_i.
 * Substitutions are column-oriented: forward, x_r -= l_rk x_k for k = 0, 1,
 * ... in turn; backward, for k = nb-1 down to 0, x_k /= u_kk and then
 * x_r -= u_rk x_k for r < k (each x_r subtracts its terms in decreasing k).
 * Argument numbers: n 1, A/LU 2, lda 3, ipiv 4, nb 5, slices 6 (0..the slice
 * limit of the current kind), X 7, ldx 8.
 */
int ozaki_zgetrf(int64_t n, ozaki_z *A, int64_t lda, int64_t *ipiv, int64_t nb, int slices);
int ozaki_zgetri(int64_t n, const ozaki_z *LU, int64_t lda, const int64_t *ipiv, ozaki_z *X,
                 int64_t ldx, int64_t nb, int slices);

/*
 * Native FP64 GEMM on the FP64 matrix cores (the comparator the paper uses as
 * ground truth: native FP64 GEMM, Section 3.2). Same arguments and error
 * numbering as ozaki_dgemm / ozaki_zgemm without `slices`. Ordinary FP64
 * rounding (fused multiply-adds in an order fixed by the kernel); alpha/beta
 * and quick returns as above; non-finite inputs propagate as IEEE arithmetic.
 */
int ozaki_native_dgemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
                       double alpha, const double *A, int64_t lda, const double *B,
                       int64_t ldb, double beta, double *C, int64_t ldc);
int ozaki_native_zgemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
                       ozaki_z alpha, const ozaki_z *A, int64_t lda, const ozaki_z *B,
                       int64_t ldb, ozaki_z beta, ozaki_z *C, int64_t ldc);

/*
 * Batched complex GEMM: `batch` independent problems
 *   C_b <- alpha_b op(A_b) op(B_b) + beta_b C_b,   b = 0 .. batch-1,
 * each emulated exactly as ozaki_zgemm would with slices[b] slices (the results
 * are bit-identical to batch separate ozaki_zgemm calls). Every argument is a
 * HOST array of length `batch`; A, B and C hold device pointers. This serves
 * the many small and uneven block products of a KKR/LSMS inversion (Sections
 * 3.2 and 4 of the paper).
 *   slices       host array of per-problem slice counts (1..OZAKI_S_MAX), or
 *                NULL for automatic selection (ozaki_load_selector must have
 *                been called; the residual probe raises any count that falls
 *                short of the target). The automatic mode returns
 *                OZAKI_ERR_NO_SELECTOR when no selector is loaded.
 *   slices_used  host array receiving the slice count used per problem, or
 *                NULL.
 * Execution: one batched exponent scan, one batched split and one grouped
 * persistent GEMM per distinct slice count walk global task and tile tables.
 * With graphs on (the default), the sequence is captured into a HIP graph on
 * the first call with a given argument set (pointers, sizes, scalars, slices)
 * and replayed on later identical calls; the plan (device descriptors and
 * packed-operand workspace, owned by the library) is cached with it.
 * Errors: -i for argument i of the first invalid problem, numbered transa 1,
 * transb 2, m 3, n 4, k 5, alpha 6, A 7, lda 8, B 9, ldb 10, beta 11, C 12,
 * ldc 13, batch 14, slices 15; a NULL host array gives its argument number.
 */
int ozaki_zgemm_batched(const char *transa, const char *transb, const int64_t *m,
                        const int64_t *n, const int64_t *k, const ozaki_z *alpha,
                        const ozaki_z *const *A, const int64_t *lda, const ozaki_z *const *B,
                        const int64_t *ldb, const ozaki_z *beta, ozaki_z *const *C,
                        const int64_t *ldc, int64_t batch, const int *slices, int *slices_used);

/*
 * Selector for the automatic mode of ozaki_zgemm_batched (slices == NULL):
 * params are the OZAKI_MLP_PARAMS FP32 MLP parameters (host array, copied).
 * A problem gets s = ceil(prediction + margin) slices (clamped to 1..12); its
 * product is formed in library memory (alpha = 1, beta = 0, before the
 * 2^(e_i + f_j) scaling) with its operands split to s + 1 slices, then probed
 * (ozaki_probe's estimate, 2 vectors, seed 0x5eed0000 + round). If
 * max_i est[i] * kappa > target, the next diagonal is added to the stored sums
 * on the device (with trunc-7 slices this is exactly the product at s + 1) and
 * the probe runs again; a product still over the target is formed again at
 * s + 2 in a further pass, and so on up to s = 12. C is then finished with
 * alpha and beta by the fused epilogue's formula, so the result equals
 * ozaki_zgemm at the final s bit for bit. The automatic mode synchronises the
 * stream twice per pass (the predictions, then the pass's final slice counts)
 * and is not captured into graphs.
 * Errors: params -1, margin -2 (outside [-4, 8]), target -3 (<= 0), kappa -4 (< 1).
 */
int ozaki_load_selector(const float *params, float margin, double target, double kappa);

/* 1 (default): capture and replay HIP graphs in ozaki_zgemm_batched and in
 * ozaki_zgetrf / ozaki_zgetri (one graph per argument set, captured on the
 * first call; not while phase timing is on); 0: launch the same kernels
 * directly on every call. */
int ozaki_batched_graphs(int on);
/* Release every cached batched plan and graph (device memory included). */
int ozaki_batched_cache_clear(void);

/*
 * Tile autotuner of the fused slice GEMM. The paper takes its emulation
 * library as shipped (Section 3.1); the tile candidates and the tuning table
 * are this library's own.
 * A tuning id below 14 is 2 * tile configuration + tile order (0: down the
 * output rows, 1: along the columns); ids 14 .. 20 are configurations 0 .. 6
 * walking the tiles in groups of 16 tile rows, ids 21 .. 27 in groups of 8
 * tile rows with each XCD's workgroups on consecutive tiles.
 * ozaki_tune_configs() gives their number. Every id computes bit-identical
 * results: only the
 * workgroup shape, the LDS ring depth and the order in which the persistent
 * workgroups walk the output tiles differ.
 * The table maps (kind, slices, bucket of m, of n' = n or 2n, of the 32-deep
 * contraction blocks of k' = k or 2k; bucket = ceil(log2)) to an id; ozaki_dgemm,
 * ozaki_zgemm and ozaki_debug_diagonals look their shape up there (default 0).
 * The environment variable OZAKI_GEMM_CONFIG=<id> forces one id for every call;
 * OZAKI_TUNE_CACHE=<file> loads a saved table before the first lookup.
 * The batched path uses id 8 (four-wave 64 x 64 tiles, two workgroups per CU)
 * unless OZAKI_BATCHED_CONFIG=<id> is set.
 *
 * ozaki_autotune: times the fused GEMM kernel of every id on an m x n x k
 *   product with `slices` slices on the library's stream: packed operands of
 *   pseudo-random digits in the library workspace (the kernel's clock depends
 *   on its operand bits), a temporary m x n output allocated and freed inside,
 *   one untimed round, then 5 rounds of `reps` launches per id round-robin; the
 *   stream is synchronised. It keeps the id with the smallest median time per
 *   launch in the table and returns it in *best and that time in *best_ms
 *   (either may be NULL).
 *   Errors: kind -1 ('d' or 'z'), m -2, n -3, k -4 (each >= 1), slices -5,
 *   reps -6 (1..1000); OZAKI_ERR_* for device failures.
 * ozaki_tune_set: records `id` for the bucket of the shape (id < 0 removes the
 *   entry); id -6 if >= ozaki_tune_configs(). ozaki_tune_get: the id a call of
 *   that shape would use (>= 0) or a negative argument error as for autotune.
 * ozaki_tune_save / ozaki_tune_load: the table as a JSON file (path -1 if NULL;
 *   OZAKI_ERR_IO if the file cannot be opened or is malformed). Loading merges
 *   the entries into the table when the file's "arch" equals the current
 *   device's architecture name and ignores them otherwise.
 * The table is process-wide and not thread-safe.
 */
/*
 * Cap on the number of workgroups of the persistent slice GEMM (single and
 * batched products; 0, the default, launches one grid sized to the CU
 * count). With a cap below the tile count every workgroup walks several
 * output tiles in turn, reusing its int64 carry space; results are
 * bit-identical for every cap. For tests of that reuse at small sizes and for
 * leaving CUs to concurrent work. Errors: -1 for a negative cap.
 */
int ozaki_set_grid_limit(int64_t max_workgroups);

int ozaki_autotune(char kind, int64_t m, int64_t n, int64_t k, int slices, int reps, int *best,
                   double *best_ms);
int ozaki_tune_set(char kind, int64_t m, int64_t n, int64_t k, int slices, int id);
int ozaki_tune_get(char kind, int64_t m, int64_t n, int64_t k, int slices);
int ozaki_tune_configs(void);
int ozaki_tune_save(const char *path);
int ozaki_tune_load(const char *path);
int ozaki_tune_clear(void);

/*
 * Randomized FP64 residual probe of a computed product C ~ op(A) op(B)
 * (as left by a call with alpha = 1, beta = 0). For nvec sign vectors x_v
 * (entries +-1 from the top bit of SplitMix64(seed + v*n + j), v < nvec) it
 * computes r_v = C x_v - op(A)(op(B) x_v) with compensated (Dot2) sums and
 * u = |op(A)| (|op(B)| 1) (complex modulus entrywise), and writes
 *   est[i] = sqrt(mean_v |r_v,i|^2) * sqrt(n) / u_i      (device array, m doubles)
 * an estimate of the componentwise error scale max_j |C - C*|_ij / (|A||B|)_ij
 * of row i: est[i] is 0 when u_i = 0 and r = 0, +Inf when u_i = 0 and r != 0,
 * NaN when an input is not finite. The selector's slice count is checked
 * against it (ozaki_zgemm_batched with slices == NULL). kind 'd' or 'z'.
 * Errors: kind -1, transa -2, transb -3, m -4, n -5, k -6, A -7, lda -8, B -9,
 * ldb -10, C -11, ldc -12, nvec -13 (1..4), est -15.
 */
int ozaki_probe(char kind, char transa, char transb, int64_t m, int64_t n, int64_t k,
                const void *A, int64_t lda, const void *B, int64_t ldb, const void *C,
                int64_t ldc, int nvec, uint64_t seed, double *est);

/*
 * Selector features of one product (64 floats, device array `feat`): the
 * fraction of entries of op(A) lying delta = e_i - E(a_il) binades below their
 * row maximum, bins min(delta, 30) and a last bin for zeros (32 values); the
 * same over the columns of op(B), bins min(delta, 29) and zeros (31 values);
 * log2(k) / 16. E is the frexp exponent (the larger of the real and imaginary
 * parts for complex data). An entry delta binades down keeps 7s - delta of
 * its bits, which is what the slice count has to cover; the paper notes that
 * accuracy depends on both the precision and the operator (abstract).
 * kind 'd' or 'z'; errors as ozaki_probe (kind -1, transa -2, transb -3, m -4,
 * n -5, k -6, lda -8, ldb -10), feat -11.
 */
int ozaki_features(char kind, char transa, char transb, int64_t m, int64_t n, int64_t k,
                   const void *A, int64_t lda, const void *B, int64_t ldb, float *feat);

/*
 * Selector MLP: 64 -> 128 -> 128 -> 1 with ReLU, predicting the slice count
 * a product needs from its features. OZAKI_MLP_PARAMS FP32 parameters in the
 * order W1[128][64], b1[128], W2[128][128], b2[128], w3[128], b3; the matrix
 * products run on BF16 matrix cores (weights and layer inputs rounded to BF16
 * with round-to-nearest-even, FP32 accumulation).
 * `state` is a caller-owned device buffer of ozaki_mlp_state_bytes() bytes:
 * parameters at byte 0, Adam first and second moments and the gradient after
 * them (OZAKI_MLP_PARAMS floats each, in that order), then BF16 copies.
 * `scratch` is a device buffer of ozaki_mlp_scratch_bytes(batch) bytes; the
 * backward pass reads the activations the forward pass left there. Its
 * layout (bp = batch rounded up to a multiple of 32; regions in this order,
 * each starting at a multiple of 256 bytes; rows >= batch are zero): Xh
 * (bp x 64 BF16, row-major), Xh^T, H1 (bp x 128 FP32, after the ReLU), H1h
 * (BF16), H1h^T, H2 (FP32), H2h, H2h^T, then after a backward pass dH2h
 * (bp x 128 BF16), dH2h^T, dH1h (BF16), dH1h^T.
 *   init      He-uniform weights from SplitMix64(seed + index), zero biases
 *   refresh   rebuild the BF16 copies after writing parameters directly
 *   forward   y[b] for b < batch from X[b][64] (device, FP32)
 *   backward  loss (1/B) sum w_b (y_b - t_b)^2, w_b = under_weight when
 *             y_b < t_b else 1; writes the gradient into the state and the
 *             loss into *loss (device scalar, may be NULL)
 *   adam      one Adam step (bias-corrected, step >= 1) from the stored gradient
 */
#define OZAKI_MLP_PARAMS 24961
size_t ozaki_mlp_state_bytes(void);
size_t ozaki_mlp_scratch_bytes(int64_t batch);
int ozaki_mlp_init(void *state, uint64_t seed);
int ozaki_mlp_refresh(void *state);
int ozaki_mlp_forward(const void *state, int64_t batch, const float *X, float *y, void *scratch);
int ozaki_mlp_backward(void *state, int64_t batch, const float *y, const float *target,
                       float under_weight, float *loss, void *scratch);
int ozaki_mlp_adam(void *state, float lr, float beta1, float beta2, float eps, int64_t step);

/* Stream for all later work (a hipStream_t; NULL = null stream). */
int ozaki_set_stream(void *hip_stream);

/*
 * Caller-owned device workspace (NULL, 0 = use the library's own buffer).
 * The library keeps the pointer until it is replaced; a call that needs more
 * than `bytes` returns OZAKI_ERR_WORKSPACE. ozaki_workspace_bytes gives the
 * size a call needs (kind 'd' or 'z').
 */
int ozaki_set_workspace(void *device_ptr, size_t bytes);
size_t ozaki_workspace_bytes(char kind, int64_t m, int64_t n, int64_t k, int slices);

/*
 * Phase timing for measurement. While enabled, every emulated GEMM records a
 * pair of HIP events around each of its phases on the call's stream:
 *   OZAKI_PHASE_SCAN  exponent scan of op(A) rows and op(B) columns
 *   OZAKI_PHASE_SPLIT slicing of both operands into packed INT8 slices
 *   OZAKI_PHASE_GEMM  fused slice-pair INT8 GEMM + FP64 recombination
 *                     (Ozaki-II: the INT8 residue products)
 *   OZAKI_PHASE_RECON Ozaki-II only: CRT rebuild, scaling and alpha/beta
 * (Ozaki-II records its residue step as OZAKI_PHASE_SPLIT.)
 * ozaki_timing_read waits for the recorded events, writes the summed
 * milliseconds per phase into ms[0..OZAKI_PHASES-1] (host array) and the
 * number of timed calls into *calls (may be NULL), then clears the record.
 * Recording adds one event pair per phase and call; leave it off otherwise.
 */
#define OZAKI_PHASES 4
#define OZAKI_PHASE_SCAN 0
#define OZAKI_PHASE_SPLIT 1
#define OZAKI_PHASE_GEMM 2
#define OZAKI_PHASE_RECON 3
int ozaki_timing_enable(int on);
int ozaki_timing_read(double *ms, int64_t *calls);

/* Release the library's own device buffers: the workspace, the scratch of
 * the automatic slice mode and the LU flags (safe to call more than once). */
int ozaki_finalize(void);

/* Static text for a status code. */
const char *ozaki_status_string(int status);

/*
 * Parity hooks. They run the same kernels as the GEMM entry points and copy
 * intermediate results out in plain layouts; all output pointers are device
 * pointers. kind is 'd' (X is double) or 'z' (X is ozaki_z).
 *
 * ozaki_debug_exponents: the exponent step on op(X) rows. side 'A': X is the
 * A operand, rows are the `rows` rows of op(X) (an rows x L matrix);
 * side 'B': X is the B operand, "rows" are the columns of op(X) (L x rows).
 * Writes exps[r] (int32, e or f; 0 for a zero or flagged row) and flags[r]
 * (uint8, 1 when the row holds Inf or NaN). Argument errors: -1 kind,
 * -2 side, -3 trans, -4 rows, -5 L, -7 ldx, -8/-9 null outputs.
 */
int ozaki_debug_exponents(char kind, char side, char trans, int64_t rows, int64_t L,
                          const void *X, int64_t ldx, int32_t *exps, uint8_t *flags);

/*
 * ozaki_debug_split: the digits d_1..d_s of op(X) rows (side 'A') or op(X)
 * columns (side 'B'). Output layout: int8 digits[((p * rows + r) * L + l) * c + part]
 * with p = 0..s-1, c = 1 (real) or 2 (complex, part 0 = Re, 1 = Im).
 * Argument errors as ozaki_debug_exponents, -8 slices, -9 null output.
 */
int ozaki_debug_split(char kind, char side, char trans, int64_t rows, int64_t L,
                      const void *X, int64_t ldx, int slices, int8_t *digits);

/*
 * ozaki_debug_diagonals: the exact diagonal sums S_t, t = 2..s+1, of
 * op(A) op(B). Output layout: int64 S[(((t-2) * n + j) * m + i) * c + part],
 * c = 1 (real) or 2 (complex, part 0 = Re, 1 = Im). Argument errors as the
 * GEMM entry points (kind is argument 0: -100 when not 'd'/'z'), slices -14,
 * null output -15.
 */
int ozaki_debug_diagonals(char kind, char transa, char transb, int64_t m, int64_t n,
                          int64_t k, const void *A, int64_t lda, const void *B, int64_t ldb,
                          int slices, int64_t *S);

#ifdef __cplusplus
}
#endif

#endif /* OZAKI_H */
