// Internal launch interface between the host runtime (ozaki_api.hip) and the
// kernel files of libozaki. Not part of the public C ABI.
#pragma once

#include "ozaki_common.hpp"

namespace oz {

// Exponent step: code[r] = max over row r of expo_code (code must hold zeros
// on entry; launch_fill_i32 provides them).
hipError_t launch_fill_i32(int *p, int64_t n, int value, hipStream_t st);
// Pseudo-random digits in [-127, 127] (timing data of the autotuner).
hipError_t launch_fill_digits(int8_t *p, int64_t n, uint64_t seed, hipStream_t st);
hipError_t launch_scan(const View &v, bool cplx, int *code, hipStream_t st);

// Slicing step: writes all nrb*32 x nkb*32 packed rows/entries of S slices.
// side_b selects the B-operand construction for complex data (rows 2j and
// 2j+1 hold (Re, -Im) and (Im, Re) of column j along the contraction).
// b8 selects the 8-bit balanced slices (S <= kS8Max) instead of trunc-7.
constexpr int kS8Max = 8;
hipError_t launch_split(const View &v, bool cplx, bool side_b, const int *code, int S,
                        int8_t *out, int64_t nrb, int64_t nkb, hipStream_t st, bool b8 = false);

// Batched scan and split: task tables in device memory. A scan task covers
// all rows of one operand view over its whole contraction (codes are stored,
// no zero fill needed); a split task writes one packed operand.
struct ScanTask {
  View v;
  int *code;
  int cplx;
  int rows_fast;  // v.sr == 1: 64 rows per block, else 4 rows per block
};
struct SplitTask {
  View v;
  const int *code;
  int8_t *out;
  int64_t nrb, nkb;
  int S;
  int cplx;
  int side_b;
};
int64_t scan_task_blocks(const ScanTask &t);
int64_t split_task_blocks(const SplitTask &t);
// start[t] = first block of task t (prefix sums of the task block counts).
hipError_t launch_scan_batched(const ScanTask *tasks, const int64_t *start, int ntasks,
                               int64_t nblocks, hipStream_t st);
hipError_t launch_split_batched(const SplitTask *tasks, const int64_t *start, int ntasks,
                                int64_t nblocks, hipStream_t st);

// Debug helpers.
hipError_t launch_unpack(const int8_t *packed, bool cplx, bool side_b, int64_t R, int64_t L,
                         int S, int64_t nrb, int64_t nkb, int8_t *digits, hipStream_t st);
hipError_t launch_codes_to_exps(const int *code, int64_t R, int32_t *exps, uint8_t *flags,
                                hipStream_t st);

// C <- beta C (beta_zero: C <- 0 without reading C).
hipError_t launch_scale(bool cplx, int64_t m, int64_t n, double br, double bi, bool beta_zero,
                        void *C, int64_t ldc, hipStream_t st);

// Fused slice-pair GEMM + recombination: one product C = alpha op(A) op(B)
// + beta C given its packed operands and exponent codes.
struct GemmProblem {
  const int8_t *SP;  // packed B' (rows j' of the output's column side)
  const int8_t *SQ;  // packed A' (rows i)
  int64_t nrbP, nrbQ, nkb;
  int64_t m, nprime;  // output rows i < m, output "rows" j' < nprime (n or 2n)
  const int *codeA, *codeB;
  double ar, ai, br, bi;
  int beta_zero;
  int cplx;
  int wbits, woff;  // diagonal t (2..S+1) carries weight 2^(woff - wbits t): 7, 0 or 8, 4
  void *C;
  int64_t ldc;
  int64_t *raw;  // raw diagonal output (debug) or nullptr
  int unscaled;  // store the recombined sum itself (no 2^(e_i + f_j), no alpha/beta)
};

// Kernel arguments: either one problem (grouped == 0) or a table of problems
// walked through a tile table (tile t belongs to problem tile_prob[t] and is
// its tile number tile_local[t]).
struct GemmArgs {
  GemmProblem one;
  const GemmProblem *probs;
  const int *tile_prob;
  const int *tile_local;
  int64_t ntiles;
  int64_t *flush_ws;  // int64 per-workgroup carry space (chunked K only)
  int64_t kb_chunk;   // contraction blocks per exact INT32 chunk
  int chunked;        // some problem has nkb > kb_chunk
  int split;          // single product: nkb fits two INT32 sets per diagonal (see split_pm)
  int order;          // tile order (set from the tuning id at launch)
  int64_t max_groups; // cap on the persistent grid (0: no cap beyond the CU count)
};

// Tile counts of a problem for a configuration (host side).
int64_t gemm_tiles(int S, int cfg, int64_t m, int64_t nprime);
// Launch a grouped GEMM over the tile table in `a` (every problem has S slices).
hipError_t launch_ozgemm_grouped(int S, int cfg, const GemmArgs &a, int num_cu, hipStream_t st);

// Contraction blocks (of 32) that one INT32 accumulation may cover for S
// slices: S * 32 * kb * 127^2 < 2^31 (8-bit slices: 128^2).
int64_t kb_chunk_for(int S, bool b8 = false);
// Contraction blocks up to which a chunked single product instead splits each
// diagonal's slice pairs over two INT32 sets (configurations with one A'
// block per wave), so that it needs no int64 carry.
int64_t kb_split_for(int S, bool b8 = false);
// Tuning ids of the fused GEMM (0 .. gemm_num_configs() - 1): 2 * tile
// configuration + tile order.
int gemm_num_configs();
// Bytes of int64 carry space the GEMM needs when nkb > kb_chunk (valid for
// every configuration).
size_t gemm_flush_bytes(int S, int cfg, int num_cu);
hipError_t launch_ozgemm(int S, int cfg, const GemmArgs &a, int num_cu, hipStream_t st);

// Selector features and MLP (see ozaki_selector.hip).
struct FeatTask {
  View v;
  const int *code;
  int *hist;  // nbins integer counts of this operand side
  int cplx;
  int rows_fast;
  int nbins;  // 32 for op(A) rows, 31 for op(B) columns
};
int64_t feat_task_blocks(const FeatTask &t);
hipError_t launch_feat_hist(const FeatTask *tasks, const int64_t *start, int ntasks, int64_t nblocks,
                            hipStream_t st);
// dims[3p..3p+2] = m, n, k of problem p; hist[64p..] holds A bins 0..31 and B
// bins 32..62.
hipError_t launch_feat_finish(const int *hist, const int64_t *dims, float *feat, int64_t np,
                              hipStream_t st);
int64_t mlp_params();
size_t mlp_state_bytes();
size_t mlp_scratch_bytes(int64_t batch);
hipError_t mlp_init(void *state, uint64_t seed, hipStream_t st);
hipError_t mlp_refresh(void *state, hipStream_t st);
hipError_t mlp_forward(const void *state, int64_t b, const float *X, float *y, void *scratch,
                       hipStream_t st);
hipError_t mlp_backward(void *state, int64_t b, const float *y, const float *target, float under,
                        float *loss, void *scratch, hipStream_t st);
hipError_t mlp_adam(void *state, float lr, float b1, float b2, float eps, int64_t step,
                    hipStream_t st);

// Randomized residual probe (see ozaki_probe.hip). A task probes one product
// in four stages over chunks of its contraction (chl) and columns (chj); its
// scratch (w, ub and the chunk records p1, p2) comes from probe_task.
struct ProbeTask {
  View va, vb;
  const void *C;
  int64_t ldc;
  int cplx;
  int nv;
  uint64_t seed;
  double *w, *ub, *est, *p1, *p2;
  int64_t chl, chj, ncl, ncj;
  int64_t blk[4];  // batched: first block of this task in each stage
  // optional: C holds recombined sums still to be scaled by 2^(e_i + f_j)
  // (exponent codes of its rows and columns), and a skip flag (the task runs
  // only while flag[id] == 1)
  const int *codeA, *codeB;
  const int *flag;
  int64_t id;
};
// C = alpha P + beta C over complex problems (P: m x n, leading dimension m).
struct AxpbyTask {
  const void *P;
  void *C;
  int64_t m, n, ldc;
  double ar, ai, br, bi;
  int beta_zero;
  const int *codeA, *codeB;  // optional: P = RN-scaled P 2^(e_i + f_j) first
};
int64_t axpby_task_blocks(const AxpbyTask &t);
// Scratch bytes of one probe, its task (scratch at ws), blocks per stage, and
// the launches: one task, or a table of tasks whose blk[] hold the prefix sums
// of probe_stage_blocks (nblk[s] blocks in stage s).
size_t probe_workspace_bytes(int64_t m, int64_t n, int64_t k);
ProbeTask probe_task(const View &va, const View &vb, bool cplx, const void *C, int64_t ldc, int nv,
                     uint64_t seed, void *ws, double *est);
int64_t probe_stage_blocks(const ProbeTask &t, int stage);
hipError_t launch_probe_batched(const ProbeTask *tasks, int ntasks, const int64_t *nblk,
                                hipStream_t st);
hipError_t launch_axpby_batched(const AxpbyTask *tasks, const int64_t *start, int ntasks,
                                int64_t nblocks, hipStream_t st);
int probe_max_vectors();
hipError_t launch_probe_max_batched(const ProbeTask *tasks, int ntasks, double *out,
                                    hipStream_t st);
// Automatic-mode decision for n problems after a probe round: flag[e] (the
// problems probed this round: all when `first`, else those with flag[e] == 1)
// becomes 1 when emax[e] * kappa > target and s[e] < cap[e] (then s[e] is
// raised by one), 2 when the target is missed but s[e] == cap[e] < smax,
// else 0.
hipError_t launch_probe_decide(const double *emax, int64_t n, double kappa, double target,
                               int smax, int *s, const int *cap, int *flag, int first,
                               hipStream_t st);
// One more diagonal for the problems with flag[id] == 1: diagonal d = s[id] + 1
// (trunc-7 slices, the new slice count s[id]) over the problem's packed
// operands, added to its recombined sums P (unscaled, column-major, leading
// dimension m) as P = RN(P + S_d 2^(woff - wbits d)). Tiles of 64 x 64 (j' x
// i) from a tile table.
struct DiagTask {
  const int8_t *SP, *SQ;  // packed B' and A' (as GemmProblem)
  int64_t nrbP, nrbQ, nkb;
  int64_t m, nprime;
  void *P;
  int cplx;
  int wbits, woff;
  int64_t id;
};
int64_t diag_tiles(int64_t m, int64_t nprime);
hipError_t launch_add_diagonal(const DiagTask *tasks, const int *tile_task, const int *tile_local,
                               int64_t ntiles, const int *s, const int *flag, hipStream_t st);
hipError_t launch_probe(const View &va, const View &vb, bool cplx, const void *C, int64_t ldc,
                        int nv, uint64_t seed, void *ws, double *est, hipStream_t st);

// Ozaki-II (see ozaki2.hip): N pairwise-coprime moduli, integer conversion
// with beta bits per operand entry, INT8 residue planes, INT32 modular
// products and the CRT rebuild.
constexpr int kModMax = 20;
// The k-th modulus (0-based; 0 outside 0..kModMax-1).
int crt_modulus(int k);
// floor(log2(m_0 ... m_{n-1})), or -1 for n outside 1..kModMax.
int crt_log2_floor(int n);
// beta = min(63, floor((floor(log2 M) - 1 - ceil(log2 K')) / 2)); below 1
// means too few moduli for the contraction length.
int crt_beta(int n, int64_t kprime);
// Residues of X' (rows of op(A), or of B' for side_b) into n planes in the
// packed fragment layout of the slices (nrb 32-row blocks, nkb 32-entry
// contraction blocks, nkb a multiple of 4; plane k at out + k nrb nkb KiB);
// padded rows and contraction entries hold zero residues.
hipError_t launch_residues(const View &v, bool cplx, bool side_b, const int *code, int n, int beta,
                           int8_t *out, int64_t nrb, int64_t nkb, hipStream_t st);
// Fused Ozaki-II product: per output tile the n modular INT8 products, each
// reduced at once to its Garner digit, then the rebuilt integer rounded to
// FP64, scaled by 2^(e_i + f_j - 2 beta) and alpha/beta applied.
struct Oz2Args {
  const int8_t *RA, *RB;  // packed residue planes of A' (nrbQ blocks) and B' (nrbP blocks)
  int64_t nrbQ, nrbP, nkb;
  int64_t m, nprime;      // output rows i < m, output "rows" j' < nprime (n or 2n)
  const int *codeA, *codeB;
  int beta;
  double ar, ai, br, bi;
  int beta_zero;
  int cplx;
  void *C;
  int64_t ldc;
};
hipError_t launch_oz2gemm(int n, const Oz2Args &a, int num_cu, hipStream_t st);

// Blocked LU and inverse (see ozaki_lu.hip): one pivot column (pivot search,
// swap over the panel columns [p0, p1) and panel update), the panel's
// multipliers once its columns are done; the
// row interchanges ipiv[c0..c1) (c1 - c0 <= kLuMaxBlock) turned into
// destination/source row slots in `pairs` (kLuPairWords int64: destinations,
// then sources, at offset 2 * kLuMaxBlock) and applied to the columns
// [q0, q1) and [q2, q3); a triangular solve with nb x nb unit lower /
// non-unit upper T on ncols columns of X; the identity; a scalar store.
constexpr int64_t kLuMaxBlock = 1024;  // panel / block width limit (one thread per block row)
hipError_t launch_lu_column(double2 *A, int64_t lda, int64_t n, int64_t c, int64_t p0, int64_t p1,
                            int64_t *ipiv, int64_t *singular, hipStream_t st);
hipError_t launch_lu_scale(double2 *A, int64_t lda, int64_t n, int64_t p0, int64_t p1, hipStream_t st);
// The columns of the panel [p0, p1), multipliers included: leaves of up to 8
// columns factored in registers by one workgroup (k_lu_leaf, which stores the
// multipliers), each followed by the leaf's interchanges and updates on the
// other panel columns (k_lu_trail); a column whose rows do not fit a leaf goes
// through launch_lu_column and is scaled by launch_lu_scale at the end. The
// mode picks the leaf widths (automatic: the widest that fits) or forces one
// width, or columns only; every mode gives the same factors bit for bit.
enum { kLuPanelAuto = 0, kLuPanelColumns = 1, kLuPanelLeaf8 = 2, kLuPanelLeaf4 = 3, kLuPanelLeaf2 = 4 };
hipError_t launch_lu_panel(double2 *A, int64_t lda, int64_t n, int64_t p0, int64_t p1, int64_t *ipiv,
                           int64_t *singular, int mode, hipStream_t st);
constexpr int64_t kLuPairWords = 4 * kLuMaxBlock;
hipError_t launch_swap_pairs(const int64_t *ipiv, int64_t c0, int64_t c1, int64_t n,
                             int64_t *pairs, hipStream_t st);
hipError_t launch_apply_pairs(double2 *A, int64_t lda, int64_t w, const int64_t *pairs, int64_t q0,
                              int64_t q1, int64_t q2, int64_t q3, hipStream_t st);
hipError_t launch_trsm(bool upper, const double2 *T, int64_t ldt, int64_t nb, double2 *X,
                       int64_t ldx, int64_t ncols, hipStream_t st);
hipError_t launch_identity(double2 *X, int64_t ldx, int64_t n, hipStream_t st);
hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t st);

// Native FP64 matrix-core GEMM.
struct NativeArgs {
  View A;  // op(A): rows i, contraction l
  View B;  // op(B): rows j, contraction l
  int64_t m, n, k;
  int cplx;
  double ar, ai, br, bi;
  int beta_zero;
  void *C;
  int64_t ldc;
};
hipError_t launch_native(const NativeArgs &a, hipStream_t st);

// One emulated complex product (the ozaki_zgemm path) whose scratch is the
// device memory of `scratch_bytes` bytes that scratch() provides (called after
// the argument checks and quick returns): nothing is allocated, phase timing
// is skipped, OZAKI_ERR_TOO_LARGE when the product needs more.
int zgemm_fixed_scratch(char transa, char transb, int64_t m, int64_t n, int64_t k, double ar,
                        double ai, const void *A, int64_t lda, const void *B, int64_t ldb,
                        double br, double bi, void *C, int64_t ldc, int slices,
                        int (*scratch)(char **), size_t scratch_bytes);

}  // namespace oz
