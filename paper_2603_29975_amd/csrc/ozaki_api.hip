// Host runtime and C ABI of libozaki: argument checks, quick returns,
// workspace, stream binding and the launch sequence of one emulated GEMM.
//
// One emulated call is four kernel kinds on the caller's stream:
//   fill (zero the exponent codes) -> scan op(A) rows, op(B) columns ->
//   split both operands into packed INT8 slices -> fused slice GEMM with FP64
//   recombination and alpha/beta.
// An Ozaki-II call shares the fill and scan, then writes INT8 residue planes,
// runs one batched INT8 GEMM over the moduli and rebuilds C by the CRT.
// The interface mirrors a BLAS GEMM because the paper's solver reaches the
// emulation through intercepted standard BLAS calls (Section 3.1).
#include <algorithm>
#include <array>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <vector>

#include "../../include/ozaki.h"
#include "ozaki_internal.hpp"

namespace {

using namespace oz;

constexpr int kMaxDev = 16;

struct DevInfo {
  bool valid = false;
  int num_cu = 0;
  char arch[64] = {};  // gcnArchName up to the first ':'
};

struct State {
  hipStream_t stream = nullptr;
  int split = -1;  // OZAKI_SPLIT_* of the single-product calls (-1: not read from OZAKI_SPLIT yet)
  void *user_ws = nullptr;
  size_t user_ws_bytes = 0;
  int64_t grid_limit = 0;  // ozaki_set_grid_limit (0: one persistent grid per the CU count)
  void *own_ws[kMaxDev] = {};
  size_t own_ws_bytes[kMaxDev] = {};
  DevInfo dev[kMaxDev];
};

State g;

// The LU graphs hold workspace pointers: dropped whenever the workspace moves.
void clear_lu_graphs();

// Slice kind of ozaki_dgemm / ozaki_zgemm and the debug hooks: set by
// ozaki_set_split, else OZAKI_SPLIT=b8 in the environment, else trunc-7.
bool split_b8() {
  if (g.split < 0) {
    const char *e = getenv("OZAKI_SPLIT");
    g.split = (e != nullptr && (std::strcmp(e, "b8") == 0 || std::strcmp(e, "1") == 0))
                  ? OZAKI_SPLIT_BAL8
                  : OZAKI_SPLIT_TRUNC7;
  }
  return g.split == OZAKI_SPLIT_BAL8;
}
int max_slices(bool b8) { return b8 ? kS8Max : OZAKI_S_MAX; }

// ---------------------------------------------------------------- timing
struct Mark {
  int phase;
  hipEvent_t start, stop;
};
struct Timing {
  bool on = false;
  int64_t calls = 0;
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
};
Timing g_tm;

hipEvent_t take_event() {
  if (!g_tm.pool.empty()) {
    hipEvent_t e = g_tm.pool.back();
    g_tm.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records the start of `phase` on the stream; returns the mark index or -1.
int phase_begin(int phase, hipStream_t st) {
  if (!g_tm.on) return -1;
  Mark mk{phase, take_event(), take_event()};
  if (mk.start == nullptr || mk.stop == nullptr) return -1;
  if (hipEventRecord(mk.start, st) != hipSuccess) return -1;
  g_tm.marks.push_back(mk);
  return (int)g_tm.marks.size() - 1;
}

void phase_end(int idx, hipStream_t st) {
  if (idx < 0) return;
  (void)hipEventRecord(g_tm.marks[idx].stop, st);
}

char up(char c) { return (char)std::toupper((unsigned char)c); }
bool trans_ok(char c) {
  c = up(c);
  return c == 'N' || c == 'T' || c == 'C';
}

int current_device(int *dev) {
  if (hipGetDevice(dev) != hipSuccess) return OZAKI_ERR_NO_DEVICE;
  if (*dev < 0 || *dev >= kMaxDev) return OZAKI_ERR_NO_DEVICE;
  DevInfo &d = g.dev[*dev];
  if (!d.valid) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, *dev) != hipSuccess || cu <= 0)
      return OZAKI_ERR_NO_DEVICE;
    d.num_cu = cu;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, *dev) != hipSuccess) return OZAKI_ERR_NO_DEVICE;
    size_t i = 0;
    for (; i + 1 < sizeof(d.arch) && prop.gcnArchName[i] && prop.gcnArchName[i] != ':'; ++i)
      d.arch[i] = prop.gcnArchName[i];
    d.arch[i] = 0;
    d.valid = true;
  }
  return OZAKI_OK;
}

// Workspace of at least `bytes`, from the caller's buffer or the library's own
// grow-only buffer on the current device.
int get_workspace(size_t bytes, void **out) {
  if (bytes == 0) bytes = 256;
  if (g.user_ws != nullptr) {
    if (bytes > g.user_ws_bytes) return OZAKI_ERR_WORKSPACE;
    *out = g.user_ws;
    return OZAKI_OK;
  }
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  if (g.own_ws_bytes[dev] < bytes) {
    clear_lu_graphs();
    if (g.own_ws[dev] != nullptr) {
      // hipFree waits for work still using the old buffer.
      if (hipFree(g.own_ws[dev]) != hipSuccess) return OZAKI_ERR_HIP;
      g.own_ws[dev] = nullptr;
      g.own_ws_bytes[dev] = 0;
    }
    const size_t grow = std::max(bytes, (size_t)64 << 20);
    void *p = nullptr;
    if (hipMalloc(&p, grow) != hipSuccess) {
      (void)hipGetLastError();
      return OZAKI_ERR_ALLOC;
    }
    g.own_ws[dev] = p;
    g.own_ws_bytes[dev] = grow;
  }
  *out = g.own_ws[dev];
  return OZAKI_OK;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Sizes of the packed operands of one emulated product.
struct Plan {
  int S;
  bool cplx;
  bool b8;                    // 8-bit balanced slices instead of trunc-7
  int64_t m, n, k;
  int64_t kprime, kpad, nkb;
  int64_t nprime;             // rows of B' (n or 2n)
  int64_t nrbQ, nrbP;         // 32-row blocks of A' and B' (padded to 128 rows)
  size_t off_codeA, off_codeB, off_SA, off_SB, off_flush, total;
  int64_t kb_chunk;
};

Plan make_plan(bool cplx, int64_t m, int64_t n, int64_t k, int S, int num_cu, bool b8 = false) {
  Plan p{};
  p.S = S;
  p.cplx = cplx;
  p.b8 = b8;
  p.m = m;
  p.n = n;
  p.k = k;
  p.kprime = cplx ? 2 * k : k;
  p.kpad = round_up(std::max<int64_t>(p.kprime, 1), kKPad);
  p.nkb = p.kpad / 32;
  p.nprime = cplx ? 2 * n : n;
  p.nrbQ = round_up(std::max<int64_t>(m, 1), kRowPad) / 32;
  p.nrbP = round_up(std::max<int64_t>(p.nprime, 1), kRowPad) / 32;
  p.kb_chunk = kb_chunk_for(S, b8);
  size_t off = 0;
  p.off_codeA = off;
  off += align256(sizeof(int) * (size_t)std::max<int64_t>(m, 1));
  p.off_codeB = off;
  off += align256(sizeof(int) * (size_t)std::max<int64_t>(n, 1));
  p.off_SA = off;
  off += align256((size_t)S * p.nrbQ * 32 * p.kpad);
  p.off_SB = off;
  off += align256((size_t)S * p.nrbP * 32 * p.kpad);
  p.off_flush = off;
  if (p.nkb > p.kb_chunk) off += align256(gemm_flush_bytes(S, 0, num_cu));
  p.total = off;
  return p;
}

View view_opA(const void *A, char trans, int64_t m, int64_t k, int64_t lda, bool cplx) {
  View v;
  v.base = A;
  v.R = m;
  v.L = k;
  if (up(trans) == 'N') {
    v.sr = 1;
    v.sl = lda;
  } else {
    v.sr = lda;
    v.sl = 1;
  }
  v.conj = cplx && up(trans) == 'C';
  return v;
}

// Columns j of op(B) (k x n) as the rows of the view.
View view_opB(const void *B, char trans, int64_t k, int64_t n, int64_t ldb, bool cplx) {
  View v;
  v.base = B;
  v.R = n;
  v.L = k;
  if (up(trans) == 'N') {
    v.sr = ldb;
    v.sl = 1;
  } else {
    v.sr = 1;
    v.sl = ldb;
  }
  v.conj = cplx && up(trans) == 'C';
  return v;
}

int hip_rc(hipError_t e) { return e == hipSuccess ? OZAKI_OK : OZAKI_ERR_HIP; }

// ---------------------------------------------------------------- autotune
// Tuning table of the fused GEMM: for each (real/complex, s, size bucket) the
// fastest tuning id found by ozaki_autotune. A bucket is the ceiling of log2
// of m, of the rows n' of B' and of the 32-deep contraction blocks.
struct TuneEntry {
  int id;
  double ms;
};
using TuneKey = std::array<int, 5>;
std::map<TuneKey, TuneEntry> g_tune;
bool g_tune_env_loaded = false;

int log2_bucket(int64_t x) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < x) ++b;
  return b;
}

TuneKey tune_key(bool cplx, int S, int64_t m, int64_t nprime, int64_t nkb) {
  return {cplx ? 1 : 0, S, log2_bucket(m), log2_bucket(nprime), log2_bucket(nkb)};
}

int tune_load(const char *path);

// Tuning id of one emulated product: OZAKI_GEMM_CONFIG (a tuning id) wins,
// then the tuning table (seeded once from the file named by OZAKI_TUNE_CACHE),
// then the default 0.
int gemm_config(bool cplx, int S, int64_t m, int64_t nprime, int64_t nkb) {
  static int env = -2;
  if (env == -2) {
    const char *e = getenv("OZAKI_GEMM_CONFIG");
    env = (e != nullptr && *e) ? atoi(e) : -1;
    if (env >= gemm_num_configs()) env = -1;
  }
  if (env >= 0) return env;
  if (!g_tune_env_loaded) {
    g_tune_env_loaded = true;
    const char *f = getenv("OZAKI_TUNE_CACHE");
    if (f != nullptr && *f) (void)tune_load(f);
  }
  const auto it = g_tune.find(tune_key(cplx, S, m, nprime, nkb));
  return it == g_tune.end() ? 0 : it->second.id;
}

// BLAS argument checks; returns 0 or -(argument number).
int check_gemm_args(char transa, char transb, int64_t m, int64_t n, int64_t k, int64_t lda,
                    int64_t ldb, int64_t ldc) {
  if (!trans_ok(transa)) return -1;
  if (!trans_ok(transb)) return -2;
  if (m < 0) return -3;
  if (n < 0) return -4;
  if (k < 0) return -5;
  const int64_t nrowa = up(transa) == 'N' ? m : k;
  const int64_t nrowb = up(transb) == 'N' ? k : n;
  if (lda < std::max<int64_t>(1, nrowa)) return -8;
  if (ldb < std::max<int64_t>(1, nrowb)) return -10;
  if (ldc < std::max<int64_t>(1, m)) return -13;
  return 0;
}

// Scan and split both operands into the workspace described by `p`.
int prepare(const Plan &p, char *ws, const View &va, const View &vb, hipStream_t st,
            bool timed = true) {
  int *codeA = reinterpret_cast<int *>(ws + p.off_codeA);
  int *codeB = reinterpret_cast<int *>(ws + p.off_codeB);
  int8_t *SA = reinterpret_cast<int8_t *>(ws + p.off_SA);
  int8_t *SB = reinterpret_cast<int8_t *>(ws + p.off_SB);
  int rc;
  int mk = timed ? phase_begin(OZAKI_PHASE_SCAN, st) : -1;
  // codeA and codeB lie back to back (codeB at off_codeB): one fill zeroes both
  if ((rc = hip_rc(launch_fill_i32(codeA, (int64_t)((p.off_codeB - p.off_codeA) / sizeof(int)) + p.n,
                                   0, st))))
    return rc;
  if ((rc = hip_rc(launch_scan(va, p.cplx, codeA, st)))) return rc;
  if ((rc = hip_rc(launch_scan(vb, p.cplx, codeB, st)))) return rc;
  phase_end(mk, st);
  mk = timed ? phase_begin(OZAKI_PHASE_SPLIT, st) : -1;
  if ((rc = hip_rc(launch_split(va, p.cplx, false, codeA, p.S, SA, p.nrbQ, p.nkb, st, p.b8))))
    return rc;
  if ((rc = hip_rc(launch_split(vb, p.cplx, true, codeB, p.S, SB, p.nrbP, p.nkb, st, p.b8))))
    return rc;
  phase_end(mk, st);
  return OZAKI_OK;
}

GemmProblem gemm_problem(const Plan &p, char *ws, double ar, double ai, double br, double bi,
                         bool beta_zero, void *C, int64_t ldc, int64_t *raw) {
  GemmProblem a{};
  a.SP = reinterpret_cast<const int8_t *>(ws + p.off_SB);
  a.SQ = reinterpret_cast<const int8_t *>(ws + p.off_SA);
  a.nrbP = p.nrbP;
  a.nrbQ = p.nrbQ;
  a.nkb = p.nkb;
  a.m = p.m;
  a.nprime = p.nprime;
  a.codeA = reinterpret_cast<const int *>(ws + p.off_codeA);
  a.codeB = reinterpret_cast<const int *>(ws + p.off_codeB);
  a.ar = ar;
  a.ai = ai;
  a.br = br;
  a.bi = bi;
  a.beta_zero = beta_zero ? 1 : 0;
  a.cplx = p.cplx ? 1 : 0;
  a.wbits = p.b8 ? 8 : kDigitBits;
  a.woff = p.b8 ? 4 : 0;
  a.C = C;
  a.ldc = ldc;
  a.raw = raw;
  return a;
}

GemmArgs gemm_args(const Plan &p, char *ws, double ar, double ai, double br, double bi,
                   bool beta_zero, void *C, int64_t ldc, int64_t *raw) {
  GemmArgs a{};
  a.one = gemm_problem(p, ws, ar, ai, br, bi, beta_zero, C, ldc, raw);
  a.flush_ws = reinterpret_cast<int64_t *>(ws + p.off_flush);
  a.kb_chunk = p.kb_chunk;
  a.chunked = p.nkb > p.kb_chunk ? 1 : 0;
  a.split = (a.chunked && p.nkb <= kb_split_for(p.S, p.b8)) ? 1 : 0;
  a.max_groups = g.grid_limit;
  return a;
}

// One emulated product. fixed_ws == nullptr: scratch from get_workspace and
// phase timing as enabled; otherwise the scratch is the device memory that
// fixed_ws provides (called once the arguments have passed their checks;
// fixed_cap bytes, OZAKI_ERR_TOO_LARGE beyond them) and nothing is allocated
// or timed.
int emulated_gemm_ws(bool cplx, char transa, char transb, int64_t m, int64_t n, int64_t k,
                     double ar, double ai, const void *A, int64_t lda, const void *B, int64_t ldb,
                     double br, double bi, void *C, int64_t ldc, int slices,
                     int (*fixed_ws)(char **), size_t fixed_cap) {
  int rc = check_gemm_args(transa, transb, m, n, k, lda, ldb, ldc);
  if (rc) return rc;
  const bool b8 = split_b8();
  if (slices < 1 || slices > max_slices(b8)) return -14;
  if (m == 0 || n == 0) return OZAKI_OK;
  if (C == nullptr) return -12;
  const bool alpha_zero = ar == 0.0 && ai == 0.0;
  const bool beta_zero = br == 0.0 && bi == 0.0;
  const bool beta_one = br == 1.0 && bi == 0.0;
  if (alpha_zero || k == 0) {
    if (beta_one) return OZAKI_OK;
    return hip_rc(launch_scale(cplx, m, n, br, bi, beta_zero, C, ldc, g.stream));
  }
  if (A == nullptr) return -7;
  if (B == nullptr) return -9;
  int dev = 0;
  if ((rc = current_device(&dev))) return rc;
  const Plan p = make_plan(cplx, m, n, k, slices, g.dev[dev].num_cu, b8);
  char *ws = nullptr;
  if (fixed_ws == nullptr) {
    void *wsv = nullptr;
    if ((rc = get_workspace(p.total, &wsv))) return rc;
    ws = static_cast<char *>(wsv);
  } else {
    if (p.total > fixed_cap) return OZAKI_ERR_TOO_LARGE;
    if ((rc = fixed_ws(&ws))) return rc;
  }
  const bool timed = fixed_ws == nullptr;
  const View va = view_opA(A, transa, m, k, lda, cplx);
  const View vb = view_opB(B, transb, k, n, ldb, cplx);
  if ((rc = prepare(p, ws, va, vb, g.stream, timed))) return rc;
  const GemmArgs ga = gemm_args(p, ws, ar, ai, br, bi, beta_zero, C, ldc, nullptr);
  const int mk = timed ? phase_begin(OZAKI_PHASE_GEMM, g.stream) : -1;
  rc = hip_rc(launch_ozgemm(slices, gemm_config(cplx, slices, m, p.nprime, p.nkb), ga,
                            g.dev[dev].num_cu, g.stream));
  phase_end(mk, g.stream);
  if (timed && g_tm.on) ++g_tm.calls;
  return rc;
}

int emulated_gemm(bool cplx, char transa, char transb, int64_t m, int64_t n, int64_t k,
                  double ar, double ai, const void *A, int64_t lda, const void *B, int64_t ldb,
                  double br, double bi, void *C, int64_t ldc, int slices) {
  return emulated_gemm_ws(cplx, transa, transb, m, n, k, ar, ai, A, lda, B, ldb, br, bi, C, ldc,
                          slices, nullptr, 0);
}

int native_gemm(bool cplx, char transa, char transb, int64_t m, int64_t n, int64_t k, double ar,
                double ai, const void *A, int64_t lda, const void *B, int64_t ldb, double br,
                double bi, void *C, int64_t ldc) {
  int rc = check_gemm_args(transa, transb, m, n, k, lda, ldb, ldc);
  if (rc) return rc;
  if (m == 0 || n == 0) return OZAKI_OK;
  if (C == nullptr) return -12;
  const bool alpha_zero = ar == 0.0 && ai == 0.0;
  const bool beta_zero = br == 0.0 && bi == 0.0;
  const bool beta_one = br == 1.0 && bi == 0.0;
  if (alpha_zero || k == 0) {
    if (beta_one) return OZAKI_OK;
    return hip_rc(launch_scale(cplx, m, n, br, bi, beta_zero, C, ldc, g.stream));
  }
  if (A == nullptr) return -7;
  if (B == nullptr) return -9;
  NativeArgs a{};
  a.A = view_opA(A, transa, m, k, lda, cplx);
  a.B = view_opB(B, transb, k, n, ldb, cplx);
  a.m = m;
  a.n = n;
  a.k = k;
  a.cplx = cplx ? 1 : 0;
  a.ar = ar;
  a.ai = ai;
  a.br = br;
  a.bi = bi;
  a.beta_zero = beta_zero ? 1 : 0;
  a.C = C;
  a.ldc = ldc;
  return hip_rc(launch_native(a, g.stream));
}

// ---------------------------------------------------------------- Ozaki-II
// Workspace of one Ozaki-II product: exponent codes, then the residue planes
// of A' (N planes of m rows) and of B' (N planes of n' rows) in the packed
// fragment layout (rows padded to 128, K' to 128).
struct Plan2 {
  int N, beta;
  bool cplx;
  int64_t m, n, k, kprime, kpad, nprime, nkb, nrbQ, nrbP;
  size_t off_codeA, off_codeB, off_RA, off_RB, total;
};

// 0, or the negative argument number of a size the path cannot take: -5 for
// K' above OZAKI2_K_MAX, -14 for too few moduli (beta < 1).
int make_plan2(bool cplx, int64_t m, int64_t n, int64_t k, int N, Plan2 *p) {
  *p = Plan2{};
  p->N = N;
  p->cplx = cplx;
  p->m = m;
  p->n = n;
  p->k = k;
  p->kprime = cplx ? 2 * k : k;
  p->nprime = cplx ? 2 * n : n;
  if (p->kprime > OZAKI2_K_MAX) return -5;
  p->beta = crt_beta(N, std::max<int64_t>(p->kprime, 1));
  if (p->beta < 1) return -14;
  p->kpad = round_up(std::max<int64_t>(p->kprime, 1), 128);
  p->nkb = p->kpad / 32;
  p->nrbQ = round_up(std::max<int64_t>(m, 1), kRowPad) / 32;
  p->nrbP = round_up(std::max<int64_t>(p->nprime, 1), kRowPad) / 32;
  size_t off = 0;
  p->off_codeA = off;
  off += align256(sizeof(int) * (size_t)std::max<int64_t>(m, 1));
  p->off_codeB = off;
  off += align256(sizeof(int) * (size_t)std::max<int64_t>(n, 1));
  p->off_RA = off;
  off += align256((size_t)N * p->nrbQ * p->nkb * kFragBytes);
  p->off_RB = off;
  off += align256((size_t)N * p->nrbP * p->nkb * kFragBytes);
  p->total = off;
  return 0;
}

int ozaki2_gemm_impl(bool cplx, char transa, char transb, int64_t m, int64_t n, int64_t k,
                     double ar, double ai, const void *A, int64_t lda, const void *B, int64_t ldb,
                     double br, double bi, void *C, int64_t ldc, int moduli) {
  int rc = check_gemm_args(transa, transb, m, n, k, lda, ldb, ldc);
  if (rc) return rc;
  if (moduli < OZAKI2_MODULI_MIN || moduli > OZAKI2_MODULI_MAX) return -14;
  if (m == 0 || n == 0) return OZAKI_OK;
  if (C == nullptr) return -12;
  const bool alpha_zero = ar == 0.0 && ai == 0.0;
  const bool beta_zero = br == 0.0 && bi == 0.0;
  const bool beta_one = br == 1.0 && bi == 0.0;
  if (alpha_zero || k == 0) {
    if (beta_one) return OZAKI_OK;
    return hip_rc(launch_scale(cplx, m, n, br, bi, beta_zero, C, ldc, g.stream));
  }
  if (A == nullptr) return -7;
  if (B == nullptr) return -9;
  Plan2 p;
  if ((rc = make_plan2(cplx, m, n, k, moduli, &p))) return rc;
  int dev = 0;
  if ((rc = current_device(&dev))) return rc;
  void *wsv = nullptr;
  if ((rc = get_workspace(p.total, &wsv))) return rc;
  char *ws = static_cast<char *>(wsv);
  int *codeA = reinterpret_cast<int *>(ws + p.off_codeA);
  int *codeB = reinterpret_cast<int *>(ws + p.off_codeB);
  int8_t *RA = reinterpret_cast<int8_t *>(ws + p.off_RA);
  int8_t *RB = reinterpret_cast<int8_t *>(ws + p.off_RB);
  const View va = view_opA(A, transa, m, k, lda, cplx);
  const View vb = view_opB(B, transb, k, n, ldb, cplx);
  hipStream_t st = g.stream;

  int mk = phase_begin(OZAKI_PHASE_SCAN, st);
  if ((rc = hip_rc(launch_fill_i32(codeA, (int64_t)((p.off_codeB - p.off_codeA) / sizeof(int)) + n,
                                   0, st))))
    return rc;
  if ((rc = hip_rc(launch_scan(va, cplx, codeA, st)))) return rc;
  if ((rc = hip_rc(launch_scan(vb, cplx, codeB, st)))) return rc;
  phase_end(mk, st);

  mk = phase_begin(OZAKI_PHASE_SPLIT, st);
  if ((rc = hip_rc(launch_residues(va, cplx, false, codeA, moduli, p.beta, RA, p.nrbQ, p.nkb, st))))
    return rc;
  if ((rc = hip_rc(launch_residues(vb, cplx, true, codeB, moduli, p.beta, RB, p.nrbP, p.nkb, st))))
    return rc;
  phase_end(mk, st);

  // the modular products and the rebuild: one fused kernel
  mk = phase_begin(OZAKI_PHASE_GEMM, st);
  Oz2Args ga{};
  ga.RA = RA;
  ga.RB = RB;
  ga.nrbQ = p.nrbQ;
  ga.nrbP = p.nrbP;
  ga.nkb = p.nkb;
  ga.m = m;
  ga.nprime = p.nprime;
  ga.codeA = codeA;
  ga.codeB = codeB;
  ga.beta = p.beta;
  ga.ar = ar;
  ga.ai = ai;
  ga.br = br;
  ga.bi = bi;
  ga.beta_zero = beta_zero ? 1 : 0;
  ga.cplx = cplx ? 1 : 0;
  ga.C = C;
  ga.ldc = ldc;
  rc = hip_rc(launch_oz2gemm(moduli, ga, g.dev[dev].num_cu, st));
  phase_end(mk, st);
  if (g_tm.on) ++g_tm.calls;
  return rc;
}

// ---------------------------------------------------------------- blocked LU
// C <- C - A B (complex, column-major blocks) through the emulated ZGEMM
// (slices > 0, the current slice kind) or the native FP64 one (slices == 0).
int lu_update(int slices, int64_t m, int64_t n, int64_t k, const double2 *A, int64_t lda,
              const double2 *B, int64_t ldb, double2 *C, int64_t ldc) {
  if (m <= 0 || n <= 0 || k <= 0) return OZAKI_OK;
  if (slices > 0)
    return emulated_gemm(true, 'N', 'N', m, n, k, -1.0, 0.0, A, lda, B, ldb, 1.0, 0.0, C, ldc,
                         slices);
  return native_gemm(true, 'N', 'N', m, n, k, -1.0, 0.0, A, lda, B, ldb, 1.0, 0.0, C, ldc);
}

// Per device: the singular-column flag (one int64), then the row
// interchange slots (kLuPairWords int64).
int64_t *g_lu_flag[kMaxDev] = {};

int lu_workspace(int64_t **out) {
  int dev = 0;
  if (int rc = current_device(&dev)) return rc;
  if (g_lu_flag[dev] == nullptr &&
      hipMalloc(&g_lu_flag[dev], sizeof(int64_t) * (1 + kLuPairWords)) != hipSuccess) {
    g_lu_flag[dev] = nullptr;
    return OZAKI_ERR_ALLOC;
  }
  *out = g_lu_flag[dev];
  return OZAKI_OK;
}

// How ozaki_zgetrf factors its panels: OZAKI_LU_PANEL=columns (one pivot and
// one update launch per column), leaf8 / leaf4 / leaf2 (that leaf width
// wherever its rows fit, else columns), anything else the widest leaf that
// fits. Read at every call; all modes give the same factors bit for bit.
int lu_panel_mode() {
  const char *e = getenv("OZAKI_LU_PANEL");
  if (e == nullptr) return kLuPanelAuto;
  if (std::strcmp(e, "columns") == 0) return kLuPanelColumns;
  if (std::strcmp(e, "leaf8") == 0) return kLuPanelLeaf8;
  if (std::strcmp(e, "leaf4") == 0) return kLuPanelLeaf4;
  if (std::strcmp(e, "leaf2") == 0) return kLuPanelLeaf2;
  return kLuPanelAuto;
}

int lu_args(int64_t n, const void *A, int64_t lda, const void *ipiv, int64_t nb, int slices) {
  if (n < 0) return -1;
  if (A == nullptr && n > 0) return -2;
  if (lda < std::max<int64_t>(1, n)) return -3;
  if (ipiv == nullptr && n > 0) return -4;
  if (nb < 1 || nb > kLuMaxBlock) return -5;
  if (slices < 0 || slices > max_slices(split_b8())) return -6;
  return 0;
}

// The launch sequence of a factorization ('F') or an inverse ('I'), run on
// the library's stream. With graphs on (ozaki_batched_graphs) and phase timing
// off, the sequence is captured once per argument set into a HIP graph on a
// private stream and replayed afterwards: a 2048 factorization is some 4,100
// small dependent launches, and a replayed graph spares their host
// submission. The workspace of the emulated updates is sized before capture
// (no allocation inside it); every launch parameter is fixed by the
// arguments, and the pivots reach later kernels through device memory only.
struct LuGraph {
  std::vector<uint8_t> sig;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};
std::list<LuGraph> g_lu_graphs;  // most recent first
constexpr size_t kLuGraphCache = 4;
hipStream_t g_lu_cap = nullptr;

template <typename Enqueue>
int lu_run(char what, int64_t n, ozaki_z *A, int64_t lda, int64_t *ipiv, ozaki_z *X, int64_t ldx,
           int64_t nb, int slices, Enqueue enqueue);

// View of op(X) for the debug hooks (see ozaki.h for `side`).
int debug_view(char kind, char side, char trans, int64_t rows, int64_t L, const void *X,
               int64_t ldx, View *v, bool *cplx) {
  kind = up(kind);
  side = up(side);
  if (kind != 'D' && kind != 'Z') return -1;
  if (side != 'A' && side != 'B') return -2;
  if (!trans_ok(trans)) return -3;
  if (rows < 0) return -4;
  if (L < 0) return -5;
  *cplx = kind == 'Z';
  if (side == 'A') {
    const int64_t need = up(trans) == 'N' ? rows : L;
    if (ldx < std::max<int64_t>(1, need)) return -7;
    *v = view_opA(X, trans, rows, L, ldx, *cplx);
  } else {
    const int64_t need = up(trans) == 'N' ? L : rows;
    if (ldx < std::max<int64_t>(1, need)) return -7;
    *v = view_opB(X, trans, L, rows, ldx, *cplx);
  }
  if (rows > 0 && L > 0 && X == nullptr) return -6;
  return 0;
}


// ---------------------------------------------------------------- batched
// A batched plan: device descriptors (problems, task and tile tables) and the
// packed-operand workspace of every problem in one allocation, plus the HIP
// graph of its launch sequence.
struct ScaleOp {
  int64_t m, n, ldc;
  double br, bi;
  bool beta_zero;
  void *C;
};

struct GroupDesc {
  int S;
  int64_t ntiles;
  size_t off_tile_prob, off_tile_local;
  bool chunked;
};

struct BatchedPlan {
  std::vector<uint8_t> sig;  // exact argument signature
  int dev = 0;
  void *mem = nullptr;
  bool owns_mem = true;  // false: mem belongs to a caller's buffer
  size_t off_probs = 0, off_scan = 0, off_scan_start = 0, off_split = 0, off_split_start = 0,
         off_flush = 0;
  int nscan = 0, nsplit = 0;
  int64_t scan_blocks = 0, split_blocks = 0;
  std::vector<GroupDesc> groups;
  std::vector<ScaleOp> scales;
  std::vector<int> used;  // slices used per problem
  int tune_id = 0;        // tile configuration of the grouped GEMM
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct BatchedState {
  bool graphs = true;
  std::list<BatchedPlan *> cache;  // most recent first
  hipStream_t cap = nullptr;       // private stream used for graph capture
};
BatchedState g_bat;
constexpr size_t kPlanCache = 4;

void free_plan(BatchedPlan *pl) {
  if (pl == nullptr) return;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->mem && pl->owns_mem) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(pl->dev);
    (void)hipFree(pl->mem);
    (void)hipSetDevice(cur);
  }
  delete pl;
}

template <typename T>
void sig_put(std::vector<uint8_t> &v, const T &x) {
  const uint8_t *b = reinterpret_cast<const uint8_t *>(&x);
  v.insert(v.end(), b, b + sizeof(T));
}

// Enqueue the plan's kernels on `st`.
int enqueue_plan(const BatchedPlan &pl, hipStream_t st, bool capturing) {
  char *base = static_cast<char *>(pl.mem);
  int rc;
  // phase events only when launching directly (never inside a graph capture)
  const bool timed = !capturing;
  int mk = timed ? phase_begin(OZAKI_PHASE_SCAN, st) : -1;
  if ((rc = hip_rc(launch_scan_batched(reinterpret_cast<const ScanTask *>(base + pl.off_scan),
                                       reinterpret_cast<const int64_t *>(base + pl.off_scan_start),
                                       pl.nscan, pl.scan_blocks, st))))
    return rc;
  phase_end(mk, st);
  mk = timed ? phase_begin(OZAKI_PHASE_SPLIT, st) : -1;
  if ((rc = hip_rc(launch_split_batched(reinterpret_cast<const SplitTask *>(base + pl.off_split),
                                        reinterpret_cast<const int64_t *>(base + pl.off_split_start),
                                        pl.nsplit, pl.split_blocks, st))))
    return rc;
  phase_end(mk, st);
  mk = timed ? phase_begin(OZAKI_PHASE_GEMM, st) : -1;
  for (const GroupDesc &gd : pl.groups) {
    GemmArgs a{};
    a.probs = reinterpret_cast<const GemmProblem *>(base + pl.off_probs);
    a.tile_prob = reinterpret_cast<const int *>(base + gd.off_tile_prob);
    a.tile_local = reinterpret_cast<const int *>(base + gd.off_tile_local);
    a.ntiles = gd.ntiles;
    a.flush_ws = reinterpret_cast<int64_t *>(base + pl.off_flush);
    a.kb_chunk = kb_chunk_for(gd.S);
    a.chunked = gd.chunked ? 1 : 0;
    a.max_groups = g.grid_limit;
    if ((rc = hip_rc(launch_ozgemm_grouped(gd.S, pl.tune_id, a, g.dev[pl.dev].num_cu, st))))
      return rc;
  }
  phase_end(mk, st);
  if (timed && g_tm.on) ++g_tm.calls;
  for (const ScaleOp &sc : pl.scales)
    if ((rc = hip_rc(launch_scale(true, sc.m, sc.n, sc.br, sc.bi, sc.beta_zero, sc.C, sc.ldc, st))))
      return rc;
  return OZAKI_OK;
}

// Builds (or finds) the plan of a validated batched call.
// Tile configuration of the grouped GEMM of batched calls: OZAKI_BATCHED_CONFIG
// (a tuning id) or the default 8, the four-wave 64 x 64 tiles (two workgroups
// per CU), which waste less padding on the small problems of a batch.
int batched_tune_id() {
  static int id = -2;
  if (id == -2) {
    const char *e = getenv("OZAKI_BATCHED_CONFIG");
    id = (e != nullptr && *e) ? atoi(e) : -1;
    if (id >= gemm_num_configs()) id = -1;
  }
  return id >= 0 ? id : 8;
}

// Lays out one batched plan: problem descriptors, scan and split task tables,
// tile tables (one group per slice count, longest contraction first) and the
// workspace of every emulated problem. alloc(total) provides the device memory
// (nullptr on failure); the descriptor tables are returned in `host`, to be
// copied to the start of that memory by the caller.
template <typename Alloc>
int build_plan(const char *transa, const char *transb, const int64_t *m, const int64_t *n,
               const int64_t *k, const ozaki_z *alpha, const ozaki_z *const *A,
               const int64_t *lda, const ozaki_z *const *B, const int64_t *ldb,
               const ozaki_z *beta, ozaki_z *const *C, const int64_t *ldc, int64_t batch,
               const int *slices, int num_cu, BatchedPlan *pl, Alloc alloc,
               std::vector<uint8_t> &host, const int *split_slices = nullptr,
               bool unscaled = false, int *const *ext_codeA = nullptr,
               int *const *ext_codeB = nullptr) {
  // ext_codeA/B (per batch entry): exponent codes already computed; the plan
  // then has no scan of its own and its split and GEMM read these
  const bool ext = ext_codeA != nullptr && ext_codeB != nullptr;
  std::vector<int64_t> prob_b;
  pl->used.assign((size_t)batch, 0);
  pl->tune_id = batched_tune_id();
  std::vector<GemmProblem> probs;
  std::vector<ScanTask> scans;
  std::vector<SplitTask> splits;
  std::vector<int> prob_S;
  std::vector<size_t> prob_ws;  // workspace offset of each emulated problem
  std::vector<Plan> plans;
  size_t ws_total = 0;
  size_t flush_bytes = 0;
  for (int64_t b = 0; b < batch; ++b) {
    pl->used[b] = slices[b];
    if (m[b] == 0 || n[b] == 0) continue;
    const bool alpha_zero = alpha[b].re == 0.0 && alpha[b].im == 0.0;
    const bool beta_zero = beta[b].re == 0.0 && beta[b].im == 0.0;
    const bool beta_one = beta[b].re == 1.0 && beta[b].im == 0.0;
    if (alpha_zero || k[b] == 0) {
      if (!beta_one) pl->scales.push_back({m[b], n[b], ldc[b], beta[b].re, beta[b].im, beta_zero, C[b]});
      continue;
    }
    // the operands are split to split_slices[b] >= slices[b] digits (trunc-7
    // digits at s are a prefix of those at more slices); the GEMM takes the
    // first slices[b]
    const int S_split = split_slices != nullptr ? std::max(split_slices[b], slices[b]) : slices[b];
    Plan p = make_plan(true, m[b], n[b], k[b], S_split, num_cu);
    p.S = slices[b];
    p.kb_chunk = kb_chunk_for(slices[b]);
    plans.push_back(p);
    prob_ws.push_back(ws_total);
    ws_total += align256(p.off_flush);  // codes and packed operands (carry space is shared)
    prob_S.push_back(slices[b]);
    if (p.nkb > p.kb_chunk) flush_bytes = std::max(flush_bytes, gemm_flush_bytes(p.S, 0, num_cu));
    GemmProblem gp = gemm_problem(p, nullptr, alpha[b].re, alpha[b].im, beta[b].re, beta[b].im,
                                  beta_zero, C[b], ldc[b], nullptr);
    gp.unscaled = unscaled ? 1 : 0;
    probs.push_back(gp);
    const View va = view_opA(A[b], transa[b], m[b], k[b], lda[b], true);
    const View vb = view_opB(B[b], transb[b], k[b], n[b], ldb[b], true);
    prob_b.push_back(b);
    if (!ext) {
      scans.push_back({va, nullptr, 1, va.sr == 1 ? 1 : 0});
      scans.push_back({vb, nullptr, 1, vb.sr == 1 ? 1 : 0});
    }
    splits.push_back({va, nullptr, nullptr, p.nrbQ, p.nkb, S_split, 1, 0});
    splits.push_back({vb, nullptr, nullptr, p.nrbP, p.nkb, S_split, 1, 1});
  }
  const size_t np = probs.size();

  // tile tables, one group per distinct slice count, longest contraction first
  std::map<int, std::vector<std::pair<int, int>>> tiles;  // S -> (problem, local tile)
  for (size_t i = 0; i < np; ++i) {
    const int64_t nt = gemm_tiles(prob_S[i], pl->tune_id, plans[i].m, plans[i].nprime);
    for (int64_t t = 0; t < nt; ++t) tiles[prob_S[i]].push_back({(int)i, (int)t});
  }
  for (auto &kv : tiles)
    std::stable_sort(kv.second.begin(), kv.second.end(),
                     [&](const std::pair<int, int> &x, const std::pair<int, int> &y) {
                       return plans[x.first].nkb > plans[y.first].nkb;
                     });

  // device layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(std::max<size_t>(bytes, 1));
    return o;
  };
  pl->off_probs = take(np * sizeof(GemmProblem));
  pl->nscan = (int)scans.size();
  pl->off_scan = take(scans.size() * sizeof(ScanTask));
  pl->off_scan_start = take((scans.size() + 1) * sizeof(int64_t));
  pl->nsplit = (int)splits.size();
  pl->off_split = take(splits.size() * sizeof(SplitTask));
  pl->off_split_start = take((splits.size() + 1) * sizeof(int64_t));
  for (auto &kv : tiles) {
    GroupDesc gd{};
    gd.S = kv.first;
    gd.ntiles = (int64_t)kv.second.size();
    gd.off_tile_prob = take(kv.second.size() * sizeof(int));
    gd.off_tile_local = take(kv.second.size() * sizeof(int));
    gd.chunked = false;
    for (auto &pt : kv.second) gd.chunked = gd.chunked || plans[pt.first].nkb > plans[pt.first].kb_chunk;
    pl->groups.push_back(gd);
  }
  pl->off_flush = take(flush_bytes);
  const size_t desc_bytes = off;
  const size_t off_ws = take(ws_total);
  const size_t total = off;

  char *base = alloc(total);
  if (base == nullptr) return OZAKI_ERR_ALLOC;
  pl->mem = base;

  // patch device pointers into the descriptors
  for (size_t i = 0; i < np; ++i) {
    char *w = base + off_ws + prob_ws[i];
    const Plan &p = plans[i];
    GemmProblem &gp = probs[i];
    gp.SP = reinterpret_cast<const int8_t *>(w + p.off_SB);
    gp.SQ = reinterpret_cast<const int8_t *>(w + p.off_SA);
    int *ca = ext ? ext_codeA[prob_b[i]] : reinterpret_cast<int *>(w + p.off_codeA);
    int *cb = ext ? ext_codeB[prob_b[i]] : reinterpret_cast<int *>(w + p.off_codeB);
    gp.codeA = ca;
    gp.codeB = cb;
    if (!ext) {
      scans[2 * i].code = ca;
      scans[2 * i + 1].code = cb;
    }
    splits[2 * i].code = ca;
    splits[2 * i].out = reinterpret_cast<int8_t *>(w + p.off_SA);
    splits[2 * i + 1].code = cb;
    splits[2 * i + 1].out = reinterpret_cast<int8_t *>(w + p.off_SB);
  }
  host.assign(desc_bytes, 0);
  auto put = [&](size_t o, const void *src, size_t bytes) {
    if (bytes) std::memcpy(host.data() + o, src, bytes);
  };
  put(pl->off_probs, probs.data(), np * sizeof(GemmProblem));
  put(pl->off_scan, scans.data(), scans.size() * sizeof(ScanTask));
  put(pl->off_split, splits.data(), splits.size() * sizeof(SplitTask));
  std::vector<int64_t> start(scans.size() + 1, 0);
  for (size_t t = 0; t < scans.size(); ++t) start[t + 1] = start[t] + scan_task_blocks(scans[t]);
  pl->scan_blocks = start.back();
  put(pl->off_scan_start, start.data(), start.size() * sizeof(int64_t));
  start.assign(splits.size() + 1, 0);
  for (size_t t = 0; t < splits.size(); ++t) start[t + 1] = start[t] + split_task_blocks(splits[t]);
  pl->split_blocks = start.back();
  put(pl->off_split_start, start.data(), start.size() * sizeof(int64_t));
  size_t gi = 0;
  for (auto &kv : tiles) {
    std::vector<int> tp(kv.second.size()), tl(kv.second.size());
    for (size_t x = 0; x < kv.second.size(); ++x) {
      tp[x] = kv.second[x].first;
      tl[x] = kv.second[x].second;
    }
    put(pl->groups[gi].off_tile_prob, tp.data(), tp.size() * sizeof(int));
    put(pl->groups[gi].off_tile_local, tl.data(), tl.size() * sizeof(int));
    ++gi;
  }
  return OZAKI_OK;
}

int get_plan(const char *transa, const char *transb, const int64_t *m, const int64_t *n,
             const int64_t *k, const ozaki_z *alpha, const ozaki_z *const *A, const int64_t *lda,
             const ozaki_z *const *B, const int64_t *ldb, const ozaki_z *beta, ozaki_z *const *C,
             const int64_t *ldc, int64_t batch, const int *slices, BatchedPlan **out) {
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  std::vector<uint8_t> sig;
  sig_put(sig, dev);
  sig_put(sig, batch);
  for (int64_t b = 0; b < batch; ++b) {
    sig_put(sig, up(transa[b]));
    sig_put(sig, up(transb[b]));
    sig_put(sig, m[b]);
    sig_put(sig, n[b]);
    sig_put(sig, k[b]);
    sig_put(sig, alpha[b]);
    sig_put(sig, A[b]);
    sig_put(sig, lda[b]);
    sig_put(sig, B[b]);
    sig_put(sig, ldb[b]);
    sig_put(sig, beta[b]);
    sig_put(sig, C[b]);
    sig_put(sig, ldc[b]);
    sig_put(sig, slices[b]);
  }
  for (auto it = g_bat.cache.begin(); it != g_bat.cache.end(); ++it) {
    if ((*it)->sig == sig) {
      BatchedPlan *pl = *it;
      g_bat.cache.erase(it);
      g_bat.cache.push_front(pl);
      *out = pl;
      return OZAKI_OK;
    }
  }

  BatchedPlan *pl = new BatchedPlan();
  pl->sig = std::move(sig);
  pl->dev = dev;
  std::vector<uint8_t> host;
  rc = build_plan(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, batch, slices,
                  g.dev[dev].num_cu, pl,
                  [](size_t bytes) -> char * {
                    void *p = nullptr;
                    if (hipMalloc(&p, bytes) != hipSuccess) {
                      (void)hipGetLastError();
                      return nullptr;
                    }
                    return static_cast<char *>(p);
                  },
                  host);
  if (rc) {
    free_plan(pl);
    return rc;
  }

  if (hipMemcpy(pl->mem, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    free_plan(pl);
    return OZAKI_ERR_HIP;
  }

  if (g_bat.graphs) {
    if (g_bat.cap == nullptr && hipStreamCreateWithFlags(&g_bat.cap, hipStreamNonBlocking) != hipSuccess) {
      free_plan(pl);
      return OZAKI_ERR_HIP;
    }
    if (hipStreamBeginCapture(g_bat.cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      free_plan(pl);
      return OZAKI_ERR_HIP;
    }
    const int erc = enqueue_plan(*pl, g_bat.cap, true);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(g_bat.cap, &graph);
    pl->graph = graph;
    if (erc != OZAKI_OK || e != hipSuccess ||
        hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGetLastError();
      free_plan(pl);
      return OZAKI_ERR_HIP;
    }
  }

  g_bat.cache.push_front(pl);
  while (g_bat.cache.size() > kPlanCache) {
    BatchedPlan *old = g_bat.cache.back();
    g_bat.cache.pop_back();
    free_plan(old);
  }
  *out = pl;
  return OZAKI_OK;
}

// Validated fixed-slice batched call: plan (cached) + graph replay or launches.
int run_fixed_batched(const char *transa, const char *transb, const int64_t *m, const int64_t *n,
                      const int64_t *k, const ozaki_z *alpha, const ozaki_z *const *A,
                      const int64_t *lda, const ozaki_z *const *B, const int64_t *ldb,
                      const ozaki_z *beta, ozaki_z *const *C, const int64_t *ldc, int64_t batch,
                      const int *slices) {
  BatchedPlan *pl = nullptr;
  int rc = get_plan(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, batch, slices, &pl);
  if (rc) return rc;
  if (pl->exec != nullptr) return hip_rc(hipGraphLaunch(pl->exec, g.stream));
  return enqueue_plan(*pl, g.stream, false);
}

// ---------------------------------------------------------------- automatic slices
struct SelectorState {
  bool loaded = false;
  int dev = -1;
  void *state = nullptr;  // MLP state (device)
  float margin = 0.5f;
  double target = 1e-11;
  double kappa = 8.0;     // probe estimate times kappa must meet the target
  void *ws = nullptr;     // grow-only scratch of the automatic mode
  size_t ws_bytes = 0;
  void *plan_ws = nullptr;  // grow-only memory of the per-round batched plans
  size_t plan_ws_bytes = 0;
};
SelectorState g_sel;

// Memory for one round's batched plan in the automatic mode (grow-only; the
// previous round's work is complete before the next plan is laid out).
char *sel_plan_memory(size_t bytes) {
  if (g_sel.plan_ws_bytes < bytes) {
    if (g_sel.plan_ws != nullptr) {
      (void)hipFree(g_sel.plan_ws);
      g_sel.plan_ws = nullptr;
      g_sel.plan_ws_bytes = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_sel.plan_ws = p;
    g_sel.plan_ws_bytes = bytes;
  }
  return static_cast<char *>(g_sel.plan_ws);
}

int load_selector(const float *params, float margin, double target, double kappa) {
  if (params == nullptr) return -1;
  if (!(margin >= -4.0f && margin <= 8.0f)) return -2;
  if (!(target > 0.0)) return -3;
  if (!(kappa >= 1.0)) return -4;
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  if (g_sel.state != nullptr && g_sel.dev != dev) {
    (void)hipFree(g_sel.state);
    g_sel.state = nullptr;
  }
  if (g_sel.state == nullptr) {
    if (hipMalloc(&g_sel.state, mlp_state_bytes()) != hipSuccess) {
      (void)hipGetLastError();
      return OZAKI_ERR_ALLOC;
    }
    if (hipMemset(g_sel.state, 0, mlp_state_bytes()) != hipSuccess) return OZAKI_ERR_HIP;
  }
  if (hipMemcpy(g_sel.state, params, sizeof(float) * mlp_params(), hipMemcpyHostToDevice) != hipSuccess)
    return OZAKI_ERR_HIP;
  if ((rc = hip_rc(mlp_refresh(g_sel.state, nullptr)))) return rc;
  if (hipDeviceSynchronize() != hipSuccess) return OZAKI_ERR_HIP;
  g_sel.dev = dev;
  g_sel.margin = margin;
  g_sel.target = target;
  g_sel.kappa = kappa;
  g_sel.loaded = true;
  return OZAKI_OK;
}

int auto_ws(size_t bytes, char **out) {
  if (g_sel.ws_bytes < bytes) {
    if (g_sel.ws) (void)hipFree(g_sel.ws);
    g_sel.ws = nullptr;
    g_sel.ws_bytes = 0;
    if (hipMalloc(&g_sel.ws, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return OZAKI_ERR_ALLOC;
    }
    g_sel.ws_bytes = bytes;
  }
  *out = static_cast<char *>(g_sel.ws);
  return OZAKI_OK;
}

// Slices per problem from the selector, checked by the residual probe. Every
// product is formed at its predicted s with its operands split one slice
// deeper, into library memory as the recombined sums before the final
// 2^(e_i + f_j) scaling (alpha = 1, beta = 0). The probe and the decision run
// on the device: a product that misses the target gets its next diagonal
// added to the stored sums (the trunc-7 prefix property: the result is then
// exactly the product at s + 1) and is probed again. The host synchronises
// twice per pass (the predictions, then the final slice counts); a product
// still missing the target after that is formed again two slices higher in a
// further pass. C is finished with alpha and beta exactly as the fused
// epilogue would, so the result equals a fixed-s call at the final s bit for
// bit.
constexpr uint64_t kProbeSeed = 0x5eed0000ull;  // round r of the automatic mode probes with seed + r
constexpr int kProbeVectors = 2;

int auto_batched(const char *transa, const char *transb, const int64_t *m, const int64_t *n,
                 const int64_t *k, const ozaki_z *alpha, const ozaki_z *const *A,
                 const int64_t *lda, const ozaki_z *const *B, const int64_t *ldb,
                 const ozaki_z *beta, ozaki_z *const *C, const int64_t *ldc, int64_t batch,
                 int *slices_used) {
  if (!g_sel.loaded) return OZAKI_ERR_NO_SELECTOR;
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  if (dev != g_sel.dev) return OZAKI_ERR_NO_SELECTOR;
  hipStream_t st = g.stream;
  std::vector<int> used((size_t)batch, 0);
  std::vector<int64_t> E;  // emulated problems
  std::vector<ScaleOp> scales;
  for (int64_t b = 0; b < batch; ++b) {
    if (m[b] == 0 || n[b] == 0) continue;
    const bool alpha_zero = alpha[b].re == 0.0 && alpha[b].im == 0.0;
    const bool beta_zero = beta[b].re == 0.0 && beta[b].im == 0.0;
    const bool beta_one = beta[b].re == 1.0 && beta[b].im == 0.0;
    if (alpha_zero || k[b] == 0) {
      if (!beta_one) scales.push_back({m[b], n[b], ldc[b], beta[b].re, beta[b].im, beta_zero, C[b]});
      continue;
    }
    E.push_back(b);
  }
  const int64_t ne = (int64_t)E.size();
  // scratch layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(std::max<size_t>(bytes, 1));
    return o;
  };
  std::vector<size_t> o_codeA(ne), o_codeB(ne), o_P(ne), o_w(ne), o_est(ne);
  int64_t diag_tiles_all = 0;
  for (int64_t e = 0; e < ne; ++e) {
    const int64_t b = E[e];
    o_codeA[e] = take(sizeof(int) * m[b]);
    o_codeB[e] = take(sizeof(int) * n[b]);
    o_P[e] = take(sizeof(ozaki_z) * m[b] * n[b]);
    o_w[e] = take(probe_workspace_bytes(m[b], n[b], k[b]));
    o_est[e] = take(sizeof(double) * m[b]);
    diag_tiles_all += diag_tiles(m[b], 2 * n[b]);
  }
  const size_t o_hist = take(sizeof(int) * 64 * ne), o_dims = take(sizeof(int64_t) * 3 * ne),
               o_feat = take(sizeof(float) * 64 * ne), o_y = take(sizeof(float) * ne),
               o_scan = take(sizeof(ScanTask) * 2 * ne), o_scan_s = take(sizeof(int64_t) * (2 * ne + 1)),
               o_ft = take(sizeof(FeatTask) * 2 * ne), o_ft_s = take(sizeof(int64_t) * (2 * ne + 1)),
               o_pt = take(sizeof(ProbeTask) * ne), o_ax = take(sizeof(AxpbyTask) * ne),
               o_ax_s = take(sizeof(int64_t) * (ne + 1)), o_mlp = take(mlp_scratch_bytes(ne)),
               o_emax = take(sizeof(double) * ne), o_s = take(sizeof(int) * ne),
               o_cap = take(sizeof(int) * ne), o_flag = take(sizeof(int) * ne),
               o_dt = take(sizeof(DiagTask) * ne), o_dtp = take(sizeof(int) * diag_tiles_all),
               o_dtl = take(sizeof(int) * diag_tiles_all);
  char *ws = nullptr;
  if ((rc = auto_ws(off, &ws))) return rc;
  auto h2d = [&](size_t o, const void *src, size_t bytes) {
    return bytes ? hip_rc(hipMemcpyAsync(ws + o, src, bytes, hipMemcpyHostToDevice, st)) : OZAKI_OK;
  };

  // features and selector
  std::vector<ScanTask> scans;
  std::vector<FeatTask> feats;
  std::vector<int64_t> dims;
  for (int64_t e = 0; e < ne; ++e) {
    const int64_t b = E[e];
    const View va = view_opA(A[b], transa[b], m[b], k[b], lda[b], true);
    const View vb = view_opB(B[b], transb[b], k[b], n[b], ldb[b], true);
    int *ca = reinterpret_cast<int *>(ws + o_codeA[e]);
    int *cb = reinterpret_cast<int *>(ws + o_codeB[e]);
    int *h = reinterpret_cast<int *>(ws + o_hist) + 64 * e;
    scans.push_back({va, ca, 1, va.sr == 1 ? 1 : 0});
    scans.push_back({vb, cb, 1, vb.sr == 1 ? 1 : 0});
    feats.push_back({va, ca, h, 1, va.sr == 1 ? 1 : 0, 32});
    feats.push_back({vb, cb, h + 32, 1, vb.sr == 1 ? 1 : 0, 31});
    dims.push_back(m[b]);
    dims.push_back(n[b]);
    dims.push_back(k[b]);
  }
  std::vector<int64_t> ss(2 * ne + 1, 0), fs(2 * ne + 1, 0);
  for (size_t t = 0; t < scans.size(); ++t) ss[t + 1] = ss[t] + scan_task_blocks(scans[t]);
  for (size_t t = 0; t < feats.size(); ++t) fs[t + 1] = fs[t] + feat_task_blocks(feats[t]);
  if ((rc = h2d(o_scan, scans.data(), scans.size() * sizeof(ScanTask)))) return rc;
  if ((rc = h2d(o_scan_s, ss.data(), ss.size() * sizeof(int64_t)))) return rc;
  if ((rc = h2d(o_ft, feats.data(), feats.size() * sizeof(FeatTask)))) return rc;
  if ((rc = h2d(o_ft_s, fs.data(), fs.size() * sizeof(int64_t)))) return rc;
  if ((rc = h2d(o_dims, dims.data(), dims.size() * sizeof(int64_t)))) return rc;
  if ((rc = hip_rc(launch_fill_i32(reinterpret_cast<int *>(ws + o_hist), 64 * ne, 0, st)))) return rc;
  if ((rc = hip_rc(launch_scan_batched(reinterpret_cast<const ScanTask *>(ws + o_scan),
                                       reinterpret_cast<const int64_t *>(ws + o_scan_s),
                                       (int)scans.size(), ss.back(), st))))
    return rc;
  if ((rc = hip_rc(launch_feat_hist(reinterpret_cast<const FeatTask *>(ws + o_ft),
                                    reinterpret_cast<const int64_t *>(ws + o_ft_s),
                                    (int)feats.size(), fs.back(), st))))
    return rc;
  if ((rc = hip_rc(launch_feat_finish(reinterpret_cast<const int *>(ws + o_hist),
                                      reinterpret_cast<const int64_t *>(ws + o_dims),
                                      reinterpret_cast<float *>(ws + o_feat), ne, st))))
    return rc;
  if ((rc = hip_rc(mlp_forward(g_sel.state, ne, reinterpret_cast<const float *>(ws + o_feat),
                               reinterpret_cast<float *>(ws + o_y), ws + o_mlp, st))))
    return rc;
  std::vector<float> y(ne);
  if (ne && (rc = hip_rc(hipMemcpyAsync(y.data(), ws + o_y, sizeof(float) * ne,
                                        hipMemcpyDeviceToHost, st))))
    return rc;
  if ((rc = hip_rc(hipStreamSynchronize(st)))) return rc;
  std::vector<int> s_of(ne);
  for (int64_t e = 0; e < ne; ++e) {
    const double v = std::ceil((double)y[e] + (double)g_sel.margin);
    s_of[e] = (int)std::min<double>(OZAKI_S_MAX, std::max<double>(1.0, std::isfinite(v) ? v : OZAKI_S_MAX));
  }

  int *s_dev = reinterpret_cast<int *>(ws + o_s);
  int *cap_dev = reinterpret_cast<int *>(ws + o_cap);
  int *flag_dev = reinterpret_cast<int *>(ws + o_flag);
  double *emax = reinterpret_cast<double *>(ws + o_emax);
  const ProbeTask *pt_dev = reinterpret_cast<const ProbeTask *>(ws + o_pt);
  std::vector<int64_t> pending(ne);
  for (int64_t e = 0; e < ne; ++e) pending[e] = e;
  for (int pass = 0; !pending.empty() && pass <= OZAKI_S_MAX; ++pass) {
    const size_t np = pending.size();
    std::vector<char> ta(np), tb(np);
    std::vector<int64_t> mm(np), nn(np), kk(np), la(np), lb(np), lc(np);
    std::vector<ozaki_z> one(np, ozaki_z{1.0, 0.0}), zero(np, ozaki_z{0.0, 0.0});
    std::vector<const ozaki_z *> pa(np), pb(np);
    std::vector<ozaki_z *> pc(np);
    std::vector<int> sl(np), cap(np);
    std::vector<int *> eca(np), ecb(np);  // the feature scan's codes: no second scan
    for (size_t x = 0; x < np; ++x) {
      const int64_t e = pending[x], b = E[e];
      eca[x] = reinterpret_cast<int *>(ws + o_codeA[e]);
      ecb[x] = reinterpret_cast<int *>(ws + o_codeB[e]);
      ta[x] = transa[b];
      tb[x] = transb[b];
      mm[x] = m[b];
      nn[x] = n[b];
      kk[x] = k[b];
      la[x] = lda[b];
      lb[x] = ldb[b];
      lc[x] = m[b];
      pa[x] = A[b];
      pb[x] = B[b];
      pc[x] = reinterpret_cast<ozaki_z *>(ws + o_P[e]);
      sl[x] = s_of[e];
      cap[x] = std::min(OZAKI_S_MAX, s_of[e] + 1);
    }
    // this pass's products at their slice counts, split one slice deeper,
    // stored unscaled: a one-off plan in the automatic mode's own memory,
    // launched directly (no cache, no graph)
    BatchedPlan rp;
    rp.dev = dev;
    rp.owns_mem = false;
    std::vector<uint8_t> host;
    if ((rc = build_plan(ta.data(), tb.data(), mm.data(), nn.data(), kk.data(), one.data(), pa.data(),
                         la.data(), pb.data(), lb.data(), zero.data(), pc.data(), lc.data(),
                         (int64_t)np, sl.data(), g.dev[dev].num_cu, &rp, sel_plan_memory, host,
                         cap.data(), true, eca.data(), ecb.data())))
      return rc;
    if ((rc = hip_rc(hipMemcpyAsync(rp.mem, host.data(), host.size(), hipMemcpyHostToDevice, st))))
      return rc;
    if ((rc = enqueue_plan(rp, st, false))) return rc;

    // probe tasks (recombined sums scaled on the fly by the feature scan's
    // codes, which equal the plan's), decision state, one-diagonal tasks
    const GemmProblem *gps = reinterpret_cast<const GemmProblem *>(host.data() + rp.off_probs);
    std::vector<ProbeTask> pts(np);
    std::vector<DiagTask> dts(np);
    std::vector<int> dtp, dtl;
    int64_t nblk[4] = {0, 0, 0, 0};
    for (size_t x = 0; x < np; ++x) {
      const int64_t e = pending[x], b = E[e];
      ProbeTask &pt = pts[x];
      pt = probe_task(view_opA(A[b], transa[b], m[b], k[b], lda[b], true),
                      view_opB(B[b], transb[b], k[b], n[b], ldb[b], true), true, pc[x], m[b],
                      kProbeVectors, kProbeSeed, ws + o_w[e],
                      reinterpret_cast<double *>(ws + o_est[e]));
      pt.codeA = reinterpret_cast<const int *>(ws + o_codeA[e]);
      pt.codeB = reinterpret_cast<const int *>(ws + o_codeB[e]);
      pt.flag = flag_dev;
      pt.id = (int64_t)x;
      for (int stage = 0; stage < 4; ++stage) {
        pt.blk[stage] = nblk[stage];
        nblk[stage] += probe_stage_blocks(pt, stage);
      }
      const GemmProblem &gp = gps[x];
      dts[x] = DiagTask{gp.SP, gp.SQ, gp.nrbP, gp.nrbQ, gp.nkb, gp.m, gp.nprime, pc[x], 1,
                        kDigitBits, 0, (int64_t)x};
      const int64_t nt = diag_tiles(gp.m, gp.nprime);
      for (int64_t t = 0; t < nt; ++t) {
        dtp.push_back((int)x);
        dtl.push_back((int)t);
      }
    }
    std::vector<int> ones(np, 1);
    if ((rc = h2d(o_s, sl.data(), np * sizeof(int)))) return rc;
    if ((rc = h2d(o_cap, cap.data(), np * sizeof(int)))) return rc;
    if ((rc = h2d(o_flag, ones.data(), np * sizeof(int)))) return rc;  // round 0 probes all
    if ((rc = h2d(o_dt, dts.data(), np * sizeof(DiagTask)))) return rc;
    if ((rc = h2d(o_dtp, dtp.data(), dtp.size() * sizeof(int)))) return rc;
    if ((rc = h2d(o_dtl, dtl.data(), dtl.size() * sizeof(int)))) return rc;
    // one host copy of the task table per round: an asynchronous copy may
    // read its host buffer after the call returns
    std::vector<ProbeTask> pts1 = pts;
    for (int round = 0; round < 2; ++round) {
      std::vector<ProbeTask> &pr = round == 0 ? pts : pts1;
      for (size_t x = 0; x < np; ++x) pr[x].seed = kProbeSeed + (uint64_t)(2 * pass + round);
      if ((rc = h2d(o_pt, pr.data(), np * sizeof(ProbeTask)))) return rc;
      if ((rc = hip_rc(launch_probe_batched(pt_dev, (int)np, nblk, st)))) return rc;
      if ((rc = hip_rc(launch_probe_max_batched(pt_dev, (int)np, emax, st)))) return rc;
      if ((rc = hip_rc(launch_probe_decide(emax, (int64_t)np, g_sel.kappa, g_sel.target, OZAKI_S_MAX,
                                           s_dev, cap_dev, flag_dev, round == 0 ? 1 : 0, st))))
        return rc;
      if (round == 0 &&
          (rc = hip_rc(launch_add_diagonal(reinterpret_cast<const DiagTask *>(ws + o_dt),
                                           reinterpret_cast<const int *>(ws + o_dtp),
                                           reinterpret_cast<const int *>(ws + o_dtl),
                                           (int64_t)dtp.size(), s_dev, flag_dev, st))))
        return rc;
    }
    std::vector<int> s_fin(np), f_fin(np);
    if ((rc = hip_rc(hipMemcpyAsync(s_fin.data(), s_dev, np * sizeof(int), hipMemcpyDeviceToHost, st))))
      return rc;
    if ((rc = hip_rc(hipMemcpyAsync(f_fin.data(), flag_dev, np * sizeof(int), hipMemcpyDeviceToHost,
                                    st))))
      return rc;
    // also keeps `host` and the task vectors alive until their copies are done
    if ((rc = hip_rc(hipStreamSynchronize(st)))) return rc;
    std::vector<int64_t> next;
    for (size_t x = 0; x < np; ++x) {
      const int64_t e = pending[x];
      s_of[e] = s_fin[x];
      if (f_fin[x] == 2) {  // missed at the deepest slice of this pass: form it again higher
        s_of[e] = std::min(OZAKI_S_MAX, s_fin[x] + 1);
        next.push_back(e);
      }
    }
    pending.swap(next);
  }

  // finish: C = alpha 2^(e_i + f_j) P + beta C
  std::vector<AxpbyTask> ax(ne);
  std::vector<int64_t> as(ne + 1, 0);
  for (int64_t e = 0; e < ne; ++e) {
    const int64_t b = E[e];
    ax[e] = {ws + o_P[e], C[b], m[b], n[b], ldc[b], alpha[b].re, alpha[b].im, beta[b].re, beta[b].im,
             (beta[b].re == 0.0 && beta[b].im == 0.0) ? 1 : 0,
             reinterpret_cast<const int *>(ws + o_codeA[e]), reinterpret_cast<const int *>(ws + o_codeB[e])};
    as[e + 1] = as[e] + axpby_task_blocks(ax[e]);
    used[b] = s_of[e];
  }
  if ((rc = h2d(o_ax, ax.data(), ne * sizeof(AxpbyTask)))) return rc;
  if ((rc = h2d(o_ax_s, as.data(), (ne + 1) * sizeof(int64_t)))) return rc;
  if ((rc = hip_rc(launch_axpby_batched(reinterpret_cast<const AxpbyTask *>(ws + o_ax),
                                        reinterpret_cast<const int64_t *>(ws + o_ax_s), (int)ne,
                                        as.back(), st))))
    return rc;
  for (const ScaleOp &sc : scales)
    if ((rc = hip_rc(launch_scale(true, sc.m, sc.n, sc.br, sc.bi, sc.beta_zero, sc.C, sc.ldc, st))))
      return rc;
  if ((rc = hip_rc(hipStreamSynchronize(st)))) return rc;  // host tables above go out of scope
  if (slices_used != nullptr)
    for (int64_t b = 0; b < batch; ++b) slices_used[b] = used[b];
  return OZAKI_OK;
}

// Tuning cache file (JSON). One entry per line so that the reader below can
// take it line by line; any JSON reader can read it too:
//   {"format": "ozaki-tune-1", "arch": "gfx950", "entries": [
//    {"kind": "z", "slices": 7, "mb": 11, "nb": 12, "kb": 7, "id": 0, "ms": 0.8205},
//    ...]}
// Entries of another architecture are ignored.
int tune_load(const char *path) {
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  FILE *f = fopen(path, "r");
  if (f == nullptr) return OZAKI_ERR_IO;
  char line[512];
  bool arch_ok = false, seen_arch = false;
  std::map<TuneKey, TuneEntry> got;
  while (fgets(line, sizeof line, f) != nullptr) {
    const char *a = strstr(line, "\"arch\"");
    if (a != nullptr) {
      char arch[64] = {};
      if (sscanf(a, "\"arch\": \"%63[^\"]\"", arch) != 1) {
        fclose(f);
        return OZAKI_ERR_IO;
      }
      seen_arch = true;
      arch_ok = strcmp(arch, g.dev[dev].arch) == 0;
    }
    const char *e = strstr(line, "{\"kind\"");
    if (e == nullptr) continue;
    char kind = 0;
    int S, mb, nb, kb, id;
    double ms;
    if (sscanf(e, "{\"kind\": \"%c\", \"slices\": %d, \"mb\": %d, \"nb\": %d, \"kb\": %d, "
                  "\"id\": %d, \"ms\": %lf}",
               &kind, &S, &mb, &nb, &kb, &id, &ms) != 7 ||
        (kind != 'd' && kind != 'z') || S < 1 || S > OZAKI_S_MAX || id < 0 ||
        id >= gemm_num_configs()) {
      fclose(f);
      return OZAKI_ERR_IO;
    }
    got[{kind == 'z' ? 1 : 0, S, mb, nb, kb}] = TuneEntry{id, ms};
  }
  fclose(f);
  if (!seen_arch) return OZAKI_ERR_IO;
  if (arch_ok)
    for (const auto &kv : got) g_tune[kv.first] = kv.second;
  return OZAKI_OK;
}

int tune_save(const char *path) {
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  FILE *f = fopen(path, "w");
  if (f == nullptr) return OZAKI_ERR_IO;
  fprintf(f, "{\"format\": \"ozaki-tune-1\", \"arch\": \"%s\", \"entries\": [\n", g.dev[dev].arch);
  size_t i = 0;
  for (const auto &kv : g_tune) {
    const TuneKey &k = kv.first;
    fprintf(f,
            " {\"kind\": \"%c\", \"slices\": %d, \"mb\": %d, \"nb\": %d, \"kb\": %d, \"id\": %d, "
            "\"ms\": %.6f}%s\n",
            k[0] ? 'z' : 'd', k[1], k[2], k[3], k[4], kv.second.id, kv.second.ms,
            ++i < g_tune.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  return fclose(f) == 0 ? OZAKI_OK : OZAKI_ERR_IO;
}

// Times every tuning id of the fused GEMM on one shape and records the
// fastest. The packed operands are filled with pseudo-random digits (the
// kernel's power draw, and with it the clock, depends on the operand bits; all
// zeros would time a faster chip), the exponent codes with e = 0. The ids are
// timed round-robin, `reps` launches per id and round, after one untimed
// round; an id's time is its median over the rounds.
int autotune(bool cplx, int64_t m, int64_t n, int64_t k, int S, int reps, int *best,
             double *best_ms) {
  constexpr int kRounds = 5;
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  const Plan p = make_plan(cplx, m, n, k, S, g.dev[dev].num_cu);
  void *wsv = nullptr;
  if ((rc = get_workspace(p.total, &wsv))) return rc;
  char *ws = static_cast<char *>(wsv);
  const hipStream_t st = g.stream;
  if ((rc = hip_rc(launch_fill_i32(reinterpret_cast<int *>(ws + p.off_codeA), m, kCodeBias, st))))
    return rc;
  if ((rc = hip_rc(launch_fill_i32(reinterpret_cast<int *>(ws + p.off_codeB), n, kCodeBias, st))))
    return rc;
  if ((rc = hip_rc(launch_fill_digits(reinterpret_cast<int8_t *>(ws + p.off_SA),
                                      (int64_t)(p.off_SB - p.off_SA), 0x5eed0001ull, st))))
    return rc;
  if ((rc = hip_rc(launch_fill_digits(reinterpret_cast<int8_t *>(ws + p.off_SB),
                                      (int64_t)(p.off_flush - p.off_SB), 0x5eed0002ull, st))))
    return rc;
  void *C = nullptr;
  const size_t cbytes = (size_t)m * n * (cplx ? 16 : 8);
  if (hipMalloc(&C, cbytes) != hipSuccess) {
    (void)hipGetLastError();
    return OZAKI_ERR_ALLOC;
  }
  const int nid = gemm_num_configs();
  std::vector<std::vector<double>> t(nid);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = OZAKI_ERR_HIP;
  const GemmArgs ga = gemm_args(p, ws, 1.0, 0.0, 0.0, 0.0, true, C, m, nullptr);
  for (int round = 0; rc == OZAKI_OK && round <= kRounds; ++round) {
    for (int id = 0; rc == OZAKI_OK && id < nid; ++id) {
      if ((rc = hip_rc(hipEventRecord(e0, st)))) break;
      for (int r = 0; rc == OZAKI_OK && r < reps; ++r)
        rc = hip_rc(launch_ozgemm(S, id, ga, g.dev[dev].num_cu, st));
      if (rc) break;
      if ((rc = hip_rc(hipEventRecord(e1, st)))) break;
      if ((rc = hip_rc(hipEventSynchronize(e1)))) break;
      float msf = 0.f;
      if ((rc = hip_rc(hipEventElapsedTime(&msf, e0, e1)))) break;
      if (round > 0) t[id].push_back((double)msf / reps);  // round 0 warms up
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (hipFree(C) != hipSuccess && rc == OZAKI_OK) rc = OZAKI_ERR_HIP;
  if (rc) return rc;
  int best_id = 0;
  double best_t = 0.0;
  for (int id = 0; id < nid; ++id) {
    std::vector<double> v = t[id];
    std::sort(v.begin(), v.end());
    const double med = v[v.size() / 2];
    if (id == 0 || med < best_t) {
      best_id = id;
      best_t = med;
    }
  }
  g_tune[tune_key(cplx, S, m, p.nprime, p.nkb)] = TuneEntry{best_id, best_t};
  if (best) *best = best_id;
  if (best_ms) *best_ms = best_t;
  return OZAKI_OK;
}

int tune_shape(char kind, int64_t m, int64_t n, int64_t k, int slices, bool *cplx) {
  kind = up(kind);
  if (kind != 'D' && kind != 'Z') return -1;
  if (m <= 0) return -2;
  if (n <= 0) return -3;
  if (k <= 0) return -4;
  if (slices < 1 || slices > OZAKI_S_MAX) return -5;
  *cplx = kind == 'Z';
  return OZAKI_OK;
}

template <typename Enqueue>
int lu_run(char what, int64_t n, ozaki_z *A, int64_t lda, int64_t *ipiv, ozaki_z *X, int64_t ldx,
           int64_t nb, int slices, Enqueue enqueue) {
  if (!g_bat.graphs || g_tm.on) return enqueue(g.stream);
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  std::vector<uint8_t> sig;
  sig_put(sig, what);
  sig_put(sig, dev);
  sig_put(sig, n);
  sig_put(sig, A);
  sig_put(sig, lda);
  sig_put(sig, ipiv);
  sig_put(sig, X);
  sig_put(sig, ldx);
  sig_put(sig, nb);
  sig_put(sig, slices);
  sig_put(sig, split_b8());
  for (auto it = g_lu_graphs.begin(); it != g_lu_graphs.end(); ++it) {
    if (it->sig == sig) {
      g_lu_graphs.splice(g_lu_graphs.begin(), g_lu_graphs, it);
      return hip_rc(hipGraphLaunch(g_lu_graphs.front().exec, g.stream));
    }
  }
  // the largest emulated update of either sequence is at most n x n x nb
  if (slices > 0) {
    void *wsv = nullptr;
    const Plan p = make_plan(true, n, n, std::min(nb, n), slices, g.dev[dev].num_cu, split_b8());
    if ((rc = get_workspace(p.total, &wsv))) return rc;
  }
  if (g_lu_cap == nullptr && hipStreamCreateWithFlags(&g_lu_cap, hipStreamNonBlocking) != hipSuccess)
    return OZAKI_ERR_HIP;
  if (hipStreamBeginCapture(g_lu_cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return OZAKI_ERR_HIP;
  const hipStream_t user = g.stream;
  g.stream = g_lu_cap;  // the emulated and native updates launch on g.stream
  const int erc = enqueue(g_lu_cap);
  g.stream = user;
  LuGraph lg;
  lg.sig = std::move(sig);
  const hipError_t e = hipStreamEndCapture(g_lu_cap, &lg.graph);
  if (erc != OZAKI_OK || e != hipSuccess ||
      hipGraphInstantiate(&lg.exec, lg.graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    if (lg.exec) (void)hipGraphExecDestroy(lg.exec);
    if (lg.graph) (void)hipGraphDestroy(lg.graph);
    return erc != OZAKI_OK ? erc : OZAKI_ERR_HIP;
  }
  if (g_lu_graphs.size() >= kLuGraphCache) {
    LuGraph &old = g_lu_graphs.back();
    (void)hipGraphExecDestroy(old.exec);
    (void)hipGraphDestroy(old.graph);
    g_lu_graphs.pop_back();
  }
  g_lu_graphs.push_front(std::move(lg));
  return hip_rc(hipGraphLaunch(g_lu_graphs.front().exec, g.stream));
}

void clear_lu_graphs() {
  for (LuGraph &lg : g_lu_graphs) {
    (void)hipGraphExecDestroy(lg.exec);
    (void)hipGraphDestroy(lg.graph);
  }
  g_lu_graphs.clear();
}

}  // namespace

namespace oz {
int zgemm_fixed_scratch(char transa, char transb, int64_t m, int64_t n, int64_t k, double ar,
                        double ai, const void *A, int64_t lda, const void *B, int64_t ldb,
                        double br, double bi, void *C, int64_t ldc, int slices,
                        int (*scratch)(char **), size_t scratch_bytes) {
  return emulated_gemm_ws(true, transa, transb, m, n, k, ar, ai, A, lda, B, ldb, br, bi, C, ldc,
                          slices, scratch, scratch_bytes);
}
}  // namespace oz

extern "C" {

int ozaki_dgemm(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
                const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                double *C, int64_t ldc, int slices) {
  return emulated_gemm(false, transa, transb, m, n, k, alpha, 0.0, A, lda, B, ldb, beta, 0.0, C,
                       ldc, slices);
}

int ozaki_zgemm(char transa, char transb, int64_t m, int64_t n, int64_t k, ozaki_z alpha,
                const ozaki_z *A, int64_t lda, const ozaki_z *B, int64_t ldb, ozaki_z beta,
                ozaki_z *C, int64_t ldc, int slices) {
  return emulated_gemm(true, transa, transb, m, n, k, alpha.re, alpha.im, A, lda, B, ldb, beta.re,
                       beta.im, C, ldc, slices);
}

int ozaki2_dgemm(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
                 const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                 double *C, int64_t ldc, int moduli) {
  return ozaki2_gemm_impl(false, transa, transb, m, n, k, alpha, 0.0, A, lda, B, ldb, beta, 0.0, C,
                          ldc, moduli);
}

int ozaki2_zgemm(char transa, char transb, int64_t m, int64_t n, int64_t k, ozaki_z alpha,
                 const ozaki_z *A, int64_t lda, const ozaki_z *B, int64_t ldb, ozaki_z beta,
                 ozaki_z *C, int64_t ldc, int moduli) {
  return ozaki2_gemm_impl(true, transa, transb, m, n, k, alpha.re, alpha.im, A, lda, B, ldb,
                          beta.re, beta.im, C, ldc, moduli);
}

int ozaki_zgetrf(int64_t n, ozaki_z *A, int64_t lda, int64_t *ipiv, int64_t nb, int slices) {
  int rc = lu_args(n, A, lda, ipiv, nb, slices);
  if (rc) return rc;
  if (n == 0) return OZAKI_OK;
  int64_t *flag = nullptr;
  if ((rc = lu_workspace(&flag))) return rc;
  double2 *a = reinterpret_cast<double2 *>(A);
  const int mode = lu_panel_mode();
  auto enqueue = [&](hipStream_t st) -> int {
    int r;
    int64_t *pairs = flag + 1;
    if ((r = hip_rc(launch_set_i64(flag, n, st)))) return r;
    for (int64_t j0 = 0; j0 < n; j0 += nb) {
      const int64_t j1 = std::min(n, j0 + nb), w = j1 - j0;
      if ((r = hip_rc(launch_lu_panel(a, lda, n, j0, j1, ipiv, flag, mode, st)))) return r;
      if ((r = hip_rc(launch_swap_pairs(ipiv, j0, j1, n, pairs, st)))) return r;
      if ((r = hip_rc(launch_apply_pairs(a, lda, w, pairs, 0, j0, j1, n, st)))) return r;
      if (j1 < n) {
        // U12 = L11^-1 A12, then A22 -= L21 U12
        if ((r = hip_rc(launch_trsm(false, a + j0 + j0 * lda, lda, w, a + j0 + j1 * lda, lda,
                                    n - j1, st))))
          return r;
        if ((r = lu_update(slices, n - j1, n - j1, w, a + j1 + j0 * lda, lda, a + j0 + j1 * lda, lda,
                           a + j1 + j1 * lda, lda)))
          return r;
      }
    }
    return OZAKI_OK;
  };
  if ((rc = lu_run((char)('a' + mode), n, A, lda, ipiv, nullptr, 0, nb, slices, enqueue))) return rc;
  int64_t first_zero = n;
  if (hipMemcpyAsync(&first_zero, flag, sizeof(int64_t), hipMemcpyDeviceToHost, g.stream) != hipSuccess ||
      hipStreamSynchronize(g.stream) != hipSuccess)
    return OZAKI_ERR_HIP;
  return first_zero < n ? OZAKI_ERR_SINGULAR : OZAKI_OK;
}

int ozaki_zgetri(int64_t n, const ozaki_z *LU, int64_t lda, const int64_t *ipiv, ozaki_z *X,
                 int64_t ldx, int64_t nb, int slices) {
  int rc = lu_args(n, LU, lda, ipiv, nb, slices);
  if (rc) return rc;
  if (X == nullptr && n > 0) return -7;  // X and ldx are checked as arguments 7 and 8
  if (ldx < std::max<int64_t>(1, n)) return -8;
  if (n == 0) return OZAKI_OK;
  int64_t *flag = nullptr;
  if ((rc = lu_workspace(&flag))) return rc;
  const double2 *lu = reinterpret_cast<const double2 *>(LU);
  double2 *x = reinterpret_cast<double2 *>(X);
  auto enqueue = [&](hipStream_t st) -> int {
    int r;
    int64_t *pairs = flag + 1;
    // X = P I (the interchanges in blocks of nb, in order), then Y = L^-1 X
    // (blocks top down), then X = U^-1 Y (bottom up)
    if ((r = hip_rc(launch_identity(x, ldx, n, st)))) return r;
    for (int64_t i0 = 0; i0 < n; i0 += nb) {
      const int64_t i1 = std::min(n, i0 + nb);
      if ((r = hip_rc(launch_swap_pairs(ipiv, i0, i1, n, pairs, st)))) return r;
      if ((r = hip_rc(launch_apply_pairs(x, ldx, i1 - i0, pairs, 0, n, 0, 0, st)))) return r;
    }
    for (int64_t i0 = 0; i0 < n; i0 += nb) {
      const int64_t i1 = std::min(n, i0 + nb), w = i1 - i0;
      if ((r = hip_rc(launch_trsm(false, lu + i0 + i0 * lda, lda, w, x + i0, ldx, n, st)))) return r;
      if ((r = lu_update(slices, n - i1, n, w, lu + i1 + i0 * lda, lda, x + i0, ldx, x + i1, ldx)))
        return r;
    }
    for (int64_t i0 = (n - 1) / nb * nb; i0 >= 0; i0 -= nb) {
      const int64_t i1 = std::min(n, i0 + nb), w = i1 - i0;
      if ((r = hip_rc(launch_trsm(true, lu + i0 + i0 * lda, lda, w, x + i0, ldx, n, st)))) return r;
      if ((r = lu_update(slices, i0, n, w, lu + i0 * lda, lda, x + i0, ldx, x, ldx))) return r;
    }
    return OZAKI_OK;
  };
  return lu_run('I', n, const_cast<ozaki_z *>(LU), lda, const_cast<int64_t *>(ipiv), X, ldx, nb,
                slices, enqueue);
}

int ozaki2_moduli(int moduli, int32_t *out) {
  if (moduli < OZAKI2_MODULI_MIN || moduli > OZAKI2_MODULI_MAX) return -1;
  if (out == nullptr) return -2;
  for (int q = 0; q < moduli; ++q) out[q] = crt_modulus(q);
  return OZAKI_OK;
}

int ozaki2_beta_bits(int moduli, int64_t kprime) {
  if (moduli < OZAKI2_MODULI_MIN || moduli > OZAKI2_MODULI_MAX) return -1;
  if (kprime < 1 || kprime > OZAKI2_K_MAX) return -2;
  const int b = crt_beta(moduli, kprime);
  return b < 1 ? 0 : b;
}

size_t ozaki2_workspace_bytes(char kind, int64_t m, int64_t n, int64_t k, int moduli) {
  kind = up(kind);
  if ((kind != 'D' && kind != 'Z') || m < 0 || n < 0 || k < 0 || moduli < OZAKI2_MODULI_MIN ||
      moduli > OZAKI2_MODULI_MAX)
    return 0;
  Plan2 p;
  if (make_plan2(kind == 'Z', m, n, k, moduli, &p)) return 0;
  return p.total;
}

int ozaki_native_dgemm(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
                       const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                       double *C, int64_t ldc) {
  return native_gemm(false, transa, transb, m, n, k, alpha, 0.0, A, lda, B, ldb, beta, 0.0, C, ldc);
}

int ozaki_native_zgemm(char transa, char transb, int64_t m, int64_t n, int64_t k, ozaki_z alpha,
                       const ozaki_z *A, int64_t lda, const ozaki_z *B, int64_t ldb, ozaki_z beta,
                       ozaki_z *C, int64_t ldc) {
  return native_gemm(true, transa, transb, m, n, k, alpha.re, alpha.im, A, lda, B, ldb, beta.re,
                     beta.im, C, ldc);
}

int ozaki_zgemm_batched(const char *transa, const char *transb, const int64_t *m, const int64_t *n,
                        const int64_t *k, const ozaki_z *alpha, const ozaki_z *const *A,
                        const int64_t *lda, const ozaki_z *const *B, const int64_t *ldb,
                        const ozaki_z *beta, ozaki_z *const *C, const int64_t *ldc, int64_t batch,
                        const int *slices, int *slices_used) {
  if (batch < 0) return -14;
  if (batch == 0) return OZAKI_OK;
  if (!transa) return -1;
  if (!transb) return -2;
  if (!m) return -3;
  if (!n) return -4;
  if (!k) return -5;
  if (!alpha) return -6;
  if (!A) return -7;
  if (!lda) return -8;
  if (!B) return -9;
  if (!ldb) return -10;
  if (!beta) return -11;
  if (!C) return -12;
  if (!ldc) return -13;
  for (int64_t b = 0; b < batch; ++b) {
    int rc = check_gemm_args(transa[b], transb[b], m[b], n[b], k[b], lda[b], ldb[b], ldc[b]);
    if (rc) return rc;
    if (slices != nullptr && (slices[b] < 1 || slices[b] > OZAKI_S_MAX)) return -15;
    if (m[b] == 0 || n[b] == 0) continue;
    if (C[b] == nullptr) return -12;
    const bool alpha_zero = alpha[b].re == 0.0 && alpha[b].im == 0.0;
    if (alpha_zero || k[b] == 0) continue;
    if (A[b] == nullptr) return -7;
    if (B[b] == nullptr) return -9;
  }
  if (slices == nullptr)
    return auto_batched(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, batch,
                        slices_used);
  int rc = run_fixed_batched(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, batch,
                             slices);
  if (rc == OZAKI_OK && slices_used != nullptr)
    for (int64_t b = 0; b < batch; ++b) slices_used[b] = slices[b];
  return rc;
}

int ozaki_autotune(char kind, int64_t m, int64_t n, int64_t k, int slices, int reps, int *best,
                   double *best_ms) {
  bool cplx = false;
  int rc = tune_shape(kind, m, n, k, slices, &cplx);
  if (rc) return rc;
  if (reps < 1 || reps > 1000) return -6;
  return autotune(cplx, m, n, k, slices, reps, best, best_ms);
}

int ozaki_tune_set(char kind, int64_t m, int64_t n, int64_t k, int slices, int id) {
  bool cplx = false;
  int rc = tune_shape(kind, m, n, k, slices, &cplx);
  if (rc) return rc;
  if (id >= gemm_num_configs()) return -6;
  const Plan p = make_plan(cplx, m, n, k, slices, 1);
  const TuneKey key = tune_key(cplx, slices, m, p.nprime, p.nkb);
  if (id < 0)
    g_tune.erase(key);
  else
    g_tune[key] = TuneEntry{id, 0.0};
  return OZAKI_OK;
}

int ozaki_tune_get(char kind, int64_t m, int64_t n, int64_t k, int slices) {
  bool cplx = false;
  int rc = tune_shape(kind, m, n, k, slices, &cplx);
  if (rc) return rc;
  const Plan p = make_plan(cplx, m, n, k, slices, 1);
  return gemm_config(cplx, slices, m, p.nprime, p.nkb);
}

int ozaki_tune_configs(void) { return gemm_num_configs(); }

int ozaki_tune_save(const char *path) {
  if (path == nullptr) return -1;
  return tune_save(path);
}

int ozaki_tune_load(const char *path) {
  if (path == nullptr) return -1;
  return tune_load(path);
}

int ozaki_tune_clear(void) {
  g_tune.clear();
  return OZAKI_OK;
}

int ozaki_load_selector(const float *params, float margin, double target, double kappa) {
  return load_selector(params, margin, target, kappa);
}

int ozaki_batched_graphs(int on) {
  const bool want = on != 0;
  if (want != g_bat.graphs) {
    for (BatchedPlan *pl : g_bat.cache) free_plan(pl);
    g_bat.cache.clear();
    clear_lu_graphs();
  }
  g_bat.graphs = want;
  return OZAKI_OK;
}

int ozaki_batched_cache_clear(void) {
  for (BatchedPlan *pl : g_bat.cache) free_plan(pl);
  g_bat.cache.clear();
  clear_lu_graphs();
  return OZAKI_OK;
}

int ozaki_probe(char kind, char transa, char transb, int64_t m, int64_t n, int64_t k, const void *A,
                int64_t lda, const void *B, int64_t ldb, const void *C, int64_t ldc, int nvec,
                uint64_t seed, double *est) {
  kind = up(kind);
  if (kind != 'D' && kind != 'Z') return -1;
  const bool cplx = kind == 'Z';
  int rc = check_gemm_args(transa, transb, m, n, k, lda, ldb, ldc);
  if (rc) {
    // GEMM numbering -> probe numbering (kind is argument 1 here)
    switch (rc) {
      case -8: return -8;
      case -10: return -10;
      case -13: return -12;
      default: return rc - 1;
    }
  }
  if (nvec < 1 || nvec > probe_max_vectors()) return -13;
  if (m == 0) return OZAKI_OK;
  if (est == nullptr) return -15;
  if (n > 0 && C == nullptr) return -11;
  if (k > 0 && A == nullptr) return -7;
  if (k > 0 && n > 0 && B == nullptr) return -9;
  void *wsv = nullptr;
  if ((rc = get_workspace(probe_workspace_bytes(m, n, k), &wsv))) return rc;
  const View va = view_opA(A, transa, m, k, lda, cplx);
  const View vb = view_opB(B, transb, k, n, ldb, cplx);
  return hip_rc(launch_probe(va, vb, cplx, C, ldc, nvec, seed, wsv, est, g.stream));
}

int ozaki_features(char kind, char transa, char transb, int64_t m, int64_t n, int64_t k,
                   const void *A, int64_t lda, const void *B, int64_t ldb, float *feat) {
  kind = up(kind);
  if (kind != 'D' && kind != 'Z') return -1;
  const bool cplx = kind == 'Z';
  int rc = check_gemm_args(transa, transb, m, n, k, lda, ldb, std::max<int64_t>(1, m));
  if (rc) {
    switch (rc) {
      case -8: return -8;
      case -10: return -10;
      default: return rc - 1;
    }
  }
  if (m == 0 || n == 0 || k == 0) return -4 - (m == 0 ? 0 : (n == 0 ? 1 : 2));
  if (feat == nullptr) return -11;
  if (A == nullptr) return -7;
  if (B == nullptr) return -9;
  // workspace: codes (m + n), histogram (64), dims (3), task tables
  const size_t oc = 0, ocb = align256(sizeof(int) * m), oh = ocb + align256(sizeof(int) * n),
               od = oh + 256, ot = od + 256, os = ot + align256(2 * sizeof(FeatTask)),
               total = os + 256;
  void *wsv = nullptr;
  if ((rc = get_workspace(total, &wsv))) return rc;
  char *ws = static_cast<char *>(wsv);
  int *codeA = reinterpret_cast<int *>(ws + oc);
  int *codeB = reinterpret_cast<int *>(ws + ocb);
  int *hist = reinterpret_cast<int *>(ws + oh);
  const View va = view_opA(A, transa, m, k, lda, cplx);
  const View vb = view_opB(B, transb, k, n, ldb, cplx);
  FeatTask tk[2] = {{va, codeA, hist, cplx ? 1 : 0, va.sr == 1 ? 1 : 0, 32},
                    {vb, codeB, hist + 32, cplx ? 1 : 0, vb.sr == 1 ? 1 : 0, 31}};
  int64_t start[3] = {0, feat_task_blocks(tk[0]), 0};
  start[2] = start[1] + feat_task_blocks(tk[1]);
  const int64_t dims[3] = {m, n, k};
  hipStream_t st = g.stream;
  if ((rc = hip_rc(hipMemcpyAsync(ws + od, dims, sizeof(dims), hipMemcpyHostToDevice, st)))) return rc;
  if ((rc = hip_rc(hipMemcpyAsync(ws + ot, tk, sizeof(tk), hipMemcpyHostToDevice, st)))) return rc;
  if ((rc = hip_rc(hipMemcpyAsync(ws + os, start, sizeof(start), hipMemcpyHostToDevice, st)))) return rc;
  if ((rc = hip_rc(launch_fill_i32(codeA, m, 0, st)))) return rc;
  if ((rc = hip_rc(launch_fill_i32(codeB, n, 0, st)))) return rc;
  if ((rc = hip_rc(launch_fill_i32(hist, 64, 0, st)))) return rc;
  if ((rc = hip_rc(launch_scan(va, cplx, codeA, st)))) return rc;
  if ((rc = hip_rc(launch_scan(vb, cplx, codeB, st)))) return rc;
  if ((rc = hip_rc(launch_feat_hist(reinterpret_cast<const FeatTask *>(ws + ot),
                                    reinterpret_cast<const int64_t *>(ws + os), 2, start[2], st))))
    return rc;
  rc = hip_rc(launch_feat_finish(hist, reinterpret_cast<const int64_t *>(ws + od), feat, 1, st));
  if (rc == OZAKI_OK) rc = hip_rc(hipStreamSynchronize(st));  // host arrays above go out of scope
  return rc;
}

size_t ozaki_mlp_state_bytes(void) { return mlp_state_bytes(); }
size_t ozaki_mlp_scratch_bytes(int64_t batch) { return batch < 0 ? 0 : mlp_scratch_bytes(batch); }

int ozaki_mlp_init(void *state, uint64_t seed) {
  if (state == nullptr) return -1;
  return hip_rc(mlp_init(state, seed, g.stream));
}

int ozaki_mlp_refresh(void *state) {
  if (state == nullptr) return -1;
  return hip_rc(mlp_refresh(state, g.stream));
}

int ozaki_mlp_forward(const void *state, int64_t batch, const float *X, float *y, void *scratch) {
  if (state == nullptr) return -1;
  if (batch < 0) return -2;
  if (batch == 0) return OZAKI_OK;
  if (X == nullptr) return -3;
  if (y == nullptr) return -4;
  if (scratch == nullptr) return -5;
  return hip_rc(mlp_forward(state, batch, X, y, scratch, g.stream));
}

int ozaki_mlp_backward(void *state, int64_t batch, const float *y, const float *target,
                       float under_weight, float *loss, void *scratch) {
  if (state == nullptr) return -1;
  if (batch < 0) return -2;
  if (batch == 0) return OZAKI_OK;
  if (y == nullptr) return -3;
  if (target == nullptr) return -4;
  if (!(under_weight > 0.0f)) return -5;
  if (scratch == nullptr) return -7;
  return hip_rc(mlp_backward(state, batch, y, target, under_weight, loss, scratch, g.stream));
}

int ozaki_mlp_adam(void *state, float lr, float beta1, float beta2, float eps, int64_t step) {
  if (state == nullptr) return -1;
  if (!(lr > 0.0f)) return -2;
  if (!(beta1 >= 0.0f && beta1 < 1.0f)) return -3;
  if (!(beta2 >= 0.0f && beta2 < 1.0f)) return -4;
  if (!(eps > 0.0f)) return -5;
  if (step < 1) return -6;
  return hip_rc(mlp_adam(state, lr, beta1, beta2, eps, step, g.stream));
}

int ozaki_set_stream(void *hip_stream) {
  g.stream = reinterpret_cast<hipStream_t>(hip_stream);
  return OZAKI_OK;
}

int ozaki_set_workspace(void *device_ptr, size_t bytes) {
  clear_lu_graphs();
  if (device_ptr == nullptr) {
    g.user_ws = nullptr;
    g.user_ws_bytes = 0;
    return OZAKI_OK;
  }
  if (bytes == 0) return -2;
  g.user_ws = device_ptr;
  g.user_ws_bytes = bytes;
  return OZAKI_OK;
}

size_t ozaki_workspace_bytes(char kind, int64_t m, int64_t n, int64_t k, int slices) {
  kind = up(kind);
  const bool b8 = split_b8();
  if ((kind != 'D' && kind != 'Z') || m < 0 || n < 0 || k < 0 || slices < 1 ||
      slices > max_slices(b8))
    return 0;
  int dev = 0;
  int num_cu = 256;
  if (current_device(&dev) == OZAKI_OK) num_cu = g.dev[dev].num_cu;
  return make_plan(kind == 'Z', m, n, k, slices, num_cu, b8).total;
}

int ozaki_set_split(int mode) {
  if (mode != OZAKI_SPLIT_TRUNC7 && mode != OZAKI_SPLIT_BAL8) return -1;
  g.split = mode;
  return OZAKI_OK;
}

int ozaki_get_split(void) { return split_b8() ? OZAKI_SPLIT_BAL8 : OZAKI_SPLIT_TRUNC7; }

int ozaki_set_grid_limit(int64_t max_workgroups) {
  if (max_workgroups < 0) return -1;
  g.grid_limit = max_workgroups;
  return OZAKI_OK;
}

int ozaki_timing_enable(int on) {
  g_tm.on = on != 0;
  return OZAKI_OK;
}

int ozaki_timing_read(double *ms, int64_t *calls) {
  if (ms == nullptr) return -1;
  for (int p = 0; p < OZAKI_PHASES; ++p) ms[p] = 0.0;
  int rc = OZAKI_OK;
  for (Mark &mk : g_tm.marks) {
    float t = 0.0f;
    if (hipEventSynchronize(mk.stop) != hipSuccess ||
        hipEventElapsedTime(&t, mk.start, mk.stop) != hipSuccess)
      rc = OZAKI_ERR_HIP;
    else if (mk.phase >= 0 && mk.phase < OZAKI_PHASES)
      ms[mk.phase] += (double)t;
    g_tm.pool.push_back(mk.start);
    g_tm.pool.push_back(mk.stop);
  }
  g_tm.marks.clear();
  if (calls != nullptr) *calls = g_tm.calls;
  g_tm.calls = 0;
  return rc;
}

int ozaki_finalize(void) {
  int rc = OZAKI_OK;
  clear_lu_graphs();
  for (int d = 0; d < kMaxDev; ++d) {
    if (g.own_ws[d] != nullptr) {
      int cur = 0;
      if (hipGetDevice(&cur) != hipSuccess) rc = OZAKI_ERR_HIP;
      if (hipSetDevice(d) != hipSuccess || hipFree(g.own_ws[d]) != hipSuccess) rc = OZAKI_ERR_HIP;
      (void)hipSetDevice(cur);
      g.own_ws[d] = nullptr;
      g.own_ws_bytes[d] = 0;
    }
  }
  // scratch of the automatic slice mode (the selector itself stays loaded)
  for (void **p : {&g_sel.ws, &g_sel.plan_ws}) {
    if (*p == nullptr) continue;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) rc = OZAKI_ERR_HIP;
    if (hipSetDevice(g_sel.dev) != hipSuccess || hipFree(*p) != hipSuccess) rc = OZAKI_ERR_HIP;
    (void)hipSetDevice(cur);
    *p = nullptr;
  }
  g_sel.ws_bytes = 0;
  g_sel.plan_ws_bytes = 0;
  for (int d = 0; d < kMaxDev; ++d) {
    if (g_lu_flag[d] != nullptr) {
      int cur = 0;
      if (hipGetDevice(&cur) != hipSuccess) rc = OZAKI_ERR_HIP;
      if (hipSetDevice(d) != hipSuccess || hipFree(g_lu_flag[d]) != hipSuccess) rc = OZAKI_ERR_HIP;
      (void)hipSetDevice(cur);
      g_lu_flag[d] = nullptr;
    }
  }
  return rc;
}

const char *ozaki_status_string(int status) {
  if (status < 0) return "invalid argument";
  switch (status) {
    case OZAKI_OK: return "success";
    case OZAKI_ERR_HIP: return "HIP runtime error";
    case OZAKI_ERR_ALLOC: return "device workspace allocation failed";
    case OZAKI_ERR_WORKSPACE: return "caller workspace too small";
    case OZAKI_ERR_TOO_LARGE: return "product needs more scratch than the fixed device array holds";
    case OZAKI_ERR_NO_DEVICE: return "no usable device";
    case OZAKI_ERR_INTERNAL: return "internal error";
    case OZAKI_ERR_NO_SELECTOR: return "automatic slice selection needs a loaded selector";
    case OZAKI_ERR_IO: return "tuning cache file missing, unwritable or malformed";
    case OZAKI_ERR_SINGULAR: return "exactly zero pivot: the matrix is singular";
    default: return "unknown status";
  }
}

int ozaki_debug_exponents(char kind, char side, char trans, int64_t rows, int64_t L, const void *X,
                          int64_t ldx, int32_t *exps, uint8_t *flags) {
  View v;
  bool cplx = false;
  int rc = debug_view(kind, side, trans, rows, L, X, ldx, &v, &cplx);
  if (rc) return rc;
  if (rows == 0) return OZAKI_OK;
  if (exps == nullptr) return -8;
  if (flags == nullptr) return -9;
  void *wsv = nullptr;
  if ((rc = get_workspace(align256(sizeof(int) * rows), &wsv))) return rc;
  int *code = static_cast<int *>(wsv);
  if ((rc = hip_rc(launch_fill_i32(code, rows, 0, g.stream)))) return rc;
  if ((rc = hip_rc(launch_scan(v, cplx, code, g.stream)))) return rc;
  return hip_rc(launch_codes_to_exps(code, rows, exps, flags, g.stream));
}

int ozaki_debug_split(char kind, char side, char trans, int64_t rows, int64_t L, const void *X,
                      int64_t ldx, int slices, int8_t *digits) {
  View v;
  bool cplx = false;
  int rc = debug_view(kind, side, trans, rows, L, X, ldx, &v, &cplx);
  if (rc) return rc;
  const bool b8 = split_b8();
  if (slices < 1 || slices > max_slices(b8)) return -8;
  if (rows == 0 || L == 0) return OZAKI_OK;
  if (digits == nullptr) return -9;
  const bool side_b = up(side) == 'B';
  const int64_t prows = (cplx && side_b) ? 2 * rows : rows;
  const int64_t kpad = round_up(cplx ? 2 * L : L, kKPad);
  const int64_t nrb = round_up(prows, kRowPad) / 32;
  const size_t code_bytes = align256(sizeof(int) * rows);
  const size_t total = code_bytes + align256((size_t)slices * nrb * 32 * kpad);
  void *wsv = nullptr;
  if ((rc = get_workspace(total, &wsv))) return rc;
  int *code = static_cast<int *>(wsv);
  int8_t *packed = static_cast<int8_t *>(wsv) + code_bytes;
  if ((rc = hip_rc(launch_fill_i32(code, rows, 0, g.stream)))) return rc;
  if ((rc = hip_rc(launch_scan(v, cplx, code, g.stream)))) return rc;
  if ((rc = hip_rc(launch_split(v, cplx, side_b, code, slices, packed, nrb, kpad / 32, g.stream,
                                b8))))
    return rc;
  return hip_rc(launch_unpack(packed, cplx, side_b, rows, L, slices, nrb, kpad / 32, digits, g.stream));
}

int ozaki_debug_diagonals(char kind, char transa, char transb, int64_t m, int64_t n, int64_t k,
                          const void *A, int64_t lda, const void *B, int64_t ldb, int slices,
                          int64_t *S) {
  kind = up(kind);
  if (kind != 'D' && kind != 'Z') return -100;
  const bool cplx = kind == 'Z';
  int rc = check_gemm_args(transa, transb, m, n, k, lda, ldb, std::max<int64_t>(1, m));
  if (rc) return rc;
  const bool b8 = split_b8();
  if (slices < 1 || slices > max_slices(b8)) return -14;
  if (m == 0 || n == 0 || k == 0) return OZAKI_OK;
  if (S == nullptr) return -15;
  if (A == nullptr) return -7;
  if (B == nullptr) return -9;
  int dev = 0;
  if ((rc = current_device(&dev))) return rc;
  const Plan p = make_plan(cplx, m, n, k, slices, g.dev[dev].num_cu, b8);
  void *wsv = nullptr;
  if ((rc = get_workspace(p.total, &wsv))) return rc;
  char *ws = static_cast<char *>(wsv);
  const View va = view_opA(A, transa, m, k, lda, cplx);
  const View vb = view_opB(B, transb, k, n, ldb, cplx);
  if ((rc = prepare(p, ws, va, vb, g.stream))) return rc;
  const GemmArgs ga = gemm_args(p, ws, 1.0, 0.0, 0.0, 0.0, true, nullptr, m, S);
  // raw diagonal output exists in tile configuration 0 only (either order)
  return hip_rc(launch_ozgemm(slices, gemm_config(cplx, slices, m, p.nprime, p.nkb) & 1, ga,
                              g.dev[dev].num_cu, g.stream));
}

}  // extern "C"
