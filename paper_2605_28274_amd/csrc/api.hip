// C ABI of libsylv: context creation, the factorized CG / BiCGSTAB iteration drivers
// (Algorithms 4.1 and 4.2), the FP64 true residual and factor export.
//
// The host only sequences kernels: every scalar of the recurrences stays on the device, and
// the host polls the device's stop flag every `check_every` iterations (iterations enqueued
// after the stop return at kernel entry).
#include <algorithm>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"

namespace {

constexpr size_t ALIGN = 256;
constexpr size_t CORE_SCRATCH = 16384;  // doubles of reduction partials of the core kernels

struct Layout {
  // sizes
  int64_t n = 0, m = 0, s = 0, Jmax = 0, rmax = 0, ldb = 0, ldc = 0, rc_rows = 0;
  int lyap = 0, method = 0, max_iter = 0, fp32 = 0;
  int64_t esz = 8;  // bytes per basis element
  size_t partial_cap = 0;
  // byte offsets into the workspace
  size_t off_V, off_W, off_H, off_G, off_X, off_R, off_P, off_Q, off_S, off_T;
  size_t off_U, off_Uw, off_coefV, off_coefW, off_btrp, off_btci, off_btval, off_tscr;
  size_t off_cscr, off_partials, off_counters, off_ds, off_ssv, off_ssw, off_rt, off_rl, off_rr, off_hist;
  size_t off_Lx, off_M2, off_d1, off_d2, off_c2, off_cpart, cpart_cap = 0;
  size_t off_Ex[5] = {0, 0, 0, 0, 0};  // further cores of CGS and GPBiCG
  // solution compression: l <= lc columns of the randomized range (rmax x lc panels)
  int64_t lc = 0;
  size_t off_cOm = 0, off_cY = 0, off_cZ = 0, off_cB = 0, off_cG = 0, off_cU = 0, off_cUk = 0,
         off_cYk = 0, off_csig = 0, off_cidx = 0, off_cpt = 0, off_cinfo = 0;
  size_t off_dots, off_flag, off_panV, off_panW, off_sellA, off_sellB;
  // outer refinement: correction contexts and the buffers of the sketch and of the residual of
  // the summed iterates (child: a correction context, whose operators belong to the parent)
  int child = 0, refine_max = 0, refine_q = 0, refine_iter = 0;
  size_t child_bytes = 0, off_child = 0;
  int64_t rows_max = 0, smax = 0, cmax = 0, ldE = 0, child_rmax = 0;
  size_t tn_cap = 0;
  size_t off_Om, off_Zb, off_Yb, off_Eb, off_Fb, off_Pp, off_Qp, off_sa, off_sb, off_sc2, off_sd,
      off_sk, off_sT, off_tn, off_atrp, off_atci, off_atval, off_atscr, off_GL, off_GN, off_Mc,
      off_T1, off_Es, off_rinfo, off_gpart;
  size_t gpart_cap = 0;  // doubles of split-K / stream-K partial tiles of the residual Grams
  // split-BF16 residual Grams: packed chunk, column maxima / exponents, FP32 partials
  int gram_prec = 0;
  int64_t cpad = 0;
  size_t off_pack = 0, off_cmaxb = 0, off_cexp = 0, off_bpart = 0, bpart_floats = 0;
  size_t total = 0;
};

constexpr int NLD = 64;         // row stride (doubles) of the narrow panels of the refinement
constexpr int64_t COMPRESS_LMAX = 256;  // columns of the randomized range at most
constexpr int REFINE_CAP = 4;   // correction solves at most

size_t bump(size_t &cur, size_t bytes) {
  const size_t o = (cur + ALIGN - 1) / ALIGN * ALIGN;
  cur = o + bytes;
  return o;
}

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Methods on block Lanczos bases (one operator per iteration: CG, CR) and on block Arnoldi
// bases (two per iteration: BiCGSTAB, CGS, GPBiCG).
bool lanczos_method(int m) { return m == SYLV_METHOD_CG || m == SYLV_METHOD_CR; }
bool known_method(int m) { return m >= SYLV_METHOD_CG && m <= SYLV_METHOD_GPBICG; }
// Blocks of each basis generated in max_iter iterations (with the step issued ahead).
int64_t blocks_needed(int m, int max_iter) {
  if (m == SYLV_METHOD_CG) return (int64_t)max_iter + 2;
  if (m == SYLV_METHOD_CR) return (int64_t)max_iter + 3;
  return 2 * (int64_t)max_iter + 2;
}
// Extra core buffers of the methods beyond X, R, P, Q, S, T.
int extra_cores(int m) {
  return m == SYLV_METHOD_CGS ? 2 : (m == SYLV_METHOD_GPBICG ? 5 : 0);
}

int check_csr_header(const sylv_csr &M, int64_t rows) {
  if (M.rows != rows || M.rows < 0 || M.rows > INT32_MAX || M.nnz < 0 ||
      M.nnz >= ((int64_t)1 << 31))
    return SYLV_ERR_INVALID;
  if (!M.row_ptr || (M.nnz > 0 && (!M.col_idx || !M.values))) return SYLV_ERR_INVALID;
  return 0;
}

int make_layout(const sylv_problem *pb, const sylv_options *op, Layout &L, bool child = false) {
  if (!pb || !op) return SYLV_ERR_INVALID;
  L.child = child ? 1 : 0;
  if (pb->n <= 0 || pb->m <= 0 || pb->s < 1 || pb->s > SYLV_MAX_S) return SYLV_ERR_INVALID;
  // column indices are int32: at most 2^31 - 1 rows (this also keeps every size below in int64)
  if (pb->n > INT32_MAX || pb->m > INT32_MAX) return SYLV_ERR_INVALID;
  if (pb->s > std::min(pb->n, pb->m)) return SYLV_ERR_INVALID;
  if (pb->lyapunov && pb->n != pb->m) return SYLV_ERR_INVALID;
  if (op->max_iter < 1 || !known_method(op->method)) return SYLV_ERR_INVALID;
  // outer refinement drives CG and BiCGSTAB corrections only
  if (op->refine_max > 0 && op->method > SYLV_METHOD_BICGSTAB) return SYLV_ERR_INVALID;
  if (op->precision != SYLV_FP64 && op->precision != SYLV_MIXED_FP32 &&
      op->precision != SYLV_MIXED_BF16SPLIT)
    return SYLV_ERR_INVALID;
  if (op->streams < 0 || op->streams > 2) return SYLV_ERR_INVALID;
  if (op->reorth < 0 || op->reorth > 2) return SYLV_ERR_INVALID;
  if (op->gram_precision < 0 || op->gram_precision > 2 || op->verify < 0 || op->verify > 1)
    return SYLV_ERR_INVALID;
  if (!lanczos_method(op->method) && op->reorth == 2 &&
      !arnoldi_lagged_supported(pb->s, op->precision == SYLV_MIXED_FP32))
    return SYLV_ERR_INVALID;
  if (!pb->C1 || pb->ldc1 < pb->s) return SYLV_ERR_INVALID;
  if (!pb->lyapunov && (!pb->C2 || pb->ldc2 < pb->s)) return SYLV_ERR_INVALID;
  int e = check_csr_header(pb->A, pb->n);
  if (e) return e;
  if (!pb->lyapunov && (e = check_csr_header(pb->B, pb->m))) return e;
  L.n = pb->n;
  L.m = pb->m;
  L.s = pb->s;
  L.lyap = pb->lyapunov ? 1 : 0;
  L.method = op->method;
  L.max_iter = op->max_iter;
  L.fp32 = op->precision == SYLV_MIXED_FP32;
  L.esz = L.fp32 ? 4 : 8;
  // blocks generated: CG k+2 after k+1 iterations, CR k+3; two-operator methods 2k+3
  L.Jmax = blocks_needed(op->method, op->max_iter);
  L.rmax = L.Jmax * L.s;
  if (L.rmax > (1 << 20)) return SYLV_ERR_INVALID;
  // multiple of 64 columns (whole 64-wide tiles of the residual Grams stay inside a row),
  // never a multiple of 4 KiB (row strides that map every row to the same memory channel)
  L.ldb = round_up(L.rmax, 64);
  if ((L.ldb * L.esz) % 4096 == 0) L.ldb += 64;
  L.ldc = round_up(L.rmax, 64);
  const int64_t maxrows = std::max(L.n, L.m);
  L.rc_rows = std::min<int64_t>(maxrows, 16384);
  const int64_t tiles = (L.ldb + 255) / 256;
  const int64_t t16 = L.ldc / 16;
  L.partial_cap = std::max<size_t>(
      {(size_t)(256 * tiles * 256 * L.s), (size_t)(t16 * t16 * 2 + 64), (size_t)1024 * 66,
       arnoldi_partials_needed((int)L.s, L.n, L.lyap ? 0 : L.m, L.ldb)});
  size_t cur = 0;
  const size_t c2 = (size_t)L.ldc * L.ldc * sizeof(double);
  L.off_V = bump(cur, (size_t)L.n * L.ldb * L.esz);
  L.off_W = L.lyap ? L.off_V : bump(cur, (size_t)L.m * L.ldb * L.esz);
  L.off_H = bump(cur, c2);
  L.off_G = L.lyap ? L.off_H : bump(cur, c2);
  L.off_X = bump(cur, c2);
  L.off_R = bump(cur, c2);
  L.off_P = bump(cur, c2);
  L.off_Q = bump(cur, c2);
  if (L.method != SYLV_METHOD_CG) {
    L.off_S = bump(cur, c2);
    L.off_T = bump(cur, c2);
  } else {
    L.off_S = L.off_T = 0;
  }
  for (int i = 0; i < extra_cores(L.method); ++i) L.off_Ex[i] = bump(cur, c2);
  L.off_U = bump(cur, (size_t)L.n * L.s * 8);
  L.off_Uw = bump(cur, (size_t)L.m * L.s * 8);
  L.off_coefV = bump(cur, (size_t)L.ldb * 2 * L.s * 8);  // 2 s columns in the lagged step
  L.off_coefW = bump(cur, (size_t)L.ldb * 2 * L.s * 8);
  const int64_t bnnz = (L.lyap || child) ? 0 : pb->B.nnz;
  L.off_btrp = bump(cur, (size_t)(L.m + 1) * 4);
  L.off_btci = bump(cur, (size_t)std::max<int64_t>(bnnz, 1) * 4);
  L.off_btval = bump(cur, (size_t)std::max<int64_t>(bnnz, 1) * 8);
  L.off_tscr = bump(cur, csr_transpose_scratch(L.m));
  L.off_partials = bump(cur, L.partial_cap * 8);
  L.off_cscr = bump(cur, CORE_SCRATCH * 8);
  L.off_counters = bump(cur, CNT_MAX * sizeof(int));
  L.off_ds = bump(cur, sizeof(DevState));
  L.off_ssv = bump(cur, sizeof(SideState));
  L.off_ssw = bump(cur, sizeof(SideState));
  L.off_rt = bump(cur, SYLV_MAX_S * SYLV_MAX_S * 8);
  L.off_rl = bump(cur, SYLV_MAX_S * SYLV_MAX_S * 8);
  L.off_rr = bump(cur, SYLV_MAX_S * SYLV_MAX_S * 8);
  L.off_hist = bump(cur, (size_t)4 * L.Jmax * 8);
  // true-residual buffers: R^ core, band scratch, right-hand-side QR defects and a copy of C2
  L.off_Lx = bump(cur, c2);
  L.off_M2 = bump(cur, c2);
  L.off_d1 = bump(cur, (size_t)L.n * L.s * 8);
  L.off_d2 = L.lyap ? L.off_d1 : bump(cur, (size_t)L.m * L.s * 8);
  L.off_c2 = bump(cur, (size_t)L.m * L.s * 8);  // C2 (C1 for Lyapunov)
  // stream-K partial tiles of the core operator (BiCGSTAB): one 64 x 64 tile per output tile
  // and per chunk (at most 512 chunks), for cores of up to 1024 tiles
  if (L.method != SYLV_METHOD_CG) {
    const int64_t T = L.ldc / 64 + 1;
    L.cpart_cap = (size_t)(512 + std::min<int64_t>(T * T, 1024)) * 4096;
    L.off_cpart = bump(cur, L.cpart_cap * 8);
  }
  L.off_panV = bump(cur, (size_t)LZ_RING * L.n * L.s * L.esz);
  L.off_panW = L.lyap ? L.off_panV : bump(cur, (size_t)LZ_RING * L.m * L.s * L.esz);
  L.off_sellA = child ? 0 : bump(cur, sell_bytes(L.n, pb->A.nnz));
  L.off_sellB = (L.lyap || child) ? L.off_sellA : bump(cur, sell_bytes(L.m, pb->B.nnz));
  L.off_dots = bump(cur, 16 * 8);
  if (!child) {
    L.lc = std::min<int64_t>(COMPRESS_LMAX, L.rmax);
    const size_t panel = (size_t)L.rmax * L.lc * 8, wide = (size_t)L.lc * L.ldc * 8;
    L.off_cOm = bump(cur, panel);
    L.off_cY = bump(cur, wide);
    L.off_cZ = bump(cur, wide);
    L.off_cB = bump(cur, wide);
    L.off_cG = bump(cur, (size_t)L.lc * L.lc * 8);
    L.off_cU = bump(cur, panel);
    L.off_cUk = bump(cur, panel);
    L.off_cYk = bump(cur, panel);
    L.off_csig = bump(cur, (size_t)L.lc * 8 * 2);
    L.off_cidx = bump(cur, (size_t)L.lc * 4);
    L.off_cpt = bump(cur, 1024 * 8);
    L.off_cinfo = bump(cur, 64);
  }
  L.off_flag = bump(cur, 16 * sizeof(int));
  if (!child && op->refine_max > 0) {
    if (op->refine_max > REFINE_CAP || op->refine_rank < 1 || op->refine_rank > SYLV_MAX_S ||
        op->refine_max_iter < 1)
      return SYLV_ERR_INVALID;
    L.refine_max = op->refine_max;
    L.refine_q = op->refine_rank;
    L.refine_iter = op->refine_max_iter;
    // a correction is a Sylvester problem with a rank <= refine_q right-hand side (for Lyapunov
    // with B = A^T, since the residual need not be semidefinite)
    sylv_problem cp = *pb;
    cp.s = std::min<int64_t>(L.refine_q, std::min(pb->n, pb->m));
    cp.lyapunov = 0;
    cp.B = pb->lyapunov ? pb->A : pb->B;
    cp.B.rows = pb->m;
    cp.C1 = cp.C2 = reinterpret_cast<const double *>(ALIGN);
    cp.ldc1 = cp.ldc2 = NLD;
    sylv_options co = *op;
    co.max_iter = L.refine_iter;
    co.refine_max = 0;
    Layout CL;
    if ((e = make_layout(&cp, &co, CL, true))) return e;
    L.child_bytes = (CL.total + ALIGN - 1) / ALIGN * ALIGN;
    L.off_child = bump(cur, L.child_bytes * L.refine_max);
    L.rows_max = std::max(L.n, L.m);
    const size_t panel = (size_t)L.rows_max * NLD * 8;
    L.off_Om = bump(cur, panel);
    L.off_Zb = bump(cur, panel);
    L.off_Yb = bump(cur, panel);
    L.off_Eb = bump(cur, panel);
    L.off_Fb = bump(cur, panel);
    L.off_Pp = bump(cur, (size_t)L.refine_max * L.n * NLD * 8);
    L.off_Qp = bump(cur, (size_t)L.refine_max * L.m * NLD * 8);
    L.smax = std::max(L.rmax, CL.rmax) + 2 * SYLV_MAX_S;
    const size_t small = (size_t)L.smax * NLD * 8;
    L.off_sa = bump(cur, small);
    L.off_sb = bump(cur, small);
    L.off_sc2 = bump(cur, small);
    L.off_sd = bump(cur, small);
    L.off_sk = bump(cur, small);
    L.off_sT = bump(cur, small);
    L.tn_cap = tn_partials_needed(L.rows_max, L.smax, SYLV_MAX_S);
    L.off_tn = bump(cur, L.tn_cap * 8);
    L.off_atrp = bump(cur, (size_t)(L.n + 1) * 4);
    L.off_atci = bump(cur, (size_t)std::max<int64_t>(pb->A.nnz, 1) * 4);
    L.off_atval = bump(cur, (size_t)std::max<int64_t>(pb->A.nnz, 1) * 8);
    L.off_atscr = bump(cur, csr_transpose_scratch(L.n));
    L.child_rmax = CL.rmax;
    L.off_rinfo = bump(cur, 64 * 8);
  }
  if (!child) {
    // residual of the (summed) iterate, R = L M N^T over the stacked tall factors of every
    // step: L = [V_j+, E_A,j, D1_j, ...; P_i], N = [W_j+, E_B,j, D2_j, C2_j, ...; Q_i]
    const int64_t q1 = L.refine_q;
    L.cmax = round_up(2 * L.rmax + 4 * L.s + L.refine_max * (2 * L.child_rmax + 5 * q1), 64);
    const size_t cc = (size_t)L.cmax * L.cmax * 8;
    L.off_GL = bump(cur, cc);
    L.off_GN = bump(cur, cc);
    L.off_Mc = bump(cur, cc);
    L.off_T1 = bump(cur, cc);
    L.ldE = round_up(L.rmax + 2 * L.s, 64) +
            L.refine_max * round_up(L.child_rmax + 2 * L.refine_q, 64) + 64;
    L.off_Es = bump(cur, (size_t)L.rc_rows * L.ldE * 8);
    L.gpart_cap = gram_part_doubles(L.cmax, L.rc_rows);
    L.off_gpart = bump(cur, L.gpart_cap * 8);
    // SYLV_MIXED_BF16SPLIT: FP64 bases with the split-BF16 residual Grams (at least form 1)
    L.gram_prec = op->precision == SYLV_MIXED_BF16SPLIT ? std::max(op->gram_precision, 1)
                                                        : op->gram_precision;
    if (L.gram_prec > 0) {
      L.cpad = bf16_pack_width(L.cmax);
      L.off_pack = bump(cur, bf16_pack_bytes(L.rc_rows, L.cpad));
      L.off_cmaxb = bump(cur, (size_t)L.cpad * 8);
      L.off_cexp = bump(cur, (size_t)L.cpad * 4);
      L.bpart_floats = bf16_part_floats(L.cpad, L.rc_rows);
      L.off_bpart = bump(cur, L.bpart_floats * 4);
    }
  }
  L.total = cur + ALIGN;
  return 0;
}

// Optional kernel timing: HIP events around each launch of an instrumented kernel family, read
// back after the solve. Launches of iterations past the stop are discarded.
struct Prof {
  struct Rec {
    int fam, iter;
    hipEvent_t a, b;
    double bytes, flops;
  };
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Rec> recs;
  hipEvent_t start = nullptr;
  int iter = 0;
  int64_t launches[FAM_COUNT] = {};
  double ms[FAM_COUNT] = {}, bytes[FAM_COUNT] = {}, flops[FAM_COUNT] = {};
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void reset_stats() {
    for (int f = 0; f < FAM_COUNT; ++f) launches[f] = 0, ms[f] = bytes[f] = flops[f] = 0.0;
  }
  // Accumulates the recorded launches of iterations < iters (the stream must be idle).
  void flush(int iters) {
    for (const Rec &r : recs) {
      if (r.iter >= iters || !r.a || !r.b) continue;
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) continue;
      launches[r.fam] += 1;
      ms[r.fam] += t;
      bytes[r.fam] += r.bytes;
      flops[r.fam] += r.flops;
    }
    recs.clear();
    used = 0;
  }
  ~Prof() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

struct Ctx {
  Layout L;
  Prof *prof = nullptr;
  hipStream_t st = nullptr;
  sylv_csr A{}, B{};
  double closure_tol = 1e-12;
  int check_every = 16;
  int record_history = 1;
  char *ws = nullptr;
  SideDesc sv{}, sw{};
  double *H, *G, *X, *R, *P, *Q, *S, *T, *Rt, *RL, *RR, *hist;
  double *Ex[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double *cpart = nullptr;  // split-K scratch of the core operator
  DevState *ds;
  SideState *ssv, *ssw;
  Scratch sc{};   // Krylov steps (Arnoldi / Lanczos) and the residual evaluation
  Scratch scc{};  // core recurrences (they run concurrently with the Krylov steps)
  // Krylov steps run on their own stream (kst), one iteration ahead of the core recurrences on
  // st: the bases do not depend on the iterates, so each iteration's core work overlaps the
  // next iteration's basis extension. kst == st when the context was created without it.
  hipStream_t kst = nullptr;
  bool own_kst = false;
  bool lagged = false;  // block Arnoldi with the second pass one step later
  hipEvent_t ev_k[4] = {nullptr, nullptr, nullptr, nullptr};  // Krylov step done (ring)
  hipEvent_t ev_c[3] = {nullptr, nullptr, nullptr};        // core iteration done (ring)
  hipEvent_t ev_s = nullptr;                               // stream join
  int32_t *btrp, *btci;
  double *btval;
  int *flag;
  double *dots;
  // host state
  int solved = 0, method = 0, status = 0, iters = 0, max_iter_run = 0;
  int64_t rank = 0;
  double relres = 0.0;
  DevState *h_ds = nullptr;  // pinned
  std::vector<double> h_hist;
  // outer refinement
  Ctx *parent = nullptr;
  std::vector<Ctx *> kids;   // correction contexts of the last refined solve
  std::vector<int> kid_k;    // their right-hand-side ranks
  sylv_csr AT{};             // A^T (refinement only)
  double refine_inner_tol = 0.0;
  double rel_true = -1.0;    // FP64 true residual of the summed iterate (refined solves)
  int outer_steps = 0;
  int in_refine = 0;         // the refinement's own first solve is running
  int verify = 1;            // check the true residual after a converged solve
  int64_t comp_k = -1;       // rank of the compressed solution (-1: none since the last solve)
  double comp_err = 0.0;     // its relative Frobenius error
  int res_valid = 0;         // abs_res / rel_res hold the residual of the current iterate
  double res_abs = 0.0, res_rel = 0.0;
};

template <typename T>
T *at(Ctx *c, size_t off) {
  return reinterpret_cast<T *>(c->ws + off);
}

}  // namespace

void prof_begin(const Scratch &sc, hipStream_t st) {
  Prof *p = reinterpret_cast<Prof *>(sc.prof);
  if (!p) return;
  p->start = p->get();
  if (p->start) (void)hipEventRecord(p->start, st);
}

void prof_end(const Scratch &sc, int fam, double bytes, double flops, hipStream_t st) {
  Prof *p = reinterpret_cast<Prof *>(sc.prof);
  if (!p || !p->start) return;
  hipEvent_t e = p->get();
  if (!e) return;
  (void)hipEventRecord(e, st);
  p->recs.push_back(Prof::Rec{fam, p->iter, p->start, e, bytes, flops});
  p->start = nullptr;
}

namespace {

void set_iter(Ctx *c, int k) {
  if (c->prof) c->prof->iter = k;
}

int read_state(Ctx *c) {
  HIPOK(hipMemcpyAsync(c->h_ds, c->ds, sizeof(DevState), hipMemcpyDeviceToHost, c->st));
  HIPOK(hipStreamSynchronize(c->st));
  return 0;
}

int begin_solve(Ctx *c, double tol, int max_iter, int method) {
  const Layout &L = c->L;
  // the workspace holds the bases and cores of the method it was sized for
  if (method != L.method && !(method == SYLV_METHOD_CG && L.method == SYLV_METHOD_BICGSTAB))
    return SYLV_ERR_WORKSPACE;
  const int64_t need_blocks = blocks_needed(method, max_iter);
  if (max_iter < 1 || need_blocks > L.Jmax || !(tol >= 0.0)) return SYLV_ERR_INVALID;
  const size_t c2 = (size_t)L.ldc * L.ldc * 8;
  double *zero[] = {c->H, c->G, c->X, c->R, c->P, c->Q, c->S, c->T,
                    c->Ex[0], c->Ex[1], c->Ex[2], c->Ex[3], c->Ex[4]};
  for (double *z : zero)
    if (z) HIPOK(hipMemsetAsync(z, 0, c2, c->st));
  // the compact copy of block 1 (V_1, W_1) is the first SpMM input; earlier solves reused it.
  // The other ring slots start at zero: the block Lanczos ring writes whole groups of slots
  // into the basis, and slots of blocks a solve never formed must hold finite values.
  const size_t e = (size_t)L.esz;
  HIPOK(hipMemsetAsync(c->sv.panel[1], 0, (size_t)(LZ_RING - 1) * L.n * L.s * e, c->st));
  if (!L.lyap)
    HIPOK(hipMemsetAsync(c->sw.panel[1], 0, (size_t)(LZ_RING - 1) * L.m * L.s * e, c->st));
  HIPOK(hipMemcpy2DAsync(c->sv.panel[0], L.s * e, c->sv.basis, L.ldb * e, L.s * e, L.n,
                         hipMemcpyDeviceToDevice, c->st));
  if (!L.lyap)
    HIPOK(hipMemcpy2DAsync(c->sw.panel[0], L.s * e, c->sw.basis, L.ldb * e, L.s * e, L.m,
                           hipMemcpyDeviceToDevice, c->st));
  // R0 = R_L R_R^T from the first-block factors kept since sylv_create
  int err = launch_setup_scalars((int)L.s, c->RL, c->RR, c->R, c->P, c->Rt, L.ldc, tol, c->ds,
                                 c->st);
  if (err) return err;
  c->solved = 0;
  c->res_valid = 0;
  c->comp_k = -1;
  c->method = method;
  c->max_iter_run = max_iter;
  return 0;
}

int end_solve(Ctx *c, int max_iter, double seconds, sylv_result *res) {
  int e = read_state(c);
  if (e) return e;
  const DevState &d = *c->h_ds;
  if (d.done) {
    c->status = d.status;
    c->iters = d.iters;
  } else {
    c->status = SYLV_NOT_CONVERGED;
    c->iters = max_iter;
  }
  c->relres = d.relres;
  if (c->prof) c->prof->flush(c->iters);
  c->rank = lanczos_method(c->method) ? (int64_t)c->iters * c->L.s
                                       : 2 * (int64_t)c->iters * c->L.s;
  if (c->iters == 0) c->relres = 1.0;
  c->h_hist.assign((size_t)4 * max_iter, 0.0);
  HIPOK(hipMemcpy(c->h_hist.data(), c->hist, sizeof(double) * 4 * max_iter, hipMemcpyDeviceToHost));
  c->solved = 1;
  if (res) {
    res->status = c->status;
    res->iters = c->iters;
    res->rank_v = res->rank_w = c->rank;
    res->rel_res_recursive = c->relres;
    res->seconds = seconds;
    res->outer_steps = 0;
    res->rel_res_true = -1.0;
  }
  return c->status;
}

// Creates a context; with a parent, a correction context of the outer refinement: the problem's
// operators (CSR validated, B^T and the sliced-ELLPACK copies) are the parent's.
// Streams and events of the overlapped Krylov / core schedule (kst = st when not overlapped).
int make_streams(Ctx *c, bool overlap) {
  c->kst = c->st;
  for (hipEvent_t *e : {&c->ev_k[0], &c->ev_k[1], &c->ev_k[2], &c->ev_k[3], &c->ev_c[0],
                        &c->ev_c[1], &c->ev_c[2], &c->ev_s})
    HIPOK(hipEventCreateWithFlags(e, hipEventDisableTiming));
  if (overlap) {
    HIPOK(hipStreamCreateWithFlags(&c->kst, hipStreamNonBlocking));
    c->own_kst = true;
  }
  return 0;
}

void free_streams(Ctx *c) {
  for (hipEvent_t e : {c->ev_k[0], c->ev_k[1], c->ev_k[2], c->ev_k[3], c->ev_c[0], c->ev_c[1],
                       c->ev_c[2], c->ev_s})
    if (e) (void)hipEventDestroy(e);
  if (c->own_kst && c->kst) (void)hipStreamDestroy(c->kst);
  c->own_kst = false;
  c->kst = nullptr;
}

// b waits for the work queued so far on a (no-op when they are the same stream).
int join(Ctx *c, hipStream_t a, hipStream_t b) {
  if (a == b) return 0;
  HIPOK(hipEventRecord(c->ev_s, a));
  HIPOK(hipStreamWaitEvent(b, c->ev_s, 0));
  return 0;
}

int ctx_create(void **out, const sylv_problem *pb, const sylv_options *op, void *workspace,
               size_t ws_bytes, void *stream, Ctx *parent, bool overlap = true) {
  if (!out) return SYLV_ERR_INVALID;
  *out = nullptr;
  Layout L;
  int e = make_layout(pb, op, L, parent != nullptr);
  if (e) return e;
  if (!workspace || ws_bytes < L.total) return SYLV_ERR_WORKSPACE;
  Ctx *c = new (std::nothrow) Ctx();
  if (!c) return SYLV_ERR_INVALID;
  c->L = L;
  c->st = reinterpret_cast<hipStream_t>(stream);
  c->A = pb->A;
  c->B = pb->B;
  c->closure_tol = op->closure_tol > 0 ? op->closure_tol : (L.fp32 ? 1e-6 : 1e-12);
  c->parent = parent;
  c->refine_inner_tol = op->refine_inner_tol;
  c->check_every = op->check_every > 0 ? op->check_every : 16;
  c->verify = op->verify;
  c->record_history = op->record_history;
  c->lagged = !lanczos_method(L.method) && op->reorth != 1 &&
              arnoldi_lagged_supported((int)L.s, L.fp32);
  c->ws = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(workspace) + ALIGN - 1) / ALIGN * ALIGN);
  if (hipHostMalloc(reinterpret_cast<void **>(&c->h_ds), sizeof(DevState)) != hipSuccess) {
    delete c;
    return SYLV_ERR_HIP;
  }
  c->H = at<double>(c, L.off_H);
  c->G = at<double>(c, L.off_G);
  c->X = at<double>(c, L.off_X);
  c->R = at<double>(c, L.off_R);
  c->P = at<double>(c, L.off_P);
  c->Q = at<double>(c, L.off_Q);
  c->S = L.off_S ? at<double>(c, L.off_S) : nullptr;
  c->T = L.off_T ? at<double>(c, L.off_T) : nullptr;
  for (int i = 0; i < extra_cores(L.method); ++i) c->Ex[i] = at<double>(c, L.off_Ex[i]);
  c->Rt = at<double>(c, L.off_rt);
  c->RL = at<double>(c, L.off_rl);
  c->RR = at<double>(c, L.off_rr);
  c->hist = at<double>(c, L.off_hist);
  c->cpart = L.cpart_cap ? at<double>(c, L.off_cpart) : nullptr;
  c->ds = at<DevState>(c, L.off_ds);
  c->ssv = at<SideState>(c, L.off_ssv);
  c->ssw = L.lyap ? c->ssv : at<SideState>(c, L.off_ssw);
  c->sc.partials = at<double>(c, L.off_partials);
  c->sc.partial_cap = L.partial_cap;
  c->sc.counters = at<int>(c, L.off_counters);
  c->scc.partials = at<double>(c, L.off_cscr);
  c->scc.partial_cap = CORE_SCRATCH;
  c->scc.counters = c->sc.counters;
  c->btrp = at<int32_t>(c, L.off_btrp);
  c->btci = at<int32_t>(c, L.off_btci);
  c->btval = at<double>(c, L.off_btval);
  c->flag = at<int>(c, L.off_flag);
  c->dots = at<double>(c, L.off_dots);

  auto fail = [&](int code) {
    hipHostFree(c->h_ds);
    free_streams(c);
    delete c;
    return code;
  };
  // second stream for the Krylov steps: requested, or automatic for bases of 16384+ rows
  const int64_t krows = L.n + (L.lyap ? 0 : L.m);
  overlap = overlap && (op->streams == 2 || (op->streams == 0 && krows >= 16384));
  if ((e = make_streams(c, overlap))) return fail(e);
  hipStream_t st = c->st;
  if (hipMemsetAsync(c->sc.counters, 0, CNT_MAX * sizeof(int), st) != hipSuccess ||
      hipMemsetAsync(c->ds, 0, sizeof(DevState), st) != hipSuccess ||
      hipMemsetAsync(c->flag, 0, 16 * sizeof(int), st) != hipSuccess)
    return fail(SYLV_ERR_HIP);
  // validate CSR structure on the device (a correction context reuses the parent's operators)
  if (!parent && (e = launch_csr_validate(L.n, pb->A.nnz, pb->A.row_ptr, pb->A.col_idx, c->flag, st)))
    return fail(e);
  if (!parent && !L.lyap &&
      (e = launch_csr_validate(L.m, pb->B.nnz, pb->B.row_ptr, pb->B.col_idx, c->flag + 1, st)))
    return fail(e);
  int hflag[2] = {0, 0};
  if (hipMemcpyAsync(hflag, c->flag, sizeof(hflag), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(SYLV_ERR_HIP);
  if (hflag[0] || hflag[1]) return fail(SYLV_ERR_INVALID);
  // W side operator: B^T
  if (!L.lyap && !parent) {
    if ((e = launch_csr_transpose(L.m, pb->B.nnz, pb->B.row_ptr, pb->B.col_idx, pb->B.values,
                                  c->btrp, c->btci, c->btval, at<void>(c, L.off_tscr), st)))
      return fail(e);
  }
  char *panv = at<char>(c, L.off_panV), *panw = at<char>(c, L.off_panW);
  c->sv = SideDesc{L.n, pb->A.nnz, pb->A.row_ptr, pb->A.col_idx, pb->A.values,
                   at<void>(c, L.off_V), L.ldb, c->H, at<double>(c, L.off_U),
                   at<double>(c, L.off_coefV), c->ssv, {}, L.fp32, SellMat{}};
  for (int k = 0; k < LZ_RING; ++k) c->sv.panel[k] = panv + k * L.n * L.s * L.esz;
  if (L.lyap) {
    c->sw = c->sv;
  } else {
    c->sw = SideDesc{L.m, pb->B.nnz, c->btrp, c->btci, c->btval, at<void>(c, L.off_W), L.ldb,
                     c->G, at<double>(c, L.off_Uw), at<double>(c, L.off_coefW), c->ssw, {},
                     L.fp32, SellMat{}};
    for (int k = 0; k < LZ_RING; ++k) c->sw.panel[k] = panw + k * L.m * L.s * L.esz;
  }
  if (parent) {
    // operators of the parent: V side A; W side B^T (A when the parent is a Lyapunov problem)
    const SideDesc &pw = parent->L.lyap ? parent->sv : parent->sw;
    c->sv.rp = parent->sv.rp;
    c->sv.ci = parent->sv.ci;
    c->sv.val = parent->sv.val;
    c->sv.nnz = parent->sv.nnz;
    c->sv.sell = parent->sv.sell;
    c->sw.rp = pw.rp;
    c->sw.ci = pw.ci;
    c->sw.val = pw.val;
    c->sw.nnz = pw.nnz;
    c->sw.sell = pw.sell;
  }
  // SELL copies of A and B^T for the Krylov SpMM (CSR stays in use if the padding is large)
  if (!parent) c->sv.sell = SellMat{};
  if (!parent) {
    int nar = 0;
    e = build_sell(L.n, pb->A.nnz, pb->A.row_ptr, pb->A.col_idx, pb->A.values,
                   at<void>(c, L.off_sellA), st, true, &nar);
    if (e == 0) {
      c->sv.sell = sell_view(L.n, pb->A.nnz, at<void>(c, L.off_sellA));
      c->sv.sell.narrow = nar;
    } else if (e != SYLV_ERR_WORKSPACE) {
      return fail(e);
    }
  }
  if (parent) {
  } else if (L.lyap) {
    c->sw.sell = c->sv.sell;
  } else {
    c->sw.sell = SellMat{};
    int nar = 0;
    e = build_sell(L.m, pb->B.nnz, c->btrp, c->btci, c->btval, at<void>(c, L.off_sellB), st,
                   true, &nar);
    if (e == 0) {
      c->sw.sell = sell_view(L.m, pb->B.nnz, at<void>(c, L.off_sellB));
      c->sw.sell.narrow = nar;
    } else if (e != SYLV_ERR_WORKSPACE) {
      return fail(e);
    }
  }
  // QR factorizations C1 = V_1 R_L, C2 = W_1 R_R (Alg. 4.1 step 1, Alg. 4.2 step 2)
  const int s = (int)L.s;
  if ((e = launch_first_block(s, c->sv, pb->C1, pb->ldc1, c->closure_tol, c->sc, c->ds, st)))
    return fail(e);
  if (hipMemcpyAsync(c->RL, c->ssv->Hs1, sizeof(double) * SYLV_MAX_S * SYLV_MAX_S,
                     hipMemcpyDeviceToDevice, st) != hipSuccess)
    return fail(SYLV_ERR_HIP);
  SideState hs[2];
  if (hipMemcpyAsync(&hs[0], c->ssv, sizeof(SideState), hipMemcpyDeviceToHost, st) != hipSuccess)
    return fail(SYLV_ERR_HIP);
  if (!L.lyap) {
    if ((e = launch_first_block(s, c->sw, pb->C2, pb->ldc2, c->closure_tol, c->sc, c->ds, st)))
      return fail(e);
    if (hipMemcpyAsync(c->RR, c->ssw->Hs1, sizeof(double) * SYLV_MAX_S * SYLV_MAX_S,
                       hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(&hs[1], c->ssw, sizeof(SideState), hipMemcpyDeviceToHost, st) != hipSuccess)
      return fail(SYLV_ERR_HIP);
  } else {
    if (hipMemcpyAsync(c->RR, c->RL, sizeof(double) * SYLV_MAX_S * SYLV_MAX_S,
                       hipMemcpyDeviceToDevice, st) != hipSuccess)
      return fail(SYLV_ERR_HIP);
    hs[1] = hs[0];
  }
  // right-hand-side QR defects D1 = C1 - V_1 R_L, D2 = C2 - W_1 R_R and a copy of C2, for the
  // true residual (C1, C2 are not read after creation)
  {
    const double *C2in = L.lyap ? pb->C1 : pb->C2;
    const int64_t ld2 = L.lyap ? pb->ldc1 : pb->ldc2;
    if ((e = launch_qr_defect(L.n, s, pb->C1, pb->ldc1, c->sv.basis, L.fp32, L.ldb, c->RL,
                              at<double>(c, L.off_d1), st)))
      return fail(e);
    if (!L.lyap && (e = launch_qr_defect(L.m, s, pb->C2, pb->ldc2, c->sw.basis, L.fp32, L.ldb,
                                         c->RR, at<double>(c, L.off_d2), st)))
      return fail(e);
    if (hipMemcpy2DAsync(at<double>(c, L.off_c2), s * 8, C2in, ld2 * 8, s * 8, L.m,
                         hipMemcpyDeviceToDevice, st) != hipSuccess)
      return fail(SYLV_ERR_HIP);
  }
  // A^T for the refinement's products with the transposed residual
  if (L.refine_max > 0) {
    int32_t *atrp = at<int32_t>(c, L.off_atrp), *atci = at<int32_t>(c, L.off_atci);
    double *atval = at<double>(c, L.off_atval);
    if ((e = launch_csr_transpose(L.n, pb->A.nnz, pb->A.row_ptr, pb->A.col_idx, pb->A.values, atrp,
                                  atci, atval, at<void>(c, L.off_atscr), st)))
      return fail(e);
    c->AT = sylv_csr{L.n, pb->A.nnz, atrp, atci, atval};
  }
  if (hipStreamSynchronize(st) != hipSuccess) return fail(SYLV_ERR_HIP);
  for (int i = 0; i < 2; ++i) {
    if (!std::isfinite(hs[i].ref2)) return fail(SYLV_ERR_INVALID);
    if (hs[i].mode != 0) return fail(SYLV_ERR_RHS_RANK);
  }
  *out = c;
  return 0;
}



// ---- outer refinement (mixed precision) ----
// The residual of the summed iterate X = sum_j V_j X_j W_j^T, where step 0 solves the problem
// and step j >= 1 the correction equation with right-hand side P_j Q_j^T, is
//   R = sum_j D_j - sum_{j>=1} P_j Q_j^T,
//   D_j = D1 C2^T + V_1 R_L D2^T + V_j+ R^_j W_j+^T - E_A,j X_j W_j^T - V_j X_j E_B,j^T
// (the defect form of each step: E_A = A V - V+ H, E_B = B^T W - W+ G, R^ = C_core - L(X),
// D1 = C1 - V_1 R_L, D2 = C2 - W_1 R_R for the step's right-hand side C1 C2^T).
// Products of R and R^T with narrow panels need only the factors; the FP64 norm of R is the
// trace <G_L M, M G_N> over the Grams of the stacked tall factors.

// R^_j = [R0 0; 0 0] - L(X_j) into the step's Lx buffer.
int compute_rhat(Ctx *cj) {
  const Layout &L = cj->L;
  const int s = (int)L.s;
  const int64_t p = cj->rank, q = p + s;
  double *Lx = at<double>(cj, L.off_Lx);
  int e = launch_core_op(s, (int)p, cj->H, cj->G, cj->X, Lx, L.ldc, nullptr, cj->st);
  if (e) return e;
  return launch_rhat(s, (int)q, Lx, cj->Rt, Lx, L.ldc, cj->st);
}

// Y (left rows x qz) += D_j Z (trans: D_j^T Z), Z (right rows x qz); narrow panels of stride
// NLD; R^_j must be current in the step's Lx buffer. D_j includes the right-hand-side defect
// D1 C2^T + V_1 R_L D2^T (the QR of C1, C2 holds only to the basis storage precision).
int apply_step(Ctx *P, Ctx *cj, bool trans, int qz, const double *Z, double *Y) {
  const Layout &PL = P->L, &CL = cj->L;
  hipStream_t st = P->st;
  const SideDesc &Ls = trans ? cj->sw : cj->sv;
  const SideDesc &Rs = trans ? cj->sv : cj->sw;
  const double *Hl = trans ? cj->G : cj->H, *Hr = trans ? cj->H : cj->G;
  // transpose of the right side's operator: B (of B^T) or A^T
  const sylv_csr &MrT = (trans || PL.lyap) ? P->AT : P->B;
  const int64_t p = cj->rank, q = p + CL.s, ldc = CL.ldc, ldb = CL.ldb;
  if (p == 0) return 0;
  const bool f32 = CL.fp32;
  double *a = at<double>(P, PL.off_sa), *b = at<double>(P, PL.off_sb);
  double *c2 = at<double>(P, PL.off_sc2), *d = at<double>(P, PL.off_sd);
  double *Zb = at<double>(P, PL.off_Zb), *Eb = at<double>(P, PL.off_Eb);
  double *Fb = at<double>(P, PL.off_Fb), *tn = at<double>(P, PL.off_tn);
  const double *Rh = at<double>(cj, CL.off_Lx);
  const int64_t xr = trans ? 1 : ldc, xc = trans ? ldc : 1;
  const int s = (int)CL.s;
  const double *D1 = at<double>(cj, CL.off_d1), *D2 = at<double>(cj, CL.off_d2);
  const double *C2 = at<double>(cj, CL.off_c2);
  int e;
  // right-hand-side defect D1 C2^T + V_1 R_L D2^T (transposed: C2 D1^T + D2 R_L^T V_1^T)
  if (!trans) {
    if ((e = launch_tn(Rs.rows, s, qz, C2, false, s, Z, NLD, a, NLD, tn, PL.tn_cap, st))) return e;
    if ((e = launch_nn(Ls.rows, s, qz, 1.0, D1, false, s, a, NLD, 1.0, Y, NLD, st))) return e;
    if ((e = launch_tn(Rs.rows, s, qz, D2, false, s, Z, NLD, b, NLD, tn, PL.tn_cap, st))) return e;
    if ((e = launch_gemm(s, qz, s, 1.0, cj->RL, s, 1, b, NLD, 1, 0.0, c2, NLD, st))) return e;
    if ((e = launch_nn(Ls.rows, s, qz, 1.0, Ls.basis, f32, ldb, c2, NLD, 1.0, Y, NLD, st)))
      return e;
  } else {
    if ((e = launch_tn(Rs.rows, s, qz, D1, false, s, Z, NLD, a, NLD, tn, PL.tn_cap, st))) return e;
    if ((e = launch_nn(Ls.rows, s, qz, 1.0, C2, false, s, a, NLD, 1.0, Y, NLD, st))) return e;
    if ((e = launch_tn(Rs.rows, s, qz, Rs.basis, f32, ldb, Z, NLD, b, NLD, tn, PL.tn_cap, st)))
      return e;
    if ((e = launch_gemm(s, qz, s, 1.0, cj->RL, 1, s, b, NLD, 1, 0.0, c2, NLD, st))) return e;
    if ((e = launch_nn(Ls.rows, s, qz, 1.0, D2, false, s, c2, NLD, 1.0, Y, NLD, st))) return e;
  }
  // a = R+^T Z; b = E_R^T Z = R_p^T (M_R^T Z) - H_R^T a
  if ((e = launch_tn(Rs.rows, (int)q, qz, Rs.basis, f32, ldb, Z, NLD, a, NLD, tn, PL.tn_cap, st)))
    return e;
  if ((e = launch_spmm(qz, Rs.rows, MrT.row_ptr, MrT.col_idx, MrT.values, Z, NLD, Zb, NLD, st)))
    return e;
  if ((e = launch_tn(Rs.rows, (int)p, qz, Rs.basis, f32, ldb, Zb, NLD, b, NLD, tn, PL.tn_cap, st)))
    return e;
  if ((e = launch_gemm(p, qz, q, -1.0, Hr, 1, ldc, a, NLD, 1, 1.0, b, NLD, st))) return e;
  // d = R^ a + H_L X a_p - [X b; 0]; c2 = X a_p
  if ((e = launch_gemm(q, qz, q, 1.0, Rh, xr, xc, a, NLD, 1, 0.0, d, NLD, st))) return e;
  if ((e = launch_gemm(p, qz, p, 1.0, cj->X, xr, xc, a, NLD, 1, 0.0, c2, NLD, st))) return e;
  if ((e = launch_gemm(q, qz, p, 1.0, Hl, ldc, 1, c2, NLD, 1, 1.0, d, NLD, st))) return e;
  if ((e = launch_gemm(p, qz, p, -1.0, cj->X, xr, xc, b, NLD, 1, 1.0, d, NLD, st))) return e;
  // Y += L+ d - M_L (L_p c2)
  if ((e = launch_nn(Ls.rows, (int)q, qz, 1.0, Ls.basis, f32, ldb, d, NLD, 1.0, Y, NLD, st)))
    return e;
  if ((e = launch_nn(Ls.rows, (int)p, qz, 1.0, Ls.basis, f32, ldb, c2, NLD, 0.0, Eb, NLD, st)))
    return e;
  if ((e = launch_spmm(qz, Ls.rows, Ls.rp, Ls.ci, Ls.val, Eb, NLD, Fb, NLD, st))) return e;
  return launch_axpy_narrow(Ls.rows, qz, -1.0, Fb, NLD, Y, NLD, st);
}

double *pp_panel(Ctx *P, int i) { return at<double>(P, P->L.off_Pp) + (size_t)i * P->L.n * NLD; }
double *qq_panel(Ctx *P, int i) { return at<double>(P, P->L.off_Qp) + (size_t)i * P->L.m * NLD; }

// Y (n x qz) += R Z (trans: Y (m x qz) += R^T Z) over the steps and the compressed right-hand
// sides of the corrections so far.
int apply_residual(Ctx *P, const std::vector<Ctx *> &steps, bool trans, int qz, const double *Z,
                   double *Y) {
  const Layout &PL = P->L;
  double *sk = at<double>(P, PL.off_sk), *tn = at<double>(P, PL.off_tn);
  int e;
  for (Ctx *cj : steps)
    if ((e = apply_step(P, cj, trans, qz, Z, Y))) return e;
  for (size_t i = 0; i + 1 < steps.size(); ++i) {
    // - P_i Q_i^T Z  (trans: - Q_i P_i^T Z)
    const int k = P->kid_k[i];
    const double *Rp = trans ? pp_panel(P, (int)i) : qq_panel(P, (int)i);
    const double *Lp = trans ? qq_panel(P, (int)i) : pp_panel(P, (int)i);
    const int64_t rr = trans ? PL.n : PL.m, lr = trans ? PL.m : PL.n;
    if ((e = launch_tn(rr, k, qz, Rp, false, NLD, Z, NLD, sk, NLD, tn, PL.tn_cap, P->st))) return e;
    if ((e = launch_nn(lr, k, qz, -1.0, Lp, false, NLD, sk, NLD, 1.0, Y, NLD, P->st))) return e;
  }
  return 0;
}

// Frobenius norm of the residual R = L M N^T of the (summed) iterate from the Grams of the
// stacked tall factors: per step j, L gets [V_j+, E_A,j, D1_j] and N gets [W_j+, E_B,j, D2_j,
// C2_j]; per correction i, L gets P_i and N gets Q_i. With D1 = C1 - V_1 R_L and
// D2 = C2 - W_1 R_R (the right-hand side's QR defects, O(u) of the basis storage precision),
//   R_j = D1 C2^T + V_1 R_L D2^T + V+ R^ W+^T - E_A X W^T - V X E_B^T,
// and ||R||^2 = <G_L M, M G_N>. No term cancels against ||C1 C2^T||: every block is of the size
// of the residual or of a defect.
int stacked_residual(Ctx *P, const std::vector<Ctx *> &steps, double *abs_res, double *rel_res) {
  const Layout &PL = P->L;
  hipStream_t st = P->st;
  int e;
  struct Seg {
    const char *ptr;  // rowed: row r at ptr + r ld esz; else E-buffer columns (chunk rows)
    bool f32, rowed;
    int64_t ld, cols, esz;
    bool defect;      // basis defects, QR defects and the C2 columns beside them
  };
  double *Es = at<double>(P, PL.off_Es);
  for (Ctx *cj : steps)
    if (cj->rank > 0 && (e = compute_rhat(cj))) return e;
  // E-buffer columns per step (64-column aligned): [E_A | D1] on the V side, [E_B | D2 | C2] on
  // the W side, so each side of a step is two Gram segments (basis, defects)
  std::vector<int64_t> eoff(steps.size());
  int64_t eo = 0;
  for (size_t j = 0; j < steps.size(); ++j) {
    eoff[j] = eo;
    eo += round_up(steps[j]->rank + 2 * steps[j]->L.s, 64);
  }
  if (eo > PL.ldE) return SYLV_ERR_WORKSPACE;
  struct Idx {
    int v, e, w, eb;
  };
  std::vector<Idx> idx(steps.size(), Idx{-1, -1, -1, -1});
  std::vector<Seg> segL, segN;
  std::vector<int> pL, qN;
  // compact sources copied per chunk into the E buffer: (step, column offset, source, columns)
  struct Fill {
    int64_t col;
    const double *src;
    int cols;
  };
  std::vector<Fill> fillL, fillN;
  for (size_t j = 0; j < steps.size(); ++j) {
    Ctx *cj = steps[j];
    if (cj->rank == 0) continue;
    const Layout &CL = cj->L;
    const int64_t p = cj->rank, q = p + CL.s, s = CL.s;
    const char *eb = reinterpret_cast<const char *>(Es + eoff[j]);
    idx[j].v = (int)segL.size();
    segL.push_back(Seg{static_cast<const char *>(cj->sv.basis), (bool)CL.fp32, true, CL.ldb, q,
                       CL.esz, false});
    idx[j].e = (int)segL.size();
    segL.push_back(Seg{eb, false, false, PL.ldE, p + s, 8, true});
    fillL.push_back(Fill{eoff[j] + p, at<double>(cj, CL.off_d1), (int)s});
    idx[j].w = (int)segN.size();
    segN.push_back(Seg{static_cast<const char *>(cj->sw.basis), (bool)CL.fp32, true, CL.ldb, q,
                       CL.esz, false});
    idx[j].eb = (int)segN.size();
    segN.push_back(Seg{eb, false, false, PL.ldE, p + 2 * s, 8, true});
    fillN.push_back(Fill{eoff[j] + p, at<double>(cj, CL.off_d2), (int)s});
    fillN.push_back(Fill{eoff[j] + p + s, at<double>(cj, CL.off_c2), (int)s});
  }
  for (size_t i = 0; i + 1 < steps.size(); ++i) {
    pL.push_back((int)segL.size());
    segL.push_back(Seg{reinterpret_cast<const char *>(pp_panel(P, (int)i)), false, true, NLD,
                       P->kid_k[i], 8, false});
    qN.push_back((int)segN.size());
    segN.push_back(Seg{reinterpret_cast<const char *>(qq_panel(P, (int)i)), false, true, NLD,
                       P->kid_k[i], 8, false});
  }
  auto offsets = [](const std::vector<Seg> &segs) {
    std::vector<int64_t> o(segs.size() + 1, 0);
    for (size_t a = 0; a < segs.size(); ++a) o[a + 1] = o[a] + segs[a].cols;
    return o;
  };
  const std::vector<int64_t> offL = offsets(segL), offN = offsets(segN);
  const int64_t cL = offL.back(), cN = offN.back(), ldG = PL.cmax;
  if (cL > PL.cmax || cN > PL.cmax) return SYLV_ERR_WORKSPACE;
  double *GL = at<double>(P, PL.off_GL), *GN = at<double>(P, PL.off_GN);
  double *Mc = at<double>(P, PL.off_Mc), *T1 = at<double>(P, PL.off_T1);
  double *gpart = at<double>(P, PL.off_gpart);
  auto side_pass = [&](bool w, const std::vector<Seg> &segs, const std::vector<int64_t> &offs,
                       double *G) -> int {
    const int64_t rows = w ? PL.m : PL.n;
    int ee;
    for (Ctx *cj : steps) {
      if (cj->rank == 0 || lanczos_method(cj->L.method)) continue;
      const SideDesc &sd = w ? cj->sw : cj->sv;
      const int64_t q = cj->rank + cj->L.s;
      const int qk = (int)std::min<int64_t>(round_up(q, 32), cj->L.ldb);
      if ((ee = launch_zero_cols(sd.rows, sd.basis, cj->L.fp32, cj->L.ldb, (int)q, qk, st)))
        return ee;
    }
    for (int64_t r0 = 0; r0 < rows; r0 += PL.rc_rows) {
      const int64_t r1 = std::min(rows, r0 + PL.rc_rows), nr = r1 - r0;
      for (size_t j = 0; j < steps.size(); ++j) {
        Ctx *cj = steps[j];
        if (cj->rank == 0) continue;
        const Layout &CL = cj->L;
        const SideDesc &sd = w ? cj->sw : cj->sv;
        const double *Hm = w ? cj->G : cj->H;
        const int p = (int)cj->rank, q = p + (int)CL.s;
        double *Ej = Es + eoff[j];
        prof_begin(P->sc, st);
        if (lanczos_method(CL.method)) {
          if ((ee = launch_defect_band(r0, r1, sd.rp, sd.ci, sd.val, sd.basis, CL.fp32, CL.ldb, p, q,
                                       (int)CL.s, Hm, CL.ldc, at<double>(cj, CL.off_M2), CL.ldc,
                                       r0 == 0, Ej, PL.ldE, st)))
            return ee;
        } else {
          if ((ee = launch_spmm_rows((int)CL.s, r0, r1, sd.rp, sd.ci, sd.val, sd.basis, CL.fp32,
                                     CL.ldb, p, Ej, PL.ldE, st)))
            return ee;
          const char *vb = static_cast<const char *>(sd.basis) + r0 * CL.ldb * CL.esz;
          if ((ee = launch_defect_gemm(nr, p, q, (int)CL.s, vb, CL.fp32, CL.ldb, Hm, CL.ldc, Ej,
                                       PL.ldE, st)))
            return ee;
        }
        // algorithmic: the basis rows read once, the defect rows written once; flops of the
        // operator rows (their average length) and the band (3 s entries per column), or of the
        // dense Hessenberg product
        const double row_nnz = sd.rows > 0 ? (double)sd.nnz / (double)sd.rows : 0.0;
        const double dflops = lanczos_method(CL.method)
                                  ? 2.0 * nr * p * (row_nnz + 3.0 * CL.s)
                                  : 2.0 * nr * p * (row_nnz + (double)q);
        prof_end(P->sc, FAM_RES_DEFECT, (double)nr * (CL.esz * q + 8.0 * p), dflops, st);
      }
      // compact sources (QR defects, C2) next to the defects
      for (const Fill &f : (w ? fillN : fillL))
        if ((ee = launch_copy_block((int)nr, f.cols, 1.0, f.src + r0 * f.cols, f.cols, false,
                                    Es + f.col, PL.ldE, st)))
          return ee;
      const double beta = r0 == 0 ? 0.0 : 1.0;
      // split BF16 for the blocks with a defect operand (gram_precision 1) or for all (2)
      auto bf16_block = [&](size_t a, size_t b) {
        return PL.gram_prec == 2 || (PL.gram_prec == 1 && (segs[a].defect || segs[b].defect));
      };
      bool any_bf16 = false;
      for (size_t a = 0; a < segs.size(); ++a)
        for (size_t b = 0; b <= a; ++b) any_bf16 = any_bf16 || bf16_block(a, b);
      if (any_bf16) {
        if (segs.size() > (size_t)BF_MAX_SEGS) return SYLV_ERR_WORKSPACE;
        BfSegs bs{};
        for (size_t a = 0; a < segs.size(); ++a) {
          const Seg &A = segs[a];
          bs.s[a] = BfSeg{A.ptr + (A.rowed ? r0 * A.ld * A.esz : 0), A.ld, offs[a], A.cols,
                          (int)A.esz, 0};
        }
        bs.count = (int)segs.size();
        prof_begin(P->sc, st);
        if ((ee = launch_bf16_pack(bs, nr, offs.back(), PL.cpad,
                                   at<unsigned long long>(P, PL.off_cmaxb), at<int>(P, PL.off_cexp),
                                   at<char>(P, PL.off_pack), st)))
          return ee;
        double pb = 0.0;
        for (const Seg &A : segs) pb += (double)nr * A.cols * A.esz;
        prof_end(P->sc, FAM_RES_PACK, pb + 4.0 * (double)nr * offs.back(), 0.0, st);
      }
      // the FP64 blocks of the chunk as one launch on 128 x 128 tiles (whole-tile rounds across
      // all of them) when they are large enough and the partial slots fit
      std::vector<char> batched(segs.size() * segs.size(), 0);
      {
        GramJob jobs[GRAM_JOBS_MAX];
        int nj = 0;
        double jbytes = 0.0, jfl = 0.0;
        for (size_t a = 0; a < segs.size() && nj < GRAM_JOBS_MAX; ++a)
          for (size_t b = 0; b <= a && nj < GRAM_JOBS_MAX; ++b) {
            const Seg &A = segs[a], &B = segs[b];
            if (bf16_block(a, b) || A.f32 || B.f32) continue;
            const char *pa = A.ptr + (A.rowed ? r0 * A.ld * A.esz : 0);
            const char *pb = B.ptr + (B.rowed ? r0 * B.ld * B.esz : 0);
            jobs[nj++] = GramJob{GramSeq{0, 0, a == b ? 1 : 0}, A.cols, B.cols,
                                 reinterpret_cast<const double *>(pa), A.ld,
                                 reinterpret_cast<const double *>(pb), B.ld,
                                 G + offs[a] * ldG + offs[b], ldG, 0};
            batched[a * segs.size() + b] = 1;
            jbytes += (double)nr * (a == b ? A.cols * A.esz : A.cols * A.esz + B.cols * B.esz);
            jfl += (a == b ? (double)A.cols * (A.cols + 1) : 2.0 * A.cols * B.cols) * nr;
          }
        int je = 1;
        if (nj > 1) {
          prof_begin(P->sc, st);
          je = launch_gram_jobs(jobs, nj, nr, beta, st, gpart, PL.gpart_cap);
          if (je < 0) return je;
          if (je == 0) prof_end(P->sc, FAM_RES_GRAM, jbytes, jfl, st);
        }
        if (je != 0) std::fill(batched.begin(), batched.end(), 0);
      }
      for (size_t a = 0; a < segs.size(); ++a)
        for (size_t b = 0; b <= a; ++b) {
          const Seg &A = segs[a], &B = segs[b];
          if (batched[a * segs.size() + b]) continue;
          // useful flops of the block (lower triangle only when a == b)
          const double fl = (a == b ? (double)A.cols * (A.cols + 1) : 2.0 * A.cols * B.cols) * nr;
          if (bf16_block(a, b)) {
            prof_begin(P->sc, st);
            if ((ee = launch_gram_bf16(A.cols, B.cols, nr, at<char>(P, PL.off_pack), PL.cpad,
                                       at<int>(P, PL.off_cexp), offs[a], offs[b], beta,
                                       G + offs[a] * ldG + offs[b], ldG, a == b, st,
                                       at<float>(P, PL.off_bpart), PL.bpart_floats)))
              return ee;
            // three BF16 products per FP64-equivalent product; operands read as packed hi/lo
            prof_end(P->sc, FAM_RES_BF16, 4.0 * nr * (a == b ? A.cols : A.cols + B.cols), 3.0 * fl,
                     st);
            continue;
          }
          const char *pa = A.ptr + (A.rowed ? r0 * A.ld * A.esz : 0);
          const char *pb = B.ptr + (B.rowed ? r0 * B.ld * B.esz : 0);
          prof_begin(P->sc, st);
          if ((ee = launch_gram(A.cols, B.cols, nr, pa, A.f32, A.ld, pb, B.f32, B.ld, beta,
                                G + offs[a] * ldG + offs[b], ldG, a == b, st, gpart, PL.gpart_cap)))
            return ee;
          prof_end(P->sc, FAM_RES_GRAM,
                   (double)nr * (a == b ? A.cols * A.esz : A.cols * A.esz + B.cols * B.esz), fl,
                   st);
        }
    }
    return launch_mirror(offs.back(), G, ldG, st);
  };
  // Lyapunov with a single step: B^T = A, W = V, G = H, so the W-side factors are the V-side
  // ones followed by C1 (E_B = E_A, D2 = D1, C2 = C1) and G_L is the leading cL x cL block of
  // G_N; one pass over the rows serves both sides.
  const bool shared = PL.lyap && steps.size() == 1;
  if (!shared && (e = side_pass(false, segL, offL, GL))) return e;
  if ((e = side_pass(true, segN, offN, GN))) return e;
  if (shared && (e = launch_copy_block((int)cL, (int)cL, 1.0, GN, ldG, false, GL, ldG, st)))
    return e;
  // M (cL x cN)
  HIPOK(hipMemset2DAsync(Mc, ldG * 8, 0, cN * 8, cL, st));
  auto put = [&](int64_t r, int64_t c, int rows, int cols, double alpha, const double *src,
                 int64_t lds) -> int {
    return launch_copy_block(rows, cols, alpha, src, lds, false, Mc + r * ldG + c, ldG, st);
  };
  for (size_t j = 0; j < steps.size(); ++j) {
    Ctx *cj = steps[j];
    if (cj->rank == 0) continue;
    const Layout &CL = cj->L;
    const int p = (int)cj->rank, q = p + (int)CL.s, s = (int)CL.s;
    const Idx &x = idx[j];
    const int64_t d1 = offL[x.e] + p, d2 = offN[x.eb] + p, c2 = d2 + s;
    if ((e = put(offL[x.v], offN[x.w], q, q, 1.0, at<double>(cj, CL.off_Lx), CL.ldc))) return e;
    if ((e = put(offL[x.e], offN[x.w], p, p, -1.0, cj->X, CL.ldc))) return e;
    if ((e = put(offL[x.v], offN[x.eb], p, p, -1.0, cj->X, CL.ldc))) return e;
    if ((e = launch_diag_fill(s, 1.0, Mc + d1 * ldG + c2, ldG, st))) return e;
    if ((e = put(offL[x.v], d2, s, s, 1.0, cj->RL, s))) return e;
  }
  for (size_t i = 0; i + 1 < steps.size(); ++i) {
    if ((e = launch_diag_fill(P->kid_k[i], -1.0, Mc + offL[pL[i]] * ldG + offN[qN[i]], ldG, st)))
      return e;
  }
  // ||R||^2 = <G_L M, M G_N>: G_L M as A^T B on the symmetric Gram; M G_N into G_L's storage
  if ((e = launch_gram(cL, cN, cL, GL, false, ldG, Mc, false, ldG, 0.0, T1, ldG, false, st, gpart,
                       PL.gpart_cap)))
    return e;
  if ((e = launch_gemm_nn(cL, cN, cN, Mc, ldG, GN, ldG, GL, ldG, st))) return e;
  if ((e = launch_dot(cL, cN, T1, ldG, GL, ldG, P->dots, P->sc, st))) return e;
  double r2 = 0.0;
  HIPOK(hipMemcpyAsync(&r2, P->dots, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  const double ar = std::sqrt(std::max(r2, 0.0));
  if (abs_res) *abs_res = ar;
  if (rel_res) *rel_res = ar / P->h_ds->normR0;
  return 0;
}

std::vector<Ctx *> refine_steps(Ctx *P) {
  std::vector<Ctx *> v{P};
  v.insert(v.end(), P->kids.begin(), P->kids.end());
  return v;
}

// True residual of the current (summed) iterate, kept until the next solve.
int true_residual(Ctx *c, double *abs_res, double *rel_res) {
  if (!c->res_valid) {
    int e = read_state(c);
    if (e) return e;
    if (c->prof) c->prof->iter = 0;
    if (c->rank == 0 && c->kids.empty()) {
      c->res_abs = c->h_ds->normR0;
      c->res_rel = 1.0;
    } else if ((e = stacked_residual(c, refine_steps(c), &c->res_abs, &c->res_rel))) {
      return e;
    }
    if (c->prof) c->prof->flush(1);  // the residual's launches (stream idle after its read-back)
    c->res_valid = 1;
  }
  if (abs_res) *abs_res = c->res_abs;
  if (rel_res) *rel_res = c->res_rel;
  return 0;
}

// Solve with outer refinement: the first solve (to max(tol, refine_inner_tol)); then, while the
// sketched residual norm ||R Omega||_F / sqrt(q) (an unbiased estimate of ||R||_F^2 when squared)
// exceeds tol / 2 and corrections remain, compress R to P (R^T P)^T through the sketch
// Y = R R^T R Omega (one power step) and solve the correction equation with that right-hand
// side. The FP64 true
// residual of the summed iterate is evaluated at the end; if it misses tol while corrections
// remain, the loop resumes.
int refined_solve(Ctx *P, int method, double tol, int max_iter, sylv_result *res) {
  const Layout &PL = P->L;
  hipStream_t st = P->st;
  auto t0 = std::chrono::steady_clock::now();
  for (Ctx *k : P->kids) sylv_destroy(k);
  P->kids.clear();
  P->kid_k.clear();
  P->rel_true = -1.0;
  P->outer_steps = 0;
  sylv_result r0{};
  P->in_refine = 1;
  int e = (method == SYLV_METHOD_CG)
              ? sylv_factored_cg(P, std::max(tol, P->refine_inner_tol), max_iter, &r0)
              : sylv_factored_bicgstab(P, std::max(tol, P->refine_inner_tol), max_iter, &r0);
  P->in_refine = 0;
  if (e < 0) return e;
  const int first_status = e;
  const double normR0 = P->h_ds->normR0;
  int total_iters = r0.iters;
  double rel = -1.0, absr = 0.0;
  const int q = (int)std::min<int64_t>(PL.refine_q, std::min(PL.n, PL.m));
  double *Om = at<double>(P, PL.off_Om), *Yb = at<double>(P, PL.off_Yb);
  double *sk = at<double>(P, PL.off_sk), *sT = at<double>(P, PL.off_sT);
  double *tn = at<double>(P, PL.off_tn);
  int *info = at<int>(P, PL.off_rinfo);
  double *dinfo = at<double>(P, PL.off_rinfo) + 8;
  int J = 0;
  while (true) {
    bool more = J < PL.refine_max;
    if (more) {
      std::vector<Ctx *> steps = refine_steps(P);
      for (Ctx *cj : steps)
        if (cj->rank > 0 && (e = compute_rhat(cj))) return e;
      // sketch Y = R Omega and its Gram
      if ((e = launch_gauss_fill(PL.m, q, 0x5EEDull + (uint64_t)J, Om, NLD, st))) return e;
      HIPOK(hipMemset2DAsync(Yb, NLD * 8, 0, q * 8, PL.n, st));
      if ((e = apply_residual(P, steps, false, q, Om, Yb))) return e;
      if ((e = launch_tn(PL.n, q, q, Yb, false, NLD, Yb, NLD, sk, NLD, tn, PL.tn_cap, st)))
        return e;
      if ((e = launch_orth_small(q, sk, NLD, sT, NLD, info, dinfo, st))) return e;
      int k = 0;
      double tr = 0.0;
      HIPOK(hipMemcpyAsync(&k, info, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPOK(hipMemcpyAsync(&tr, dinfo, sizeof(double), hipMemcpyDeviceToHost, st));
      HIPOK(hipStreamSynchronize(st));
      const double est = std::sqrt(std::max(tr, 0.0) / q);
      more = k > 0 && est > 0.5 * tol * normR0;
      if (more) {
        // one power step, Y = R (R^T Y), sharpens the sketch toward R's dominant left subspace
        HIPOK(hipMemset2DAsync(Om, NLD * 8, 0, q * 8, PL.m, st));
        if ((e = apply_residual(P, steps, true, q, Yb, Om))) return e;
        HIPOK(hipMemset2DAsync(Yb, NLD * 8, 0, q * 8, PL.n, st));
        if ((e = apply_residual(P, steps, false, q, Om, Yb))) return e;
        if ((e = launch_tn(PL.n, q, q, Yb, false, NLD, Yb, NLD, sk, NLD, tn, PL.tn_cap, st)))
          return e;
        if ((e = launch_orth_small(q, sk, NLD, sT, NLD, info, dinfo, st))) return e;
        HIPOK(hipMemcpyAsync(&k, info, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPOK(hipStreamSynchronize(st));
        k = std::max(k, 1);  // a vanishing sketch leaves P_J = 0, which the QR below rejects
        ++J;
        // P_J = Y T (orthonormal), Q_J = R^T P_J
        double *PJ = pp_panel(P, J - 1), *QJ = qq_panel(P, J - 1);
        if ((e = launch_nn(PL.n, q, k, 1.0, Yb, false, NLD, sT, NLD, 0.0, PJ, NLD, st))) return e;
        HIPOK(hipMemset2DAsync(QJ, NLD * 8, 0, k * 8, PL.m, st));
        if ((e = apply_residual(P, steps, true, k, PJ, QJ))) return e;
        if ((e = launch_tn(PL.m, k, k, QJ, false, NLD, QJ, NLD, sk, NLD, tn, PL.tn_cap, st)))
          return e;
        if ((e = launch_orth_small(k, sk, NLD, sT + (size_t)16 * NLD, NLD, info + 1, dinfo + 1,
                                   st)))
          return e;
        double qn2 = 0.0;
        HIPOK(hipMemcpyAsync(&qn2, dinfo + 1, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPOK(hipStreamSynchronize(st));
        // correction equation A Y + Y B = P_J Q_J^T (Sylvester form also for Lyapunov problems)
        sylv_problem cp{PL.n, PL.m, k, P->A, PL.lyap ? P->AT : P->B, 0, PJ, NLD, QJ, NLD};
        cp.B.rows = PL.m;
        sylv_options co{};
        sylv_default_options(&co);
        co.method = method;
        co.max_iter = PL.refine_iter;
        co.check_every = P->check_every;
        co.closure_tol = P->closure_tol;
        co.precision = PL.fp32 ? SYLV_MIXED_FP32 : SYLV_FP64;
        void *kid = nullptr;
        char *kws = P->ws + PL.off_child + (size_t)(J - 1) * PL.child_bytes;
        e = ctx_create(&kid, &cp, &co, kws, PL.child_bytes, st, P);
        if (e == SYLV_ERR_RHS_RANK) {
          more = false;
        } else if (e) {
          return e;
        } else {
          Ctx *K = reinterpret_cast<Ctx *>(kid);
          const double qn = std::sqrt(std::max(qn2, 0.0));
          const double tolJ =
              std::min(0.5, std::max(tol, 0.3 * tol * normR0 / std::max(qn, 1e-300)));
          sylv_result rk{};
          e = (method == SYLV_METHOD_CG) ? sylv_factored_cg(K, tolJ, PL.refine_iter, &rk)
                                         : sylv_factored_bicgstab(K, tolJ, PL.refine_iter, &rk);
          if (e < 0) {
            sylv_destroy(K);
            return e;
          }
          total_iters += rk.iters;
          P->kids.push_back(K);
          P->kid_k.push_back(k);
          continue;
        }
      }
    }
    // the estimate is below tol / 2 (or no correction remains): FP64 true residual of the sum
    if ((e = stacked_residual(P, refine_steps(P), &absr, &rel))) return e;
    if (rel <= tol || J >= PL.refine_max || !more) break;
  }
  P->rel_true = rel;
  P->res_abs = absr;
  P->res_rel = rel;
  P->res_valid = 1;
  P->outer_steps = (int)P->kids.size();
  int status = rel <= tol ? SYLV_OK
                          : (first_status == SYLV_BREAKDOWN ? SYLV_BREAKDOWN : SYLV_NOT_CONVERGED);
  P->status = status;
  int64_t rank = P->rank;
  for (Ctx *k : P->kids) rank += k->rank;
  if (res) {
    *res = r0;
    res->status = status;
    res->iters = total_iters;
    res->rank_v = res->rank_w = rank;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    res->outer_steps = P->outer_steps;
    res->rel_res_true = rel;
  }
  return status;
}

}  // namespace

int create_context(void **out, const sylv_problem *pb, const sylv_options *op, void *workspace,
                   size_t ws_bytes, void *stream, bool overlap) {
  return ctx_create(out, pb, op, workspace, ws_bytes, stream, nullptr, overlap);
}

thread_local char g_last_error[512] = "";

void note_hip_error(hipError_t e, const char *what) {
  snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

void note_error(const char *msg) { snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }

extern "C" {

const char *sylv_last_error(void) { return g_last_error; }

void sylv_default_options(sylv_options *opt) {
  if (!opt) return;
  opt->method = SYLV_METHOD_BICGSTAB;
  opt->max_iter = 200;
  opt->check_every = 16;
  opt->record_history = 1;
  opt->closure_tol = 0.0;  // precision default
  opt->precision = SYLV_FP64;
  opt->refine_max = 0;
  opt->refine_max_iter = 100;
  opt->refine_rank = 8;
  opt->refine_inner_tol = 0.0;
  opt->streams = 0;
  opt->reorth = 0;
  opt->gram_precision = 0;
  opt->verify = 1;
}

size_t sylv_workspace_bytes(const sylv_problem *prob, const sylv_options *opt) {
  Layout L;
  if (make_layout(prob, opt, L)) return 0;
  return L.total;
}

const char *sylv_status_string(int status) {
  switch (status) {
    case SYLV_OK: return "converged";
    case SYLV_NOT_CONVERGED: return "not converged (max_iter reached)";
    case SYLV_BREAKDOWN: return "breakdown";
    case SYLV_ERR_INVALID: return "invalid argument";
    case SYLV_ERR_HIP: return "HIP runtime error";
    case SYLV_ERR_WORKSPACE: return "workspace too small or misaligned";
    case SYLV_ERR_RHS_RANK: return "right-hand-side factor is rank deficient";
    case SYLV_ERR_STATE: return "call out of order";
    default: return "unknown status";
  }
}

int sylv_create(void **out, const sylv_problem *pb, const sylv_options *op, void *workspace,
                size_t ws_bytes, void *stream) {
  return ctx_create(out, pb, op, workspace, ws_bytes, stream, nullptr);
}

void sylv_destroy(void *ctx) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return;
  for (Ctx *k : c->kids) sylv_destroy(k);
  if (c->h_ds) hipHostFree(c->h_ds);
  free_streams(c);
  delete c->prof;
  delete c;
}

int sylv_set_profiling(void *ctx, int on) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  if (on) {
    if (!c->prof) c->prof = new (std::nothrow) Prof();
    if (!c->prof) return SYLV_ERR_INVALID;
    c->prof->reset_stats();
  } else {
    delete c->prof;
    c->prof = nullptr;
  }
  c->sc.prof = c->prof;
  return 0;
}

int sylv_get_kernel_stats(void *ctx, sylv_kernel_stat *out, int cap, int *count) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c || !c->prof) return SYLV_ERR_STATE;
  if (count) *count = FAM_COUNT;
  for (int f = 0; f < FAM_COUNT && f < cap && out; ++f) {
    out[f].family = f;
    out[f].launches = c->prof->launches[f];
    out[f].ms = c->prof->ms[f];
    out[f].bytes = c->prof->bytes[f];
    out[f].flops = c->prof->flops[f];
  }
  return 0;
}

const char *sylv_kernel_family_name(int family) {
  static const char *names[FAM_COUNT] = {"spmm",     "gram",          "update",   "block_qr",
                                         "core_op",  "core_band",     "core_elem", "upd_gram",
                                         "res_gram", "res_gram_bf16", "res_pack", "res_defect"};
  return (family >= 0 && family < FAM_COUNT) ? names[family] : "unknown";
}

static int cg_body(void *ctx, double tol, int max_iter, sylv_result *res) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  if (c->L.refine_max > 0 && !c->in_refine)
    return refined_solve(c, SYLV_METHOD_CG, tol, max_iter, res);
  const Layout &L = c->L;
  const int s = (int)L.s;
  auto t0 = std::chrono::steady_clock::now();
  int e = begin_solve(c, tol, max_iter, SYLV_METHOD_CG);
  if (e) return e;
  const hipStream_t ks = c->kst, cs = c->st;
  // Lyapunov (G = H, C2 = C1): every core is symmetric (Section 4.3)
  const bool sym = L.lyap != 0;
  int steps = 0;  // Lanczos steps issued: blocks 0 .. steps exist
  if ((e = join(c, cs, ks))) return e;  // the Krylov stream sees the solve's set-up
  for (int k = 0; k < max_iter; ++k) {
    const int p = (k + 1) * s;
    set_iter(c, k);
    // (k+1)-th block Lanczos step on both sides (Alg. 4.1 steps 4-5), on the Krylov stream at
    // most one iteration ahead of the core recurrences (it waits for core iteration k - 2)
    if (ks != cs && k >= 2) HIPOK(hipStreamWaitEvent(ks, c->ev_c[(k - 2) % 3], 0));
    if ((e = launch_lanczos_pair(s, c->sv, L.lyap ? nullptr : &c->sw, k, L.ldc, c->closure_tol,
                                 c->sc, c->ds, ks)))
      return e;
    steps = k + 1;
    if (ks != cs) {
      HIPOK(hipEventRecord(c->ev_k[0], ks));
      HIPOK(hipStreamWaitEvent(cs, c->ev_k[0], 0));
    }
    // P_k = R_k + beta_{k-1} P_{k-1} (step 14 of the previous iteration; P_0 = R_0 with
    // beta = 0) into the other P buffer, with <P_k, Q_k> (steps 6-7); the Q buffer serves as
    // the second P buffer. Symmetric cores store the lower triangle only.
    const double q2 = (double)(p + s) * (p + s), half = sym ? 0.5 : 1.0;
    double *Pprev = (k & 1) ? c->Q : c->P, *Pk = (k & 1) ? c->P : c->Q;
    prof_begin(c->sc, c->st);
    if ((e = launch_cg_pq(s, p, sym, c->H, c->G, c->R, Pprev, Pk, L.ldc, c->scc, c->ds, c->st)))
      return e;
    prof_end(c->sc, FAM_CORE_BAND, half * 8.0 * 3.0 * p * p,
             half * 2.0 * 2.0 * 3.0 * s * q2, c->st);
    // alpha, X and R updates (steps 7-9), stopping test, rho and beta (steps 10-13)
    prof_begin(c->sc, c->st);
    if ((e = launch_cg_xr(s, p, sym, c->H, c->G, Pk, c->X, c->R, L.ldc, c->scc, c->ds, c->hist,
                          k, max_iter, c->st)))
      return e;
    prof_end(c->sc, FAM_CORE_ELEM, half * 8.0 * (3.0 * p * p + 2.0 * q2),
             half * (2.0 * 2.0 * 3.0 * s * q2 + 4.0 * q2), c->st);
    if (ks != cs) HIPOK(hipEventRecord(c->ev_c[k % 3], cs));
    if ((k + 1) % c->check_every == 0 && k + 1 < max_iter) {
      if ((e = read_state(c))) return e;
      if (c->h_ds->done) break;
    }
  }
  // basis columns of the newest blocks still held only in the ring
  if ((steps + 1) % LZ_RING != 0 &&
      (e = launch_lanczos_flush(s, c->sv, L.lyap ? nullptr : &c->sw, steps + 1, ks)))
    return e;
  if ((e = join(c, ks, cs))) return e;
  // the upper triangle of the symmetric solution core from its lower one
  if (sym && (e = launch_mirror(std::min<int64_t>(L.ldc, (int64_t)(max_iter + 1) * s), c->X,
                                L.ldc, c->st)))
    return e;
  if (hipStreamSynchronize(c->st) != hipSuccess) return SYLV_ERR_HIP;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return end_solve(c, max_iter, secs, res);
}

static int bicg_body(void *ctx, double tol, int max_iter, sylv_result *res) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  if (c->L.refine_max > 0 && !c->in_refine)
    return refined_solve(c, SYLV_METHOD_BICGSTAB, tol, max_iter, res);
  const Layout &L = c->L;
  const int s = (int)L.s;
  auto t0 = std::chrono::steady_clock::now();
  int e = begin_solve(c, tol, max_iter, SYLV_METHOD_BICGSTAB);
  if (e) return e;
  const hipStream_t ks = c->kst, cs = c->st;
  if ((e = join(c, cs, ks))) return e;  // the Krylov stream sees the solve's set-up
  int next_step = 0;                    // first Arnoldi step not yet enqueued
  const int *done = &c->ds->done;
  // algorithmic flops of eq. (3.11) with block Hessenberg H, G ((p+s) x p, J = p/s column
  // blocks, column block c holding c+2 row blocks): 2 nnz(H) p + 2 nnz(G) p
  auto coreop_flops = [s](double p) {
    const double J = p / s;
    return 4.0 * p * s * s * (J * (J + 1) / 2 + J);
  };
  auto coreop_bytes = [s](double p) {
    const double J = p / s;
    return 8.0 * (2.0 * s * s * (J * (J + 1) / 2 + J) + p * p + (p + s) * (p + s));
  };
  for (int k = 0; k < max_iter; ++k) {
    const int p = (2 * k + 1) * s;
    set_iter(c, k);
    const SideDesc *sw = L.lyap ? nullptr : &c->sw;
    // Block Arnoldi steps (Alg. 4.2 steps 5-6 and 10-11) on the Krylov stream, at most one
    // iteration ahead of the core recurrences (they wait for core iteration k - 2); the core
    // work waits for the step that completes the columns of H and G it reads: step j writes
    // column block j, or, with the lagged second pass, completes column block j - 1
    const int need1 = 2 * k + (c->lagged ? 1 : 0), need2 = need1 + 1;
    if (ks != cs && k >= 2) HIPOK(hipStreamWaitEvent(ks, c->ev_c[(k - 2) % 3], 0));
    for (; next_step <= need2; ++next_step) {
      if ((e = launch_arnoldi_pair(s, c->sv, sw, next_step, L.ldc, c->closure_tol, c->sc, c->ds,
                                   ks, c->lagged)))
        return e;
      if (ks != cs) HIPOK(hipEventRecord(c->ev_k[next_step % 4], ks));
    }
    if (ks != cs) HIPOK(hipStreamWaitEvent(cs, c->ev_k[need1 % 4], 0));
    // Q_k (step 7), alpha_k (step 8), S_k (step 9)
    prof_begin(c->sc, c->st);
    if ((e = launch_core_op(s, p, c->H, c->G, c->P, c->Q, L.ldc, done, c->st, c->cpart,
                            L.cpart_cap)))
      return e;
    prof_end(c->sc, FAM_CORE_OP, coreop_bytes(p), coreop_flops(p), c->st);
    const double q1 = (double)(p + s) * (p + s), q2 = (double)(p + 2 * s) * (p + 2 * s);
    prof_begin(c->sc, c->st);
    if ((e = launch_bicg_s(s, p, c->Q, c->R, c->S, c->Rt, L.ldc, c->ds, c->hist, k, max_iter,
                           c->st)))
      return e;
    prof_end(c->sc, FAM_CORE_ELEM, 8.0 * 3.0 * q1, 2.0 * q1, c->st);
    // the (2k+2)-th Arnoldi block (steps 10-11) is needed from here on
    if (ks != cs) HIPOK(hipStreamWaitEvent(cs, c->ev_k[need2 % 4], 0));
    // T_k (step 12), omega_k (step 13), rho_{k+1}, beta_k (steps 18-19)
    prof_begin(c->sc, c->st);
    if ((e = launch_core_op(s, p + s, c->H, c->G, c->S, c->T, L.ldc, done, c->st, c->cpart,
                            L.cpart_cap)))
      return e;
    prof_end(c->sc, FAM_CORE_OP, coreop_bytes(p + s), coreop_flops(p + s), c->st);
    prof_begin(c->sc, c->st);
    if ((e = launch_bicg_omega(s, p, c->T, c->S, L.ldc, c->scc, c->ds, c->st)))
      return e;
    prof_end(c->sc, FAM_CORE_ELEM, 8.0 * 2.0 * q2, 4.0 * q2, c->st);
    // X, R, P updates and the stopping test (steps 14-15, 20)
    prof_begin(c->sc, c->st);
    if ((e = launch_bicg_update(s, p, c->X, c->R, c->P, c->Q, c->S, c->T, c->Rt, L.ldc, c->scc,
                                c->ds, c->hist, k, max_iter, c->st)))
      return e;
    prof_end(c->sc, FAM_CORE_ELEM, 8.0 * 8.0 * q2, 12.0 * q2, c->st);
    if (ks != cs) HIPOK(hipEventRecord(c->ev_c[k % 3], cs));
    if ((k + 1) % c->check_every == 0 && k + 1 < max_iter) {
      if ((e = read_state(c))) return e;
      if (c->h_ds->done) break;
    }
  }
  if ((e = join(c, ks, cs))) return e;
  if (hipStreamSynchronize(c->st) != hipSuccess) return SYLV_ERR_HIP;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return end_solve(c, max_iter, secs, res);
}

// ---- solution compression: truncated SVD of the core (randomized range with one power step,
// one-sided Jacobi on the projected core, exact error of the truncated core) ----
static int compress_core(Ctx *c, double rel_tol, int64_t max_rank) {
  const Layout &L = c->L;
  const hipStream_t st = c->st;
  const int64_t r = c->rank, ldc = L.ldc, lm = L.lc;
  double *X = c->X, *T = c->Q;  // a free core buffer after the solve holds the rank-k core
  double *Om = at<double>(c, L.off_cOm), *Y = at<double>(c, L.off_cY), *Z = at<double>(c, L.off_cZ);
  double *Bm = at<double>(c, L.off_cB), *G = at<double>(c, L.off_cG), *U = at<double>(c, L.off_cU);
  double *Uk = at<double>(c, L.off_cUk), *Yk = at<double>(c, L.off_cYk);
  double *sig = at<double>(c, L.off_csig), *sigk = sig + lm, *pt = at<double>(c, L.off_cpt);
  int *idx = at<int>(c, L.off_cidx), *info = at<int>(c, L.off_cinfo);
  c->comp_k = 0;
  c->comp_err = 0.0;
  if (r == 0) return 0;
  double nx = 0.0;
  int e = diff_norm(r, r, X, ldc, nullptr, 0, pt, nullptr, &nx, st);
  if (e) return e;
  if (nx == 0.0) return 0;
  // rows of M (l x r) orthonormal: one-sided Jacobi, then normalized (rows of negligible norm
  // dropped: Y's rank is below l)
  std::vector<double> hs(lm);
  std::vector<double> f(lm);
  auto orth_rows = [&](double *M, int l) -> int {
    int ee;
    if ((ee = launch_jacobi_rows(l, r, M, ldc, G, lm, info, st))) return ee;
    if ((ee = launch_row_norms(l, r, M, ldc, sig, st))) return ee;
    HIPOK(hipMemcpyAsync(hs.data(), sig, sizeof(double) * l, hipMemcpyDeviceToHost, st));
    HIPOK(hipStreamSynchronize(st));
    const double mx = *std::max_element(hs.begin(), hs.begin() + l);
    for (int i = 0; i < l; ++i) f[i] = (hs[i] > 1e-14 * mx) ? 1.0 / hs[i] : 0.0;
    HIPOK(hipMemcpyAsync(sig, f.data(), sizeof(double) * l, hipMemcpyHostToDevice, st));
    return launch_scale_rows(l, r, M, ldc, sig, st);
  };
  int l = (int)std::min<int64_t>(r, std::min<int64_t>(lm, std::max<int64_t>(64, 2 * max_rank)));
  for (;;) {
    if ((e = launch_gauss_fill(r, l, 0xC0FFEEull + (uint64_t)l, Om, lm, st))) return e;
    // Y^T = Omega^T Xc^T (l x r), orthonormal rows; one power step Y^T = (Q^T Xc) Xc^T
    if ((e = launch_gemm(l, r, r, 1.0, Om, 1, lm, X, 1, ldc, 0.0, Y, ldc, st))) return e;
    if ((e = orth_rows(Y, l))) return e;
    // (each product is followed by an orthonormalization, so a direction keeps its singular
    // value relative to the largest once, not its square: small ones stay above rounding)
    if ((e = launch_gemm(l, r, r, 1.0, Y, ldc, 1, X, ldc, 1, 0.0, Z, ldc, st))) return e;
    if ((e = orth_rows(Z, l))) return e;
    if ((e = launch_gemm(l, r, r, 1.0, Z, ldc, 1, X, 1, ldc, 0.0, Y, ldc, st))) return e;
    if ((e = orth_rows(Y, l))) return e;
    // B = Q^T Xc (l x r); G B = D with orthogonal rows, sigma_i = ||D_i||
    if ((e = launch_gemm(l, r, r, 1.0, Y, ldc, 1, X, ldc, 1, 0.0, Bm, ldc, st))) return e;
    if ((e = launch_jacobi_rows(l, r, Bm, ldc, G, lm, info, st))) return e;
    if ((e = launch_row_norms(l, r, Bm, ldc, sig, st))) return e;
    HIPOK(hipMemcpyAsync(hs.data(), sig, sizeof(double) * l, hipMemcpyDeviceToHost, st));
    HIPOK(hipStreamSynchronize(st));
    std::vector<int> ord(l);
    for (int i = 0; i < l; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return hs[a] > hs[b]; });
    // smallest k whose singular-value tail meets the tolerance
    std::vector<double> tail(l + 1, 0.0);
    for (int i = l - 1; i >= 0; --i) tail[i] = tail[i + 1] + hs[ord[i]] * hs[ord[i]];
    int k = l;
    for (int i = 0; i <= l; ++i)
      if (std::sqrt(tail[i]) <= rel_tol * nx) {
        k = i;
        break;
      }
    if (max_rank >= 0) k = (int)std::min<int64_t>(k, max_rank);
    // U = Q G^T (r x l); U_k, Y_k and sigma_k in descending order
    if ((e = launch_gemm(r, l, l, 1.0, Y, 1, ldc, G, 1, lm, 0.0, U, lm, st))) return e;
    HIPOK(hipMemcpyAsync(idx, ord.data(), sizeof(int) * l, hipMemcpyHostToDevice, st));
    std::vector<double> hk(l);
    for (int i = 0; i < l; ++i) hk[i] = hs[ord[i]];
    HIPOK(hipMemcpyAsync(sigk, hk.data(), sizeof(double) * l, hipMemcpyHostToDevice, st));
    double err = 0.0;
    if (k > 0) {
      if ((e = launch_gather_cols(r, k, idx, U, lm, sig, Uk, lm, st))) return e;  // U_k sigma_k
      if ((e = launch_gather_rows_t(r, k, idx, Bm, ldc, sig, Yk, lm, st))) return e;
      if ((e = launch_gemm(r, r, k, 1.0, Uk, lm, 1, Yk, 1, lm, 0.0, T, ldc, st))) return e;
      if ((e = diff_norm(r, r, X, ldc, T, ldc, pt, &err, nullptr, st))) return e;
      if ((e = launch_gather_cols(r, k, idx, U, lm, nullptr, Uk, lm, st))) return e;  // U_k
    } else {
      err = nx;
    }
    c->comp_k = k;
    c->comp_err = err / nx;
    if (err <= rel_tol * nx * (1.0 + 1e-12) || l >= r || l >= lm || (max_rank >= 0 && k >= max_rank))
      return 0;
    l = (int)std::min<int64_t>({2 * (int64_t)l, r, lm});
  }
}

// ---- further factorized methods (CR on block Lanczos bases; CGS and GPBiCG on block Arnoldi
// bases), on the context's stream: each iteration issues the basis steps its core products
// need, then the core products (eq. (3.11)) and the elementwise core recurrences ----

// Arnoldi steps up to `need` (inclusive), one at a time.
static int arnoldi_upto(Ctx *c, int &next_step, int need) {
  const SideDesc *sw = c->L.lyap ? nullptr : &c->sw;
  for (; next_step <= need; ++next_step) {
    int e = launch_arnoldi_pair((int)c->L.s, c->sv, sw, next_step, c->L.ldc, c->closure_tol, c->sc,
                                c->ds, c->st, c->lagged);
    if (e) return e;
  }
  return 0;
}

static int poll_done(Ctx *c, int k, int max_iter, bool &stop) {
  stop = false;
  if ((k + 1) % c->check_every == 0 && k + 1 < max_iter) {
    int e = read_state(c);
    if (e) return e;
    stop = c->h_ds->done != 0;
  }
  return 0;
}

static int finish(Ctx *c, int max_iter, std::chrono::steady_clock::time_point t0,
                  sylv_result *res) {
  if (hipStreamSynchronize(c->st) != hipSuccess) return SYLV_ERR_HIP;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return end_solve(c, max_iter, secs, res);
}

// Factorized conjugate residual: S = F(R) by eq. (3.11) each iteration (block Lanczos step k+1
// first), Q = F(P) by recurrence; alpha = <R, S> / <Q, Q>, beta = <R+, S+> / <R, S>.
static int cr_body(void *ctx, double tol, int max_iter, sylv_result *res) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  const Layout &L = c->L;
  const int s = (int)L.s;
  auto t0 = std::chrono::steady_clock::now();
  int e = begin_solve(c, tol, max_iter, SYLV_METHOD_CR);
  if (e) return e;
  const hipStream_t st = c->st;
  const int *done = &c->ds->done;
  const SideDesc *sw = L.lyap ? nullptr : &c->sw;
  int steps = 0;
  auto step = [&](int j) {
    steps = j + 1;
    return launch_lanczos_pair(s, c->sv, sw, j, L.ldc, c->closure_tol, c->sc, c->ds, st);
  };
  // S_0 = F(R_0), Q_0 = S_0, rho_0 = <R_0, S_0>, <Q_0, Q_0>
  if ((e = step(0))) return e;
  if ((e = launch_core_op(s, s, c->H, c->G, c->R, c->S, L.ldc, done, st, c->cpart, L.cpart_cap)))
    return e;
  if ((e = launch_cr_init(2 * s, c->R, c->S, c->Q, L.ldc, c->scc, c->ds, st))) return e;
  for (int k = 0; k < max_iter; ++k) {
    const int q = (k + 2) * s;  // R_{k+1}, Q_k: q x q; S_{k+1}: (q + s) x (q + s)
    set_iter(c, k);
    if ((e = launch_cr_xr(q, c->X, c->R, c->P, c->Q, L.ldc, c->scc, c->ds, c->hist, k, max_iter,
                          st)))
      return e;
    if ((e = step(k + 1))) return e;
    if ((e = launch_core_op(s, q, c->H, c->G, c->R, c->S, L.ldc, done, st, c->cpart,
                            L.cpart_cap)))
      return e;
    if ((e = launch_cr_beta_pq(q + s, c->R, c->S, c->P, c->Q, L.ldc, c->scc, c->ds, c->hist, k,
                               max_iter, st)))
      return e;
    bool stop;
    if ((e = poll_done(c, k, max_iter, stop))) return e;
    if (stop) break;
  }
  if ((steps + 1) % LZ_RING != 0 && (e = launch_lanczos_flush(s, c->sv, sw, steps + 1, st)))
    return e;
  return finish(c, max_iter, t0, res);
}

// Factorized CGS: V = F(P), alpha = rho / <R~0, V(1:s,1:s)>, Q = U - alpha V, W = U + Q,
// X += alpha W, R -= alpha F(W), beta = rho+ / rho, U = R + beta Q, P = U + beta (Q + beta P).
static int cgs_body(void *ctx, double tol, int max_iter, sylv_result *res) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  const Layout &L = c->L;
  const int s = (int)L.s;
  auto t0 = std::chrono::steady_clock::now();
  int e = begin_solve(c, tol, max_iter, SYLV_METHOD_CGS);
  if (e) return e;
  const hipStream_t st = c->st;
  const int *done = &c->ds->done;
  double *U = c->Ex[0], *V = c->S, *Qb = c->Q, *Wk = c->T, *AW = c->Ex[1];
  if ((e = launch_copy_block(s, s, 1.0, c->R, L.ldc, false, U, L.ldc, st))) return e;  // U_0 = R_0
  int next_step = 0;
  for (int k = 0; k < max_iter; ++k) {
    const int p = (2 * k + 1) * s, q = p + s;
    const int need1 = 2 * k + (c->lagged ? 1 : 0);
    set_iter(c, k);
    if ((e = arnoldi_upto(c, next_step, need1))) return e;
    if ((e = launch_core_op(s, p, c->H, c->G, c->P, V, L.ldc, done, st, c->cpart, L.cpart_cap)))
      return e;
    if ((e = launch_alpha_corner(s, c->Rt, V, L.ldc, c->ds, c->hist, k, max_iter, st))) return e;
    if ((e = launch_cgs_qwx(q, U, V, Qb, Wk, c->X, L.ldc, c->ds, st))) return e;
    if ((e = arnoldi_upto(c, next_step, need1 + 1))) return e;
    if ((e = launch_core_op(s, q, c->H, c->G, Wk, AW, L.ldc, done, st, c->cpart, L.cpart_cap)))
      return e;
    if ((e = launch_axpy_rho_beta(s, q + s, AW, c->R, c->Rt, L.ldc, false, c->scc, c->ds, c->hist,
                                  k, max_iter, st)))
      return e;
    if ((e = launch_cgs_up(q + s, c->R, Qb, U, c->P, L.ldc, c->ds, st))) return e;
    bool stop;
    if ((e = poll_done(c, k, max_iter, stop))) return e;
    if (stop) break;
  }
  return finish(c, max_iter, t0, res);
}

// Factorized GPBiCG: p = r + beta (p - u), F(p), alpha, y and t, F(t), zeta and eta from the
// two-term minimization (eta = 0 on the first iteration), u, z, x and r updates, beta, w.
static int gpbicg_body(void *ctx, double tol, int max_iter, sylv_result *res) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  const Layout &L = c->L;
  const int s = (int)L.s;
  auto t0 = std::chrono::steady_clock::now();
  int e = begin_solve(c, tol, max_iter, SYLV_METHOD_GPBICG);
  if (e) return e;
  const hipStream_t st = c->st;
  const int *done = &c->ds->done;
  double *AP = c->Q, *T = c->S, *Tm = c->T, *AT = c->Ex[0], *Y = c->Ex[1], *U = c->Ex[2],
         *Z = c->Ex[3], *Wv = c->Ex[4];
  int next_step = 0;
  for (int k = 0; k < max_iter; ++k) {
    const int p = (2 * k + 1) * s, q = p + s;
    const int need1 = 2 * k + (c->lagged ? 1 : 0);
    set_iter(c, k);
    if ((e = launch_gp_p(p, c->R, U, c->P, L.ldc, c->ds, st))) return e;
    if ((e = arnoldi_upto(c, next_step, need1))) return e;
    if ((e = launch_core_op(s, p, c->H, c->G, c->P, AP, L.ldc, done, st, c->cpart, L.cpart_cap)))
      return e;
    if ((e = launch_alpha_corner(s, c->Rt, AP, L.ldc, c->ds, c->hist, k, max_iter, st))) return e;
    if ((e = launch_gp_yt(q, Tm, c->R, Wv, AP, Y, T, L.ldc, c->ds, st))) return e;
    if ((e = arnoldi_upto(c, next_step, need1 + 1))) return e;
    if ((e = launch_core_op(s, q, c->H, c->G, T, AT, L.ldc, done, st, c->cpart, L.cpart_cap)))
      return e;
    if ((e = launch_gp_zeta(q + s, AT, Y, T, L.ldc, k == 0, c->scc, c->ds, c->hist, k, max_iter,
                            st)))
      return e;
    if ((e = launch_gp_update(q + s, AP, Tm, c->P, T, Y, AT, c->R, U, Z, c->X, L.ldc, c->scc,
                              c->ds, st)))
      return e;
    if ((e = launch_axpy_rho_beta(s, q + s, nullptr, c->R, c->Rt, L.ldc, true, c->scc, c->ds,
                                  c->hist, k, max_iter, st)))
      return e;
    if ((e = launch_gp_w(q + s, AT, AP, Wv, L.ldc, c->ds, st))) return e;
    std::swap(T, Tm);  // t_k becomes t_{k-1} of the next iteration
    bool stop;
    if ((e = poll_done(c, k, max_iter, stop))) return e;
    if (stop) break;
  }
  return finish(c, max_iter, t0, res);
}

// A solve followed, when the context verifies, by the true residual of the converged iterate:
// if it misses tol (the recursive residual of the recurrence drifted from the true one), the
// solve runs again with the recursive target lowered in proportion, at most twice.
static int solve_verified(void *ctx, int method, double tol, int max_iter, sylv_result *res) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  auto run = [&](double t) {
    switch (method) {
      case SYLV_METHOD_CG: return cg_body(ctx, t, max_iter, res);
      case SYLV_METHOD_BICGSTAB: return bicg_body(ctx, t, max_iter, res);
      case SYLV_METHOD_CR: return cr_body(ctx, t, max_iter, res);
      case SYLV_METHOD_CGS: return cgs_body(ctx, t, max_iter, res);
      default: return gpbicg_body(ctx, t, max_iter, res);
    }
  };
  auto t0 = std::chrono::steady_clock::now();
  int st = run(tol);
  const bool verify = c->verify && !c->parent && !c->in_refine && c->L.refine_max == 0;
  if (st != SYLV_OK || !verify) return st;
  double target = tol;
  for (int round = 0;; ++round) {
    double a = 0.0, r = 0.0;
    int e = true_residual(c, &a, &r);
    if (e) return e;
    if (r <= tol || round == 2) {
      if (r > tol) c->status = SYLV_NOT_CONVERGED;
      if (res) {
        res->status = c->status;
        res->rel_res_true = r;
        res->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      }
      return c->status;
    }
    target *= std::min(0.5, 0.5 * tol / r);
    st = run(target);
    if (st != SYLV_OK) return st;
  }
}

}  // extern "C"

// ---- batch groups ----

static void group_sides(Ctx *const *cs, int n, std::vector<GroupSide> &out) {
  out.clear();
  for (int i = 0; i < n; ++i) {
    Ctx *c = cs[i];
    const Layout &L = c->L;
    const int64_t pair = L.n + (L.lyap ? 0 : L.m);
    out.push_back(GroupSide{c->sv, c->sc, 0, pair, L.ldc, &c->ds->done});
    if (!L.lyap) out.push_back(GroupSide{c->sw, c->sc, 1, pair, L.ldc, &c->ds->done});
  }
}

static bool group_compatible(Ctx *const *cs, int n) {
  if (n < 1) return false;
  for (int i = 0; i < n; ++i) {
    if (!group_eligible(cs[i])) return false;
    const Layout &a = cs[0]->L, &b = cs[i]->L;
    if (b.method != a.method || b.s != a.s || b.lyap != a.lyap ||
        cs[i]->closure_tol != cs[0]->closure_tol || cs[i]->st != cs[0]->st)
      return false;
  }
  return true;
}

bool group_eligible(void *ctx) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c || c->parent || c->L.fp32 || c->L.refine_max > 0 || c->kst != c->st) return false;
  if (c->L.method == SYLV_METHOD_CG) return true;
  return c->L.method == SYLV_METHOD_BICGSTAB && c->lagged;
}

static size_t group_split(Ctx *const *cs, int n, size_t &kbytes) {
  std::vector<GroupSide> sides;
  group_sides(cs, n, sides);
  kbytes = krylov_group_bytes((int)cs[0]->L.s, cs[0]->L.method == SYLV_METHOD_CG, sides.data(),
                              (int)sides.size());
  if (kbytes == 0) return 0;
  return kbytes + (sizeof(CoreInst) * n + 255) / 256 * 256 + 256 + (sizeof(int) * n + 255) / 256 * 256;
}

size_t group_bytes(void *const *ctxs, int n) {
  Ctx *const *cs = reinterpret_cast<Ctx *const *>(ctxs);
  if (!ctxs || !group_compatible(cs, n)) return 0;
  size_t kb = 0;
  return group_split(cs, n, kb);
}

void group_release(GroupRun &g) {
  for (hipGraphExec_t e : g.exec)
    if (e) (void)hipGraphExecDestroy(e);
  g.exec.clear();
  if (g.vst) (void)hipStreamDestroy(g.vst);
  g.vst = nullptr;
  if (g.h_poll) (void)hipHostFree(g.h_poll);
  g.h_poll = nullptr;
}

static int group_capture(GroupRun &g, int seg, int k0, int k1);

int group_prepare(GroupRun &g, void *const *ctxs, int n, void *dev, size_t bytes, bool graphs,
                  int max_iter) {
  Ctx *const *cs = reinterpret_cast<Ctx *const *>(ctxs);
  if (!ctxs || !group_compatible(cs, n)) return SYLV_ERR_INVALID;
  size_t kb = 0;
  const size_t need = group_split(cs, n, kb);
  if (need == 0) return SYLV_ERR_WORKSPACE;
  if (!dev || bytes < need || (reinterpret_cast<uintptr_t>(dev) & 255)) return SYLV_ERR_WORKSPACE;
  const Layout &L0 = cs[0]->L;
  g.ctx.assign(ctxs, ctxs + n);
  g.method = L0.method;
  g.s = (int)L0.s;
  g.sym = L0.lyap;
  g.st = cs[0]->st;
  g.closure_tol = cs[0]->closure_tol;
  g.graphs = graphs;
  g.graph_max_iter = -1;
  std::vector<GroupSide> sides;
  group_sides(cs, n, sides);
  char *p = static_cast<char *>(dev);
  if (int e = krylov_group_create(&g.kg, &g.ka, g.s, g.method == SYLV_METHOD_CG, sides.data(),
                                  (int)sides.size(), p, kb, g.st))
    return e;
  std::vector<CoreInst> tab(n);
  g.min_ldc = INT64_MAX;
  for (int i = 0; i < n; ++i) {
    Ctx *c = cs[i];
    tab[i] = CoreInst{c->H, c->G, c->X, c->R, c->P, c->Q, c->S, c->T, c->Rt, c->scc.partials,
                      c->ds, c->hist, c->L.ldc, 0, 0};
    g.min_ldc = std::min<int64_t>(g.min_ldc, c->L.ldc);
  }
  g.tab = reinterpret_cast<CoreInst *>(p + kb);
  g.poll = reinterpret_cast<int *>(p + kb + (sizeof(CoreInst) * n + 255) / 256 * 256);
  g.list = g.poll + 64;
  HIPOK(hipMemcpyAsync(g.tab, tab.data(), sizeof(CoreInst) * n, hipMemcpyHostToDevice, g.st));
  HIPOK(hipStreamSynchronize(g.st));
  if (!g.h_poll &&
      hipHostMalloc(reinterpret_cast<void **>(&g.h_poll), sizeof(int) * 8) != hipSuccess)
    return SYLV_ERR_HIP;
  if (!graphs && !g.vst && hipStreamCreateWithFlags(&g.vst, hipStreamNonBlocking) != hipSuccess)
    return SYLV_ERR_HIP;
  if (graphs) {
    // every segment up to max_iter is captured now, while no other work of the library runs:
    // a capture in progress is invalidated by synchronous calls elsewhere in the process
    g.graph_max_iter = max_iter;
    for (int seg = 0; seg * GROUP_SEG < max_iter; ++seg)
      if (int e = group_capture(g, seg, seg * GROUP_SEG, std::min(max_iter, (seg + 1) * GROUP_SEG)))
        return e;
  }
  return 0;
}

// The launches of iteration k of every problem of the group (no host synchronization, so they
// can be captured in a graph).
static int group_iteration(GroupRun &g, int k) {
  const int s = g.s;
  const hipStream_t st = g.st;
  // graphs run over every problem; otherwise the launches cover the problems still running
  const KGroup &kv = g.graphs ? g.kg : g.ka;
  const int *list = g.graphs ? nullptr : g.list;
  const int n = g.graphs ? (int)g.ctx.size() : g.na;
  int e;
  if (g.method == SYLV_METHOD_CG) {
    if ((e = launch_krylov_group(kv, k, g.closure_tol, st))) return e;
    return launch_cg_group(s, g.sym != 0, (k + 1) * s, k, g.tab, list, n, st);
  }
  // lagged block Arnoldi: the core work of iteration k needs steps up to 2k + 2
  for (int j = (k == 0 ? 0 : 2 * k + 1); j <= 2 * k + 2; ++j)
    if ((e = launch_krylov_group(kv, j, g.closure_tol, st))) return e;
  const int p = (2 * k + 1) * s;
  const int64_t T = (p + 2 * s + 63) / 64 * 64;
  if (T > g.min_ldc) return SYLV_ERR_WORKSPACE;
  if ((e = launch_core_op_group(s, p, 0, g.tab, list, n, st))) return e;
  if ((e = launch_bicg_group_s(s, p, k, g.tab, list, n, st))) return e;
  if ((e = launch_core_op_group(s, p + s, 1, g.tab, list, n, st))) return e;
  if ((e = launch_bicg_group_omega(s, p, g.tab, list, n, st))) return e;
  return launch_bicg_group_update(s, p, k, g.tab, list, n, st);
}

// The poll after `steps` iterations: the problems still running (and, for the compacted
// launches, the tables restricted to them), read back by the host. Block Lanczos first moves
// the ring's partial group of blocks to the bases of the problems still in the launches, so
// that a problem leaving them has all its basis columns in place.
static int group_poll(GroupRun &g, int steps) {
  const int n = (int)g.ctx.size();
  int nread = 1;
  if (!g.graphs) {
    if (g.method == SYLV_METHOD_CG && steps > 0 && (steps + 1) % LZ_RING != 0)
      if (int e = launch_krylov_group_flush(g.ka, steps + 1, g.st)) return e;
    if (int e = launch_krylov_group_compact(g.kg, g.ka, g.poll + 1, g.st)) return e;
    nread = 2 + GK_COUNT;
  }
  if (int e = launch_group_active(g.tab, n, g.poll, g.list, g.st)) return e;
  HIPOK(hipMemcpyAsync(g.h_poll, g.poll, sizeof(int) * nread, hipMemcpyDeviceToHost, g.st));
  HIPOK(hipStreamSynchronize(g.st));
  g.na = g.h_poll[0];
  if (!g.graphs) {
    g.ka.nsides = g.h_poll[1];
    for (int k = 0; k < GK_COUNT; ++k) g.ka.nblk[k] = g.h_poll[2 + k];
  }
  return 0;
}

// Iterations [k0, k1) of segment seg as one graph (captured, not run).
static int group_capture(GroupRun &g, int seg, int k0, int k1) {
  if ((int)g.exec.size() <= seg) g.exec.resize(seg + 1, nullptr);
  if (g.exec[seg]) return 0;
  HIPOK(hipStreamBeginCapture(g.st, hipStreamCaptureModeThreadLocal));
  int e = 0;
  for (int k = k0; k < k1 && !e; ++k) e = group_iteration(g, k);
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(g.st, &graph);
  if (e) {
    if (graph) (void)hipGraphDestroy(graph);
    return e;
  }
  HIPOK(ce);
  const hipError_t ie = hipGraphInstantiate(&g.exec[seg], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPOK(ie);
  return 0;
}

// Iterations [k0, k1): the segment's graph when it was captured for this max_iter, else the
// launches themselves.
static int group_segment(GroupRun &g, int seg, int k0, int k1, bool replay) {
  if (replay && seg < (int)g.exec.size() && g.exec[seg]) {
    HIPOK(hipGraphLaunch(g.exec[seg], g.st));
    return 0;
  }
  for (int k = k0; k < k1; ++k)
    if (int e = group_iteration(g, k)) return e;
  return 0;
}

// The end of one problem's solve: the symmetric core completed (Lyapunov CG), the state and
// history read back, and, for a converged problem that verifies, its FP64 true residual. A true
// residual that misses tol is left for a solve of its own (*again), which must not run while
// the group still launches (the problem's stop flag would be cleared).
static int group_finish(GroupRun &g, Ctx *c, double tol, int max_iter, double secs,
                        sylv_result *r, bool *again) {
  *again = false;
  if (g.method == SYLV_METHOD_CG && g.sym) {
    const Layout &L = c->L;
    if (int e = launch_mirror(std::min<int64_t>(L.ldc, (int64_t)(max_iter + 1) * L.s), c->X,
                              L.ldc, c->st))
      return e;
  }
  const int st = end_solve(c, max_iter, secs, r);
  if (st < 0) return st;
  if (st == SYLV_OK && c->verify) {
    double a = 0.0, rel = 0.0;
    if (int e = true_residual(c, &a, &rel)) return e;
    r->rel_res_true = rel;
    *again = rel > tol;
  }
  return 0;
}

int group_solve(GroupRun &g, double tol, int max_iter, sylv_result *res) {
  const int n = (int)g.ctx.size();
  if (n < 1 || !res) return SYLV_ERR_INVALID;
  auto t0 = std::chrono::steady_clock::now();
  auto secs = [&] {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  Ctx *const *cs = reinterpret_cast<Ctx *const *>(g.ctx.data());
  for (int i = 0; i < n; ++i)
    if (int e = begin_solve(cs[i], tol, max_iter, g.method)) return e;
  const bool replay = g.graphs && g.graph_max_iter == max_iter;
  // compacted launches: a problem that has left the launches is finished (state, history, true
  // residual) by a second host thread on the side stream while this one keeps launching
  std::vector<char> queued(n, 0), again(n, 0), running(n, 1);
  std::vector<int> list(n);
  std::mutex mu;
  std::condition_variable cv;
  std::deque<int> todo;
  bool closed = false;
  int ferr = 0;
  std::string fmsg;
  int dev = 0;
  HIPOK(hipGetDevice(&dev));
  const bool side = !g.graphs && g.vst;
  std::thread finisher;
  if (side)
    finisher = std::thread([&] {
      if (hipSetDevice(dev) != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        ferr = SYLV_ERR_HIP;
      }
      for (;;) {
        int i;
        {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&] { return closed || !todo.empty(); });
          if (todo.empty()) return;
          i = todo.front();
          todo.pop_front();
          if (ferr) continue;
        }
        Ctx *c = cs[i];
        c->st = c->kst = g.vst;
        bool ag = false;
        const int e = group_finish(g, c, tol, max_iter, secs(), &res[i], &ag);
        c->st = c->kst = g.st;
        again[i] = ag;
        if (e) {
          std::lock_guard<std::mutex> lk(mu);
          ferr = e;
          fmsg = sylv_last_error();
        }
      }
    });
  auto stop_finisher = [&] {
    if (!side) return 0;
    {
      std::lock_guard<std::mutex> lk(mu);
      closed = true;
    }
    cv.notify_all();
    finisher.join();
    if (ferr) note_error(fmsg.c_str());
    return ferr;
  };
  auto run = [&]() -> int {
    if (!g.graphs)
      if (int e = group_poll(g, 0)) return e;  // every problem starts in the launches
    int steps = 0;  // iterations enqueued
    if (int e = group_segment(g, 0, 0, std::min(max_iter, GROUP_SEG), replay)) return e;
    for (int seg = 0;; ++seg) {
      steps = std::min(max_iter, (seg + 1) * GROUP_SEG);
      if (steps >= max_iter) break;
      if (int e = group_poll(g, steps)) return e;
      if (g.na == 0) break;
      if (side) {
        HIPOK(hipMemcpyAsync(list.data(), g.list, sizeof(int) * g.na, hipMemcpyDeviceToHost,
                             g.st));
        HIPOK(hipStreamSynchronize(g.st));
        std::fill(running.begin(), running.end(), 0);
        for (int j = 0; j < g.na; ++j) running[list[j]] = 1;
        {
          std::lock_guard<std::mutex> lk(mu);
          for (int i = 0; i < n; ++i)
            if (!running[i] && !queued[i]) {
              queued[i] = 1;
              todo.push_back(i);
            }
        }
        cv.notify_one();
      }
      if (int e = group_segment(g, seg + 1, steps, std::min(max_iter, steps + GROUP_SEG), replay))
        return e;
    }
    // basis columns of the newest blocks still held only in the ring (the problems that were in
    // the last launches; the others were written at the poll that removed them)
    const KGroup &last = g.graphs ? g.kg : g.ka;
    if (g.method == SYLV_METHOD_CG && (steps + 1) % LZ_RING != 0 && last.nsides > 0)
      if (int e = launch_krylov_group_flush(last, steps + 1, g.st)) return e;
    HIPOK(hipStreamSynchronize(g.st));
    return 0;
  };
  const int e1 = run();
  const int e2 = stop_finisher();
  if (e1) return e1;
  if (e2) return e2;
  for (int i = 0; i < n; ++i) {
    if (queued[i]) continue;
    bool ag = false;
    if (int e = group_finish(g, cs[i], tol, max_iter, secs(), &res[i], &ag)) return e;
    again[i] = ag;
  }
  // verification as for a single solve: a converged iterate whose true residual misses tol is
  // solved again alone with a lower recursive target
  int worst = 0;
  for (int i = 0; i < n; ++i) {
    Ctx *c = cs[i];
    int st = res[i].status;
    if (again[i]) {
      double target = tol, r = res[i].rel_res_true;
      for (int round = 1;; ++round) {
        target *= std::min(0.5, 0.5 * tol / r);
        st = g.method == SYLV_METHOD_CG ? cg_body(c, target, max_iter, &res[i])
                                        : bicg_body(c, target, max_iter, &res[i]);
        if (st != SYLV_OK) break;
        double a = 0.0;
        if (int e = true_residual(c, &a, &r)) return e;
        res[i].rel_res_true = r;
        if (r <= tol || round == 2) {
          if (r > tol) c->status = SYLV_NOT_CONVERGED;
          st = c->status;
          break;
        }
      }
    }
    res[i].status = st;
    worst = std::max(worst, st);
  }
  return worst;
}

extern "C" {

int sylv_factored_cg(void *ctx, double tol, int max_iter, sylv_result *res) {
  return solve_verified(ctx, SYLV_METHOD_CG, tol, max_iter, res);
}

int sylv_factored_bicgstab(void *ctx, double tol, int max_iter, sylv_result *res) {
  return solve_verified(ctx, SYLV_METHOD_BICGSTAB, tol, max_iter, res);
}

int sylv_compress(void *ctx, double rel_tol, int64_t max_rank, int64_t *rank, double *rel_err) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c || !(rel_tol >= 0.0)) return SYLV_ERR_INVALID;
  if (!c->solved || c->parent || !c->kids.empty()) return SYLV_ERR_STATE;
  if (c->L.fp32) return SYLV_ERR_INVALID;
  int e = compress_core(c, rel_tol, max_rank);
  if (e) {
    c->comp_k = -1;
    return e;
  }
  if (rank) *rank = c->comp_k;
  if (rel_err) *rel_err = c->comp_err;
  return c->comp_err <= rel_tol * (1.0 + 1e-12) ? 0 : SYLV_NOT_CONVERGED;
}

int sylv_get_compressed(void *ctx, double *Z1, int64_t ldz1, double *sigma, double *Z2,
                        int64_t ldz2, int64_t *rank) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  if (c->comp_k < 0) return SYLV_ERR_STATE;
  const Layout &L = c->L;
  const int64_t k = c->comp_k, r = c->rank, lm = L.lc;
  if (rank) *rank = k;
  if (k == 0) return 0;
  if ((Z1 && ldz1 < k) || (Z2 && ldz2 < k)) return SYLV_ERR_INVALID;
  hipStream_t st = c->st;
  int e;
  const double *V = static_cast<const double *>(c->sv.basis);
  const double *W = static_cast<const double *>(c->sw.basis);
  if (Z1 && (e = launch_gemm(L.n, k, r, 1.0, V, L.ldb, 1, at<double>(c, L.off_cUk), lm, 1, 0.0, Z1,
                             ldz1, st)))
    return e;
  if (Z2 && (e = launch_gemm(L.m, k, r, 1.0, W, L.ldb, 1, at<double>(c, L.off_cYk), lm, 1, 0.0, Z2,
                             ldz2, st)))
    return e;
  if (sigma)
    HIPOK(hipMemcpyAsync(sigma, at<double>(c, L.off_csig) + lm, sizeof(double) * k,
                         hipMemcpyDeviceToDevice, st));
  HIPOK(hipStreamSynchronize(st));
  return 0;
}

int sylv_factored_cr(void *ctx, double tol, int max_iter, sylv_result *res) {
  return solve_verified(ctx, SYLV_METHOD_CR, tol, max_iter, res);
}

int sylv_factored_cgs(void *ctx, double tol, int max_iter, sylv_result *res) {
  return solve_verified(ctx, SYLV_METHOD_CGS, tol, max_iter, res);
}

int sylv_factored_gpbicg(void *ctx, double tol, int max_iter, sylv_result *res) {
  return solve_verified(ctx, SYLV_METHOD_GPBICG, tol, max_iter, res);
}

int sylv_get_factors(void *ctx, double *V, int64_t ldv, double *Xc, int64_t ldx, double *W,
                     int64_t ldw, int64_t *rank_v, int64_t *rank_w) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  if (!c->solved) return SYLV_ERR_STATE;
  // the summed iterate of a refined solve: V = [V_0 V_1 ...], Xc = diag(X_0, X_1, ...)
  std::vector<Ctx *> steps = refine_steps(c);
  int64_t r = 0;
  for (Ctx *cj : steps) r += cj->rank;
  if (rank_v) *rank_v = r;
  if (rank_w) *rank_w = r;
  if (r == 0) return 0;
  if ((V && ldv < r) || (Xc && ldx < r) || (W && ldw < r)) return SYLV_ERR_INVALID;
  if (Xc && steps.size() > 1) HIPOK(hipMemset2DAsync(Xc, ldx * 8, 0, r * 8, r, c->st));
  int64_t off = 0;
  for (Ctx *cj : steps) {
    const Layout &L = cj->L;
    const int64_t rj = cj->rank;
    if (rj == 0) continue;
    auto copy_basis = [&](double *dst, int64_t ldd, const SideDesc &sd) -> int {
      if (L.fp32)
        return launch_widen(sd.rows, rj, static_cast<const float *>(sd.basis), L.ldb, dst, ldd,
                            c->st);
      return launch_copy_rows(sd.rows, rj, static_cast<const double *>(sd.basis), L.ldb, dst,
                              ldd, c->st);
    };
    int e;
    if (V && (e = copy_basis(V + off, ldv, cj->sv))) return e;
    if (Xc)
      HIPOK(hipMemcpy2DAsync(Xc + off * ldx + off, ldx * 8, cj->X, L.ldc * 8, rj * 8, rj,
                             hipMemcpyDeviceToDevice, c->st));
    if (W && (e = copy_basis(W + off, ldw, cj->sw))) return e;
    off += rj;
  }
  HIPOK(hipStreamSynchronize(c->st));
  return 0;
}

int sylv_get_history(void *ctx, double *relres, double *alpha, double *beta, double *omega, int cap,
                     int *count) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  if (!c->solved) return SYLV_ERR_STATE;
  const int mi = c->max_iter_run;
  const int n = std::min(c->iters, cap);
  if (count) *count = c->iters;
  for (int k = 0; k < n; ++k) {
    if (relres) relres[k] = c->h_hist[k];
    if (alpha) alpha[k] = c->h_hist[mi + k];
    if (beta) beta[k] = c->h_hist[2 * mi + k];
    if (omega) omega[k] = c->h_hist[3 * mi + k];
  }
  return 0;
}

// ||A X + X B - C1 C2^T||_F of the current iterate (the summed iterate after a refined solve),
// from the Gram traces of the stacked tall factors of its defect form.
int sylv_residual_norm(void *ctx, double *abs_res, double *rel_res) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  if (!c->solved) return SYLV_ERR_STATE;
  if (c->parent) return SYLV_ERR_STATE;
  return true_residual(c, abs_res, rel_res);
}

int sylv_spmm(const sylv_csr *A, int64_t s, const double *X, int64_t ldx, double *Y, int64_t ldy,
              void *stream) {
  if (!A || s < 1 || s > SYLV_MAX_S || ldx < s || ldy < s || !X || !Y) return SYLV_ERR_INVALID;
  if (check_csr_header(*A, A->rows)) return SYLV_ERR_INVALID;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  return launch_spmm((int)s, A->rows, A->row_ptr, A->col_idx, A->values, X, ldx, Y, ldy, st);
}

size_t sylv_gram_work_bytes(int64_t M, int64_t N, int64_t K) {
  if (M < 1 || N < 1 || K < 1 || M > INT32_MAX || N > INT32_MAX || K > INT32_MAX) return 0;
  return gram_part_doubles(std::max(M, N), K) * 8;
}

int sylv_gram(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda, const double *B,
              int64_t ldb, int symmetric, int accumulate, double *C, int64_t ldc, void *work,
              size_t work_bytes, void *stream) {
  if (M < 0 || N < 0 || K < 1 || M > INT32_MAX || N > INT32_MAX || K > INT32_MAX)
    return SYLV_ERR_INVALID;
  if (M == 0 || N == 0) return 0;
  if (!A || !B || !C || ldc < N || (symmetric && M != N)) return SYLV_ERR_INVALID;
  if (lda < round_up(M, 64) || ldb < round_up(N, 64) || lda % 8 || ldb % 8)
    return SYLV_ERR_INVALID;
  if (work && reinterpret_cast<uintptr_t>(work) % 8) return SYLV_ERR_INVALID;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int e = launch_gram(M, N, K, A, false, lda, B, false, ldb, accumulate ? 1.0 : 0.0, C, ldc,
                      symmetric != 0, st, static_cast<double *>(work), work ? work_bytes / 8 : 0);
  if (e) return e;
  if (symmetric && (e = launch_mirror(M, C, ldc, st))) return e;
  HIPOK(hipStreamSynchronize(st));
  return 0;
}

int sylv_dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t a_rs,
               int64_t a_cs, const double *B, int64_t b_rs, int64_t b_cs, double beta, double *C,
               int64_t ldc, void *stream) {
  if (M < 0 || N < 0 || K < 0 || ldc < N || (M > 0 && N > 0 && (!C || (K > 0 && (!A || !B)))))
    return SYLV_ERR_INVALID;
  if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX) return SYLV_ERR_INVALID;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int e = launch_gemm(M, N, K, alpha, A, a_rs, a_cs, B, b_rs, b_cs, beta, C, ldc, st);
  if (e) return e;
  HIPOK(hipStreamSynchronize(st));
  return 0;
}

size_t sylv_sell_bytes(const sylv_csr *A) {
  if (!A || A->rows <= 0 || check_csr_header(*A, A->rows)) return 0;
  return sell_bytes(A->rows, A->nnz);
}

int sylv_sell_build(const sylv_csr *A, void *sell, size_t bytes, void *stream) {
  if (!A || !sell || A->rows <= 0 || check_csr_header(*A, A->rows)) return SYLV_ERR_INVALID;
  if (bytes < sell_bytes(A->rows, A->nnz)) return SYLV_ERR_WORKSPACE;
  return build_sell(A->rows, A->nnz, A->row_ptr, A->col_idx, A->values, sell,
                    reinterpret_cast<hipStream_t>(stream));
}

int sylv_sell_spmm(const sylv_csr *A, const void *sell, int64_t s, const double *X, int64_t ldx,
                   double *Y, int64_t ldy, void *stream) {
  if (!A || !sell || s < 1 || s > SYLV_MAX_S || ldx < s || ldy < s || !X || !Y)
    return SYLV_ERR_INVALID;
  if (A->rows <= 0 || check_csr_header(*A, A->rows)) return SYLV_ERR_INVALID;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const SellMat M = sell_view(A->rows, A->nnz, const_cast<void *>(sell));
  return launch_sell_spmm((int)s, M, X, ldx, Y, ldy, st);
}

size_t sylv_csr_transpose_scratch_bytes(int64_t rows) { return csr_transpose_scratch(rows); }

int sylv_csr_transpose(const sylv_csr *A, int32_t *out_row_ptr, int32_t *out_col_idx,
                       double *out_values, void *scratch, void *stream) {
  if (!A || !out_row_ptr || !scratch) return SYLV_ERR_INVALID;
  if (check_csr_header(*A, A->rows) || A->rows <= 0) return SYLV_ERR_INVALID;
  if (A->nnz > 0 && (!out_col_idx || !out_values)) return SYLV_ERR_INVALID;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int e = launch_csr_transpose(A->rows, A->nnz, A->row_ptr, A->col_idx, A->values, out_row_ptr,
                               out_col_idx, out_values, scratch, st);
  if (e) return e;
  HIPOK(hipStreamSynchronize(st));
  return 0;
}

}  // extern "C"
