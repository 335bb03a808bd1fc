// C ABI of libsylv: context creation, the factorized CG / BiCGSTAB iteration drivers
// (Algorithms 4.1 and 4.2), the FP64 true residual and factor export.
//
// The host only sequences kernels: every scalar of the recurrences stays on the device, and
// the host polls the device's stop flag every `check_every` iterations (iterations enqueued
// after the stop return at kernel entry).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"

namespace {

constexpr size_t ALIGN = 256;

struct Layout {
  // sizes
  int64_t n = 0, m = 0, s = 0, Jmax = 0, rmax = 0, ldb = 0, ldc = 0, rc_rows = 0;
  int lyap = 0, method = 0, max_iter = 0, fp32 = 0;
  int64_t esz = 8;  // bytes per basis element
  size_t partial_cap = 0;
  // byte offsets into the workspace
  size_t off_V, off_W, off_H, off_G, off_X, off_R, off_P, off_Q, off_S, off_T;
  size_t off_U, off_Uw, off_coefV, off_coefW, off_btrp, off_btci, off_btval, off_tscr;
  size_t off_partials, off_counters, off_ds, off_ssv, off_ssw, off_rt, off_rl, off_rr, off_hist;
  size_t off_E, off_GVV, off_GWW, off_GVE, off_GWE, off_GEEa, off_GEEb, off_Lx, off_M1, off_M2;
  size_t off_dots, off_flag, off_panV, off_panW, off_sellA, off_sellB;
  size_t total = 0;
};

size_t bump(size_t &cur, size_t bytes) {
  const size_t o = (cur + ALIGN - 1) / ALIGN * ALIGN;
  cur = o + bytes;
  return o;
}

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int check_csr_header(const sylv_csr &M, int64_t rows) {
  if (M.rows != rows || M.nnz < 0 || M.nnz >= ((int64_t)1 << 31)) return SYLV_ERR_INVALID;
  if (!M.row_ptr || (M.nnz > 0 && (!M.col_idx || !M.values))) return SYLV_ERR_INVALID;
  return 0;
}

int make_layout(const sylv_problem *pb, const sylv_options *op, Layout &L) {
  if (!pb || !op) return SYLV_ERR_INVALID;
  if (pb->n <= 0 || pb->m <= 0 || pb->s < 1 || pb->s > SYLV_MAX_S) return SYLV_ERR_INVALID;
  if (pb->s > std::min(pb->n, pb->m)) return SYLV_ERR_INVALID;
  if (pb->lyapunov && pb->n != pb->m) return SYLV_ERR_INVALID;
  if (op->max_iter < 1 || (op->method != SYLV_METHOD_CG && op->method != SYLV_METHOD_BICGSTAB))
    return SYLV_ERR_INVALID;
  if (op->precision != SYLV_FP64 && op->precision != SYLV_MIXED_FP32) return SYLV_ERR_INVALID;
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
  // blocks generated: CG k+2 after k+1 iterations; BiCGSTAB 2k+3
  L.Jmax = (op->method == SYLV_METHOD_CG) ? (int64_t)op->max_iter + 2 : 2 * (int64_t)op->max_iter + 2;
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
  if (L.method == SYLV_METHOD_BICGSTAB) {
    L.off_S = bump(cur, c2);
    L.off_T = bump(cur, c2);
  } else {
    L.off_S = L.off_T = 0;
  }
  L.off_U = bump(cur, (size_t)L.n * L.s * 8);
  L.off_Uw = bump(cur, (size_t)L.m * L.s * 8);
  L.off_coefV = bump(cur, (size_t)L.ldb * L.s * 8);
  L.off_coefW = bump(cur, (size_t)L.ldb * L.s * 8);
  const int64_t bnnz = L.lyap ? 0 : pb->B.nnz;
  L.off_btrp = bump(cur, (size_t)(L.m + 1) * 4);
  L.off_btci = bump(cur, (size_t)std::max<int64_t>(bnnz, 1) * 4);
  L.off_btval = bump(cur, (size_t)std::max<int64_t>(bnnz, 1) * 8);
  L.off_tscr = bump(cur, csr_transpose_scratch(L.m));
  L.off_partials = bump(cur, L.partial_cap * 8);
  L.off_counters = bump(cur, CNT_MAX * sizeof(int));
  L.off_ds = bump(cur, sizeof(DevState));
  L.off_ssv = bump(cur, sizeof(SideState));
  L.off_ssw = bump(cur, sizeof(SideState));
  L.off_rt = bump(cur, SYLV_MAX_S * SYLV_MAX_S * 8);
  L.off_rl = bump(cur, SYLV_MAX_S * SYLV_MAX_S * 8);
  L.off_rr = bump(cur, SYLV_MAX_S * SYLV_MAX_S * 8);
  L.off_hist = bump(cur, (size_t)4 * L.Jmax * 8);
  // true-residual buffers
  L.off_E = bump(cur, (size_t)L.rc_rows * L.ldb * 8);
  L.off_GVV = bump(cur, c2);
  L.off_GWW = bump(cur, c2);
  L.off_GVE = bump(cur, c2);
  L.off_GWE = bump(cur, c2);
  L.off_GEEa = bump(cur, c2);
  L.off_GEEb = bump(cur, c2);
  L.off_Lx = bump(cur, c2);
  L.off_M1 = bump(cur, c2);
  L.off_M2 = bump(cur, c2);
  L.off_panV = bump(cur, (size_t)2 * L.n * L.s * L.esz);
  L.off_panW = L.lyap ? L.off_panV : bump(cur, (size_t)2 * L.m * L.s * L.esz);
  L.off_sellA = bump(cur, sell_bytes(L.n, pb->A.nnz));
  L.off_sellB = L.lyap ? L.off_sellA : bump(cur, sell_bytes(L.m, pb->B.nnz));
  L.off_dots = bump(cur, 16 * 8);
  L.off_flag = bump(cur, 16 * sizeof(int));
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
    for (hipEvent_t e : pool) hipEventDestroy(e);
  }
};

struct Ctx {
  Layout L;
  Prof *prof = nullptr;
  hipStream_t st = nullptr;
  sylv_csr A{}, B{};
  double closure_tol = 1e-12;
  int check_every = 8;
  int record_history = 1;
  char *ws = nullptr;
  SideDesc sv{}, sw{};
  double *H, *G, *X, *R, *P, *Q, *S, *T, *Rt, *RL, *RR, *hist;
  DevState *ds;
  SideState *ssv, *ssw;
  Scratch sc{};
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
  if (p->start) hipEventRecord(p->start, st);
}

void prof_end(const Scratch &sc, int fam, double bytes, double flops, hipStream_t st) {
  Prof *p = reinterpret_cast<Prof *>(sc.prof);
  if (!p || !p->start) return;
  hipEvent_t e = p->get();
  if (!e) return;
  hipEventRecord(e, st);
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
  const int64_t need_blocks = (method == SYLV_METHOD_CG) ? (int64_t)max_iter + 2 : 2 * (int64_t)max_iter + 2;
  if (max_iter < 1 || need_blocks > L.Jmax || !(tol >= 0.0)) return SYLV_ERR_INVALID;
  if (method == SYLV_METHOD_BICGSTAB && L.method != SYLV_METHOD_BICGSTAB) return SYLV_ERR_WORKSPACE;
  const size_t c2 = (size_t)L.ldc * L.ldc * 8;
  double *zero[] = {c->H, c->G, c->X, c->R, c->P, c->Q, c->S, c->T};
  for (double *z : zero)
    if (z) HIPOK(hipMemsetAsync(z, 0, c2, c->st));
  // the compact copy of block 1 (V_1, W_1) is the first SpMM input; earlier solves reused it
  const size_t e = (size_t)L.esz;
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
  c->rank = (c->method == SYLV_METHOD_CG) ? (int64_t)c->iters * c->L.s
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
  }
  return c->status;
}

}  // namespace

thread_local char g_last_error[512] = "";

void note_hip_error(hipError_t e, const char *what) {
  snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

extern "C" {

const char *sylv_last_error(void) { return g_last_error; }

void sylv_default_options(sylv_options *opt) {
  if (!opt) return;
  opt->method = SYLV_METHOD_BICGSTAB;
  opt->max_iter = 200;
  opt->check_every = 8;
  opt->record_history = 1;
  opt->closure_tol = 0.0;  // precision default
  opt->precision = SYLV_FP64;
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
  if (!out) return SYLV_ERR_INVALID;
  *out = nullptr;
  Layout L;
  int e = make_layout(pb, op, L);
  if (e) return e;
  if (!workspace || ws_bytes < L.total) return SYLV_ERR_WORKSPACE;
  Ctx *c = new (std::nothrow) Ctx();
  if (!c) return SYLV_ERR_INVALID;
  c->L = L;
  c->st = reinterpret_cast<hipStream_t>(stream);
  c->A = pb->A;
  c->B = pb->B;
  c->closure_tol = op->closure_tol > 0 ? op->closure_tol : (L.fp32 ? 1e-6 : 1e-12);
  c->check_every = op->check_every > 0 ? op->check_every : 8;
  c->record_history = op->record_history;
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
  c->Rt = at<double>(c, L.off_rt);
  c->RL = at<double>(c, L.off_rl);
  c->RR = at<double>(c, L.off_rr);
  c->hist = at<double>(c, L.off_hist);
  c->ds = at<DevState>(c, L.off_ds);
  c->ssv = at<SideState>(c, L.off_ssv);
  c->ssw = L.lyap ? c->ssv : at<SideState>(c, L.off_ssw);
  c->sc.partials = at<double>(c, L.off_partials);
  c->sc.partial_cap = L.partial_cap;
  c->sc.counters = at<int>(c, L.off_counters);
  c->btrp = at<int32_t>(c, L.off_btrp);
  c->btci = at<int32_t>(c, L.off_btci);
  c->btval = at<double>(c, L.off_btval);
  c->flag = at<int>(c, L.off_flag);
  c->dots = at<double>(c, L.off_dots);

  auto fail = [&](int code) {
    hipHostFree(c->h_ds);
    delete c;
    return code;
  };
  hipStream_t st = c->st;
  if (hipMemsetAsync(c->sc.counters, 0, CNT_MAX * sizeof(int), st) != hipSuccess ||
      hipMemsetAsync(c->ds, 0, sizeof(DevState), st) != hipSuccess ||
      hipMemsetAsync(c->flag, 0, 16 * sizeof(int), st) != hipSuccess)
    return fail(SYLV_ERR_HIP);
  // validate CSR structure on the device
  if ((e = launch_csr_validate(L.n, pb->A.nnz, pb->A.row_ptr, pb->A.col_idx, c->flag, st)))
    return fail(e);
  if (!L.lyap && (e = launch_csr_validate(L.m, pb->B.nnz, pb->B.row_ptr, pb->B.col_idx,
                                          c->flag + 1, st)))
    return fail(e);
  int hflag[2] = {0, 0};
  if (hipMemcpyAsync(hflag, c->flag, sizeof(hflag), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(SYLV_ERR_HIP);
  if (hflag[0] || hflag[1]) return fail(SYLV_ERR_INVALID);
  // W side operator: B^T
  if (!L.lyap) {
    if ((e = launch_csr_transpose(L.m, pb->B.nnz, pb->B.row_ptr, pb->B.col_idx, pb->B.values,
                                  c->btrp, c->btci, c->btval, at<void>(c, L.off_tscr), st)))
      return fail(e);
  }
  char *panv = at<char>(c, L.off_panV), *panw = at<char>(c, L.off_panW);
  c->sv = SideDesc{L.n, pb->A.nnz, pb->A.row_ptr, pb->A.col_idx, pb->A.values,
                   at<void>(c, L.off_V), L.ldb, c->H, at<double>(c, L.off_U),
                   at<double>(c, L.off_coefV), c->ssv,
                   {panv, panv + L.n * L.s * L.esz}, L.fp32, SellMat{}};
  if (L.lyap) {
    c->sw = c->sv;
  } else {
    c->sw = SideDesc{L.m, pb->B.nnz, c->btrp, c->btci, c->btval, at<void>(c, L.off_W), L.ldb,
                     c->G, at<double>(c, L.off_Uw), at<double>(c, L.off_coefW), c->ssw,
                     {panw, panw + L.m * L.s * L.esz}, L.fp32, SellMat{}};
  }
  // SELL copies of A and B^T for the Krylov SpMM (CSR stays in use if the padding is large)
  c->sv.sell = SellMat{};
  e = build_sell(L.n, pb->A.nnz, pb->A.row_ptr, pb->A.col_idx, pb->A.values,
                 at<void>(c, L.off_sellA), st);
  if (e == 0) c->sv.sell = sell_view(L.n, pb->A.nnz, at<void>(c, L.off_sellA));
  else if (e != SYLV_ERR_WORKSPACE) return fail(e);
  if (L.lyap) {
    c->sw.sell = c->sv.sell;
  } else {
    c->sw.sell = SellMat{};
    e = build_sell(L.m, pb->B.nnz, c->btrp, c->btci, c->btval, at<void>(c, L.off_sellB), st);
    if (e == 0) c->sw.sell = sell_view(L.m, pb->B.nnz, at<void>(c, L.off_sellB));
    else if (e != SYLV_ERR_WORKSPACE) return fail(e);
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
  if (hipStreamSynchronize(st) != hipSuccess) return fail(SYLV_ERR_HIP);
  for (int i = 0; i < 2; ++i) {
    if (!std::isfinite(hs[i].ref2)) return fail(SYLV_ERR_INVALID);
    if (hs[i].mode != 0) return fail(SYLV_ERR_RHS_RANK);
  }
  *out = c;
  return 0;
}

void sylv_destroy(void *ctx) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return;
  if (c->h_ds) hipHostFree(c->h_ds);
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
  static const char *names[FAM_COUNT] = {"spmm",    "gram",      "update",   "block_qr",
                                         "core_op", "core_band", "core_elem"};
  return (family >= 0 && family < FAM_COUNT) ? names[family] : "unknown";
}

int sylv_factored_cg(void *ctx, double tol, int max_iter, sylv_result *res) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  const Layout &L = c->L;
  const int s = (int)L.s;
  auto t0 = std::chrono::steady_clock::now();
  int e = begin_solve(c, tol, max_iter, SYLV_METHOD_CG);
  if (e) return e;
  for (int k = 0; k < max_iter; ++k) {
    const int p = (k + 1) * s;
    set_iter(c, k);
    // (k+1)-th block Lanczos step on both sides (Alg. 4.1 steps 4-5)
    if ((e = launch_lanczos_pair(s, c->sv, L.lyap ? nullptr : &c->sw, k, L.ldc, c->closure_tol,
                                 c->sc, c->ds, c->st)))
      return e;
    // Q_k (step 6) and alpha_k (step 7)
    const double q2 = (double)(p + s) * (p + s);
    prof_begin(c->sc, c->st);
    if ((e = launch_cg_core(s, p, c->H, c->G, c->P, c->Q, L.ldc, c->sc, c->ds, c->st)))
      return e;
    prof_end(c->sc, FAM_CORE_BAND, 8.0 * ((double)p * p + q2) + 2 * 8.0 * 3 * s * (p + s),
             2.0 * 2.0 * 3.0 * s * (double)p * (p + s), c->st);
    // X, R updates, stopping test, rho, beta, P update (steps 8-14)
    prof_begin(c->sc, c->st);
    if ((e = launch_cg_update(s, p, c->X, c->R, c->P, c->Q, L.ldc, c->sc, c->ds, c->hist, k,
                              max_iter, c->st)))
      return e;
    prof_end(c->sc, FAM_CORE_ELEM, 8.0 * 9.0 * q2, 8.0 * q2, c->st);
    if ((k + 1) % c->check_every == 0 && k + 1 < max_iter) {
      if ((e = read_state(c))) return e;
      if (c->h_ds->done) break;
    }
  }
  if (hipStreamSynchronize(c->st) != hipSuccess) return SYLV_ERR_HIP;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return end_solve(c, max_iter, secs, res);
}

int sylv_factored_bicgstab(void *ctx, double tol, int max_iter, sylv_result *res) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  const Layout &L = c->L;
  const int s = (int)L.s;
  auto t0 = std::chrono::steady_clock::now();
  int e = begin_solve(c, tol, max_iter, SYLV_METHOD_BICGSTAB);
  if (e) return e;
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
    // (2k+1)-th block Arnoldi step on both sides (Alg. 4.2 steps 5-6)
    if ((e = launch_arnoldi_pair(s, c->sv, sw, 2 * k, L.ldc, c->closure_tol, c->sc, c->ds, c->st)))
      return e;
    // Q_k (step 7), alpha_k (step 8), S_k (step 9)
    prof_begin(c->sc, c->st);
    if ((e = launch_core_op(s, p, c->H, c->G, c->P, c->Q, L.ldc, done, c->st))) return e;
    prof_end(c->sc, FAM_CORE_OP, coreop_bytes(p), coreop_flops(p), c->st);
    const double q1 = (double)(p + s) * (p + s), q2 = (double)(p + 2 * s) * (p + 2 * s);
    prof_begin(c->sc, c->st);
    if ((e = launch_bicg_s(s, p, c->Q, c->R, c->S, c->Rt, L.ldc, c->ds, c->hist, k, max_iter,
                           c->st)))
      return e;
    prof_end(c->sc, FAM_CORE_ELEM, 8.0 * 3.0 * q1, 2.0 * q1, c->st);
    // (2k+2)-th Arnoldi step (steps 10-11)
    if ((e = launch_arnoldi_pair(s, c->sv, sw, 2 * k + 1, L.ldc, c->closure_tol, c->sc, c->ds,
                                 c->st)))
      return e;
    // T_k (step 12), omega_k (step 13), rho_{k+1}, beta_k (steps 18-19)
    prof_begin(c->sc, c->st);
    if ((e = launch_core_op(s, p + s, c->H, c->G, c->S, c->T, L.ldc, done, c->st))) return e;
    prof_end(c->sc, FAM_CORE_OP, coreop_bytes(p + s), coreop_flops(p + s), c->st);
    prof_begin(c->sc, c->st);
    if ((e = launch_bicg_omega(s, p, c->T, c->S, L.ldc, c->sc, c->ds, c->st)))
      return e;
    prof_end(c->sc, FAM_CORE_ELEM, 8.0 * 2.0 * q2, 4.0 * q2, c->st);
    // X, R, P updates and the stopping test (steps 14-15, 20)
    prof_begin(c->sc, c->st);
    if ((e = launch_bicg_update(s, p, c->X, c->R, c->P, c->Q, c->S, c->T, c->Rt, L.ldc, c->sc,
                                c->ds, c->hist, k, max_iter, c->st)))
      return e;
    prof_end(c->sc, FAM_CORE_ELEM, 8.0 * 8.0 * q2, 12.0 * q2, c->st);
    if ((k + 1) % c->check_every == 0 && k + 1 < max_iter) {
      if ((e = read_state(c))) return e;
      if (c->h_ds->done) break;
    }
  }
  if (hipStreamSynchronize(c->st) != hipSuccess) return SYLV_ERR_HIP;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return end_solve(c, max_iter, secs, res);
}

int sylv_get_factors(void *ctx, double *V, int64_t ldv, double *Xc, int64_t ldx, double *W,
                     int64_t ldw, int64_t *rank_v, int64_t *rank_w) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  if (!c->solved) return SYLV_ERR_STATE;
  const Layout &L = c->L;
  const int64_t r = c->rank;
  if (rank_v) *rank_v = r;
  if (rank_w) *rank_w = r;
  if (r == 0) return 0;
  if ((V && ldv < r) || (Xc && ldx < r) || (W && ldw < r)) return SYLV_ERR_INVALID;
  auto copy_basis = [&](double *dst, int64_t ldd, const SideDesc &sd) -> int {
    if (L.fp32)
      return launch_widen(sd.rows, r, static_cast<const float *>(sd.basis), L.ldb, dst, ldd, c->st);
    HIPOK(hipMemcpy2DAsync(dst, ldd * 8, sd.basis, L.ldb * 8, r * 8, sd.rows,
                           hipMemcpyDeviceToDevice, c->st));
    return 0;
  };
  int e;
  if (V && (e = copy_basis(V, ldv, c->sv))) return e;
  if (Xc)
    HIPOK(hipMemcpy2DAsync(Xc, ldx * 8, c->X, L.ldc * 8, r * 8, r, hipMemcpyDeviceToDevice, c->st));
  if (W && (e = copy_basis(W, ldw, c->sw))) return e;
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

// ||A X + X B - C1 C2^T||_F for X = V_p Xc W_p^T, p = rank, from Gram traces:
//   A X + X B = V_{p+s} L(Xc) W_{p+s}^T + E_A Xc W_p^T + V_p Xc E_B^T with the basis defects
//   E_A = A V_p - V_{p+s} H, E_B = B^T W_p - W_{p+s} G (eq. (3.8) holds up to them), so with
//   R^ = [R0 0; 0 0] - L(Xc) the residual is T1 - T2 - T3, T1 = V R^ W^T, T2 = E_A Xc W_p^T,
//   T3 = V_p Xc E_B^T, and every term of ||T1 - T2 - T3||^2 is a trace of small products
//   of the Grams V^T V, W^T W, V^T E_A, W^T E_B, E_A^T E_A, E_B^T E_B.
int sylv_residual_norm(void *ctx, double *abs_res, double *rel_res) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return SYLV_ERR_INVALID;
  if (!c->solved) return SYLV_ERR_STATE;
  const Layout &L = c->L;
  hipStream_t st = c->st;
  const int s = (int)L.s;
  const int64_t p = c->rank, q = p + s, ldc = L.ldc, ldb = L.ldb;
  double h_ds_norm;
  int e = read_state(c);
  if (e) return e;
  h_ds_norm = c->h_ds->normR0;
  if (p == 0) {
    if (abs_res) *abs_res = h_ds_norm;
    if (rel_res) *rel_res = 1.0;
    return 0;
  }
  double *E = at<double>(c, L.off_E);
  double *GVV = at<double>(c, L.off_GVV), *GWW = at<double>(c, L.off_GWW);
  double *GVE = at<double>(c, L.off_GVE), *GWE = at<double>(c, L.off_GWE);
  double *GEEa = at<double>(c, L.off_GEEa), *GEEb = at<double>(c, L.off_GEEb);
  double *Lx = at<double>(c, L.off_Lx), *M1 = at<double>(c, L.off_M1), *M2 = at<double>(c, L.off_M2);
  // Gram accumulation over row chunks of one side: E = M V_p - V_q H (banded for block
  // Lanczos, a Hessenberg GEMM for block Arnoldi), then V^T V and E^T E (lower tiles, mirrored
  // at the end) and V^T E.
  const bool band = (L.method == SYLV_METHOD_CG);
  auto side_grams = [&](const SideDesc &sd, const double *Hm, double *Gbb, double *Gbe,
                        double *Gee) -> int {
    char *Vb = static_cast<char *>(sd.basis);
    const bool f32 = L.fp32;
    int ee;
    if (!band) {
      const int qk = (int)std::min<int64_t>(round_up(q, 32), ldb);
      if ((ee = launch_zero_cols(sd.rows, Vb, f32, ldb, (int)q, qk, st))) return ee;
    }
    for (int64_t r0 = 0; r0 < sd.rows; r0 += L.rc_rows) {
      const int64_t r1 = std::min(sd.rows, r0 + L.rc_rows), nr = r1 - r0;
      const double beta = (r0 == 0) ? 0.0 : 1.0;
      if (band) {
        if ((ee = launch_defect_band(r0, r1, sd.rp, sd.ci, sd.val, Vb, f32, ldb, (int)p, (int)q, s,
                                     Hm, ldc, M2, ldc, r0 == 0, E, ldb, st)))
          return ee;
      } else {
        // E = M V_p (rows r0..r1), then E -= V_q(rows) H(0:q, 0:p)
        if ((ee = launch_spmm_rows(s, r0, r1, sd.rp, sd.ci, sd.val, Vb, f32, ldb, (int)p, E, ldb,
                                   st)))
          return ee;
        if ((ee = launch_defect_gemm(nr, (int)p, (int)q, s, Vb + r0 * ldb * L.esz, f32, ldb, Hm,
                                     ldc, E, ldb, st)))
          return ee;
      }
      const char *Vr = Vb + r0 * ldb * L.esz;
      if ((ee = launch_gram(q, q, nr, Vr, f32, ldb, Vr, f32, ldb, beta, Gbb, ldc, true, st)))
        return ee;
      if ((ee = launch_gram(q, p, nr, Vr, f32, ldb, E, false, ldb, beta, Gbe, ldc, false, st)))
        return ee;
      if ((ee = launch_gram(p, p, nr, E, false, ldb, E, false, ldb, beta, Gee, ldc, true, st)))
        return ee;
    }
    if ((ee = launch_mirror(q, Gbb, ldc, st))) return ee;
    return launch_mirror(p, Gee, ldc, st);
  };
  if ((e = side_grams(c->sv, c->H, GVV, GVE, GEEa))) return e;
  const double *GWWp = GVV, *GWEp = GVE, *GEEbp = GEEa;
  if (!L.lyap) {
    if ((e = side_grams(c->sw, c->G, GWW, GWE, GEEb))) return e;
    GWWp = GWW;
    GWEp = GWE;
    GEEbp = GEEb;
  }
  // R^ = [R0 0; 0 0] - L(Xc); reuse Lx as R^
  if ((e = launch_core_op(s, (int)p, c->H, c->G, c->X, Lx, ldc, nullptr, st))) return e;
  // R0 = R_L R_R^T is the saved Rt core
  if ((e = launch_rhat(s, (int)q, Lx, c->Rt, Lx, ldc, st))) return e;
  const double *Rh = Lx;
  double *dots = c->dots;
  // t1 = <GVV R^, R^ GWW>
  if ((e = launch_gemm(q, q, q, 1.0, GVV, ldc, 1, Rh, ldc, 1, 0.0, M1, ldc, st))) return e;
  if ((e = launch_gemm(q, q, q, 1.0, Rh, ldc, 1, GWWp, ldc, 1, 0.0, M2, ldc, st))) return e;
  if ((e = launch_dot(q, q, M1, ldc, M2, ldc, dots + 0, c->sc, st))) return e;
  // t12 = <R^, GVE X GWW(0:p, 0:q)>
  if ((e = launch_gemm(q, p, p, 1.0, GVE, ldc, 1, c->X, ldc, 1, 0.0, M1, ldc, st))) return e;
  if ((e = launch_gemm(q, q, p, 1.0, M1, ldc, 1, GWWp, ldc, 1, 0.0, M2, ldc, st))) return e;
  if ((e = launch_dot(q, q, Rh, ldc, M2, ldc, dots + 1, c->sc, st))) return e;
  // t13 = <R^, GVV(0:q, 0:p) X GWE^T>
  if ((e = launch_gemm(q, p, p, 1.0, GVV, ldc, 1, c->X, ldc, 1, 0.0, M1, ldc, st))) return e;
  if ((e = launch_gemm(q, q, p, 1.0, M1, ldc, 1, GWEp, 1, ldc, 0.0, M2, ldc, st))) return e;
  if ((e = launch_dot(q, q, Rh, ldc, M2, ldc, dots + 2, c->sc, st))) return e;
  // t22 = <GEE_A X, X GWW(0:p, 0:p)>
  if ((e = launch_gemm(p, p, p, 1.0, GEEa, ldc, 1, c->X, ldc, 1, 0.0, M1, ldc, st))) return e;
  if ((e = launch_gemm(p, p, p, 1.0, c->X, ldc, 1, GWWp, ldc, 1, 0.0, M2, ldc, st))) return e;
  if ((e = launch_dot(p, p, M1, ldc, M2, ldc, dots + 3, c->sc, st))) return e;
  // t33 = <GVV(0:p, 0:p) X, X GEE_B>
  if ((e = launch_gemm(p, p, p, 1.0, GVV, ldc, 1, c->X, ldc, 1, 0.0, M1, ldc, st))) return e;
  if ((e = launch_gemm(p, p, p, 1.0, c->X, ldc, 1, GEEbp, ldc, 1, 0.0, M2, ldc, st))) return e;
  if ((e = launch_dot(p, p, M1, ldc, M2, ldc, dots + 4, c->sc, st))) return e;
  // t23 = <GVE(0:p, :) X, X GWE(0:p, :)^T>
  if ((e = launch_gemm(p, p, p, 1.0, GVE, ldc, 1, c->X, ldc, 1, 0.0, M1, ldc, st))) return e;
  if ((e = launch_gemm(p, p, p, 1.0, c->X, ldc, 1, GWEp, 1, ldc, 0.0, M2, ldc, st))) return e;
  if ((e = launch_dot(p, p, M1, ldc, M2, ldc, dots + 5, c->sc, st))) return e;
  double t[6];
  HIPOK(hipMemcpyAsync(t, dots, sizeof(t), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  double r2 = t[0] - 2.0 * t[1] - 2.0 * t[2] + t[3] + t[4] + 2.0 * t[5];
  if (r2 < 0.0) r2 = 0.0;
  const double a = std::sqrt(r2);
  if (abs_res) *abs_res = a;
  if (rel_res) *rel_res = a / h_ds_norm;
  return 0;
}

int sylv_spmm(const sylv_csr *A, int64_t s, const double *X, int64_t ldx, double *Y, int64_t ldy,
              void *stream) {
  if (!A || s < 1 || s > SYLV_MAX_S || ldx < s || ldy < s || !X || !Y) return SYLV_ERR_INVALID;
  if (check_csr_header(*A, A->rows)) return SYLV_ERR_INVALID;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int e = launch_spmm((int)s, A->rows, A->row_ptr, A->col_idx, A->values, X, ldx, Y, ldy, st);
  if (e) return e;
  HIPOK(hipStreamSynchronize(st));
  return 0;
}

int sylv_dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t a_rs,
               int64_t a_cs, const double *B, int64_t b_rs, int64_t b_cs, double beta, double *C,
               int64_t ldc, void *stream) {
  if (M < 0 || N < 0 || K < 0 || ldc < N || (M > 0 && N > 0 && (!C || (K > 0 && (!A || !B)))))
    return SYLV_ERR_INVALID;
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
  int e = launch_sell_spmm((int)s, M, X, ldx, Y, ldy, st);
  if (e) return e;
  HIPOK(hipStreamSynchronize(st));
  return 0;
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
