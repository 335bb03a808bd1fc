/*
 * Host-side argument handling of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Built by the package's build script against hostsan/libsylv_hostsan.so (the library with its
 * host code instrumented) and run by tests/test_abi_hostsan.py.
 *
 * Mode "args" (no GPU needed): every entry point is called with missing pointers, sizes out of
 * range, malformed CSR headers, unknown options and sizes near the int64 limit, and must return
 * the documented error code (or 0 for the sizing calls) without touching device memory; the
 * sizing calls are swept over many valid problems so that every branch of the workspace layout
 * runs under the sanitizers. The device pointers handed in point at one-element host arrays:
 * the host code must never dereference them, and a read past them would be reported.
 *
 * Mode "solve" (needs a GPU): small factored CG, BiCGSTAB, CR, CGS and GPBiCG solves, FP32
 * bases with outer refinement, a Lyapunov solve, the residual, factors, compression, history
 * and kernel-statistics calls, batches in every form and the building-block calls, through the
 * C ABI, so that the host logic of real solves (context set-up, the stream and event
 * bookkeeping, the batch's worker and finisher threads) runs under the sanitizers too.
 *
 * Exit status: number of failed checks (0 = all passed); a sanitizer report aborts the run.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <hip/hip_runtime_api.h>

#include "sylv.h"

static int fails = 0, checks = 0;

#define CHECK(cond, ...)                  \
  do {                                    \
    ++checks;                             \
    if (!(cond)) {                        \
      ++fails;                            \
      printf("FAIL line %d: ", __LINE__); \
      printf(__VA_ARGS__);                \
      printf("\n");                       \
    }                                     \
  } while (0)

/* stand-ins for device arrays: never dereferenced by the host code */
static int32_t fake_i32[1];
static double fake_f64[1];

static sylv_csr fake_csr(int64_t rows, int64_t nnz) {
  sylv_csr a;
  a.rows = rows;
  a.nnz = nnz;
  a.row_ptr = fake_i32;
  a.col_idx = fake_i32;
  a.values = fake_f64;
  return a;
}

static sylv_problem fake_problem(int64_t n, int64_t m, int64_t s, int lyap) {
  sylv_problem p;
  memset(&p, 0, sizeof p);
  p.n = n;
  p.m = m;
  p.s = s;
  p.A = fake_csr(n, n > 0 ? 13 : 0);
  p.B = fake_csr(m, m > 0 ? 11 : 0);
  p.lyapunov = lyap;
  p.C1 = fake_f64;
  p.ldc1 = s;
  p.C2 = lyap ? NULL : fake_f64;
  p.ldc2 = s;
  return p;
}

static sylv_options opts(int method, int max_iter) {
  sylv_options o;
  sylv_default_options(&o);
  o.method = method;
  o.max_iter = max_iter;
  return o;
}

static void check_strings(void) {
  const int codes[] = {SYLV_OK, SYLV_NOT_CONVERGED, SYLV_BREAKDOWN, SYLV_ERR_INVALID, SYLV_ERR_HIP,
                       SYLV_ERR_WORKSPACE, SYLV_ERR_RHS_RANK, SYLV_ERR_STATE, 3, -6, 1 << 30,
                       -(1 << 30), INT32_MAX, INT32_MIN};
  for (size_t i = 0; i < sizeof codes / sizeof codes[0]; ++i) {
    const char *t = sylv_status_string(codes[i]);
    CHECK(t && strlen(t) > 0, "status string of %d", codes[i]);
  }
  for (int f = -3; f < 40; ++f) {
    const char *t = sylv_kernel_family_name(f);
    CHECK(t && strlen(t) > 0, "family name %d", f);
  }
  CHECK(strcmp(sylv_kernel_family_name(INT32_MIN), "unknown") == 0, "family INT32_MIN");
  CHECK(strcmp(sylv_kernel_family_name(INT32_MAX), "unknown") == 0, "family INT32_MAX");
  const char *e = sylv_last_error();
  CHECK(e != NULL, "last error text");
  sylv_default_options(NULL);
}

static void check_workspace_sizing(void) {
  const int64_t big = (int64_t)1 << 40;
  sylv_options o = opts(SYLV_METHOD_CG, 50);
  sylv_problem p = fake_problem(300, 200, 2, 0);
  CHECK(sylv_workspace_bytes(&p, &o) > 0, "valid problem");
  CHECK(sylv_workspace_bytes(NULL, &o) == 0, "null problem");
  CHECK(sylv_workspace_bytes(&p, NULL) == 0, "null options");

  /* sizes: zero, negative, s outside 1..8 or above min(n, m), up to the int64 limit */
  const int64_t bad_nms[][3] = {{0, 200, 1},    {300, 0, 1},   {-5, 200, 1},     {300, -1, 1},
                                {300, 200, 0},  {300, 200, 9}, {300, 200, -1},   {3, 200, 4},
                                {300, 2, 4},    {INT64_MAX, 200, 1},             {300, INT64_MAX, 1},
                                {INT64_MIN, 200, 1},           {big, 200, 1},    {300, big, 1},
                                {INT64_MAX, INT64_MAX, 8},     {(int64_t)1 << 31, 200, 1}};
  for (size_t i = 0; i < sizeof bad_nms / sizeof bad_nms[0]; ++i) {
    sylv_problem q = fake_problem(bad_nms[i][0], bad_nms[i][1], bad_nms[i][2], 0);
    q.A.rows = q.n;
    q.B.rows = q.m;
    q.A.nnz = 10;
    q.B.nnz = 10;
    CHECK(sylv_workspace_bytes(&q, &o) == 0, "sizes %lld %lld %lld", (long long)bad_nms[i][0],
          (long long)bad_nms[i][1], (long long)bad_nms[i][2]);
  }
  /* Lyapunov with n != m; Lyapunov ignores B and C2 */
  sylv_problem q = fake_problem(300, 200, 2, 1);
  CHECK(sylv_workspace_bytes(&q, &o) == 0, "lyapunov n != m");
  q = fake_problem(300, 300, 2, 1);
  q.B = fake_csr(-7, -7);
  q.B.row_ptr = NULL;
  CHECK(sylv_workspace_bytes(&q, &o) > 0, "lyapunov ignores B");

  /* malformed CSR headers and right-hand sides */
  for (int which = 0; which < 12; ++which) {
    q = fake_problem(300, 200, 2, 0);
    switch (which) {
      case 0: q.A.rows = 299; break;
      case 1: q.B.rows = 201; break;
      case 2: q.A.nnz = -1; break;
      case 3: q.B.nnz = (int64_t)1 << 31; break;
      case 4: q.A.row_ptr = NULL; break;
      case 5: q.B.col_idx = NULL; break;
      case 6: q.A.values = NULL; break;
      case 7: q.C1 = NULL; break;
      case 8: q.C2 = NULL; break;
      case 9: q.ldc1 = 1; break;
      case 10: q.ldc2 = -4; break;
      default: q.A.nnz = INT64_MIN; break;
    }
    CHECK(sylv_workspace_bytes(&q, &o) == 0, "malformed input %d", which);
  }
  /* an empty matrix (nnz 0) is a valid operator without column or value arrays */
  q = fake_problem(300, 200, 2, 0);
  q.A.nnz = 0;
  q.A.col_idx = NULL;
  q.A.values = NULL;
  CHECK(sylv_workspace_bytes(&q, &o) > 0, "nnz 0");

  /* options out of range */
  for (int which = 0; which < 16; ++which) {
    sylv_options b = opts(SYLV_METHOD_BICGSTAB, 40);
    switch (which) {
      case 0: b.method = -1; break;
      case 1: b.method = 5; break;
      case 2: b.max_iter = 0; break;
      case 3: b.max_iter = -3; break;
      case 4: b.max_iter = INT32_MAX; break;
      case 5: b.precision = 3; break;
      case 6: b.streams = 3; break;
      case 7: b.streams = -1; break;
      case 8: b.reorth = 3; break;
      case 9: b.gram_precision = 3; break;
      case 10: b.verify = 2; break;
      case 11: b.refine_max = 5; break;
      case 12: b.refine_max = 1; b.refine_rank = 0; break;
      case 13: b.refine_max = 1; b.refine_max_iter = 0; break;
      case 14: b.method = SYLV_METHOD_CGS; b.refine_max = 1; break;
      default: b.precision = SYLV_MIXED_FP32; b.reorth = 2; break;
    }
    CHECK(sylv_workspace_bytes(&p, &b) == 0, "options %d", which);
  }

  /* valid problems: every method, precision and reorthogonalisation choice, small to large
   * sizes (the sizing call does host arithmetic only) */
  const int64_t sizes[][2] = {{8, 8}, {9, 17}, {300, 200}, {4096, 4096}, {100000, 7},
                              {1 << 20, 1 << 20}, {(int64_t)1 << 30, 64}};
  size_t last = 0;
  for (size_t si = 0; si < sizeof sizes / sizeof sizes[0]; ++si)
    for (int64_t s = 1; s <= 8; ++s)
      for (int method = 0; method <= 4; ++method)
        for (int prec = 0; prec <= 1; ++prec)
          for (int lyap = 0; lyap <= 1; ++lyap) {
            const int64_t n = sizes[si][0], m = lyap ? n : sizes[si][1];
            if (s > (n < m ? n : m)) continue;
            sylv_problem v = fake_problem(n, m, s, lyap);
            sylv_options w = opts(method, method == SYLV_METHOD_CG ? 300 : 120);
            w.precision = prec;
            if (prec && method <= SYLV_METHOD_BICGSTAB) {
              w.refine_max = 2;
              w.refine_rank = (int)s;
              w.refine_max_iter = 50;
            }
            const size_t nb = sylv_workspace_bytes(&v, &w);
            CHECK(nb > 0 && nb % 256 == 0 && nb > (size_t)n * 8, "valid %lld %lld s %lld method %d",
                  (long long)n, (long long)m, (long long)s, method);
            last = nb;
          }
  CHECK(last > 0, "sweep ran");
  /* the basis grows by s columns per iteration: more iterations, more workspace */
  sylv_options a = opts(SYLV_METHOD_CG, 100), b = opts(SYLV_METHOD_CG, 400);
  CHECK(sylv_workspace_bytes(&p, &a) < sylv_workspace_bytes(&p, &b), "grows with max_iter");
}

static void check_context_calls(void) {
  sylv_result res;
  double x = 0, y = 0;
  int64_t r1 = -1, r2 = -1;
  int cnt = -1;
  sylv_kernel_stat st[4];
  CHECK(sylv_factored_cg(NULL, 1e-8, 10, &res) == SYLV_ERR_INVALID, "cg null");
  CHECK(sylv_factored_bicgstab(NULL, 1e-8, 10, &res) == SYLV_ERR_INVALID, "bicgstab null");
  CHECK(sylv_factored_cr(NULL, 1e-8, 10, &res) == SYLV_ERR_INVALID, "cr null");
  CHECK(sylv_factored_cgs(NULL, 1e-8, 10, &res) == SYLV_ERR_INVALID, "cgs null");
  CHECK(sylv_factored_gpbicg(NULL, 1e-8, 10, NULL) == SYLV_ERR_INVALID, "gpbicg null");
  CHECK(sylv_residual_norm(NULL, &x, &y) == SYLV_ERR_INVALID, "residual null");
  CHECK(sylv_get_factors(NULL, NULL, 0, NULL, 0, NULL, 0, &r1, &r2) == SYLV_ERR_INVALID,
        "factors null");
  CHECK(sylv_compress(NULL, 1e-3, -1, &r1, &x) == SYLV_ERR_INVALID, "compress null");
  CHECK(sylv_get_compressed(NULL, NULL, 0, NULL, NULL, 0, &r1) == SYLV_ERR_INVALID,
        "compressed null");
  CHECK(sylv_get_history(NULL, NULL, NULL, NULL, NULL, 0, &cnt) == SYLV_ERR_INVALID,
        "history null");
  CHECK(sylv_set_profiling(NULL, 1) == SYLV_ERR_INVALID, "profiling null");
  CHECK(sylv_get_kernel_stats(NULL, st, 4, &cnt) == SYLV_ERR_STATE, "stats null");
  sylv_destroy(NULL);

  /* create: argument checks that come before any device work */
  sylv_problem p = fake_problem(300, 200, 2, 0);
  sylv_options o = opts(SYLV_METHOD_CG, 20);
  void *ctx = (void *)0x1;
  const size_t need = sylv_workspace_bytes(&p, &o);
  CHECK(sylv_create(NULL, &p, &o, fake_f64, need, NULL) == SYLV_ERR_INVALID, "create out null");
  CHECK(sylv_create(&ctx, NULL, &o, fake_f64, need, NULL) == SYLV_ERR_INVALID && ctx == NULL,
        "create problem null");
  ctx = (void *)0x1;
  CHECK(sylv_create(&ctx, &p, NULL, fake_f64, need, NULL) == SYLV_ERR_INVALID && ctx == NULL,
        "create options null");
  CHECK(sylv_create(&ctx, &p, &o, NULL, need, NULL) == SYLV_ERR_WORKSPACE, "no workspace");
  CHECK(sylv_create(&ctx, &p, &o, fake_f64, need - 1, NULL) == SYLV_ERR_WORKSPACE,
        "workspace one byte short");
  CHECK(sylv_create(&ctx, &p, &o, fake_f64, 0, NULL) == SYLV_ERR_WORKSPACE, "workspace 0");
  sylv_problem q = p;
  q.s = 0;
  CHECK(sylv_create(&ctx, &q, &o, fake_f64, need, NULL) == SYLV_ERR_INVALID, "create s 0");
}

static void check_batch_calls(void) {
  sylv_problem p[3] = {fake_problem(300, 200, 2, 0), fake_problem(120, 120, 1, 1),
                       fake_problem(64, 90, 4, 0)};
  sylv_options o[3] = {opts(SYLV_METHOD_CG, 40), opts(SYLV_METHOD_CG, 40),
                       opts(SYLV_METHOD_BICGSTAB, 30)};
  const size_t need = sylv_batch_workspace_bytes(3, p, o);
  size_t parts = 0;
  for (int i = 0; i < 3; ++i) parts += sylv_workspace_bytes(&p[i], &o[i]);
  CHECK(need >= parts && parts > 0, "batch bytes cover the instances");
  CHECK(sylv_batch_workspace_bytes(0, p, o) == 0, "batch count 0");
  CHECK(sylv_batch_workspace_bytes(-2, p, o) == 0, "batch count < 0");
  CHECK(sylv_batch_workspace_bytes(3, NULL, o) == 0, "batch probs null");
  CHECK(sylv_batch_workspace_bytes(3, p, NULL) == 0, "batch opts null");
  sylv_problem bad[3] = {p[0], p[1], p[2]};
  bad[2].s = 9;
  CHECK(sylv_batch_workspace_bytes(3, bad, o) == 0, "batch with an invalid instance");

  void *b = (void *)0x1;
  sylv_result res[3];
  CHECK(sylv_batch_create(NULL, 3, p, o, fake_f64, need, 2) == SYLV_ERR_INVALID, "batch out");
  CHECK(sylv_batch_create(&b, 0, p, o, fake_f64, need, 2) == SYLV_ERR_INVALID && b == NULL,
        "batch create count 0");
  CHECK(sylv_batch_create(&b, 3, NULL, o, fake_f64, need, 2) == SYLV_ERR_INVALID, "probs null");
  CHECK(sylv_batch_create(&b, 3, p, NULL, fake_f64, need, 2) == SYLV_ERR_INVALID, "opts null");
  CHECK(sylv_batch_create(&b, 3, p, o, fake_f64, need, 0) == SYLV_ERR_INVALID, "0 streams");
  CHECK(sylv_batch_create(&b, 3, p, o, fake_f64, need, 65) == SYLV_ERR_INVALID, "65 streams");
  CHECK(sylv_batch_create_ex(&b, 3, p, o, fake_f64, need, 2, 3) == SYLV_ERR_INVALID,
        "unknown form");
  CHECK(sylv_batch_create_ex(&b, 3, p, o, fake_f64, need, 2, -1) == SYLV_ERR_INVALID,
        "negative form");
  CHECK(sylv_batch_create_ex(&b, 3, bad, o, fake_f64, need, 2, SYLV_BATCH_GROUPED) ==
            SYLV_ERR_INVALID, "invalid instance");
  CHECK(sylv_batch_create_ex(&b, 3, p, o, NULL, need, 2, SYLV_BATCH_GRAPH) == SYLV_ERR_WORKSPACE,
        "batch without workspace");
  CHECK(sylv_batch_create_ex(&b, 3, p, o, fake_f64, need - 1, 2, SYLV_BATCH_GROUPED) ==
            SYLV_ERR_WORKSPACE, "batch workspace one byte short");
  CHECK(b == NULL, "failed create leaves no batch");
  CHECK(sylv_batch_solve(NULL, 1e-8, res) == SYLV_ERR_INVALID, "batch solve null");
  CHECK(sylv_batch_context(NULL, 0) == NULL, "batch context null");
  CHECK(sylv_batch_groups(NULL) == SYLV_ERR_INVALID, "batch groups null");
  sylv_batch_destroy(NULL);
}

static void check_building_blocks(void) {
  sylv_csr a = fake_csr(100, 300);
  double *X = fake_f64, *Y = fake_f64;
  int32_t *o32 = fake_i32;
  CHECK(sylv_spmm(NULL, 2, X, 2, Y, 2, NULL) == SYLV_ERR_INVALID, "spmm A null");
  CHECK(sylv_spmm(&a, 0, X, 2, Y, 2, NULL) == SYLV_ERR_INVALID, "spmm s 0");
  CHECK(sylv_spmm(&a, 9, X, 9, Y, 9, NULL) == SYLV_ERR_INVALID, "spmm s 9");
  CHECK(sylv_spmm(&a, 4, X, 3, Y, 4, NULL) == SYLV_ERR_INVALID, "spmm ldx < s");
  CHECK(sylv_spmm(&a, 4, X, 4, Y, 3, NULL) == SYLV_ERR_INVALID, "spmm ldy < s");
  CHECK(sylv_spmm(&a, 4, NULL, 4, Y, 4, NULL) == SYLV_ERR_INVALID, "spmm X null");
  CHECK(sylv_spmm(&a, 4, X, 4, NULL, 4, NULL) == SYLV_ERR_INVALID, "spmm Y null");
  sylv_csr neg = fake_csr(-100, 300);
  CHECK(sylv_spmm(&neg, 2, X, 2, Y, 2, NULL) == SYLV_ERR_INVALID, "spmm rows < 0");
  sylv_csr huge = fake_csr(INT64_MAX, 300);
  CHECK(sylv_spmm(&huge, 2, X, 2, Y, 2, NULL) == SYLV_ERR_INVALID, "spmm rows INT64_MAX");
  sylv_csr badnnz = fake_csr(100, -1);
  CHECK(sylv_spmm(&badnnz, 2, X, 2, Y, 2, NULL) == SYLV_ERR_INVALID, "spmm nnz < 0");

  CHECK(sylv_sell_bytes(NULL) == 0, "sell bytes null");
  CHECK(sylv_sell_bytes(&neg) == 0, "sell bytes rows < 0");
  CHECK(sylv_sell_bytes(&huge) == 0, "sell bytes rows INT64_MAX");
  CHECK(sylv_sell_bytes(&a) > 0, "sell bytes valid");
  sylv_csr big = fake_csr(((int64_t)1 << 31) - 1, ((int64_t)1 << 31) - 1);
  CHECK(sylv_sell_bytes(&big) > 0, "sell bytes largest valid");
  CHECK(sylv_sell_build(NULL, fake_f64, 1 << 20, NULL) == SYLV_ERR_INVALID, "sell build A null");
  CHECK(sylv_sell_build(&a, NULL, 1 << 20, NULL) == SYLV_ERR_INVALID, "sell build buffer null");
  CHECK(sylv_sell_build(&a, fake_f64, 8, NULL) == SYLV_ERR_WORKSPACE, "sell build too small");
  CHECK(sylv_sell_spmm(&a, NULL, 2, X, 2, Y, 2, NULL) == SYLV_ERR_INVALID, "sell spmm null");
  CHECK(sylv_sell_spmm(&a, fake_f64, 0, X, 2, Y, 2, NULL) == SYLV_ERR_INVALID, "sell spmm s 0");
  CHECK(sylv_sell_spmm(&neg, fake_f64, 2, X, 2, Y, 2, NULL) == SYLV_ERR_INVALID, "sell rows < 0");

  CHECK(sylv_csr_transpose_scratch_bytes(100) > 100 * 2 * sizeof(int),
        "transpose scratch valid");
  CHECK(sylv_csr_transpose_scratch_bytes(-5) == 0, "transpose scratch rows < 0");
  CHECK(sylv_csr_transpose_scratch_bytes(INT64_MAX) == 0, "transpose scratch INT64_MAX");
  CHECK(sylv_csr_transpose_scratch_bytes(INT64_MIN) == 0, "transpose scratch INT64_MIN");
  CHECK(sylv_csr_transpose(NULL, o32, o32, Y, fake_f64, NULL) == SYLV_ERR_INVALID, "tr A null");
  CHECK(sylv_csr_transpose(&a, NULL, o32, Y, fake_f64, NULL) == SYLV_ERR_INVALID, "tr out null");
  CHECK(sylv_csr_transpose(&a, o32, NULL, Y, fake_f64, NULL) == SYLV_ERR_INVALID, "tr cols null");
  CHECK(sylv_csr_transpose(&a, o32, o32, Y, NULL, NULL) == SYLV_ERR_INVALID, "tr scratch null");
  CHECK(sylv_csr_transpose(&neg, o32, o32, Y, fake_f64, NULL) == SYLV_ERR_INVALID, "tr rows<0");
  CHECK(sylv_csr_transpose(&huge, o32, o32, Y, fake_f64, NULL) == SYLV_ERR_INVALID,
        "tr rows INT64_MAX");
  CHECK(sylv_csr_transpose_noalloc(NULL, o32, o32, Y, NULL) == SYLV_ERR_INVALID, "tr0 A null");
  CHECK(sylv_csr_transpose_noalloc(&a, NULL, o32, Y, NULL) == SYLV_ERR_INVALID, "tr0 out null");
  CHECK(sylv_csr_transpose_noalloc(&a, o32, o32, NULL, NULL) == SYLV_ERR_INVALID, "tr0 vals");
  CHECK(sylv_csr_transpose_noalloc(&neg, o32, o32, Y, NULL) == SYLV_ERR_INVALID, "tr0 rows<0");
  sylv_csr over = fake_csr(SYLV_NOALLOC_TRANSPOSE_MAX_ROWS + 1, 10);
  CHECK(sylv_csr_transpose_noalloc(&over, o32, o32, Y, NULL) == SYLV_ERR_WORKSPACE,
        "tr0 above the scratch limit");
  CHECK(strstr(sylv_last_error(), "rows") != NULL, "tr0 names the limit");

  CHECK(sylv_dgemm(-1, 4, 4, 1.0, X, 4, 1, X, 4, 1, 0.0, Y, 4, NULL) == SYLV_ERR_INVALID, "M<0");
  CHECK(sylv_dgemm(4, -1, 4, 1.0, X, 4, 1, X, 4, 1, 0.0, Y, 4, NULL) == SYLV_ERR_INVALID, "N<0");
  CHECK(sylv_dgemm(4, 4, -1, 1.0, X, 4, 1, X, 4, 1, 0.0, Y, 4, NULL) == SYLV_ERR_INVALID, "K<0");
  CHECK(sylv_dgemm(4, 4, 4, 1.0, X, 4, 1, X, 4, 1, 0.0, Y, 3, NULL) == SYLV_ERR_INVALID, "ldc<N");
  CHECK(sylv_dgemm(4, 4, 4, 1.0, NULL, 4, 1, X, 4, 1, 0.0, Y, 4, NULL) == SYLV_ERR_INVALID,
        "gemm A null");
  CHECK(sylv_dgemm(4, 4, 4, 1.0, X, 4, 1, NULL, 4, 1, 0.0, Y, 4, NULL) == SYLV_ERR_INVALID,
        "gemm B null");
  CHECK(sylv_dgemm(4, 4, 4, 1.0, X, 4, 1, X, 4, 1, 0.0, NULL, 4, NULL) == SYLV_ERR_INVALID,
        "gemm C null");
  CHECK(sylv_dgemm(INT64_MAX, INT64_MAX, 4, 1.0, X, 4, 1, X, 4, 1, 0.0, Y, INT64_MAX, NULL) ==
            SYLV_ERR_INVALID, "gemm sizes beyond the grid");

  CHECK(sylv_gram_work_bytes(0, 5, 5) == 0 && sylv_gram_work_bytes(5, -1, 5) == 0 &&
            sylv_gram_work_bytes(5, 5, 0) == 0 && sylv_gram_work_bytes(INT64_MAX, 5, 5) == 0,
        "gram work bytes invalid");
  CHECK(sylv_gram_work_bytes(3000, 3000, 16384) >= (size_t)2 * 512 * 128 * 128 * 8,
        "gram work bytes of a large Gram");
  CHECK(sylv_gram_work_bytes(70, 50, 100) > 0, "gram work bytes of a small Gram");
  CHECK(sylv_gram(10, 10, 0, X, 64, X, 64, 0, 0, Y, 10, NULL, 0, NULL) == SYLV_ERR_INVALID,
        "gram K 0");
  CHECK(sylv_gram(-1, 10, 5, X, 64, X, 64, 0, 0, Y, 10, NULL, 0, NULL) == SYLV_ERR_INVALID,
        "gram M < 0");
  CHECK(sylv_gram(0, 10, 5, NULL, 0, NULL, 0, 0, 0, NULL, 0, NULL, 0, NULL) == 0, "gram M 0");
  CHECK(sylv_gram(10, 10, 5, NULL, 64, X, 64, 0, 0, Y, 10, NULL, 0, NULL) == SYLV_ERR_INVALID,
        "gram A null");
  CHECK(sylv_gram(10, 10, 5, X, 64, X, 64, 0, 0, NULL, 10, NULL, 0, NULL) == SYLV_ERR_INVALID,
        "gram C null");
  CHECK(sylv_gram(10, 10, 5, X, 60, X, 64, 0, 0, Y, 10, NULL, 0, NULL) == SYLV_ERR_INVALID,
        "gram lda below 64");
  CHECK(sylv_gram(10, 10, 5, X, 68, X, 64, 0, 0, Y, 10, NULL, 0, NULL) == SYLV_ERR_INVALID,
        "gram lda not a multiple of 8");
  CHECK(sylv_gram(10, 10, 5, X, 64, X, 64, 0, 0, Y, 9, NULL, 0, NULL) == SYLV_ERR_INVALID,
        "gram ldc < N");
  CHECK(sylv_gram(10, 12, 5, X, 64, X, 64, 1, 0, Y, 12, NULL, 0, NULL) == SYLV_ERR_INVALID,
        "gram symmetric M != N");
  CHECK(sylv_gram(10, 10, 5, X, 64, X, 64, 0, 0, Y, 10, (char *)fake_f64 + 1, 64, NULL) ==
            SYLV_ERR_INVALID, "gram misaligned work");
  CHECK(sylv_gram(INT64_MAX, 10, 5, X, INT64_MAX, X, 64, 0, 0, Y, 10, NULL, 0, NULL) ==
            SYLV_ERR_INVALID, "gram M beyond int32");
}

/* ---------------------------------------------------------------- solve mode (GPU) ---- */

static uint64_t rng_state = 12345;

static double urand(void) { /* splitmix64, uniform in [-1, 1) */
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static int hip_ok(hipError_t e, const char *what) {
  ++checks;
  if (e == hipSuccess) return 1;
  ++fails;
  printf("FAIL HIP %s: %s\n", what, hipGetErrorString(e));
  return 0;
}

static void *dev_alloc(size_t bytes) {
  void *d = NULL;
  if (!hip_ok(hipMalloc(&d, bytes ? bytes : 8), "hipMalloc")) return NULL;
  return d;
}

static void *to_dev(const void *h, size_t bytes) {
  void *d = dev_alloc(bytes);
  if (d && bytes && !hip_ok(hipMemcpy(d, h, bytes, hipMemcpyHostToDevice), "copy in")) return NULL;
  return d;
}

typedef struct {
  sylv_csr a;   /* device arrays */
  int32_t *rp;  /* host copies */
  int32_t *ci;
  double *va;
} Mat;

/* five-point convection-diffusion on an nx x ny grid (ny = 1: three-point); c = 0 gives the
 * symmetric positive definite Laplacian */
static Mat stencil(int nx, int ny, double c) {
  const int64_t n = (int64_t)nx * ny;
  Mat M;
  M.rp = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
  M.ci = (int32_t *)malloc((size_t)(5 * n) * sizeof(int32_t));
  M.va = (double *)malloc((size_t)(5 * n) * sizeof(double));
  int64_t k = 0;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int64_t r = (int64_t)j * nx + i;
      M.rp[r] = (int32_t)k;
      if (j > 0) M.ci[k] = (int32_t)(r - nx), M.va[k++] = -1.0;
      if (i > 0) M.ci[k] = (int32_t)(r - 1), M.va[k++] = -1.0 - c;
      M.ci[k] = (int32_t)r, M.va[k++] = 4.0;
      if (i + 1 < nx) M.ci[k] = (int32_t)(r + 1), M.va[k++] = -1.0 + c;
      if (j + 1 < ny) M.ci[k] = (int32_t)(r + nx), M.va[k++] = -1.0;
    }
  M.rp[n] = (int32_t)k;
  M.a.rows = n;
  M.a.nnz = k;
  M.a.row_ptr = (const int32_t *)to_dev(M.rp, (size_t)(n + 1) * sizeof(int32_t));
  M.a.col_idx = (const int32_t *)to_dev(M.ci, (size_t)k * sizeof(int32_t));
  M.a.values = (const double *)to_dev(M.va, (size_t)k * sizeof(double));
  return M;
}

static void free_mat(Mat *M) {
  hipFree((void *)M->a.row_ptr);
  hipFree((void *)M->a.col_idx);
  hipFree((void *)M->a.values);
  free(M->rp);
  free(M->ci);
  free(M->va);
}

typedef struct {
  sylv_problem p;
  Mat A, B;
  double *c1, *c2;
  int lyap;
} Prob;

static Prob make_prob(int nx, int ny, int mx, double c, int s, int lyap) {
  Prob P;
  memset(&P, 0, sizeof P);
  P.lyap = lyap;
  P.A = stencil(nx, ny, c);
  if (!lyap) P.B = stencil(mx, 1, c);
  const int64_t n = P.A.a.rows, m = lyap ? n : P.B.a.rows;
  double *h = (double *)malloc((size_t)((n > m ? n : m) * s) * sizeof(double));
  for (int64_t i = 0; i < n * s; ++i) h[i] = urand();
  P.c1 = (double *)to_dev(h, (size_t)(n * s) * sizeof(double));
  if (!lyap) {
    for (int64_t i = 0; i < m * s; ++i) h[i] = urand();
    P.c2 = (double *)to_dev(h, (size_t)(m * s) * sizeof(double));
  }
  free(h);
  P.p.n = n;
  P.p.m = m;
  P.p.s = s;
  P.p.A = P.A.a;
  P.p.B = lyap ? P.A.a : P.B.a;
  P.p.lyapunov = lyap;
  P.p.C1 = P.c1;
  P.p.ldc1 = s;
  P.p.C2 = P.c2;
  P.p.ldc2 = s;
  return P;
}

static void free_prob(Prob *P) {
  free_mat(&P->A);
  if (!P->lyap) free_mat(&P->B);
  hipFree(P->c1);
  if (P->c2) hipFree(P->c2);
}

typedef int (*solve_fn)(void *, double, int, sylv_result *);

static solve_fn method_fn(int method) {
  switch (method) {
    case SYLV_METHOD_CG: return sylv_factored_cg;
    case SYLV_METHOD_BICGSTAB: return sylv_factored_bicgstab;
    case SYLV_METHOD_CR: return sylv_factored_cr;
    case SYLV_METHOD_CGS: return sylv_factored_cgs;
    default: return sylv_factored_gpbicg;
  }
}

/* factors, history, compression and kernel statistics of a solved context */
static void inspect(const char *name, void *ctx, const Prob *P, int max_iter, int refined,
                    double tol) {
  double ab = -1, rel = -1;
  int e = sylv_residual_norm(ctx, &ab, &rel);
  CHECK(e == 0 && rel >= 0 && rel <= 1.05 * tol, "%s: true residual %d %g", name, e, rel);
  int64_t rv = -1, rw = -1;
  e = sylv_get_factors(ctx, NULL, 0, NULL, 0, NULL, 0, &rv, &rw);
  CHECK(e == 0 && rv > 0 && rw > 0, "%s: factor ranks %d", name, e);
  if (e == 0 && rv > 0 && rw > 0) {
    double *V = (double *)dev_alloc((size_t)(P->p.n * rv) * 8);
    double *X = (double *)dev_alloc((size_t)(rv * rw) * 8);
    double *W = (double *)dev_alloc((size_t)(P->p.m * rw) * 8);
    e = sylv_get_factors(ctx, V, rv, X, rw, W, rw, &rv, &rw);
    CHECK(e == 0, "%s: factors %d", name, e);
    hipFree(V);
    hipFree(X);
    hipFree(W);
  }
  double *h = (double *)malloc((size_t)max_iter * 4 * sizeof(double));
  int cnt = -1;
  e = sylv_get_history(ctx, h, h + max_iter, h + 2 * max_iter, h + 3 * max_iter, max_iter, &cnt);
  CHECK(e == 0 && cnt > 0 && cnt <= max_iter, "%s: history %d %d", name, e, cnt);
  /* a refined solve keeps the history of its last correction solve (its own R0) */
  if (e == 0 && cnt > 0 && !refined)
    CHECK(h[cnt - 1] <= tol * 1.0001, "%s: last relres %g", name, h[cnt - 1]);
  free(h);
  if (!refined) {
    int64_t k = -1;
    double err = -1;
    e = sylv_compress(ctx, 1e-6, -1, &k, &err);
    CHECK((e == 0 || e == SYLV_NOT_CONVERGED) && k > 0 && err >= 0, "%s: compress %d", name, e);
    int64_t k2 = -1;
    e = sylv_get_compressed(ctx, NULL, 0, NULL, NULL, 0, &k2);
    CHECK(e == 0 && k2 == k, "%s: compressed rank", name);
    if (e == 0 && k > 0) {
      double *Z1 = (double *)dev_alloc((size_t)(P->p.n * k) * 8);
      double *sg = (double *)dev_alloc((size_t)k * 8);
      double *Z2 = (double *)dev_alloc((size_t)(P->p.m * k) * 8);
      e = sylv_get_compressed(ctx, Z1, k, sg, Z2, k, &k2);
      CHECK(e == 0, "%s: compressed factors", name);
      hipFree(Z1);
      hipFree(sg);
      hipFree(Z2);
    }
  }
}

static void solve_one(const char *name, Prob *P, int method, int precision, int refine,
                      double tol) {
  sylv_options o = opts(method, 400);
  o.precision = precision;
  if (refine) {
    o.refine_max = 3;
    o.refine_rank = 8;
    o.refine_max_iter = 100;
  }
  const size_t nb = sylv_workspace_bytes(&P->p, &o);
  CHECK(nb > 0, "%s: workspace size", name);
  void *ws = dev_alloc(nb);
  if (!ws) return;
  void *ctx = NULL;
  int e = sylv_create(&ctx, &P->p, &o, ws, nb, NULL);
  CHECK(e == 0 && ctx, "%s: create %d (%s)", name, e, sylv_last_error());
  if (e == 0) {
    sylv_result r;
    memset(&r, 0, sizeof r);
    e = method_fn(method)(ctx, tol, o.max_iter, &r);
    CHECK(e == SYLV_OK && r.status == SYLV_OK && r.iters > 0, "%s: solve %d", name, e);
    printf("%s: %d iterations, ranks %lld x %lld\n", name, r.iters, (long long)r.rank_v,
           (long long)r.rank_w);
    fflush(stdout);
    inspect(name, ctx, P, refine ? 4 * o.max_iter : o.max_iter, refine, tol);
    if (refine) {
      int64_t k = -1;
      CHECK(sylv_compress(ctx, 1e-6, -1, &k, NULL) == SYLV_ERR_STATE, "%s: refined", name);
    } else {
      CHECK(sylv_get_kernel_stats(ctx, NULL, 0, NULL) == SYLV_ERR_STATE, "%s: stats off", name);
      CHECK(sylv_set_profiling(ctx, 1) == 0, "%s: profiling on", name);
      e = method_fn(method)(ctx, tol, o.max_iter, NULL);
      CHECK(e == SYLV_OK, "%s: profiled solve %d", name, e);
      sylv_kernel_stat st[32];
      int cnt = -1;
      e = sylv_get_kernel_stats(ctx, st, 32, &cnt);
      CHECK(e == 0 && cnt > 0 && cnt <= 32, "%s: kernel stats %d", name, e);
      int64_t launches = 0;
      for (int f = 0; f < cnt && f < 32; ++f) launches += st[f].launches;
      CHECK(launches > 0, "%s: timed launches", name);
      CHECK(sylv_set_profiling(ctx, 0) == 0, "%s: profiling off", name);
    }
    /* a solve with more iterations than the workspace holds is refused */
    CHECK(method_fn(method)(ctx, tol, o.max_iter + 1000, NULL) == SYLV_ERR_INVALID,
          "%s: max_iter beyond the workspace", name);
    sylv_destroy(ctx);
  }
  hipFree(ws);
}

static void single_solves(void) {
  Prob P = make_prob(21, 19, 150, 0.0, 2, 0);
  solve_one("cg", &P, SYLV_METHOD_CG, SYLV_FP64, 0, 1e-9);
  solve_one("cr", &P, SYLV_METHOD_CR, SYLV_FP64, 0, 1e-9);
  free_prob(&P);
  P = make_prob(19, 17, 130, 0.35, 3, 0);
  solve_one("bicgstab", &P, SYLV_METHOD_BICGSTAB, SYLV_FP64, 0, 1e-9);
  solve_one("cgs", &P, SYLV_METHOD_CGS, SYLV_FP64, 0, 1e-8);
  solve_one("gpbicg", &P, SYLV_METHOD_GPBICG, SYLV_FP64, 0, 1e-9);
  solve_one("bicgstab_fp32_refined", &P, SYLV_METHOD_BICGSTAB, SYLV_MIXED_FP32, 1, 1e-9);
  free_prob(&P);
  P = make_prob(23, 20, 0, 0.0, 2, 1);
  solve_one("lyapunov_cg", &P, SYLV_METHOD_CG, SYLV_FP64, 0, 1e-9);
  free_prob(&P);
}

static void batches(void) {
  enum { NB = 7 };
  Prob P[NB] = {make_prob(20, 18, 90, 0.0, 2, 0),  make_prob(16, 22, 70, 0.0, 2, 0),
                make_prob(18, 18, 0, 0.0, 1, 1),   make_prob(22, 15, 80, 0.3, 1, 0),
                make_prob(15, 20, 60, 0.3, 1, 0),  make_prob(14, 13, 90, 0.0, 2, 0),
                make_prob(17, 12, 75, 0.3, 1, 0)};
  const int meth[NB] = {SYLV_METHOD_CG,       SYLV_METHOD_CG, SYLV_METHOD_CG, SYLV_METHOD_BICGSTAB,
                        SYLV_METHOD_BICGSTAB, SYLV_METHOD_CR, SYLV_METHOD_CGS};
  sylv_problem probs[NB];
  sylv_options o[NB];
  for (int i = 0; i < NB; ++i) {
    probs[i] = P[i].p;
    o[i] = opts(meth[i], 300);
  }
  const size_t nb = sylv_batch_workspace_bytes(NB, probs, o);
  CHECK(nb > 0, "batch workspace size");
  void *ws = dev_alloc(nb);
  const double tol = 1e-9;
  for (int form = SYLV_BATCH_STREAMS; ws && form <= SYLV_BATCH_GRAPH; ++form) {
    void *b = NULL;
    int e = sylv_batch_create_ex(&b, NB, probs, o, ws, nb, 3, form);
    CHECK(e == 0 && b, "batch form %d: create %d (%s)", form, e, sylv_last_error());
    if (e) continue;
    CHECK(form == SYLV_BATCH_STREAMS ? sylv_batch_groups(b) == 0 : sylv_batch_groups(b) >= 2,
          "batch form %d: groups %d", form, sylv_batch_groups(b));
    for (int rep = 0; rep < 2; ++rep) {
      sylv_result res[NB];
      memset(res, 0, sizeof res);
      e = sylv_batch_solve(b, tol, res);
      CHECK(e == 0, "batch form %d: solve %d (%s)", form, e, sylv_last_error());
      for (int i = 0; i < NB; ++i) {
        CHECK(res[i].status == SYLV_OK && res[i].iters > 0, "batch form %d: instance %d", form, i);
        double ab = -1, rel = -1;
        e = sylv_residual_norm(sylv_batch_context(b, i), &ab, &rel);
        CHECK(e == 0 && rel <= 1.05 * tol, "batch form %d: instance %d residual %g", form, i, rel);
      }
    }
    CHECK(sylv_batch_context(b, NB) == NULL && sylv_batch_context(b, -1) == NULL,
          "batch context out of range");
    sylv_batch_destroy(b);
    printf("batch form %d done\n", form);
    fflush(stdout);
  }
  hipFree(ws);
  for (int i = 0; i < NB; ++i) free_prob(&P[i]);
}

static void building_block_calls(void) {
  Mat M = stencil(37, 29, 0.2);
  const int64_t n = M.a.rows, s = 3;
  double *hx = (double *)malloc((size_t)(n * s) * 8), *hy = (double *)malloc((size_t)(n * s) * 8);
  double *ref = (double *)malloc((size_t)(n * s) * 8);
  for (int64_t i = 0; i < n * s; ++i) hx[i] = urand();
  for (int64_t r = 0; r < n; ++r)
    for (int64_t c = 0; c < s; ++c) {
      double acc = 0;
      for (int32_t k = M.rp[r]; k < M.rp[r + 1]; ++k) acc += M.va[k] * hx[M.ci[k] * s + c];
      ref[r * s + c] = acc;
    }
  double *X = (double *)to_dev(hx, (size_t)(n * s) * 8), *Y = (double *)dev_alloc((size_t)(n * s) * 8);
  CHECK(sylv_spmm(&M.a, s, X, s, Y, s, NULL) == 0, "spmm");
  hip_ok(hipMemcpy(hy, Y, (size_t)(n * s) * 8, hipMemcpyDeviceToHost), "spmm out");
  double err = 0;
  for (int64_t i = 0; i < n * s; ++i) err = fmax(err, fabs(hy[i] - ref[i]));
  CHECK(err <= 1e-13, "spmm error %g", err);
  const size_t sb = sylv_sell_bytes(&M.a);
  void *sell = dev_alloc(sb);
  CHECK(sylv_sell_build(&M.a, sell, sb, NULL) == 0, "sell build");
  CHECK(sylv_sell_spmm(&M.a, sell, s, X, s, Y, s, NULL) == 0, "sell spmm");
  hip_ok(hipMemcpy(hy, Y, (size_t)(n * s) * 8, hipMemcpyDeviceToHost), "sell spmm out");
  err = 0;
  for (int64_t i = 0; i < n * s; ++i) err = fmax(err, fabs(hy[i] - ref[i]));
  CHECK(err <= 1e-13, "sell spmm error %g", err);
  hipFree(sell);

  /* both transposes give the same canonical CSR; the transpose of the transpose is A */
  const int64_t nnz = M.a.nnz;
  int32_t *rp[3], *ci[3];
  double *va[3];
  for (int t = 0; t < 3; ++t) {
    rp[t] = (int32_t *)dev_alloc((size_t)(n + 1) * 4);
    ci[t] = (int32_t *)dev_alloc((size_t)nnz * 4);
    va[t] = (double *)dev_alloc((size_t)nnz * 8);
  }
  void *scr = dev_alloc(sylv_csr_transpose_scratch_bytes(n));
  CHECK(sylv_csr_transpose(&M.a, rp[0], ci[0], va[0], scr, NULL) == 0, "transpose");
  CHECK(sylv_csr_transpose_noalloc(&M.a, rp[1], ci[1], va[1], NULL) == 0, "transpose noalloc");
  sylv_csr T = {n, nnz, rp[0], ci[0], va[0]};
  CHECK(sylv_csr_transpose_noalloc(&T, rp[2], ci[2], va[2], NULL) == 0, "transpose twice");
  hip_ok(hipDeviceSynchronize(), "transposes");
  int32_t *h32 = (int32_t *)malloc((size_t)(n + 1 + nnz) * 4 * 2);
  double *h64 = (double *)malloc((size_t)nnz * 8 * 2);
  hip_ok(hipMemcpy(h32, rp[0], (size_t)(n + 1) * 4, hipMemcpyDeviceToHost), "t rp");
  hip_ok(hipMemcpy(h32 + n + 1, rp[1], (size_t)(n + 1) * 4, hipMemcpyDeviceToHost), "t rp");
  CHECK(memcmp(h32, h32 + n + 1, (size_t)(n + 1) * 4) == 0, "transposes agree (rows)");
  hip_ok(hipMemcpy(h32, rp[2], (size_t)(n + 1) * 4, hipMemcpyDeviceToHost), "tt rp");
  CHECK(memcmp(h32, M.rp, (size_t)(n + 1) * 4) == 0, "double transpose rows");
  hip_ok(hipMemcpy(h32, ci[2], (size_t)nnz * 4, hipMemcpyDeviceToHost), "tt ci");
  CHECK(memcmp(h32, M.ci, (size_t)nnz * 4) == 0, "double transpose columns");
  hip_ok(hipMemcpy(h64, va[2], (size_t)nnz * 8, hipMemcpyDeviceToHost), "tt va");
  CHECK(memcmp(h64, M.va, (size_t)nnz * 8) == 0, "double transpose values");
  hip_ok(hipMemcpy(h64, va[0], (size_t)nnz * 8, hipMemcpyDeviceToHost), "t va");
  hip_ok(hipMemcpy(h64 + nnz, va[1], (size_t)nnz * 8, hipMemcpyDeviceToHost), "t va");
  CHECK(memcmp(h64, h64 + nnz, (size_t)nnz * 8) == 0, "transposes agree (values)");
  free(h32);
  free(h64);
  hipFree(scr);
  for (int t = 0; t < 3; ++t) {
    hipFree(rp[t]);
    hipFree(ci[t]);
    hipFree(va[t]);
  }

  /* C = A B^T through the strides (B stored n x s, read as its transpose) */
  const int64_t Mr = 70, K = 33;
  double *ha = (double *)malloc((size_t)(Mr * K) * 8), *hb = (double *)malloc((size_t)(s * K) * 8);
  double *hc = (double *)malloc((size_t)(Mr * s) * 8);
  for (int64_t i = 0; i < Mr * K; ++i) ha[i] = urand();
  for (int64_t i = 0; i < s * K; ++i) hb[i] = urand();
  double *dA = (double *)to_dev(ha, (size_t)(Mr * K) * 8), *dB = (double *)to_dev(hb, (size_t)(s * K) * 8);
  double *dC = (double *)dev_alloc((size_t)(Mr * s) * 8);
  CHECK(sylv_dgemm(Mr, s, K, 1.0, dA, K, 1, dB, 1, K, 0.0, dC, s, NULL) == 0, "dgemm");
  hip_ok(hipMemcpy(hc, dC, (size_t)(Mr * s) * 8, hipMemcpyDeviceToHost), "dgemm out");
  err = 0;
  for (int64_t i = 0; i < Mr; ++i)
    for (int64_t j = 0; j < s; ++j) {
      double acc = 0;
      for (int64_t k = 0; k < K; ++k) acc += ha[i * K + k] * hb[j * K + k];
      err = fmax(err, fabs(acc - hc[i * s + j]));
    }
  CHECK(err <= 1e-12, "dgemm error %g", err);

  /* Gram A^T A of the 70 x K panel above, stored K x 70 with leading dimension 128 */
  {
    const int64_t Mg = 70, Kg = 33, ldg = 128;
    double *hg = (double *)calloc((size_t)(Kg * ldg), 8), *hgc = (double *)malloc((size_t)(Mg * Mg) * 8);
    for (int64_t k = 0; k < Kg; ++k)
      for (int64_t i = 0; i < Mg; ++i) hg[k * ldg + i] = ha[i * Kg + k];
    double *dG = (double *)to_dev(hg, (size_t)(Kg * ldg) * 8), *dGC = (double *)dev_alloc((size_t)(Mg * Mg) * 8);
    const size_t wb = sylv_gram_work_bytes(Mg, Mg, Kg);
    void *wk = dev_alloc(wb);
    CHECK(sylv_gram(Mg, Mg, Kg, dG, ldg, dG, ldg, 1, 0, dGC, Mg, wk, wb, NULL) == 0, "gram");
    hip_ok(hipMemcpy(hgc, dGC, (size_t)(Mg * Mg) * 8, hipMemcpyDeviceToHost), "gram out");
    err = 0;
    for (int64_t i = 0; i < Mg; ++i)
      for (int64_t j = 0; j < Mg; ++j) {
        double acc = 0;
        for (int64_t k = 0; k < Kg; ++k) acc += ha[i * Kg + k] * ha[j * Kg + k];
        err = fmax(err, fabs(acc - hgc[i * Mg + j]));
      }
    CHECK(err <= 1e-12, "gram error %g", err);
    hipFree(dG);
    hipFree(dGC);
    hipFree(wk);
    free(hg);
    free(hgc);
  }
  hipFree(dA);
  hipFree(dB);
  hipFree(dC);
  free(ha);
  free(hb);
  free(hc);
  hipFree(X);
  hipFree(Y);
  free(hx);
  free(hy);
  free(ref);
  free_mat(&M);
}

int main(int argc, char **argv) {
  const char *mode = argc > 1 ? argv[1] : "args";
  if (strcmp(mode, "args") == 0) {
    check_strings();
    check_workspace_sizing();
    check_context_calls();
    check_batch_calls();
    check_building_blocks();
  } else if (strcmp(mode, "solve") == 0) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
      printf("solve: no GPU\n");
      return 100;
    }
    single_solves();
    batches();
    building_block_calls();
    /* every context, batch and buffer is released by now. The process ends without exit
     * handlers: when the HIP runtime unloads, the address sanitizer's own bookkeeping of
     * device-side allocations trips an internal check of the sanitizer runtime */
    printf("%s: %d checks, %d failed\n", mode, checks, fails);
    fflush(stdout);
    fflush(stderr);
    _exit(fails);
  } else {
    fprintf(stderr, "unknown mode %s\n", mode);
    return 100;
  }
  printf("%s: %d checks, %d failed\n", mode, checks, fails);
  return fails;
}
