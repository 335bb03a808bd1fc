// QR of the first block of each basis, C1 = V_1 R_L (Alg. 4.1 step 1, Alg. 4.2 step 2), by two
// Cholesky-QR passes with the rank test of the right-hand side. The block Lanczos and block
// Arnoldi steps are in arnoldi.hip.
// The new block is appended to the basis and its coefficients to column block j of H, so that
// M V_j = V_{j+1} H_{j+1,j} holds column block by column block (eq. (3.8)).
//
// Data layout: the basis is row-major rows x ldb (row r holds all basis entries of grid point
// r), so SpMM gathers s contiguous doubles per neighbour.
//
// Every kernel returns at entry once the solve is done (device flag), so iterations enqueued
// beyond convergence cost only their launch.
#include "common.h"

namespace {

constexpr int TPB = 256;

// First block: G = C^T C for C1 (or C2); the last workgroup runs pass 1 with ref2 = ||C||^2.
template <int S>
__global__ __launch_bounds__(TPB) void first_gram_kernel(const double *__restrict__ C, int64_t ldc,
                                                         int64_t rows, double *__restrict__ U,
                                                         double closure_tol, SideState *ss,
                                                         double *partials, int *counter) {
  double g[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) g[i] = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * TPB) {
    double u[S];
#pragma unroll
    for (int t = 0; t < S; ++t) {
      u[t] = C[r * ldc + t];
      U[r * S + t] = u[t];
    }
#pragma unroll
    for (int a = 0; a < S; ++a)
#pragma unroll
      for (int b = 0; b < S; ++b) g[a * S + b] = fma(u[a], u[b], g[a * S + b]);
  }
  __shared__ double out[S * S];
  if (reduce_grid<S * S>(g, partials, counter, out) && threadIdx.x == 0) {
    double tr = 0.0;
    for (int i = 0; i < S; ++i) tr += out[i * S + i];
    ss->ref2 = tr;
    finish_pass1(ss, S, closure_tol, out);
  }
}

// Pass 2 Gram: G2 = (U T1)^T (U T1); last workgroup finishes the QR factor.
template <int S>
__global__ __launch_bounds__(TPB) void pass2_gram_kernel(const double *__restrict__ U, int64_t rows,
                                                         SideState *ss, double *partials,
                                                         int *counter, const DevState *ds) {
  if (ds && ds->done) return;
  double T1[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) T1[i] = ss->T1[i];
  double g[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) g[i] = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * TPB) {
    double u[S], u1[S];
#pragma unroll
    for (int t = 0; t < S; ++t) u[t] = U[r * S + t];
#pragma unroll
    for (int b = 0; b < S; ++b) {
      double v = 0.0;
#pragma unroll
      for (int a = 0; a < S; ++a) v = fma(u[a], T1[a * S + b], v);
      u1[b] = v;
    }
#pragma unroll
    for (int a = 0; a < S; ++a)
#pragma unroll
      for (int b = 0; b < S; ++b) g[a * S + b] = fma(u1[a], u1[b], g[a * S + b]);
  }
  __shared__ double out[S * S];
  if (reduce_grid<S * S>(g, partials, counter, out) && threadIdx.x == 0) finish_pass2(ss, S, out);
}

// V[:, ocol:ocol+S] = U T (stored as T_ELEM); optionally writes H_{j+1,j} = Hs into H at
// (hrow, hcol).
template <int S, typename T_ELEM>
__global__ __launch_bounds__(TPB) void final_kernel(const double *__restrict__ U, int64_t rows,
                                                    T_ELEM *__restrict__ V, int64_t ldb, int ocol,
                                                    T_ELEM *__restrict__ pout, const SideState *ss,
                                                    double *H, int64_t ldh, int hrow, int hcol,
                                                    const DevState *ds) {
  if (ds && ds->done) return;
  double T[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) T[i] = ss->T[i];
  const int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (r < rows) {
    double u[S];
#pragma unroll
    for (int t = 0; t < S; ++t) u[t] = U[r * S + t];
#pragma unroll
    for (int b = 0; b < S; ++b) {
      double v = 0.0;
#pragma unroll
      for (int a = 0; a < S; ++a) v = fma(u[a], T[a * S + b], v);
      V[r * ldb + ocol + b] = (T_ELEM)v;
      pout[r * S + b] = (T_ELEM)v;
    }
  }
  if (H && blockIdx.x == 0 && threadIdx.x < S * S) {
    const int a = threadIdx.x / S, b = threadIdx.x % S;
    H[(int64_t)(hrow + a) * ldh + hcol + b] = ss->Hs1[a * S + b];
  }
}

unsigned grid_rows(int64_t rows) { return (unsigned)((rows + TPB - 1) / TPB); }

// Workgroups for the pass-2 Gram and first-block kernels: enough to cover the rows, capped so
// the single-workgroup final sum stays short.
unsigned grid_capped(int64_t rows) {
  int64_t g = (rows + TPB - 1) / TPB;
  return (unsigned)(g < 1024 ? g : 1024);
}

template <int S>
int first_block_t(const SideDesc &sd, const double *C, int64_t ldc_in, double closure_tol,
                  const Scratch &sc, hipStream_t st) {
  first_gram_kernel<S><<<grid_capped(sd.rows), TPB, 0, st>>>(
      C, ldc_in, sd.rows, sd.U, closure_tol, sd.ss, sc.partials, sc.counters + CNT_NRM);
  HIPOK(hipGetLastError());
  pass2_gram_kernel<S><<<grid_capped(sd.rows), TPB, 0, st>>>(sd.U, sd.rows, sd.ss, sc.partials,
                                                             sc.counters + CNT_NRM + 1, nullptr);
  HIPOK(hipGetLastError());
  if (sd.fp32)
    final_kernel<S, float><<<grid_rows(sd.rows), TPB, 0, st>>>(
        sd.U, sd.rows, static_cast<float *>(sd.basis), sd.ldb, 0,
        static_cast<float *>(sd.panel[0]), sd.ss, nullptr, 0, 0, 0, nullptr);
  else
    final_kernel<S, double><<<grid_rows(sd.rows), TPB, 0, st>>>(
        sd.U, sd.rows, static_cast<double *>(sd.basis), sd.ldb, 0,
        static_cast<double *>(sd.panel[0]), sd.ss, nullptr, 0, 0, 0, nullptr);
  HIPOK(hipGetLastError());
  return 0;
}

}  // namespace

#define DISPATCH_S(s, call)            \
  switch (s) {                         \
    case 1: { constexpr int S = 1; return call; } \
    case 2: { constexpr int S = 2; return call; } \
    case 3: { constexpr int S = 3; return call; } \
    case 4: { constexpr int S = 4; return call; } \
    case 5: { constexpr int S = 5; return call; } \
    case 6: { constexpr int S = 6; return call; } \
    case 7: { constexpr int S = 7; return call; } \
    case 8: { constexpr int S = 8; return call; } \
    default: return SYLV_ERR_INVALID;  \
  }

int launch_first_block(int s, const SideDesc &sd, const double *C, int64_t ldc_in,
                       double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st) {
  (void)ds;
  DISPATCH_S(s, first_block_t<S>(sd, C, ldc_in, closure_tol, sc, st));
}


