// Core recurrences of the further factorized Krylov methods (Section 4's remark that the
// factorization applies to other Krylov methods; Section 6): conjugate residual (CR, symmetric
// operators, block Lanczos bases), conjugate gradient squared (CGS) and generalized
// product-type BiCG (GPBiCG), both with two core products per iteration on block Arnoldi
// bases. The core products themselves (eq. (3.11)) run on launch_core_op; the kernels here are
// the elementwise updates of the cores (eq. (3.9)), the core inner products (eq. (3.10)) and the
// scalars, all in FP64.
//
// Cores follow the conventions of core.hip: ldc x ldc row-major buffers, zero at the start of a
// solve, an active upper-left corner that only grows (the zero padding of smaller cores is
// implicit). An elementwise kernel covers a q x q corner: rows strided over the workgroups,
// columns over the threads, one partial per workgroup for each inner product it forms; the
// one-workgroup scalar kernels sum those partials in a fixed order (deterministic) and update
// DevState. Every kernel returns at once when the solve has stopped.
#include "common.h"

namespace {

constexpr int TPB = 256;
constexpr int NBLK = 512;
// Scratch::partials: [0, 8 NBLK) the inner products a scalar kernel consumes, [8 NBLK, 9 NBLK)
// the partials of ||R||^2
constexpr int RR_OFF = 8 * NBLK;

unsigned grid_of(int q) { return (unsigned)(q < NBLK ? (q < 1 ? 1 : q) : NBLK); }

__device__ __forceinline__ void halt(DevState *ds, int status, int iters) {
  ds->status = status;
  ds->iters = iters;
  ds->done = 1;
}

template <int NV>
__device__ __forceinline__ void put_parts(double (&v)[NV], double *partials) {
  __shared__ double lds[16 * NV];
  block_sum<NV>(v, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) partials[(size_t)blockIdx.x * NV + i] = v[i];
}

// Sum of nb records of NV partials, in order, on thread 0 (one-workgroup kernels).
template <int NV>
__device__ __forceinline__ void sum_parts(const double *partials, int nb, double (&out)[NV]) {
  __shared__ double lds[16 * NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) out[i] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] += partials[(size_t)b * NV + i];
  block_sum<NV>(out, lds);
}

// <R~0, Z(1:s, 1:s)> (R~0 = R0 is s x s, row-major, ld s).
__device__ __forceinline__ double corner_dot(int s, const double *Rt, const double *Z,
                                             int64_t ldc) {
  double v = 0.0;
  for (int a = 0; a < s; ++a)
    for (int b = 0; b < s; ++b) v = fma(Rt[a * s + b], Z[(int64_t)a * ldc + b], v);
  return v;
}

// Relative residual from the ||R||^2 partials, the stopping test; true when the solve goes on.
__device__ __forceinline__ bool converge_test(double rr, DevState *ds, double *hist, int k) {
  const double rel = sqrt(rr) / ds->normR0;
  ds->relres = rel;
  hist[k] = rel;
  if (rel <= ds->tol) {
    halt(ds, SYLV_OK, k + 1);
    return false;
  }
  if (!isfinite(rel)) {
    halt(ds, SYLV_BREAKDOWN, k);
    return false;
  }
  return true;
}

// ---- CR ----
// After S_0 = F(R_0): Q_0 = S_0; partials of <R_0, S_0> and <Q_0, Q_0>.
__global__ __launch_bounds__(TPB) void cr_init_kernel(int q, const double *__restrict__ R,
                                                      const double *__restrict__ S,
                                                      double *__restrict__ Q, int64_t ldc,
                                                      double *partials) {
  double v[2] = {0.0, 0.0};
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      const double sv = S[o];
      Q[o] = sv;
      v[0] = fma(R[o], sv, v[0]);
      v[1] = fma(sv, sv, v[1]);
    }
  put_parts<2>(v, partials);
}

__global__ __launch_bounds__(TPB) void cr_init_scalar_kernel(const double *partials, int nb,
                                                             DevState *ds) {
  double d[2];
  sum_parts<2>(partials, nb, d);
  if (threadIdx.x != 0) return;
  ds->rho = d[0];
  ds->pq = d[1];
}

// alpha_k = rho_k / <Q_k, Q_k> (from ds), X += alpha P, R -= alpha Q over q x q, partials of
// ||R_{k+1}||^2.
__global__ __launch_bounds__(TPB) void cr_xr_kernel(int q, double *__restrict__ X,
                                                    double *__restrict__ R,
                                                    const double *__restrict__ P,
                                                    const double *__restrict__ Q, int64_t ldc,
                                                    double *partials, DevState *ds, double *hist,
                                                    int k, int max_iter) {
  if (ds->done) return;
  const double qq = ds->pq, rho = ds->rho;
  const double alpha = rho / qq;
  if (!(qq != 0.0) || rho == 0.0 || !isfinite(alpha)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) halt(ds, SYLV_BREAKDOWN, k);
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ds->alpha = alpha;
    hist[max_iter + k] = alpha;
  }
  double v[1] = {0.0};
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      X[o] = fma(alpha, P[o], X[o]);
      const double r = fma(-alpha, Q[o], R[o]);
      R[o] = r;
      v[0] = fma(r, r, v[0]);
    }
  put_parts<1>(v, partials + RR_OFF);
}

__global__ __launch_bounds__(TPB) void rr_converge_kernel(const double *partials, int nb,
                                                          DevState *ds, double *hist, int k) {
  if (ds->done) return;
  double d[1];
  sum_parts<1>(partials + RR_OFF, nb, d);
  if (threadIdx.x == 0) converge_test(d[0], ds, hist, k);
}

// Partials of <R_{k+1}, S_{k+1}> over q x q (S = F(R)).
__global__ __launch_bounds__(TPB) void dot_kernel2(int q, const double *__restrict__ A,
                                                   const double *__restrict__ B, int64_t ldc,
                                                   double *partials, const DevState *ds) {
  if (ds->done) return;
  double v[1] = {0.0};
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      v[0] = fma(A[o], B[o], v[0]);
    }
  put_parts<1>(v, partials);
}

// rho_{k+1} = <R, S>, beta_k = rho_{k+1} / rho_k.
__global__ __launch_bounds__(TPB) void cr_beta_kernel(const double *partials, int nb,
                                                      DevState *ds, double *hist, int k,
                                                      int max_iter) {
  if (ds->done) return;
  double d[1];
  sum_parts<1>(partials, nb, d);
  if (threadIdx.x != 0) return;
  if (d[0] == 0.0 || !isfinite(d[0])) {
    halt(ds, SYLV_BREAKDOWN, k + 1);
    return;
  }
  ds->beta = d[0] / ds->rho;
  ds->rho = d[0];
  hist[2 * max_iter + k] = ds->beta;
}

// P = R + beta P, Q = S + beta Q over q x q, partials of <Q, Q>.
__global__ __launch_bounds__(TPB) void cr_pq_kernel(int q, const double *__restrict__ R,
                                                    const double *__restrict__ S,
                                                    double *__restrict__ P,
                                                    double *__restrict__ Q, int64_t ldc,
                                                    double *partials, const DevState *ds) {
  if (ds->done) return;
  const double beta = ds->beta;
  double v[1] = {0.0};
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      P[o] = fma(beta, P[o], R[o]);
      const double qv = fma(beta, Q[o], S[o]);
      Q[o] = qv;
      v[0] = fma(qv, qv, v[0]);
    }
  put_parts<1>(v, partials);
}

__global__ __launch_bounds__(TPB) void cr_qq_kernel(const double *partials, int nb,
                                                    DevState *ds) {
  if (ds->done) return;
  double d[1];
  sum_parts<1>(partials, nb, d);
  if (threadIdx.x == 0) ds->pq = d[0];
}

// ---- CGS and GPBiCG: alpha = rho / <R~0, Z(1:s, 1:s)> for Z = F(P) ----
__global__ void alpha_corner_kernel(int s, const double *Rt, const double *Z, int64_t ldc,
                                    DevState *ds, double *hist, int k, int max_iter) {
  if (ds->done || threadIdx.x != 0 || blockIdx.x != 0) return;
  const double den = corner_dot(s, Rt, Z, ldc);
  const double alpha = ds->rho / den;
  if (den == 0.0 || ds->rho == 0.0 || !isfinite(alpha)) {
    halt(ds, SYLV_BREAKDOWN, k);
    return;
  }
  ds->alpha = alpha;
  hist[max_iter + k] = alpha;
}

// ---- CGS ----
// Q = U - alpha V, Wk = U + Q, X += alpha Wk over q x q.
__global__ __launch_bounds__(TPB) void cgs_qwx_kernel(int q, const double *__restrict__ U,
                                                      const double *__restrict__ V,
                                                      double *__restrict__ Q,
                                                      double *__restrict__ Wk,
                                                      double *__restrict__ X, int64_t ldc,
                                                      const DevState *ds) {
  if (ds->done) return;
  const double alpha = ds->alpha;
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      const double u = U[o];
      const double qv = fma(-alpha, V[o], u);
      const double w = u + qv;
      Q[o] = qv;
      Wk[o] = w;
      X[o] = fma(alpha, w, X[o]);
    }
}

// R -= alpha F(Wk) over q x q, partials of ||R||^2.
__global__ __launch_bounds__(TPB) void axpy_rr_kernel(int q, const double *__restrict__ Z,
                                                      double *__restrict__ R, int64_t ldc,
                                                      double *partials, const DevState *ds) {
  if (ds->done) return;
  const double alpha = ds->alpha;
  double v[1] = {0.0};
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      const double r = fma(-alpha, Z[o], R[o]);
      R[o] = r;
      v[0] = fma(r, r, v[0]);
    }
  put_parts<1>(v, partials + RR_OFF);
}

// Stopping test, then rho_{k+1} = <R~0, R(1:s,1:s)> and beta_k = scale rho_{k+1} / rho_k with
// scale = 1 (CGS) or alpha / zeta (GPBiCG, zeta kept in ds->omega).
__global__ __launch_bounds__(TPB) void rho_beta_kernel(int s, const double *Rt, const double *R,
                                                       int64_t ldc, const double *partials,
                                                       int nb, int gp, DevState *ds,
                                                       double *hist, int k, int max_iter) {
  if (ds->done) return;
  double d[1];
  sum_parts<1>(partials + RR_OFF, nb, d);
  if (threadIdx.x != 0) return;
  if (!converge_test(d[0], ds, hist, k)) return;
  const double rn = corner_dot(s, Rt, R, ldc);
  if (rn == 0.0 || !isfinite(rn)) {
    halt(ds, SYLV_BREAKDOWN, k + 1);
    return;
  }
  const double beta = (gp ? ds->alpha / ds->omega : 1.0) * (rn / ds->rho);
  ds->beta = beta;
  ds->rho = rn;
  hist[2 * max_iter + k] = beta;
}

// U = R + beta Q, P = U + beta (Q + beta P) over q x q.
__global__ __launch_bounds__(TPB) void cgs_up_kernel(int q, const double *__restrict__ R,
                                                     const double *__restrict__ Q,
                                                     double *__restrict__ U,
                                                     double *__restrict__ P, int64_t ldc,
                                                     const DevState *ds) {
  if (ds->done) return;
  const double beta = ds->beta;
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      const double qv = Q[o];
      const double u = fma(beta, qv, R[o]);
      U[o] = u;
      P[o] = fma(beta, fma(beta, P[o], qv), u);
    }
}

// ---- GPBiCG ----
// p_k = r_k + beta_{k-1} (p_{k-1} - u_{k-1}) over q x q (beta = 0 and u = 0 at k = 0).
__global__ __launch_bounds__(TPB) void gp_p_kernel(int q, const double *__restrict__ R,
                                                   const double *__restrict__ U,
                                                   double *__restrict__ P, int64_t ldc,
                                                   const DevState *ds) {
  if (ds->done) return;
  const double beta = ds->beta;
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      P[o] = fma(beta, P[o] - U[o], R[o]);
    }
}

// y_k = t_{k-1} - r_k - alpha w_{k-1} + alpha F(p_k), t_k = r_k - alpha F(p_k) over q x q.
__global__ __launch_bounds__(TPB) void gp_yt_kernel(int q, const double *__restrict__ Tm,
                                                    const double *__restrict__ R,
                                                    const double *__restrict__ Wv,
                                                    const double *__restrict__ AP,
                                                    double *__restrict__ Y,
                                                    double *__restrict__ T, int64_t ldc,
                                                    const DevState *ds) {
  if (ds->done) return;
  const double alpha = ds->alpha;
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      const double r = R[o], ap = AP[o];
      Y[o] = fma(alpha, ap - Wv[o], Tm[o] - r);
      T[o] = fma(-alpha, ap, r);
    }
}

// Partials of <Ft, Ft>, <y, y>, <Ft, y>, <y, t>, <Ft, t> over q x q (Ft = F(t_k)).
__global__ __launch_bounds__(TPB) void gp_dots_kernel(int q, const double *__restrict__ AT,
                                                      const double *__restrict__ Y,
                                                      const double *__restrict__ T, int64_t ldc,
                                                      double *partials, const DevState *ds) {
  if (ds->done) return;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      const double a = AT[o], y = Y[o], t = T[o];
      v[0] = fma(a, a, v[0]);
      v[1] = fma(y, y, v[1]);
      v[2] = fma(a, y, v[2]);
      v[3] = fma(y, t, v[3]);
      v[4] = fma(a, t, v[4]);
    }
  put_parts<5>(v, partials);
}

// zeta_k, eta_k: minimizers of ||t - eta y - zeta F(t)|| (eta = 0 on the first iteration).
__global__ __launch_bounds__(TPB) void gp_zeta_kernel(const double *partials, int nb, int first,
                                                      DevState *ds, double *hist, int k,
                                                      int max_iter) {
  if (ds->done) return;
  double d[5];
  sum_parts<5>(partials, nb, d);
  if (threadIdx.x != 0) return;
  const double tt = d[0], yy = d[1], ty = d[2], yt = d[3], ts = d[4];
  double zeta, eta;
  if (first) {
    zeta = ts / tt;
    eta = 0.0;
  } else {
    const double den = tt * yy - ty * ty;
    zeta = (yy * ts - yt * ty) / den;
    eta = (tt * yt - ty * ts) / den;
  }
  if (zeta == 0.0 || !isfinite(zeta) || !isfinite(eta)) {
    halt(ds, SYLV_BREAKDOWN, k);
    return;
  }
  ds->omega = zeta;
  ds->eta = eta;
  hist[3 * max_iter + k] = zeta;
}

// u_k = zeta F(p) + eta (t_{k-1} - r_k + beta u_{k-1}), z_k = zeta r_k + eta z_{k-1} - alpha u_k,
// x += alpha p_k + z_k, r_{k+1} = t_k - eta y_k - zeta F(t_k), over q x q; partials of
// ||r_{k+1}||^2.
__global__ __launch_bounds__(TPB) void gp_update_kernel(
    int q, const double *__restrict__ AP, const double *__restrict__ Tm,
    const double *__restrict__ P, const double *__restrict__ T, const double *__restrict__ Y,
    const double *__restrict__ AT, double *__restrict__ R, double *__restrict__ U,
    double *__restrict__ Z, double *__restrict__ X, int64_t ldc, double *partials,
    const DevState *ds) {
  if (ds->done) return;
  const double alpha = ds->alpha, zeta = ds->omega, eta = ds->eta, beta = ds->beta;
  double v[1] = {0.0};
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      const double r = R[o];
      const double u = fma(zeta, AP[o], eta * fma(beta, U[o], Tm[o] - r));
      const double z = fma(-alpha, u, fma(zeta, r, eta * Z[o]));
      U[o] = u;
      Z[o] = z;
      X[o] = X[o] + fma(alpha, P[o], z);
      const double rn = fma(-zeta, AT[o], fma(-eta, Y[o], T[o]));
      R[o] = rn;
      v[0] = fma(rn, rn, v[0]);
    }
  put_parts<1>(v, partials + RR_OFF);
}

// w_k = F(t_k) + beta_k F(p_k) over q x q.
__global__ __launch_bounds__(TPB) void gp_w_kernel(int q, const double *__restrict__ AT,
                                                   const double *__restrict__ AP,
                                                   double *__restrict__ Wv, int64_t ldc,
                                                   const DevState *ds) {
  if (ds->done) return;
  const double beta = ds->beta;
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      Wv[o] = fma(beta, AP[o], AT[o]);
    }
}

}  // namespace

#define LAUNCH(kern, grid, ...)                       \
  do {                                                \
    kern<<<(grid), TPB, 0, st>>>(__VA_ARGS__);        \
    HIPOK(hipGetLastError());                         \
  } while (0)

int launch_cr_init(int q, const double *R, const double *S, double *Q, int64_t ldc,
                   const Scratch &sc, DevState *ds, hipStream_t st) {
  const unsigned g = grid_of(q);
  LAUNCH(cr_init_kernel, g, q, R, S, Q, ldc, sc.partials);
  LAUNCH(cr_init_scalar_kernel, 1, sc.partials, (int)g, ds);
  return 0;
}

int launch_cr_xr(int q, double *X, double *R, const double *P, const double *Q, int64_t ldc,
                 const Scratch &sc, DevState *ds, double *hist, int k, int max_iter,
                 hipStream_t st) {
  const unsigned g = grid_of(q);
  LAUNCH(cr_xr_kernel, g, q, X, R, P, Q, ldc, sc.partials, ds, hist, k, max_iter);
  LAUNCH(rr_converge_kernel, 1, sc.partials, (int)g, ds, hist, k);
  return 0;
}

int launch_cr_beta_pq(int q, const double *R, const double *S, double *P, double *Q,
                      int64_t ldc, const Scratch &sc, DevState *ds, double *hist, int k,
                      int max_iter, hipStream_t st) {
  const unsigned g = grid_of(q);
  LAUNCH(dot_kernel2, g, q, R, S, ldc, sc.partials, ds);
  LAUNCH(cr_beta_kernel, 1, sc.partials, (int)g, ds, hist, k, max_iter);
  LAUNCH(cr_pq_kernel, g, q, R, S, P, Q, ldc, sc.partials, ds);
  LAUNCH(cr_qq_kernel, 1, sc.partials, (int)g, ds);
  return 0;
}

int launch_alpha_corner(int s, const double *Rt, const double *Z, int64_t ldc, DevState *ds,
                        double *hist, int k, int max_iter, hipStream_t st) {
  alpha_corner_kernel<<<1, 64, 0, st>>>(s, Rt, Z, ldc, ds, hist, k, max_iter);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_cgs_qwx(int q, const double *U, const double *V, double *Q, double *Wk, double *X,
                   int64_t ldc, DevState *ds, hipStream_t st) {
  LAUNCH(cgs_qwx_kernel, grid_of(q), q, U, V, Q, Wk, X, ldc, ds);
  return 0;
}

int launch_axpy_rho_beta(int s, int q, const double *Z, double *R, const double *Rt, int64_t ldc,
                         bool gpbicg, const Scratch &sc, DevState *ds, double *hist, int k,
                         int max_iter, hipStream_t st) {
  const unsigned g = grid_of(q);
  if (!gpbicg) LAUNCH(axpy_rr_kernel, g, q, Z, R, ldc, sc.partials, ds);
  LAUNCH(rho_beta_kernel, 1, s, Rt, R, ldc, sc.partials, (int)g, gpbicg ? 1 : 0, ds, hist, k,
         max_iter);
  return 0;
}

int launch_cgs_up(int q, const double *R, const double *Q, double *U, double *P, int64_t ldc,
                  DevState *ds, hipStream_t st) {
  LAUNCH(cgs_up_kernel, grid_of(q), q, R, Q, U, P, ldc, ds);
  return 0;
}

int launch_gp_p(int q, const double *R, const double *U, double *P, int64_t ldc, DevState *ds,
                hipStream_t st) {
  LAUNCH(gp_p_kernel, grid_of(q), q, R, U, P, ldc, ds);
  return 0;
}

int launch_gp_yt(int q, const double *Tm, const double *R, const double *Wv, const double *AP,
                 double *Y, double *T, int64_t ldc, DevState *ds, hipStream_t st) {
  LAUNCH(gp_yt_kernel, grid_of(q), q, Tm, R, Wv, AP, Y, T, ldc, ds);
  return 0;
}

int launch_gp_zeta(int q, const double *AT, const double *Y, const double *T, int64_t ldc,
                   bool first, const Scratch &sc, DevState *ds, double *hist, int k, int max_iter,
                   hipStream_t st) {
  const unsigned g = grid_of(q);
  LAUNCH(gp_dots_kernel, g, q, AT, Y, T, ldc, sc.partials, ds);
  LAUNCH(gp_zeta_kernel, 1, sc.partials, (int)g, first ? 1 : 0, ds, hist, k, max_iter);
  return 0;
}

int launch_gp_update(int q, const double *AP, const double *Tm, const double *P, const double *T,
                     const double *Y, const double *AT, double *R, double *U, double *Z,
                     double *X, int64_t ldc, const Scratch &sc, DevState *ds, hipStream_t st) {
  LAUNCH(gp_update_kernel, grid_of(q), q, AP, Tm, P, T, Y, AT, R, U, Z, X, ldc, sc.partials, ds);
  return 0;
}

int launch_gp_w(int q, const double *AT, const double *AP, double *Wv, int64_t ldc, DevState *ds,
                hipStream_t st) {
  LAUNCH(gp_w_kernel, grid_of(q), q, AT, AP, Wv, ldc, ds);
  return 0;
}

int more_grid(int q) { return (int)grid_of(q); }
