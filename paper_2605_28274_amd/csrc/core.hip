// Core recurrences of factorized CG (Algorithm 4.1) and factorized BiCGSTAB (Algorithm 4.2).
//
// Cores are dense row-major ldc x ldc FP64 buffers that are zero at the start of a solve. A
// core of the current size r occupies the upper-left r x r corner and every entry outside it
// is an exact zero; sizes only grow, so the block padding of the algorithms ([Z 0; 0 0]) is
// implicit and kernels may read beyond the active corner. Scalars (rho, alpha, beta, omega)
// live in DevState and are produced by the last workgroup of the reduction that needs them.
#include "common.h"

namespace {

constexpr int TPB = 256;


__global__ void setup_scalars_kernel(int s, const double *RL, const double *RR, double *R,
                                     double *P, double *Rt, int64_t ldc, double tol,
                                     DevState *ds) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  // R0 = R_L R_R^T (Alg. 4.1 step 2, Alg. 4.2 step 3)
  double nrm = 0.0;
  for (int a = 0; a < s; ++a)
    for (int b = 0; b < s; ++b) {
      double v = 0.0;
      for (int c = 0; c < s; ++c) v += RL[a * s + c] * RR[b * s + c];
      R[a * ldc + b] = v;
      P[a * ldc + b] = v;
      Rt[a * s + b] = v;
      nrm += v * v;
    }
  ds->rho = nrm;  // <R0, R0> for CG, <R~0, R0> = <R0, R0> for BiCGSTAB
  ds->rho_next = 0.0;
  ds->alpha = ds->omega = ds->beta = 0.0;
  ds->normR0 = sqrt(nrm);
  ds->tol = tol;
  ds->relres = 1.0;
  ds->done = 0;
  ds->status = 0;
  ds->iters = 0;
  ds->rho_zero = 0;
}

__device__ __forceinline__ void stop(DevState *ds, int status, int iters) {
  ds->status = status;
  ds->iters = iters;
  ds->done = 1;
}

// ---- CG (block-tridiagonal H and G from block Lanczos) ----

// Q = [H P, 0] + [P G^T; 0] over (p+s)^2 using the band |blk(i) - blk(l)| <= 1 of H and G;
// reduces <P, Q(1:p, 1:p)>; last workgroup: alpha = rho / <P, Q>.
template <int S>
__global__ __launch_bounds__(TPB) void cg_core_kernel(int p, const double *__restrict__ H,
                                                      const double *__restrict__ G,
                                                      const double *__restrict__ P,
                                                      double *__restrict__ Q, int64_t ldc,
                                                      double *partials, int *counter,
                                                      DevState *ds, double *hist, int k,
                                                      int max_iter) {
  if (ds->done) return;
  const int q = p + S;
  double v[1] = {0.0};
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < (int64_t)q * q;
       e += (int64_t)gridDim.x * TPB) {
    const int i = (int)(e / q), j = (int)(e % q);
    double acc = 0.0;
    if (j < p) {
      const int bi = i / S;
      const int l0 = bi > 0 ? (bi - 1) * S : 0;
      const int l1 = (bi + 2) * S < p ? (bi + 2) * S : p;
      for (int l = l0; l < l1; ++l) acc = fma(H[(int64_t)i * ldc + l], P[(int64_t)l * ldc + j], acc);
    }
    if (i < p) {
      const int bj = j / S;
      const int l0 = bj > 0 ? (bj - 1) * S : 0;
      const int l1 = (bj + 2) * S < p ? (bj + 2) * S : p;
      for (int l = l0; l < l1; ++l) acc = fma(P[(int64_t)i * ldc + l], G[(int64_t)j * ldc + l], acc);
    }
    Q[(int64_t)i * ldc + j] = acc;
    if (i < p && j < p) v[0] = fma(P[(int64_t)i * ldc + j], acc, v[0]);
  }
  __shared__ double out[1];
  if (reduce_grid<1>(v, partials, counter, out) && threadIdx.x == 0) {
    const double pq = out[0];
    ds->pq = pq;
    if (!(pq > 0.0) || !isfinite(pq)) {
      stop(ds, SYLV_BREAKDOWN, k);
      return;
    }
    ds->alpha = ds->rho / pq;
    hist[max_iter + k] = ds->alpha;
  }
}

// X += alpha P (p x p), R = R - alpha Q ((p+s)^2), ||R||^2; last workgroup: convergence test,
// rho_{k+1} and beta.
__global__ __launch_bounds__(TPB) void cg_update_kernel(int p, int q, double *__restrict__ X,
                                                        double *__restrict__ R,
                                                        const double *__restrict__ P,
                                                        const double *__restrict__ Q, int64_t ldc,
                                                        double *partials, int *counter,
                                                        DevState *ds, double *hist, int k,
                                                        int max_iter) {
  if (ds->done) return;
  const double alpha = ds->alpha;
  double v[1] = {0.0};
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < (int64_t)q * q;
       e += (int64_t)gridDim.x * TPB) {
    const int i = (int)(e / q), j = (int)(e % q);
    const int64_t o = (int64_t)i * ldc + j;
    if (i < p && j < p) X[o] = fma(alpha, P[o], X[o]);
    const double r = fma(-alpha, Q[o], R[o]);
    R[o] = r;
    v[0] = fma(r, r, v[0]);
  }
  __shared__ double out[1];
  if (reduce_grid<1>(v, partials, counter, out) && threadIdx.x == 0) {
    const double rr = out[0];
    const double rel = sqrt(rr) / ds->normR0;
    ds->relres = rel;
    hist[k] = rel;
    if (rel <= ds->tol) {
      stop(ds, SYLV_OK, k + 1);
      return;
    }
    ds->beta = rr / ds->rho;
    ds->rho = rr;
    hist[2 * max_iter + k] = ds->beta;
  }
}

// P = R + beta P over (p+s)^2.
__global__ __launch_bounds__(TPB) void cg_p_kernel(int q, const double *__restrict__ R,
                                                   double *__restrict__ P, int64_t ldc,
                                                   const DevState *ds) {
  if (ds->done) return;
  const double beta = ds->beta;
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < (int64_t)q * q;
       e += (int64_t)gridDim.x * TPB) {
    const int64_t o = (e / q) * ldc + e % q;
    P[o] = fma(beta, P[o], R[o]);
  }
}

// ---- BiCGSTAB (dense block Hessenberg H and G from block Arnoldi) ----

// alpha = rho / <R~0, Q(1:s,1:s)> (every workgroup forms it from the s x s corner), then
// S = [R 0; 0 0] - alpha Q over (p+s)^2.
__global__ __launch_bounds__(TPB) void bicg_s_kernel(int s, int q, const double *__restrict__ Q,
                                                     const double *__restrict__ R,
                                                     double *__restrict__ S,
                                                     const double *__restrict__ Rt, int64_t ldc,
                                                     DevState *ds, double *hist, int k,
                                                     int max_iter) {
  if (ds->done) return;
  double den = 0.0;
  for (int a = 0; a < s; ++a)
    for (int b = 0; b < s; ++b) den = fma(Rt[a * s + b], Q[(int64_t)a * ldc + b], den);
  const double alpha = ds->rho / den;
  if (den == 0.0 || !isfinite(alpha)) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) stop(ds, SYLV_BREAKDOWN, k);
    return;
  }
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    ds->alpha = alpha;
    hist[max_iter + k] = alpha;
  }
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < (int64_t)q * q;
       e += (int64_t)gridDim.x * TPB) {
    const int64_t o = (e / q) * ldc + e % q;
    S[o] = fma(-alpha, Q[o], R[o]);
  }
}

// <T, S> and <T, T> over (p+2s)^2; last workgroup: omega, rho_{k+1} = <R~0, R_{k+1}(1:s,1:s)>
// with R_{k+1}(1:s,1:s) = S(1:s,1:s) - omega T(1:s,1:s), and beta.
__global__ __launch_bounds__(TPB) void bicg_omega_kernel(int s, int q, const double *__restrict__ T,
                                                         const double *__restrict__ S,
                                                         const double *__restrict__ Rt,
                                                         int64_t ldc, double *partials,
                                                         int *counter, DevState *ds, double *hist,
                                                         int k, int max_iter) {
  if (ds->done) return;
  double v[2] = {0.0, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < (int64_t)q * q;
       e += (int64_t)gridDim.x * TPB) {
    const int64_t o = (e / q) * ldc + e % q;
    const double t = T[o];
    v[0] = fma(t, S[o], v[0]);
    v[1] = fma(t, t, v[1]);
  }
  __shared__ double out[2];
  if (reduce_grid<2>(v, partials, counter, out) && threadIdx.x == 0) {
    const double ts = out[0], tt = out[1];
    ds->ts = ts;
    ds->tt = tt;
    if (!(tt > 0.0) || !isfinite(tt)) {
      stop(ds, SYLV_BREAKDOWN, k);
      return;
    }
    const double omega = ts / tt;
    if (omega == 0.0 || !isfinite(omega)) {
      stop(ds, SYLV_BREAKDOWN, k);
      return;
    }
    double rn = 0.0;
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) {
        const int64_t o = (int64_t)a * ldc + b;
        rn = fma(Rt[a * s + b], fma(-omega, T[o], S[o]), rn);
      }
    ds->omega = omega;
    ds->rho_next = rn;
    ds->rho_zero = (rn == 0.0);
    ds->beta = (ds->alpha / omega) * (rn / ds->rho);
    hist[3 * max_iter + k] = omega;
  }
}

// X += alpha P + omega S; R = S - omega T; P = R + beta (P - omega Q) over (p+2s)^2 (old X is
// zero beyond 2ks, P beyond p, Q and S beyond p+s); ||R||^2 and the convergence test.
__global__ __launch_bounds__(TPB) void bicg_update_kernel(int q, double *__restrict__ X,
                                                          double *__restrict__ R,
                                                          double *__restrict__ P,
                                                          const double *__restrict__ Q,
                                                          const double *__restrict__ S,
                                                          const double *__restrict__ T,
                                                          int64_t ldc, double *partials,
                                                          int *counter, DevState *ds,
                                                          double *hist, int k, int max_iter) {
  if (ds->done) return;
  const double alpha = ds->alpha, omega = ds->omega, beta = ds->beta;
  double v[1] = {0.0};
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < (int64_t)q * q;
       e += (int64_t)gridDim.x * TPB) {
    const int64_t o = (e / q) * ldc + e % q;
    const double sv = S[o], pv = P[o];
    X[o] = fma(omega, sv, fma(alpha, pv, X[o]));
    const double r = fma(-omega, T[o], sv);
    R[o] = r;
    P[o] = fma(beta, fma(-omega, Q[o], pv), r);
    v[0] = fma(r, r, v[0]);
  }
  __shared__ double out[1];
  if (reduce_grid<1>(v, partials, counter, out) && threadIdx.x == 0) {
    const double rel = sqrt(out[0]) / ds->normR0;
    ds->relres = rel;
    hist[k] = rel;
    if (rel <= ds->tol) {
      stop(ds, SYLV_OK, k + 1);
      return;
    }
    if (ds->rho_zero) {
      stop(ds, SYLV_BREAKDOWN, k + 1);
      return;
    }
    ds->rho = ds->rho_next;
    hist[2 * max_iter + k] = ds->beta;
  }
}

// 1D grid-stride launch over a q x q region: at most 1024 workgroups of 256 threads.
dim3 grid_sq(int q) {
  const int64_t g = ((int64_t)q * q + TPB - 1) / TPB;
  return dim3((unsigned)(g < 1024 ? (g < 1 ? 1 : g) : 1024));
}

}  // namespace

int launch_setup_scalars(int s, const double *RL, const double *RR, double *R, double *P,
                         double *Rt, int64_t ldc, double tol, DevState *ds, hipStream_t st) {
  setup_scalars_kernel<<<1, 64, 0, st>>>(s, RL, RR, R, P, Rt, ldc, tol, ds);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_cg_core(int s, int p, const double *H, const double *G, const double *P, double *Q,
                   int64_t ldc, const Scratch &sc, DevState *ds, double *hist, int k,
                   int max_iter, hipStream_t st) {
  const dim3 g = grid_sq(p + s);
  switch (s) {
#define CASE(SS)                                                                               \
  case SS:                                                                                     \
    cg_core_kernel<SS><<<g, TPB, 0, st>>>(p, H, G, P, Q, ldc, sc.partials,                     \
                                          sc.counters + CNT_CORE, ds, hist, k, max_iter);      \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return SYLV_ERR_INVALID;
  }
  HIPOK(hipGetLastError());
  return 0;
}

int launch_cg_update(int s, int p, double *X, double *R, double *P, const double *Q, int64_t ldc,
                     const Scratch &sc, DevState *ds, double *hist, int k, int max_iter,
                     hipStream_t st) {
  const int q = p + s;
  cg_update_kernel<<<grid_sq(q), TPB, 0, st>>>(p, q, X, R, P, Q, ldc, sc.partials,
                                               sc.counters + CNT_ELEM, ds, hist, k, max_iter);
  HIPOK(hipGetLastError());
  cg_p_kernel<<<grid_sq(q), TPB, 0, st>>>(q, R, P, ldc, ds);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_bicg_s(int s, int p, const double *Q, const double *R, double *S, const double *Rt,
                   int64_t ldc, DevState *ds, double *hist, int k, int max_iter, hipStream_t st) {
  const int q = p + s;
  bicg_s_kernel<<<grid_sq(q), TPB, 0, st>>>(s, q, Q, R, S, Rt, ldc, ds, hist, k, max_iter);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_bicg_omega(int s, int p, const double *T, const double *S, const double *Rt,
                      int64_t ldc, const Scratch &sc, DevState *ds, double *hist, int k,
                      int max_iter, hipStream_t st) {
  const int q = p + 2 * s;
  bicg_omega_kernel<<<grid_sq(q), TPB, 0, st>>>(s, q, T, S, Rt, ldc, sc.partials,
                                                sc.counters + CNT_CORE + 1, ds, hist, k,
                                                max_iter);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_bicg_update(int s, int p, double *X, double *R, double *P, const double *Q,
                        const double *S, const double *T, int64_t ldc, const Scratch &sc,
                        DevState *ds, double *hist, int k, int max_iter, hipStream_t st) {
  const int q = p + 2 * s;
  bicg_update_kernel<<<grid_sq(q), TPB, 0, st>>>(q, X, R, P, Q, S, T, ldc, sc.partials,
                                                 sc.counters + CNT_ELEM, ds, hist, k, max_iter);
  HIPOK(hipGetLastError());
  return 0;
}
