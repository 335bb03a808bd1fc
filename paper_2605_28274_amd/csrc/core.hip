// Core recurrences of factorized CG (Algorithm 4.1) and factorized BiCGSTAB (Algorithm 4.2).
//
// Cores are dense row-major ldc x ldc FP64 buffers that are zero at the start of a solve. A
// core of the current size r occupies the upper-left r x r corner and every entry outside it
// is an exact zero; sizes only grow, so the block padding of the algorithms ([Z 0; 0 0]) is
// implicit and kernels may read beyond the active corner.
//
// Reductions: a kernel that produces an inner product writes one partial per workgroup; the
// kernel that consumes the scalar re-sums those partials in every workgroup, in a fixed order
// (identical result everywhere, deterministic), after the kernel boundary made them visible.
// This avoids a device-wide release fence per workgroup, which on a multi-XCD GPU writes back
// the L2. Scalars (rho, alpha, beta, omega) live in DevState; workgroup 0 records them.
#include "common.h"

namespace {

constexpr int TPB = 256;
constexpr int NBLK = 512;  // workgroups of the elementwise core kernels (and their partials)

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

// Writes this workgroup's NV block sums to partials[blockIdx.x * NV + i].
template <int NV>
__device__ __forceinline__ void put_partials(double (&v)[NV], double *partials) {
  __shared__ double lds[16 * NV];
  block_sum<NV>(v, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) partials[(size_t)blockIdx.x * NV + i] = v[i];
}

// Sums nb partial records of NV values in a fixed order; the result is returned to every
// thread (all threads must call).
template <int NV>
__device__ __forceinline__ void sum_partials(const double *partials, int nb, double (&out)[NV]) {
  __shared__ double lds[16 * NV];
  __shared__ double res[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) out[i] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] += partials[(size_t)b * NV + i];
  block_sum<NV>(out, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) res[i] = out[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) out[i] = res[i];
}

// ---- CG (block-tridiagonal H and G from block Lanczos) ----

// Q = [H P, 0] + [P G^T; 0] over (p+s)^2 using the band |blk(i) - blk(l)| <= 1 of H and G;
// partials of <P, Q(1:p, 1:p)>. Workgroup b owns 256 columns (b % gx) and the row groups
// b / gx, b / gx + gy, ... of CG_ROWS rows; thread j keeps row j's band of G in registers, and
// the band loops have fixed length 3S (masked), so CG_UNR rows are in flight at once.
constexpr int CG_ROWS = 16, CG_UNR = 4, CG_MAXWG = 4096;

template <int S>
__global__ __launch_bounds__(TPB) void cg_core_kernel(int p, int gx, int gy,
                                                      const double *__restrict__ H,
                                                      const double *__restrict__ G,
                                                      const double *__restrict__ P,
                                                      double *__restrict__ Q, int64_t ldc,
                                                      double *partials, const DevState *ds) {
  if (ds->done) return;
  const int q = p + S;
  const int cx = (int)blockIdx.x % gx, ry = (int)blockIdx.x / gx;
  const int j = cx * TPB + threadIdx.x;
  const bool jl = j < q;
  const int jc = jl ? j : q - 1;  // clamped column for loads
  const int bj = jc / S;
  const int l0 = bj > 0 ? (bj - 1) * S : 0;
  const int l1 = (bj + 2) * S < p ? (bj + 2) * S : p;
  double gb[3 * S];
#pragma unroll
  for (int t = 0; t < 3 * S; ++t) gb[t] = (l0 + t < l1) ? G[(int64_t)jc * ldc + l0 + t] : 0.0;
  double v[1] = {0.0};
  for (int i0 = ry * CG_ROWS; i0 < q; i0 += gy * CG_ROWS) {
#pragma unroll
    for (int u0 = 0; u0 < CG_ROWS; u0 += CG_UNR) {
      double acc[CG_UNR], pij[CG_UNR];
#pragma unroll
      for (int u = 0; u < CG_UNR; ++u) {
        const int i = i0 + u0 + u;
        const int ic = i < q ? i : q - 1;
        const int bi = ic / S;
        const int li0 = bi > 0 ? (bi - 1) * S : 0;
        double a = 0.0;
        // H P: row i of H meets rows li0 .. li0 + 3S of P (masked at p)
#pragma unroll
        for (int t = 0; t < 3 * S; ++t) {
          const int l = li0 + t;
          const bool in = (l < p) && (j < p);
          const double h = in ? H[(int64_t)ic * ldc + l] : 0.0;
          const double pv = in ? P[(int64_t)l * ldc + jc] : 0.0;
          a = fma(h, pv, a);
        }
        // P G^T: row i of P meets the band of row j of G (zero past p)
        if (ic < p) {
          const double *pr = P + (int64_t)ic * ldc + l0;
#pragma unroll
          for (int t = 0; t < 3 * S; ++t) a = fma((l0 + t < l1) ? pr[t] : 0.0, gb[t], a);
        }
        acc[u] = a;
        pij[u] = P[(int64_t)ic * ldc + jc];
      }
#pragma unroll
      for (int u = 0; u < CG_UNR; ++u) {
        const int i = i0 + u0 + u;
        if (i < q && jl) {
          Q[(int64_t)i * ldc + j] = acc[u];
          if (i < p && j < p) v[0] = fma(pij[u], acc[u], v[0]);
        }
      }
    }
  }
  put_partials<1>(v, partials);
}

// Grid of cg_core_kernel for a (p+s)^2 core: gx column chunks x gy row-group strides, at most
// CG_MAXWG workgroups (the consumer sums one partial per workgroup).
void cg_core_grid(int q, int &gx, int &gy) {
  gx = (q + TPB - 1) / TPB;
  const int groups = (q + CG_ROWS - 1) / CG_ROWS;
  gy = std::max(1, std::min(CG_MAXWG / gx, groups));
}

// alpha = rho / <P, Q> from cg_core's partials (breakdown when <P, Q> <= 0);
// X += alpha P (p x p), R = R - alpha Q ((p+s)^2); partials of ||R||^2.
__global__ __launch_bounds__(TPB) void cg_update_kernel(int p, int q, double *__restrict__ X,
                                                        double *__restrict__ R,
                                                        const double *__restrict__ P,
                                                        const double *__restrict__ Q, int64_t ldc,
                                                        const double *pq_part, int pq_nb,
                                                        double *partials, DevState *ds,
                                                        double *hist, int k, int max_iter) {
  if (ds->done) return;
  double pq[1];
  sum_partials<1>(pq_part, pq_nb, pq);
  if (!(pq[0] > 0.0) || !isfinite(pq[0])) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ds->pq = pq[0];
      stop(ds, SYLV_BREAKDOWN, k);
    }
    return;
  }
  const double alpha = ds->rho / pq[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ds->pq = pq[0];
    ds->alpha = alpha;
    hist[max_iter + k] = alpha;
  }
  double v[1] = {0.0};
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      if (i < p && j < p) X[o] = fma(alpha, P[o], X[o]);
      const double r = fma(-alpha, Q[o], R[o]);
      R[o] = r;
      v[0] = fma(r, r, v[0]);
    }
  put_partials<1>(v, partials);
}

// One workgroup: ||R_{k+1}|| / ||R_0|| from the partials, the stopping test, rho_{k+1} and
// beta_k (CG).
__global__ __launch_bounds__(TPB) void cg_converge_kernel(const double *rr_part, int nb,
                                                          DevState *ds, double *hist, int k,
                                                          int max_iter) {
  if (ds->done) return;
  double rr[1];
  sum_partials<1>(rr_part, nb, rr);
  if (threadIdx.x != 0) return;
  const double rel = sqrt(rr[0]) / ds->normR0;
  ds->relres = rel;
  hist[k] = rel;
  if (rel <= ds->tol) {
    stop(ds, SYLV_OK, k + 1);
    return;
  }
  ds->beta = rr[0] / ds->rho;
  ds->rho = rr[0];
  hist[2 * max_iter + k] = ds->beta;
}

// P = R + beta P over (p+s)^2.
__global__ __launch_bounds__(TPB) void cg_p_kernel(int q, const double *__restrict__ R,
                                                   double *__restrict__ P, int64_t ldc,
                                                   const DevState *ds) {
  if (ds->done) return;
  const double beta = ds->beta;
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
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
    if (blockIdx.x == 0 && threadIdx.x == 0) stop(ds, SYLV_BREAKDOWN, k);
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ds->alpha = alpha;
    hist[max_iter + k] = alpha;
  }
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      S[o] = fma(-alpha, Q[o], R[o]);
    }
}

// Partials of <T, S> and <T, T> over (p+2s)^2 (S is zero beyond p+s, so <T, S> is the
// inner product with T(1:(2k+2)s, 1:(2k+2)s) of Alg. 4.2 step 13).
__global__ __launch_bounds__(TPB) void bicg_omega_kernel(int q, const double *__restrict__ T,
                                                         const double *__restrict__ S,
                                                         int64_t ldc, double *partials,
                                                         const DevState *ds) {
  if (ds->done) return;
  double v[2] = {0.0, 0.0};
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      const double t = T[o];
      v[0] = fma(t, S[o], v[0]);
      v[1] = fma(t, t, v[1]);
    }
  put_partials<2>(v, partials);
}

// omega = <T, S> / <T, T>, rho_{k+1} = <R~0, S(1:s,1:s) - omega T(1:s,1:s)> and
// beta = (alpha / omega)(rho_{k+1} / rho_k), formed in every workgroup from the partials; then
// X += alpha P + omega S; R = S - omega T; P = R + beta (P - omega Q) over (p+2s)^2 (old X is
// zero beyond 2ks, P beyond p, Q and S beyond p+s); partials of ||R||^2.
__global__ __launch_bounds__(TPB) void bicg_update_kernel(int s, int q, double *__restrict__ X,
                                                          double *__restrict__ R,
                                                          double *__restrict__ P,
                                                          const double *__restrict__ Q,
                                                          const double *__restrict__ S,
                                                          const double *__restrict__ T,
                                                          const double *__restrict__ Rt,
                                                          int64_t ldc, const double *om_part,
                                                          int om_nb, double *partials,
                                                          DevState *ds, double *hist, int k,
                                                          int max_iter) {
  if (ds->done) return;
  double ts_tt[2];
  sum_partials<2>(om_part, om_nb, ts_tt);
  const double ts = ts_tt[0], tt = ts_tt[1];
  const double omega = ts / tt;
  if (!(tt > 0.0) || !isfinite(tt) || omega == 0.0 || !isfinite(omega)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ds->ts = ts;
      ds->tt = tt;
      stop(ds, SYLV_BREAKDOWN, k);
    }
    return;
  }
  double rn = 0.0;
  for (int a = 0; a < s; ++a)
    for (int b = 0; b < s; ++b) {
      const int64_t o = (int64_t)a * ldc + b;
      rn = fma(Rt[a * s + b], fma(-omega, T[o], S[o]), rn);
    }
  const double alpha = ds->alpha;
  const double beta = (alpha / omega) * (rn / ds->rho);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ds->ts = ts;
    ds->tt = tt;
    ds->omega = omega;
    ds->rho_next = rn;
    ds->rho_zero = (rn == 0.0);
    ds->beta = beta;
    hist[3 * max_iter + k] = omega;
  }
  double v[1] = {0.0};
  for (int i = blockIdx.x; i < q; i += gridDim.x)
    for (int j = threadIdx.x; j < q; j += TPB) {
      const int64_t o = (int64_t)i * ldc + j;
      const double sv = S[o], pv = P[o];
      X[o] = fma(omega, sv, fma(alpha, pv, X[o]));
      const double r = fma(-omega, T[o], sv);
      R[o] = r;
      P[o] = fma(beta, fma(-omega, Q[o], pv), r);
      v[0] = fma(r, r, v[0]);
    }
  put_partials<1>(v, partials);
}

// One workgroup: relative residual, stopping test, breakdown on rho_{k+1} = 0, rho update.
__global__ __launch_bounds__(TPB) void bicg_converge_kernel(const double *rr_part, int nb,
                                                            DevState *ds, double *hist, int k,
                                                            int max_iter) {
  if (ds->done) return;
  double rr[1];
  sum_partials<1>(rr_part, nb, rr);
  if (threadIdx.x != 0) return;
  const double rel = sqrt(rr[0]) / ds->normR0;
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

unsigned grid_q(int q) { return (unsigned)(q < NBLK ? (q < 1 ? 1 : q) : NBLK); }

}  // namespace

int launch_setup_scalars(int s, const double *RL, const double *RR, double *R, double *P,
                         double *Rt, int64_t ldc, double tol, DevState *ds, hipStream_t st) {
  setup_scalars_kernel<<<1, 64, 0, st>>>(s, RL, RR, R, P, Rt, ldc, tol, ds);
  HIPOK(hipGetLastError());
  return 0;
}

// Scratch::partials layout: [0, 2*NBLK) partials of the scalar being formed (<P,Q>: up to
// CG_MAXWG; <T,S>, <T,T>); [2*NBLK, 3*NBLK) the ||R||^2 partials (CG: from CG_MAXWG).
int launch_cg_core(int s, int p, const double *H, const double *G, const double *P, double *Q,
                   int64_t ldc, const Scratch &sc, DevState *ds, hipStream_t st) {
  int gx, gy;
  cg_core_grid(p + s, gx, gy);
  const unsigned g = (unsigned)(gx * gy);
  switch (s) {
#define CASE(SS)                                                                             \
  case SS:                                                                                   \
    cg_core_kernel<SS><<<g, TPB, 0, st>>>(p, gx, gy, H, G, P, Q, ldc, sc.partials, ds);      \
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
  const unsigned g = grid_q(q);
  double *rr = sc.partials + CG_MAXWG;
  int gx, gy;
  cg_core_grid(q, gx, gy);  // one <P, Q> partial per cg_core workgroup
  cg_update_kernel<<<g, TPB, 0, st>>>(p, q, X, R, P, Q, ldc, sc.partials, gx * gy, rr, ds, hist,
                                      k, max_iter);
  HIPOK(hipGetLastError());
  cg_converge_kernel<<<1, TPB, 0, st>>>(rr, (int)g, ds, hist, k, max_iter);
  HIPOK(hipGetLastError());
  cg_p_kernel<<<g, TPB, 0, st>>>(q, R, P, ldc, ds);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_bicg_s(int s, int p, const double *Q, const double *R, double *S, const double *Rt,
                  int64_t ldc, DevState *ds, double *hist, int k, int max_iter, hipStream_t st) {
  const int q = p + s;
  bicg_s_kernel<<<grid_q(q), TPB, 0, st>>>(s, q, Q, R, S, Rt, ldc, ds, hist, k, max_iter);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_bicg_omega(int s, int p, const double *T, const double *S, int64_t ldc,
                      const Scratch &sc, DevState *ds, hipStream_t st) {
  const int q = p + 2 * s;
  bicg_omega_kernel<<<grid_q(q), TPB, 0, st>>>(q, T, S, ldc, sc.partials, ds);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_bicg_update(int s, int p, double *X, double *R, double *P, const double *Q,
                       const double *S, const double *T, const double *Rt, int64_t ldc,
                       const Scratch &sc, DevState *ds, double *hist, int k, int max_iter,
                       hipStream_t st) {
  const int q = p + 2 * s;
  const unsigned g = grid_q(q);
  double *rr = sc.partials + 2 * NBLK;
  bicg_update_kernel<<<g, TPB, 0, st>>>(s, q, X, R, P, Q, S, T, Rt, ldc, sc.partials, (int)g, rr,
                                        ds, hist, k, max_iter);
  HIPOK(hipGetLastError());
  bicg_converge_kernel<<<1, TPB, 0, st>>>(rr, (int)g, ds, hist, k, max_iter);
  HIPOK(hipGetLastError());
  return 0;
}
