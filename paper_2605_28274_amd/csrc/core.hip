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
// Two passes over the cores per iteration, on 32 x 64 tiles:
//   cg_pq_kernel: P_k = R_k + beta_{k-1} P_{k-1} (Alg. 4.1 step 14 of the previous iteration,
//     written to the other P buffer) and partials of <P_k, Q_k>, with
//     Q_k = [H P_k, 0] + [P_k G^T; 0] (eq. (3.11), step 6) formed in registers, not stored;
//   cg_xr_kernel: alpha_k = rho_k / <P_k, Q_k> (step 7), Q_k formed again from the stored P_k
//     (same arithmetic on the same values, so the same Q_k), X += alpha P_k, R -= alpha Q_k
//     (steps 8-9) and partials of ||R_{k+1}||^2.
// H and G are block tridiagonal (|blk(i) - blk(l)| <= 1), so a tile's Q needs P_k on the rows of
// H's band times the tile's columns and on the tile's rows times the columns of G's band; both
// strips are staged in LDS. With SYM (Lyapunov: G = H and R_0 = R_L R_L^T) every core is
// symmetric: only entries i >= j are formed and stored, an entry above the diagonal is read
// from its mirror, and the inner products count off-diagonal entries twice.
constexpr int CT_I = 32, CT_J = 64, CG_GRID = 2048;

template <int S>
struct CgTile {
  double pc[CT_I + 4 * S][CT_J];  // P rows [ra, rb) x the tile's columns
  double hl[CT_I][2 * S];         // the tile's rows x P columns [ca, j0) (left of the tile)
  double hr[CT_I][2 * S];         // the tile's rows x P columns [j0 + 64, cb) (right of it)
  double hb[CT_I][3 * S];         // the band of H on the tile's rows
};

__host__ __device__ inline int cg_tiles_j(int q) { return (q + CT_J - 1) / CT_J; }
__host__ __device__ inline int cg_tiles(int q) { return ((q + CT_I - 1) / CT_I) * cg_tiles_j(q); }

// Next tile at or after t (stride gridDim.x) that holds an entry to form: all tiles, or with SYM
// those reaching the lower triangle.
template <bool SYM>
__device__ __forceinline__ int cg_next_tile(int t, int q) {
  const int tj = cg_tiles_j(q), nt = cg_tiles(q);
  for (; t < nt; t += gridDim.x) {
    const int i0 = (t / tj) * CT_I, j0 = (t % tj) * CT_J;
    if (!SYM || (i0 + CT_I - 1 < q - 1 ? i0 + CT_I - 1 : q - 1) >= j0) break;
  }
  return t;
}

// P_k(l, j) for l, j < p (zero outside): FORM reads R and the previous P and forms
// R + beta P_prev; otherwise it reads the stored P_k. SYM maps l < j to (j, l).
template <bool SYM, bool FORM>
__device__ __forceinline__ double cg_pval(int l, int j, int p, const double *__restrict__ R,
                                          const double *__restrict__ Pp, double beta,
                                          int64_t ldc) {
  if (l >= p || j >= p) return 0.0;
  const int64_t o = (SYM && l < j) ? (int64_t)j * ldc + l : (int64_t)l * ldc + j;
  return FORM ? fma(beta, Pp[o], R[o]) : Pp[o];
}

// Tile geometry: P rows [ra, rb) meet H's band on the tile's rows, P columns [ca, cb) meet G's
// band on its columns (both clipped to p).
struct CgGeom {
  int i0, j0, ra, rb, ca, cb;
};

template <int S>
__device__ __forceinline__ CgGeom cg_geom(int t, int p) {
  const int q = p + S, tj = cg_tiles_j(q);
  CgGeom g;
  g.i0 = (t / tj) * CT_I;
  g.j0 = (t % tj) * CT_J;
  const int imax = (g.i0 + CT_I - 1 < q - 1) ? g.i0 + CT_I - 1 : q - 1;
  const int jmax = (g.j0 + CT_J - 1 < q - 1) ? g.j0 + CT_J - 1 : q - 1;
  g.ra = (g.i0 / S - 1) * S > 0 ? (g.i0 / S - 1) * S : 0;
  g.rb = (imax / S + 2) * S < p ? (imax / S + 2) * S : p;
  g.ca = (g.j0 / S - 1) * S > 0 ? (g.j0 / S - 1) * S : 0;
  g.cb = (jmax / S + 2) * S < p ? (jmax / S + 2) * S : p;
  return g;
}

// Fills the two P strips and the H band of a tile into LDS and this thread's G band (column
// j0 + (t & 63)) into gb. No barrier: the caller brackets it.
template <int S, bool SYM, bool FORM>
__device__ __forceinline__ void cg_stage(CgTile<S> &T, const CgGeom &g, int p,
                                         const double *__restrict__ H,
                                         const double *__restrict__ G,
                                         const double *__restrict__ R,
                                         const double *__restrict__ Pp, double beta, int64_t ldc,
                                         double (&gb)[3 * S]) {
  const int q = p + S;
  const int j = g.j0 + (threadIdx.x & (CT_J - 1));
  const int jc = j < q ? j : q - 1;
  const int bj = jc / S;
  const int l0 = bj > 0 ? (bj - 1) * S : 0;
  const int l1 = (bj + 2) * S < p ? (bj + 2) * S : p;
#pragma unroll
  for (int t = 0; t < 3 * S; ++t) gb[t] = (l0 + t < l1) ? G[(int64_t)jc * ldc + l0 + t] : 0.0;
  // the tile's own rows of P sit inside the column strip; only the columns of G's band left and
  // right of the tile are staged apart
  const int nr = g.rb > g.ra ? g.rb - g.ra : 0;
  const int nl = g.j0 - g.ca, nrt = g.cb > g.j0 + CT_J ? g.cb - g.j0 - CT_J : 0;
  for (int e = threadIdx.x; e < nr * CT_J; e += TPB)
    T.pc[e / CT_J][e % CT_J] =
        cg_pval<SYM, FORM>(g.ra + e / CT_J, g.j0 + e % CT_J, p, R, Pp, beta, ldc);
  for (int e = threadIdx.x; e < CT_I * nl; e += TPB)
    T.hl[e / nl][e % nl] = cg_pval<SYM, FORM>(g.i0 + e / nl, g.ca + e % nl, p, R, Pp, beta, ldc);
  for (int e = threadIdx.x; e < CT_I * nrt; e += TPB)
    T.hr[e / nrt][e % nrt] =
        cg_pval<SYM, FORM>(g.i0 + e / nrt, g.j0 + CT_J + e % nrt, p, R, Pp, beta, ldc);
  for (int e = threadIdx.x; e < CT_I * 3 * S; e += TPB) {
    const int ii = e / (3 * S), t = e % (3 * S);
    const int ic = g.i0 + ii < q ? g.i0 + ii : q - 1;
    const int l = (ic / S > 0 ? (ic / S - 1) * S : 0) + t;
    T.hb[ii][t] = l < p ? H[(int64_t)ic * ldc + l] : 0.0;
  }
}

// Q_k on this thread's 8 entries of the tile (rows i0 + (t >> 6) + 4u, column j0 + (t & 63))
// into qv, and P_k there into pk, from the staged strips.
template <int S>
__device__ __forceinline__ void cg_tile_q(const CgTile<S> &T, const CgGeom &g, int p,
                                          const double (&gb)[3 * S], double (&qv)[8],
                                          double (&pk)[8]) {
  const int q = p + S;
  const int jj = threadIdx.x & (CT_J - 1), iw = threadIdx.x >> 6;
  const int j = g.j0 + jj;
  const int jc = j < q ? j : q - 1;
  const int bj = jc / S;
  const int l0 = bj > 0 ? (bj - 1) * S : 0;
  const int l1 = (bj + 2) * S < p ? (bj + 2) * S : p;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int ii = iw + 4 * u, i = g.i0 + ii;
    const int ic = i < q ? i : q - 1;
    const int bi = ic / S;
    const int li0 = bi > 0 ? (bi - 1) * S : 0;
    double a = 0.0;
    // H P: row i of H meets rows li0 .. li0 + 3S of P (zero at and past p)
    if (j < p) {
#pragma unroll
      for (int t = 0; t < 3 * S; ++t) {
        const int l = li0 + t;
        a = fma(T.hb[ii][t], l < g.rb ? T.pc[l - g.ra][jj] : 0.0, a);
      }
    }
    // P G^T: row i of P meets the band of row j of G
    if (ic < p) {
#pragma unroll
      for (int t = 0; t < 3 * S; ++t) {
        const int l = l0 + t;
        const double v = l < g.j0            ? T.hl[ii][l - g.ca]
                         : l < g.j0 + CT_J ? T.pc[i - g.ra][l - g.j0]
                                           : T.hr[ii][l - g.j0 - CT_J];
        a = fma(l < l1 ? v : 0.0, gb[t], a);
      }
    }
    qv[u] = a;
    pk[u] = (i < g.rb && i >= g.ra) ? T.pc[i - g.ra][jj] : 0.0;
  }
}

template <int S, bool SYM>
__device__ __forceinline__ void cg_pq_body(int p, const double *__restrict__ H,
                                                    const double *__restrict__ G,
                                                    const double *__restrict__ R,
                                                    const double *__restrict__ Pprev,
                                                    double *__restrict__ Pk, int64_t ldc,
                                                    double *partials, const DevState *ds) {
  if (ds->done) return;
  __shared__ CgTile<S> T;
  const int q = p + S, nt = cg_tiles(q);
  const double beta = ds->beta;
  double v[1] = {0.0};
  for (int t = cg_next_tile<SYM>(blockIdx.x, q); t < nt;
       t = cg_next_tile<SYM>(t + gridDim.x, q)) {
    const CgGeom g = cg_geom<S>(t, p);
    double gb[3 * S], qv[8], pk[8];
    __syncthreads();  // the previous tile's readers are done
    cg_stage<S, SYM, true>(T, g, p, H, G, R, Pprev, beta, ldc, gb);
    __syncthreads();
    cg_tile_q<S>(T, g, p, gb, qv, pk);
    const int j = g.j0 + (threadIdx.x & (CT_J - 1));
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = g.i0 + (threadIdx.x >> 6) + 4 * u;
      if (i < p && j < p && (!SYM || i >= j)) {
        Pk[(int64_t)i * ldc + j] = pk[u];
        v[0] = fma((SYM && i > j) ? 2.0 * pk[u] : pk[u], qv[u], v[0]);
      }
    }
  }
  put_partials<1>(v, partials);
}

template <int S, bool SYM>
__device__ __forceinline__ void cg_xr_body(int p, const double *__restrict__ H,
                                                    const double *__restrict__ G,
                                                    const double *__restrict__ Pk,
                                                    double *__restrict__ X,
                                                    double *__restrict__ R, int64_t ldc,
                                                    const double *pq_part, int pq_nb,
                                                    double *partials, DevState *ds,
                                                    double *hist, int k, int max_iter) {
  if (ds->done) return;
  __shared__ CgTile<S> T;
  const int q = p + S, nt = cg_tiles(q);
  // the first tile's strips load while the <P, Q> partials are summed
  int t = cg_next_tile<SYM>(blockIdx.x, q);
  CgGeom g{};
  double gb[3 * S];
  if (t < nt) {
    g = cg_geom<S>(t, p);
    cg_stage<S, SYM, false>(T, g, p, H, G, nullptr, Pk, 0.0, ldc, gb);
  }
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
  while (t < nt) {
    __syncthreads();  // the strips are in place
    double qv[8], pk[8];
    cg_tile_q<S>(T, g, p, gb, qv, pk);
    const int j = g.j0 + (threadIdx.x & (CT_J - 1));
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = g.i0 + (threadIdx.x >> 6) + 4 * u;
      if (i < q && j < q && (!SYM || i >= j)) {
        const int64_t o = (int64_t)i * ldc + j;
        if (i < p && j < p) X[o] = fma(alpha, pk[u], X[o]);
        const double r = fma(-alpha, qv[u], R[o]);
        R[o] = r;
        v[0] = fma((SYM && i > j) ? 2.0 * r : r, r, v[0]);
      }
    }
    t = cg_next_tile<SYM>(t + gridDim.x, q);
    if (t < nt) {
      g = cg_geom<S>(t, p);
      __syncthreads();  // the previous tile's readers are done
      cg_stage<S, SYM, false>(T, g, p, H, G, nullptr, Pk, 0.0, ldc, gb);
    }
  }
  put_partials<1>(v, partials);
}

// One workgroup: ||R_{k+1}|| / ||R_0|| from the partials, the stopping test, rho_{k+1} and
// beta_k (CG).
__device__ __forceinline__ void cg_converge_body(const double *rr_part, int nb,
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

// ---- BiCGSTAB (dense block Hessenberg H and G from block Arnoldi) ----

// alpha = rho / <R~0, Q(1:s,1:s)> (every workgroup forms it from the s x s corner), then
// S = [R 0; 0 0] - alpha Q over (p+s)^2.
__device__ __forceinline__ void bicg_s_body(int s, int q, const double *__restrict__ Q,
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
__device__ __forceinline__ void bicg_omega_body(int q, const double *__restrict__ T,
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
__device__ __forceinline__ void bicg_update_body(int s, int q, double *__restrict__ X,
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
__device__ __forceinline__ void bicg_converge_body(const double *rr_part, int nb,
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

// ---- kernels: one problem per launch, or one problem per blockIdx.y over a group table ----

template <int S, bool SYM>
__global__ __launch_bounds__(TPB) void cg_pq_kernel(int p, const double *H, const double *G,
                                                    const double *R, const double *Pprev,
                                                    double *Pk, int64_t ldc, double *partials,
                                                    const DevState *ds) {
  cg_pq_body<S, SYM>(p, H, G, R, Pprev, Pk, ldc, partials, ds);
}

// CG iteration k of every problem of the group: P_k is the Q buffer for even k and the P
// buffer for odd k (the other holds P_{k-1}).
template <int S, bool SYM>
__global__ __launch_bounds__(TPB) void cg_pq_group(const CoreInst *tab, const int *list, int p, int k) {
  const CoreInst &c = tab[list ? list[blockIdx.y] : blockIdx.y];
  cg_pq_body<S, SYM>(p, c.H, c.G, c.R, (k & 1) ? c.Q : c.P, (k & 1) ? c.P : c.Q, c.ldc, c.part,
                     c.ds);
}

template <int S, bool SYM>
__global__ __launch_bounds__(TPB) void cg_xr_kernel(int p, const double *H, const double *G,
                                                    const double *Pk, double *X, double *R,
                                                    int64_t ldc, const double *pq_part,
                                                    int pq_nb, double *partials, DevState *ds,
                                                    double *hist, int k, int max_iter) {
  cg_xr_body<S, SYM>(p, H, G, Pk, X, R, ldc, pq_part, pq_nb, partials, ds, hist, k, max_iter);
}

template <int S, bool SYM>
__global__ __launch_bounds__(TPB) void cg_xr_group(const CoreInst *tab, const int *list, int p, int k, int nb,
                                                   int rr_off) {
  const CoreInst &c = tab[list ? list[blockIdx.y] : blockIdx.y];
  cg_xr_body<S, SYM>(p, c.H, c.G, (k & 1) ? c.P : c.Q, c.X, c.R, c.ldc, c.part, nb,
                     c.part + rr_off, c.ds, c.hist, k, c.max_iter);
}

__global__ __launch_bounds__(TPB) void cg_converge_kernel(const double *rr_part, int nb,
                                                          DevState *ds, double *hist, int k,
                                                          int max_iter) {
  cg_converge_body(rr_part, nb, ds, hist, k, max_iter);
}

__global__ __launch_bounds__(TPB) void cg_converge_group(const CoreInst *tab, const int *list, int nb, int rr_off,
                                                         int k) {
  const CoreInst &c = tab[list ? list[blockIdx.y] : blockIdx.y];
  cg_converge_body(c.part + rr_off, nb, c.ds, c.hist, k, c.max_iter);
}

__global__ __launch_bounds__(TPB) void bicg_s_kernel(int s, int q, const double *Q,
                                                     const double *R, double *S,
                                                     const double *Rt, int64_t ldc, DevState *ds,
                                                     double *hist, int k, int max_iter) {
  bicg_s_body(s, q, Q, R, S, Rt, ldc, ds, hist, k, max_iter);
}

__global__ __launch_bounds__(TPB) void bicg_s_group(const CoreInst *tab, const int *list, int s, int q, int k) {
  const CoreInst &c = tab[list ? list[blockIdx.y] : blockIdx.y];
  bicg_s_body(s, q, c.Q, c.R, c.S, c.Rt, c.ldc, c.ds, c.hist, k, c.max_iter);
}

__global__ __launch_bounds__(TPB) void bicg_omega_kernel(int q, const double *T, const double *S,
                                                         int64_t ldc, double *partials,
                                                         const DevState *ds) {
  bicg_omega_body(q, T, S, ldc, partials, ds);
}

__global__ __launch_bounds__(TPB) void bicg_omega_group(const CoreInst *tab, const int *list, int q) {
  const CoreInst &c = tab[list ? list[blockIdx.y] : blockIdx.y];
  bicg_omega_body(q, c.T, c.S, c.ldc, c.part, c.ds);
}

__global__ __launch_bounds__(TPB) void bicg_update_kernel(int s, int q, double *X, double *R,
                                                          double *P, const double *Q,
                                                          const double *S, const double *T,
                                                          const double *Rt, int64_t ldc,
                                                          const double *om_part, int om_nb,
                                                          double *partials, DevState *ds,
                                                          double *hist, int k, int max_iter) {
  bicg_update_body(s, q, X, R, P, Q, S, T, Rt, ldc, om_part, om_nb, partials, ds, hist, k,
                   max_iter);
}

__global__ __launch_bounds__(TPB) void bicg_update_group(const CoreInst *tab, const int *list, int s, int q,
                                                         int k, int nb, int rr_off) {
  const CoreInst &c = tab[list ? list[blockIdx.y] : blockIdx.y];
  bicg_update_body(s, q, c.X, c.R, c.P, c.Q, c.S, c.T, c.Rt, c.ldc, c.part, nb, c.part + rr_off,
                   c.ds, c.hist, k, c.max_iter);
}

__global__ __launch_bounds__(TPB) void bicg_converge_kernel(const double *rr_part, int nb,
                                                            DevState *ds, double *hist, int k,
                                                            int max_iter) {
  bicg_converge_body(rr_part, nb, ds, hist, k, max_iter);
}

__global__ __launch_bounds__(TPB) void bicg_converge_group(const CoreInst *tab, const int *list, int nb,
                                                           int rr_off, int k) {
  const CoreInst &c = tab[list ? list[blockIdx.y] : blockIdx.y];
  bicg_converge_body(c.part + rr_off, nb, c.ds, c.hist, k, c.max_iter);
}

// The problems of the group still running: *count and their indices in list (in order).
__global__ void group_active_kernel(const CoreInst *tab, int n, int *count, int *list) {
  if (threadIdx.x != 0) return;
  int c = 0;
  for (int i = 0; i < n; ++i)
    if (!tab[i].ds->done) list[c++] = i;
  *count = c;
}

unsigned grid_q(int q) { return (unsigned)(q < NBLK ? (q < 1 ? 1 : q) : NBLK); }

}  // namespace

int launch_setup_scalars(int s, const double *RL, const double *RR, double *R, double *P,
                         double *Rt, int64_t ldc, double tol, DevState *ds, hipStream_t st) {
  setup_scalars_kernel<<<1, 64, 0, st>>>(s, RL, RR, R, P, Rt, ldc, tol, ds);
  HIPOK(hipGetLastError());
  return 0;
}

// Scratch::partials layout. CG: [0, CG_MAXWG) the <P, Q> partials, [CG_MAXWG, 2 CG_MAXWG)
// the ||R||^2 partials. BiCGSTAB: [0, 2*NBLK) partials of the scalar being formed (<T,S>,
// <T,T>), [2*NBLK, 3*NBLK) the ||R||^2 partials.
constexpr int CG_MAXWG = 4096;
static_assert(CG_GRID <= CG_MAXWG, "CG partials fit their ranges");

unsigned cg_grid(int q) { return (unsigned)std::min(cg_tiles(q), CG_GRID); }

int launch_cg_pq(int s, int p, bool sym, const double *H, const double *G, const double *R,
                 const double *Pprev, double *Pk, int64_t ldc, const Scratch &sc, DevState *ds,
                 hipStream_t st) {
  const unsigned g = cg_grid(p + s);
  switch (s) {
#define CASE(SS)                                                                              \
  case SS:                                                                                    \
    if (sym)                                                                                  \
      cg_pq_kernel<SS, true><<<g, TPB, 0, st>>>(p, H, G, R, Pprev, Pk, ldc, sc.partials, ds); \
    else                                                                                      \
      cg_pq_kernel<SS, false><<<g, TPB, 0, st>>>(p, H, G, R, Pprev, Pk, ldc, sc.partials, ds); \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return SYLV_ERR_INVALID;
  }
  HIPOK(hipGetLastError());
  return 0;
}

int launch_cg_xr(int s, int p, bool sym, const double *H, const double *G, const double *Pk,
                 double *X, double *R, int64_t ldc, const Scratch &sc, DevState *ds, double *hist,
                 int k, int max_iter, hipStream_t st) {
  const unsigned g = cg_grid(p + s);
  double *rr = sc.partials + CG_MAXWG;
  switch (s) {
#define CASE(SS)                                                                            \
  case SS:                                                                                  \
    if (sym)                                                                                \
      cg_xr_kernel<SS, true><<<g, TPB, 0, st>>>(p, H, G, Pk, X, R, ldc, sc.partials, (int)g, \
                                                rr, ds, hist, k, max_iter);                 \
    else                                                                                    \
      cg_xr_kernel<SS, false><<<g, TPB, 0, st>>>(p, H, G, Pk, X, R, ldc, sc.partials,       \
                                                 (int)g, rr, ds, hist, k, max_iter);        \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return SYLV_ERR_INVALID;
  }
  HIPOK(hipGetLastError());
  cg_converge_kernel<<<1, TPB, 0, st>>>(rr, (int)g, ds, hist, k, max_iter);
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

// ---- batch groups: one launch per phase for every problem of the group ----

int launch_cg_group(int s, bool sym, int p, int k, const CoreInst *tab, const int *list, int n,
                    hipStream_t st) {
  const unsigned g = cg_grid(p + s);
  const dim3 grid(g, (unsigned)n);
  switch (s) {
#define CASE(SS)                                                                        \
  case SS:                                                                              \
    if (sym) {                                                                          \
      cg_pq_group<SS, true><<<grid, TPB, 0, st>>>(tab, list, p, k);                           \
      cg_xr_group<SS, true><<<grid, TPB, 0, st>>>(tab, list, p, k, (int)g, CG_MAXWG);         \
    } else {                                                                            \
      cg_pq_group<SS, false><<<grid, TPB, 0, st>>>(tab, list, p, k);                          \
      cg_xr_group<SS, false><<<grid, TPB, 0, st>>>(tab, list, p, k, (int)g, CG_MAXWG);        \
    }                                                                                   \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return SYLV_ERR_INVALID;
  }
  HIPOK(hipGetLastError());
  cg_converge_group<<<dim3(1, (unsigned)n), TPB, 0, st>>>(tab, list, (int)g, CG_MAXWG, k);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_bicg_group_s(int s, int p, int k, const CoreInst *tab, const int *list, int n,
                        hipStream_t st) {
  const int q = p + s;
  bicg_s_group<<<dim3(grid_q(q), (unsigned)n), TPB, 0, st>>>(tab, list, s, q, k);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_bicg_group_omega(int s, int p, const CoreInst *tab, const int *list, int n,
                            hipStream_t st) {
  const int q = p + 2 * s;
  bicg_omega_group<<<dim3(grid_q(q), (unsigned)n), TPB, 0, st>>>(tab, list, q);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_bicg_group_update(int s, int p, int k, const CoreInst *tab, const int *list, int n,
                             hipStream_t st) {
  const int q = p + 2 * s;
  const unsigned g = grid_q(q);
  bicg_update_group<<<dim3(g, (unsigned)n), TPB, 0, st>>>(tab, list, s, q, k, (int)g, 2 * NBLK);
  HIPOK(hipGetLastError());
  bicg_converge_group<<<dim3(1, (unsigned)n), TPB, 0, st>>>(tab, list, (int)g, 2 * NBLK, k);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_group_active(const CoreInst *tab, int n, int *count, int *list, hipStream_t st) {
  group_active_kernel<<<1, 64, 0, st>>>(tab, n, count, list);
  HIPOK(hipGetLastError());
  return 0;
}
