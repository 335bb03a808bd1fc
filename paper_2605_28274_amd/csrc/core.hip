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

// Sums nb <= MAXB partial records of NV values in a fixed order (thread t adds records t,
// t + TPB, ... in turn, then the block sum); the result is returned to every thread (all TPB
// threads must call). The records are loaded all at once, so their latencies overlap.
template <int NV, int MAXB>
__device__ __forceinline__ void sum_partials(const double *partials, int nb, double (&out)[NV]) {
  __shared__ double lds[16 * NV];
  __shared__ double res[NV];
  constexpr int PER = (MAXB + TPB - 1) / TPB;
  double v[PER][NV];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int b = (int)threadIdx.x + u * TPB;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[u][i] = b < nb ? partials[(size_t)b * NV + i] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    out[i] = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) out[i] += v[u][i];
  }
  block_sum<NV>(out, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) res[i] = out[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) out[i] = res[i];
}

// ---- CG (block-tridiagonal H and G from block Lanczos) ----
// Two passes over the cores per iteration:
//   cg_pq_kernel: P_k = R_k + beta_{k-1} P_{k-1} (Alg. 4.1 step 14 of the previous iteration,
//     written to the other P buffer) and partials of <P_k, Q_k>, with
//     Q_k = [H P_k, 0] + [P_k G^T; 0] (eq. (3.11), step 6) formed in registers, not stored;
//   cg_xr_kernel: alpha_k = rho_k / <P_k, Q_k> (step 7), Q_k formed again from the stored P_k
//     (same arithmetic on the same values, so the same Q_k), X += alpha P_k, R -= alpha Q_k
//     (steps 8-9) and partials of ||R_{k+1}||^2.
// H and G are block tridiagonal (|blk(i) - blk(l)| <= 1): Q(i, j) needs P on the rows of H's
// band around i in column j and on row i at the columns of G's band around j. With SYM
// (Lyapunov: G = H and R_0 = R_L R_L^T) every core is symmetric: only entries i >= j are formed
// and stored, an entry above the diagonal is read from its mirror, and the inner products count
// off-diagonal entries twice.
//
// Column-panel form: a wave owns 64 consecutive columns j of the cores (one per lane) and a
// chunk of rows, which it walks one block row b at a time with P on block rows b-1, b, b+1 of
// its columns in registers: the band of H on a row of block b spans exactly those rows, so H P
// needs no exchange between lanes (the H entries of a row are the same for the whole wave; the
// chunk's band of H is staged in LDS once). P G^T needs P on the row at the columns of G's band
// around j: the row, with 2S columns on each side, goes through a small LDS buffer of the wave.
// Every P entry is read once per chunk (plus one block row above and below it and the side
// columns); the next block row, and X and R of the next outputs, are loaded while the current
// one is formed. Work items (panel, chunk) are spread over the waves of the grid; the reductions
// keep one record per workgroup.
constexpr int CG_GRID = 2048;

template <int S>
__host__ __device__ constexpr int cg_chunk_max() { return S <= 4 ? 128 : 64; }
template <int S>
__host__ __device__ inline int cg_chunk_rows(int q) {
  const int nc = (q + 63) / 64;
  int cr = (int)(((int64_t)q * nc + 4095) / 4096);
  cr = cr < 4 * S ? 4 * S : (cr > cg_chunk_max<S>() ? cg_chunk_max<S>() : cr);
  return cr / S * S;
}
template <int S>
__host__ __device__ inline int cg_items(int q) {
  const int cr = cg_chunk_rows<S>(q);
  return ((q + 63) / 64) * ((q + cr - 1) / cr);
}

// PQ: P_k = R + beta P_prev is formed and stored, v += <P_k, Q_k>. Otherwise (XR): P_k is read,
// X += alpha P_k, R -= alpha Q_k, v += ||R||^2. sc = beta (PQ) or alpha (XR).
template <int S, bool SYM, bool PQ>
__device__ __forceinline__ void cg_panels(int p, const double *__restrict__ H,
                                          const double *__restrict__ G,
                                          const double *__restrict__ Rin,
                                          const double *__restrict__ Pin, double *__restrict__ Pout,
                                          double *__restrict__ X, double *__restrict__ Rio,
                                          int64_t ldc, double sc, double &v) {
  constexpr int W = 64 + 4 * S, HB = cg_chunk_max<S>() * 3 * S;
  __shared__ double buf[TPB / 64][W];
  __shared__ double hbuf[TPB / 64][HB];  // the band of H on the chunk's rows
  // the wave index is uniform: everything derived from it (items, rows, H addresses) stays in
  // scalar registers and H is read with scalar loads
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double *bw = buf[wv], *hb = hbuf[wv];
  const int q = p + S, nc = (q + 63) / 64, cr = cg_chunk_rows<S>(q);
  const int items = nc * ((q + cr - 1) / cr);
  const double beta = PQ ? sc : 0.0;
  // P(l, j) is split in a raw load (into a and, for PQ, b: R and P_prev, or the stored P_k)
  // and the combination P = a + beta b, taken where the value is used, so that a load in
  // flight is not waited for early
  auto ld = [&](int l, int j, double &a, double &b) {
    const bool in = l >= 0 && j >= 0 && l < p && j < p;
    const int64_t o = (SYM && l < j) ? (int64_t)j * ldc + l : (int64_t)l * ldc + j;
    a = in ? (PQ ? Rin[o] : Pin[o]) : 0.0;
    b = (PQ && in) ? Pin[o] : 0.0;
  };
  auto pv = [&](double a, double b) { return PQ ? fma(beta, b, a) : a; };
  for (int it = (int)blockIdx.x * (TPB / 64) + wv; it < items; it += (int)gridDim.x * (TPB / 64)) {
    const int c = it % nc, r = it / nc;
    const int j0 = 64 * c, j = j0 + lane;
    int r0 = r * cr;
    const int r1 = (r0 + cr < q) ? r0 + cr : q;
    if (SYM && r1 <= j0) continue;  // above the diagonal: nothing to form
    if (SYM && r0 < j0) r0 = j0 / S * S;
    // G's band on column j: G(j, l) for l in [l0, l1)
    const int jc = j < q ? j : q - 1, bj = jc / S;
    const int l0 = bj > 0 ? (bj - 1) * S : 0;
    const int l1 = (bj + 2) * S < p ? (bj + 2) * S : p;
    double gb[3 * S];
#pragma unroll
    for (int t = 0; t < 3 * S; ++t)
      gb[t] = (j < q && l0 + t < l1) ? G[(int64_t)jc * ldc + l0 + t] : 0.0;
    const int gpos = l0 - j0 + 2 * S;  // buffer position of column l0
    // side column of this lane (lanes < 4S): 2S columns left and right of the panel
    const int hc = lane < 2 * S ? j0 - 2 * S + lane : j0 + 64 + (lane - 2 * S);
    const bool hl = lane < 4 * S;
    const int hpos = lane < 2 * S ? lane : 64 + lane;
    // the band of H on rows [r0, r1): row i, entry t = H(i, (i/S - 1) S + t)
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < (r1 - r0) * 3 * S; e += 64) {
      const int i = r0 + e / (3 * S), l = (i / S - 1) * S + e % (3 * S);
      hb[e] = (l >= 0 && l < p) ? H[(int64_t)i * ldc + l] : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
    // window: block rows b-1, b, b+1 at column j; the side columns on block row b
    const int b0 = r0 / S, b1 = (r1 + S - 1) / S;
    double w[3][S], hw[S];
#pragma unroll
    for (int a = 0; a < S; ++a) {
      double x0, y0, x1, y1, x2, y2, x3 = 0.0, y3 = 0.0;
      ld((b0 - 1) * S + a, j, x0, y0);
      ld(b0 * S + a, j, x1, y1);
      ld((b0 + 1) * S + a, j, x2, y2);
      if (hl) ld(b0 * S + a, hc, x3, y3);
      w[0][a] = pv(x0, y0);
      w[1][a] = pv(x1, y1);
      w[2][a] = pv(x2, y2);
      hw[a] = pv(x3, y3);
    }
    // X and R of a block row's outputs (XR); issued one block row ahead, before the P
    // prefetch, so that waiting for them leaves the later loads in flight (the counter of
    // outstanding memory operations drains in issue order)
    auto ld_xr = [&](int b, double (&xo)[S], double (&ro)[S]) {
#pragma unroll
      for (int a = 0; a < S; ++a) {
        const int i = b * S + a;
        const int64_t o = (int64_t)i * ldc + j;
        const bool in = i < r1 && j < q && (!SYM || i >= j);
        xo[a] = (in && i < p && j < p) ? X[o] : 0.0;
        ro[a] = in ? Rio[o] : 0.0;
      }
    };
    double xo[S], ro[S];
    if (!PQ) ld_xr(b0, xo, ro);
    for (int b = b0; b < b1; ++b) {
      double xn[S], rn[S], nx[S], ny[S], nh[S], nk[S];
      if (!PQ) ld_xr(b + 1, xn, rn);
      // the next block rows of P, in flight while this one is formed
#pragma unroll
      for (int a = 0; a < S; ++a) {
        ld((b + 2) * S + a, j, nx[a], ny[a]);
        nh[a] = nk[a] = 0.0;
        if (hl) ld((b + 1) * S + a, hc, nh[a], nk[a]);
      }
#pragma unroll
      for (int a = 0; a < S; ++a) {
        const int i = b * S + a;
        // H P: row i of H on block rows b-1 .. b+1
        double qv = 0.0;
        const double *hr = hb + (i - r0) * 3 * S;
#pragma unroll
        for (int t = 0; t < 3 * S; ++t) qv = fma(hr[t], w[t / S][t % S], qv);
        // P G^T: row i at the columns of G's band, through the wave's buffer
        bw[2 * S + lane] = w[1][a];
        if (hl) bw[hpos] = hw[a];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int t = 0; t < 3 * S; ++t) qv = fma(bw[gpos + t], gb[t], qv);
        __builtin_amdgcn_wave_barrier();
        const double pk = w[1][a];
        const int64_t o = (int64_t)i * ldc + j;
        if (PQ) {
          if (i < p && j < p && (!SYM || i >= j)) {
            Pout[o] = pk;
            v = fma((SYM && i > j) ? 2.0 * pk : pk, qv, v);
          }
        } else if (i < q && j < q && (!SYM || i >= j)) {
          if (i < p && j < p) X[o] = fma(sc, pk, xo[a]);
          const double rv = fma(-sc, qv, ro[a]);
          Rio[o] = rv;
          v = fma((SYM && i > j) ? 2.0 * rv : rv, rv, v);
        }
      }
#pragma unroll
      for (int a = 0; a < S; ++a) {
        w[0][a] = w[1][a];
        w[1][a] = w[2][a];
        w[2][a] = pv(nx[a], ny[a]);
        hw[a] = pv(nh[a], nk[a]);
        if (!PQ) {
          xo[a] = xn[a];
          ro[a] = rn[a];
        }
      }
    }
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
  double v[1] = {0.0};
  cg_panels<S, SYM, true>(p, H, G, R, Pprev, Pk, nullptr, nullptr, ldc, ds->beta, v[0]);
  put_partials<1>(v, partials);
}

template <int S, bool SYM>
__device__ __forceinline__ void cg_xr_body(int p, const double *__restrict__ H,
                                           const double *__restrict__ G,
                                           const double *__restrict__ Pk,
                                           double *__restrict__ X, double *__restrict__ R,
                                           int64_t ldc, const double *pq_part, int pq_nb,
                                           double *partials, DevState *ds, double *hist, int k,
                                           int max_iter) {
  if (ds->done) return;
  double pq[1];
  sum_partials<1, CG_GRID>(pq_part, pq_nb, pq);
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
  cg_panels<S, SYM, false>(p, H, G, nullptr, Pk, nullptr, X, R, ldc, alpha, v[0]);
  put_partials<1>(v, partials);
}

// One workgroup: ||R_{k+1}|| / ||R_0|| from the partials, the stopping test, rho_{k+1} and
// beta_k (CG).
__device__ __forceinline__ void cg_converge_body(const double *rr_part, int nb,
                                                          DevState *ds, double *hist, int k,
                                                          int max_iter) {
  if (ds->done) return;
  double rr[1];
  sum_partials<1, CG_GRID>(rr_part, nb, rr);
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
  sum_partials<2, NBLK>(om_part, om_nb, ts_tt);
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
  sum_partials<1, NBLK>(rr_part, nb, rr);
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

unsigned cg_grid(int s, int q) {
  int items = 0;
  switch (s) {
#define CASE(SS) \
  case SS: items = cg_items<SS>(q); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: break;
  }
  return (unsigned)std::max(1, std::min((items + TPB / 64 - 1) / (TPB / 64), CG_GRID));
}

int launch_cg_pq(int s, int p, bool sym, const double *H, const double *G, const double *R,
                 const double *Pprev, double *Pk, int64_t ldc, const Scratch &sc, DevState *ds,
                 hipStream_t st) {
  const unsigned g = cg_grid(s, p + s);
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
  const unsigned g = cg_grid(s, p + s);
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
  if (n < 1) return 0;  // no problem in the launches
  const unsigned g = cg_grid(s, p + s);
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
  if (n < 1) return 0;  // no problem in the launches
  const int q = p + s;
  bicg_s_group<<<dim3(grid_q(q), (unsigned)n), TPB, 0, st>>>(tab, list, s, q, k);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_bicg_group_omega(int s, int p, const CoreInst *tab, const int *list, int n,
                            hipStream_t st) {
  if (n < 1) return 0;  // no problem in the launches
  const int q = p + 2 * s;
  bicg_omega_group<<<dim3(grid_q(q), (unsigned)n), TPB, 0, st>>>(tab, list, q);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_bicg_group_update(int s, int p, int k, const CoreInst *tab, const int *list, int n,
                             hipStream_t st) {
  if (n < 1) return 0;  // no problem in the launches
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
