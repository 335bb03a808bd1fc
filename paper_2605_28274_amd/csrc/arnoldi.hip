// Block Arnoldi step j for both bases at once (Algorithm 4.2, steps 5-6 and 10-11): the V basis
// of K(A, C1) and the W basis of K(B^T, C2) advance in lockstep, so every launch below covers
// both: workgroups [0, nb_0) work on basis 0 and [nb_0, nb_0 + nb_1) on basis 1. This halves
// the launches of the step and fills the GPU with the smaller basis' work as well.
//
// Step (per basis, M the operator, V the row-major rows x ldb basis, U a rows x s panel):
//   U = M V_j, partials of ||U||^2                                 spmm_pair
//   two classical Gram-Schmidt sweeps:
//     C = V[:, 0:ncols]^T U  (split-K over row chunks)            gram_part_pair
//     sum of the chunk partials -> H column block j, coef         gram_reduce_pair
//     U -= V[:, 0:ncols] C   (FP64 MFMA, coef staged in LDS)       update_mfma_pair
//   partials of U^T U after the second sweep                       ugram_pair
//   first Cholesky-QR pass + closure test, partials of G2          qr2_pair
//   second pass, V_{j+1} = U T, H_{j+1,j}                          final_pair
// No kernel ends in a grid-wide fence: each reduction leaves one partial per workgroup and the
// next kernel sums them in a fixed order (deterministic) after the kernel boundary; the small
// s x s factorizations are then formed redundantly in every workgroup, and workgroup 0 records
// them.
#include <algorithm>

#include "common.h"

namespace {

constexpr int TPB = 256;
constexpr int NG = 8;          // thread groups splitting the chunk sum in gram_reduce_pair
constexpr int OPB = TPB / NG;  // outputs per gram_reduce_pair workgroup
constexpr int UCH = 128;       // rows of U staged in LDS at a time by gram_part_pair
constexpr int NQ = 4;          // 256-column groups processed together by gram_part_pair

struct ArSide {
  int64_t rows, nnz;
  const int32_t *rp, *ci;
  const double *val;
  void *basis;        // rows x ldb, element type T of the kernels (double, or float in mixed mode)
  int64_t ldb;
  double *H;
  double *U;
  double *coef;
  SideState *ss;
  SellMat sell;       // SELL copy of the operator (sell.ci == nullptr: CSR)
  const void *pin;    // compact copy of block j (SpMM input), element type T
  void *pout;         // compact copy of block j+1 (written with the new block), element type T
  double *part;    // Gram chunk partials of this basis
  double *aux;     // partials of ||M V_j||^2, U^T U and of the second-pass Gram
  int *cnt;        // counters of this basis (unused: no grid-wide reductions)
  int nb_spmm, nb_upd, nb_qr;  // workgroups whose partials sit in aux
  int b0, nb;      // workgroup range of this basis in the current launch
  int64_t rpc;     // rows per chunk (gram) or rows per workgroup (update)
};

struct ArPair {
  ArSide s[2];
  int nsides;
};

// The basis this workgroup works on (selected without dynamic indexing of the kernel argument)
// and the workgroup's index within that basis' range.
__device__ __forceinline__ ArSide side_of(const ArPair &P, int &lb, int &sd) {
  sd = (P.nsides > 1 && (int)blockIdx.x >= P.s[1].b0) ? 1 : 0;
  const ArSide A = sd ? P.s[1] : P.s[0];
  lb = (int)blockIdx.x - A.b0;
  return A;
}

template <int S, typename T>
__global__ __launch_bounds__(TPB) void spmm_pair(ArPair P, const DevState *ds) {
  if (ds->done) return;
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  double red[1] = {0.0};
  // row tiles lb, lb + nb, ... (at most ROW_WG workgroups per basis, so few partials)
  for (int64_t r0 = (int64_t)lb * TPB; r0 < A.rows; r0 += (int64_t)A.nb * TPB) {
    const int64_t r1 = (r0 + TPB < A.rows) ? r0 + TPB : A.rows;
    double acc[S];
    const int64_t r = r0 + threadIdx.x;
    if (A.sell.ci) {
      if (r < r1) sell_row<S>(A.sell, r, static_cast<const T *>(A.pin), S, acc);
    } else {
      spmm_rows<S>(r0, r1, A.rp, A.ci, A.val, static_cast<const T *>(A.pin), S, acc);
    }
    if (r < r1) {
#pragma unroll
      for (int t = 0; t < S; ++t) {
        A.U[r * S + t] = acc[t];
        red[0] = fma(acc[t], acc[t], red[0]);
      }
    }
  }
  __shared__ double lds[16];
  block_sum<1>(red, lds);
  if (threadIdx.x == 0) A.aux[lb] = red[0];
}

// Eight bytes of basis entries per load: one double, or two floats (FP32 bases).
template <typename T>
struct Pack8;
template <>
struct Pack8<double> {
  typedef double type;
  static constexpr int N = 1;
  static __device__ __forceinline__ type zero() { return 0.0; }
  static __device__ __forceinline__ void get(type v, double (&o)[1]) { o[0] = v; }
};
template <>
struct Pack8<float> {
  typedef float2 type;
  static constexpr int N = 2;
  static __device__ __forceinline__ type zero() { return make_float2(0.f, 0.f); }
  static __device__ __forceinline__ void get(type v, double (&o)[2]) {
    o[0] = (double)v.x;
    o[1] = (double)v.y;
  }
};

// Chunk partials of C = V^T U: workgroup lb owns rows [lb*rpc, (lb+1)*rpc) and all ncols
// columns; thread t accumulates the 8-byte column group t + 256 q (one double or two floats).
// part[lb][c][t] (rows of V are read once, coalesced; U rows come from LDS).
template <int S, typename T>
__global__ __launch_bounds__(TPB) void gram_part_pair(ArPair P, int ncols, const DevState *ds) {
  if (ds->done) return;
  typedef Pack8<T> PK;
  typedef typename PK::type V8;
  constexpr int E = PK::N, NV = NQ / E;
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  __shared__ double Us[UCH * S];
  const int64_t r0 = (int64_t)lb * A.rpc;
  const int64_t r1 = (r0 + A.rpc < A.rows) ? r0 + A.rpc : A.rows;
  double *part = A.part + (size_t)lb * ncols * S;
  for (int c0 = 0; c0 < ncols; c0 += TPB * NQ) {
    double acc[NV][E][S];
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
      for (int e = 0; e < E; ++e)
#pragma unroll
        for (int t = 0; t < S; ++t) acc[q][e][t] = 0.0;
    // columns past ncols load column group 0 instead (always in bounds) and are not stored, so
    // every load is unconditional and the loads of a step issue back to back
    int coff[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int c = c0 + (q * TPB + (int)threadIdx.x) * E;
      coff[q] = c < ncols ? c : 0;
    }
    for (int64_t rb = r0; rb < r1; rb += UCH) {
      const int nr = (int)((r1 - rb < UCH) ? r1 - rb : UCH);
      __syncthreads();
      for (int e = threadIdx.x; e < nr * S; e += TPB) Us[e] = A.U[rb * S + e];
      __syncthreads();
      const T *vrow = static_cast<const T *>(A.basis) + rb * A.ldb;
      // RU rows per step: the same bytes in flight per thread for either element type
      constexpr int RU = 2 * E;
      int r = 0;
      for (; r + RU <= nr; r += RU) {
        V8 v[RU][NV];
#pragma unroll
        for (int h = 0; h < RU; ++h)
#pragma unroll
          for (int q = 0; q < NV; ++q)
            v[h][q] = *reinterpret_cast<const V8 *>(vrow + (int64_t)(r + h) * A.ldb + coff[q]);
#pragma unroll
        for (int h = 0; h < RU; ++h)
#pragma unroll
          for (int q = 0; q < NV; ++q) {
            double x[E];
            PK::get(v[h][q], x);
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
              for (int t = 0; t < S; ++t)
                acc[q][e][t] = fma(x[e], Us[(r + h) * S + t], acc[q][e][t]);
          }
      }
      for (; r < nr; ++r) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          const V8 v = *reinterpret_cast<const V8 *>(vrow + (int64_t)r * A.ldb + coff[q]);
          double x[E];
          PK::get(v, x);
#pragma unroll
          for (int e = 0; e < E; ++e)
#pragma unroll
            for (int t = 0; t < S; ++t) acc[q][e][t] = fma(x[e], Us[r * S + t], acc[q][e][t]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int c = c0 + (q * TPB + (int)threadIdx.x) * E + e;
        if (c < ncols)
#pragma unroll
          for (int t = 0; t < S; ++t) part[c * S + t] = acc[q][e][t];
      }
  }
}

// Sums the nchunk partials of OPB consecutive outputs per workgroup: thread group g (of NG)
// adds chunks [g nchunk / NG, (g+1) nchunk / NG) for its output, then group 0 adds the NG
// group sums in order and writes column block j of H (store in sweep 1, add in sweep 2) and the
// compact coefficients.
__global__ __launch_bounds__(TPB) void gram_reduce_pair(ArPair P, int S, int ncols, int nchunk0,
                                                        int nchunk1, int64_t ldh, int hcol,
                                                        int pass, const DevState *ds) {
  if (ds->done) return;
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  __shared__ double gs[NG][OPB];
  const int nchunk = sd ? nchunk1 : nchunk0;
  const int nout = ncols * S;
  const int ol = threadIdx.x % OPB, g = threadIdx.x / OPB;
  const int o = lb * OPB + ol;
  const int q0 = (int)((int64_t)nchunk * g / NG), q1 = (int)((int64_t)nchunk * (g + 1) / NG);
  double a0 = 0.0, a1 = 0.0;
  if (o < nout) {
    int q = q0;
    for (; q + 2 <= q1; q += 2) {
      a0 += A.part[(size_t)q * nout + o];
      a1 += A.part[(size_t)(q + 1) * nout + o];
    }
    if (q < q1) a0 += A.part[(size_t)q * nout + o];
  }
  gs[g][ol] = a0 + a1;
  __syncthreads();
  if (g == 0 && o < nout) {
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < NG; ++q) a += gs[q][ol];
    const int c = o / S, t = o % S;
    double *h = A.H + (int64_t)c * ldh + hcol + t;
    *h = (pass == 1) ? a : *h + a;
    A.coef[o] = a;
  }
}

// Columns of the coefficient block staged in LDS at a time by update_mfma_pair (64 KiB, whole
// groups of 128 columns).
template <int S>
__host__ __device__ constexpr int UPD_KCH() {
  return (64 * 1024 / (S * 8)) / 128 * 128;
}

// U[r] -= V[r, 0:ncols] C on FP64 matrix cores (v_mfma_f64_16x16x4f64): each wave owns 16 rows,
// D (16 x 16) += A (16 rows x 4 basis columns) B (4 x 16, coefficient columns >= S are zero).
// Lane l reads 32 contiguous bytes of row l % 16 per step (KL consecutive columns, chunk l / 16),
// so the four lanes of a row cover 128 contiguous bytes; MFMA m of the step takes column
// k0 + KL (l / 16) + m as its k-slot l / 16 on both operands (the sum over k is the same). The
// coefficients sit in LDS, zero-padded past ncols; stale basis columns past ncols read as zero.
template <int S, typename T>
__global__ __launch_bounds__(TPB) void update_mfma_pair(ArPair P, int ncols, const DevState *ds) {
  if (ds->done) return;
  typedef double v4 __attribute__((ext_vector_type(4)));
  constexpr int KL = 32 / (int)sizeof(T);  // columns per lane per step
  constexpr int KG = 4 * KL;               // columns per step
  constexpr int KU = 4;                    // steps whose loads are in flight together
  extern __shared__ double Cs[];
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  const int nk = (ncols + KG - 1) / KG * KG;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int li = lane & 15, lq = lane >> 4;
  // one block of 16 rows per wave (UROWS rows per workgroup)
  const int64_t r0 = (int64_t)lb * A.rpc;
  const int64_t r1 = (r0 + A.rpc < A.rows) ? r0 + A.rpc : A.rows;
  const int64_t rb = r0 + 16 * w;
  const bool live = rb < r1;
  const int64_t row = (rb + li < r1) ? rb + li : r1 - 1;  // clamped loads, masked stores
  const T *vr = static_cast<const T *>(A.basis) + row * A.ldb + lq * KL;
  v4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  // the coefficients pass through LDS in chunks of at most 64 KiB
  for (int c0 = 0; c0 < nk; c0 += UPD_KCH<S>()) {
    const int c1 = (c0 + UPD_KCH<S>() < nk) ? c0 + UPD_KCH<S>() : nk;
    __syncthreads();
    for (int e = threadIdx.x; e < (c1 - c0) * S; e += TPB) {
      const int g = c0 * S + e;
      Cs[e] = g < ncols * S ? A.coef[g] : 0.0;
    }
    __syncthreads();
    if (!live) continue;
    for (int k0 = c0; k0 < c1; k0 += KU * KG) {
      T x[KU][KL];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        // a step past the chunk re-reads step 0 (in bounds); its products are masked below
        const int kk = k0 + u * KG < c1 ? k0 + u * KG : 0;
        if (sizeof(T) == 8) {
          const double2 *p2 = reinterpret_cast<const double2 *>(vr + kk);
          const double2 a = p2[0], b = p2[1];
          x[u][0] = (T)a.x;
          x[u][1] = (T)a.y;
          x[u][2] = (T)b.x;
          x[u][3] = (T)b.y;
        } else {
          const float4 *p4 = reinterpret_cast<const float4 *>(vr + kk);
          const float4 a = p4[0], b = p4[1];
          const float f[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
          for (int m = 0; m < KL; ++m) x[u][m] = (T)f[m];
        }
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const bool step = k0 + u * KG < c1;
#pragma unroll
        for (int m = 0; m < KL; ++m) {
          const int k = k0 + u * KG + lq * KL + m;
          const double av = (step && k < ncols) ? (double)x[u][m] : 0.0;
          const double bv = (step && li < S) ? Cs[(k - c0) * S + li] : 0.0;
          if (m & 1) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc1, 0, 0, 0);
          else acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc0, 0, 0, 0);
        }
      }
    }
  }
  // lane holds D[4 v + lq][li]: row rb + 4 v + lq, column li
  if (live && li < S) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = rb + 4 * v + lq;
      if (r < r1) A.U[r * S + li] -= acc0[v] + acc1[v];
    }
  }
}

// Partials of U^T U (rows over workgroups, one thread per row) for the first QR pass.
template <int S>
__global__ __launch_bounds__(TPB) void ugram_pair(ArPair P, const DevState *ds) {
  if (ds->done) return;
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  double g[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) g[i] = 0.0;
  for (int64_t r = (int64_t)lb * TPB + threadIdx.x; r < A.rows; r += (int64_t)A.nb * TPB) {
    double u[S];
#pragma unroll
    for (int t = 0; t < S; ++t) u[t] = A.U[r * S + t];
#pragma unroll
    for (int a = 0; a < S; ++a)
#pragma unroll
      for (int b = 0; b < S; ++b) g[a * S + b] = fma(u[a], u[b], g[a * S + b]);
  }
  __shared__ double lds[16 * S * S];
  block_sum<S * S>(g, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < S * S; ++i) A.aux[A.nb_spmm + lb * S * S + i] = g[i];
}

// Sums n partial records of NV values (stride NV) in a fixed order; every thread gets the sum.
template <int NV>
__device__ __forceinline__ void sum_records(const double *p, int n, double (&out)[NV]) {
  __shared__ double lds[16 * NV];
  __shared__ double res[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) out[i] = 0.0;
  for (int b = threadIdx.x; b < n; b += TPB)
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] += p[(size_t)b * NV + i];
  block_sum<NV>(out, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) res[i] = out[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) out[i] = res[i];
}

// First Cholesky-QR pass and closure test from the partials of ||M V_j||^2 and U^T U (every
// workgroup forms the same factors; workgroup 0 records them), then partials of
// G2 = (U T1)^T (U T1).
template <int S>
__global__ __launch_bounds__(TPB) void qr2_pair(ArPair P, double closure_tol, const DevState *ds) {
  if (ds->done) return;
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  __shared__ SideState st;
  double ref[1], G1[S * S];
  sum_records<1>(A.aux, A.nb_spmm, ref);
  sum_records<S * S>(A.aux + A.nb_spmm, A.nb_upd, G1);
  if (threadIdx.x == 0) {
    st.ref2 = ref[0];
    finish_pass1(&st, S, closure_tol, G1);
    if (lb == 0) {
      A.ss->ref2 = st.ref2;
      A.ss->mode = st.mode;
      for (int i = 0; i < S * S; ++i) {
        A.ss->T1[i] = st.T1[i];
        A.ss->Hs1[i] = st.Hs1[i];
      }
    }
  }
  __syncthreads();
  double T1[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) T1[i] = st.T1[i];
  double g[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) g[i] = 0.0;
  for (int64_t r = (int64_t)lb * TPB + threadIdx.x; r < A.rows; r += (int64_t)A.nb * TPB) {
    double u[S], u1[S];
#pragma unroll
    for (int t = 0; t < S; ++t) u[t] = A.U[r * S + t];
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
  __shared__ double lds[16 * S * S];
  block_sum<S * S>(g, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < S * S; ++i) A.aux[A.nb_spmm + A.nb_upd * S * S + lb * S * S + i] = g[i];
}

// Second Cholesky-QR pass from the G2 partials (every workgroup forms the same factor), then
// V[:, (j+1)s : (j+2)s] = U T; workgroup 0 records T and writes H_{j+1,j}.
template <int S, typename T>
__global__ __launch_bounds__(TPB) void final_pair(ArPair P, int jb, int64_t ldh,
                                                  const DevState *ds) {
  if (ds->done) return;
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  __shared__ SideState st;
  double G2[S * S];
  sum_records<S * S>(A.aux + A.nb_spmm + A.nb_upd * S * S, A.nb_qr, G2);
  if (threadIdx.x == 0) {
    st.mode = A.ss->mode;
    for (int i = 0; i < S * S; ++i) {
      st.T1[i] = A.ss->T1[i];
      st.Hs1[i] = A.ss->Hs1[i];
    }
    finish_pass2(&st, S, G2);
    if (lb == 0) {
      for (int i = 0; i < S * S; ++i) {
        A.ss->T[i] = st.T[i];
        A.ss->Hs1[i] = st.Hs1[i];
      }
      for (int a = 0; a < S; ++a)
        for (int b = 0; b < S; ++b)
          A.H[(int64_t)((jb + 1) * S + a) * ldh + jb * S + b] = st.Hs1[a * S + b];
    }
  }
  __syncthreads();
  double Tq[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) Tq[i] = st.T[i];
  for (int64_t r = (int64_t)lb * TPB + threadIdx.x; r < A.rows; r += (int64_t)A.nb * TPB) {
    double u[S];
#pragma unroll
    for (int t = 0; t < S; ++t) u[t] = A.U[r * S + t];
#pragma unroll
    for (int b = 0; b < S; ++b) {
      double v = 0.0;
#pragma unroll
      for (int a = 0; a < S; ++a) v = fma(u[a], Tq[a * S + b], v);
      static_cast<T *>(A.basis)[r * A.ldb + (jb + 1) * S + b] = (T)v;
      static_cast<T *>(A.pout)[r * S + b] = (T)v;
    }
  }
}

// ---- block Lanczos step j for both bases (Algorithm 4.1, steps 4-5) ----
// aux layout per basis: [nb_spmm] ||M V_j||^2, [nb_upd S^2] U^T U, [nb_qr S^2] second-pass Gram,
// [nb_spmm S^2] V_j^T U.
template <int S>
__device__ __forceinline__ double *aux_vju(const ArSide &A) {
  return A.aux + A.nb_spmm + (A.nb_upd + A.nb_qr) * S * S;
}

// U = M V_j - V_{j-1} H_{j-1,j} (H_{j-1,j} = H_{j,j-1}^T); partials of ||M V_j||^2 and V_j^T U.
template <int S, typename T>
__global__ __launch_bounds__(TPB) void lz_spmm_pair(ArPair P, int jb, int64_t ldh,
                                                    const DevState *ds) {
  if (ds->done) return;
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  double hup[S * S];  // hup[u][t] = H_{j-1,j}[u][t] = H[j s + t][(j-1) s + u]
#pragma unroll
  for (int u = 0; u < S; ++u)
#pragma unroll
    for (int t = 0; t < S; ++t)
      hup[u * S + t] = jb > 0 ? A.H[(int64_t)(jb * S + t) * ldh + (jb - 1) * S + u] : 0.0;
  double red[S * S + 1];
#pragma unroll
  for (int i = 0; i < S * S + 1; ++i) red[i] = 0.0;
  for (int64_t r0 = (int64_t)lb * TPB; r0 < A.rows; r0 += (int64_t)A.nb * TPB) {
    const int64_t r1 = (r0 + TPB < A.rows) ? r0 + TPB : A.rows;
    const int64_t r = r0 + threadIdx.x;
    double acc[S];
    if (A.sell.ci) {
      if (r < r1) sell_row<S>(A.sell, r, static_cast<const T *>(A.pin), S, acc);
    } else {
      spmm_rows<S>(r0, r1, A.rp, A.ci, A.val, static_cast<const T *>(A.pin), S, acc);
    }
    if (r < r1) {
#pragma unroll
      for (int t = 0; t < S; ++t) red[S * S] = fma(acc[t], acc[t], red[S * S]);
      if (jb > 0) {
        const T *vp = static_cast<const T *>(A.pout) + r * S;  // block j-1 (panel reused)
#pragma unroll
        for (int u = 0; u < S; ++u) {
          const double vu = (double)vp[u];
#pragma unroll
          for (int t = 0; t < S; ++t) acc[t] = fma(-vu, hup[u * S + t], acc[t]);
        }
      }
      const T *vj = static_cast<const T *>(A.pin) + r * S;
#pragma unroll
      for (int a = 0; a < S; ++a) {
        const double va = (double)vj[a];
#pragma unroll
        for (int t = 0; t < S; ++t) red[a * S + t] = fma(va, acc[t], red[a * S + t]);
      }
#pragma unroll
      for (int t = 0; t < S; ++t) A.U[r * S + t] = acc[t];
    }
  }
  __shared__ double lds[16 * (S * S + 1)];
  block_sum<S * S + 1>(red, lds);
  if (threadIdx.x == 0) {
    A.aux[lb] = red[S * S];
    double *vju = aux_vju<S>(A) + lb * S * S;
#pragma unroll
    for (int i = 0; i < S * S; ++i) vju[i] = red[i];
  }
}

// H_jj = V_j^T U from the partials (every workgroup forms it; workgroup 0 writes column block j
// of H: H_{j-1,j} and H_jj); U -= V_j H_jj; partials of U^T U.
template <int S, typename T>
__global__ __launch_bounds__(TPB) void lz_update_pair(ArPair P, int jb, int64_t ldh,
                                                      const DevState *ds) {
  if (ds->done) return;
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  double hjj[S * S];
  sum_records<S * S>(aux_vju<S>(A), A.nb_spmm, hjj);
  if (lb == 0 && threadIdx.x == 0) {
    for (int a = 0; a < S; ++a)
      for (int t = 0; t < S; ++t) {
        A.H[(int64_t)(jb * S + a) * ldh + jb * S + t] = hjj[a * S + t];
        if (jb > 0)
          A.H[(int64_t)((jb - 1) * S + a) * ldh + jb * S + t] =
              A.H[(int64_t)(jb * S + t) * ldh + (jb - 1) * S + a];
      }
  }
  double g[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) g[i] = 0.0;
  for (int64_t r = (int64_t)lb * TPB + threadIdx.x; r < A.rows; r += (int64_t)A.nb * TPB) {
    double u[S];
#pragma unroll
    for (int t = 0; t < S; ++t) u[t] = A.U[r * S + t];
    const T *vj = static_cast<const T *>(A.pin) + r * S;
#pragma unroll
    for (int a = 0; a < S; ++a) {
      const double va = (double)vj[a];
#pragma unroll
      for (int t = 0; t < S; ++t) u[t] = fma(-va, hjj[a * S + t], u[t]);
    }
#pragma unroll
    for (int t = 0; t < S; ++t) A.U[r * S + t] = u[t];
#pragma unroll
    for (int a = 0; a < S; ++a)
#pragma unroll
      for (int b = 0; b < S; ++b) g[a * S + b] = fma(u[a], u[b], g[a * S + b]);
  }
  __shared__ double lds[16 * S * S];
  block_sum<S * S>(g, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < S * S; ++i) A.aux[A.nb_spmm + lb * S * S + i] = g[i];
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Rows per gram chunk: large enough that the chunk partials stay a small fraction of the basis
// read (2 s / rpc), small enough for a few hundred workgroups, at most 512 chunks per basis.
int64_t gram_rpc(int s, int64_t rows, int64_t total_rows) {
  int64_t rpc = std::max<int64_t>(32 * s, cdiv(total_rows, 1024));
  rpc = std::min<int64_t>(rpc, std::max<int64_t>(16, cdiv(total_rows, 256)));
  rpc = std::max<int64_t>(rpc, cdiv(rows, 512));
  return std::max<int64_t>(rpc, 1);
}

struct Plan {
  ArPair P;
  int nchunk[2];
};

ArSide make_side(const SideDesc &d, const Scratch &sc, int idx, size_t half, size_t aux_len) {
  ArSide a{};
  a.rows = d.rows;
  a.nnz = d.nnz;
  a.rp = d.rp;
  a.ci = d.ci;
  a.val = d.val;
  a.basis = d.basis;
  a.ldb = d.ldb;
  a.H = d.H;
  a.U = d.U;
  a.coef = d.coef;
  a.ss = d.ss;
  a.sell = d.sell;
  a.part = sc.partials + (size_t)idx * half;
  a.aux = a.part + half - aux_len;
  a.cnt = sc.counters + CNT_PAIR + idx * 1536;
  return a;
}

// Sets the workgroup ranges of a launch with per-basis workgroup counts nb0, nb1.
void set_ranges(ArPair &P, int64_t nb0, int64_t nb1) {
  P.s[0].b0 = 0;
  P.s[0].nb = (int)nb0;
  P.s[1].b0 = (int)nb0;
  P.s[1].nb = (int)nb1;
}

unsigned total_blocks(const ArPair &P) {
  return (unsigned)(P.s[0].nb + (P.nsides > 1 ? P.s[1].nb : 0));
}

constexpr int64_t UROWS = 64;    // rows per update workgroup (16 per wave)
constexpr int64_t QR_MAXWG = 512;

// Workgroups of the row-tile kernels of one basis (spmm, local update, U^T U): at most ROW_WG,
// each taking row tiles lb, lb + nb, ...; fewer partial records for the next kernel to sum.
constexpr int64_t ROW_WG = 512;
int64_t nb_rows(int64_t rows) { return std::min<int64_t>(cdiv(rows, TPB), ROW_WG); }
int64_t nb_qr(int64_t rows) { return std::min<int64_t>(nb_rows(rows), QR_MAXWG); }
size_t aux_len(int s, int64_t rows) {
  return (size_t)(nb_rows(rows) + (cdiv(rows, UROWS) + nb_qr(rows) + nb_rows(rows)) * s * s + 16);
}

template <int S, typename T>
int arnoldi_pair_t(const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,
                   double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st) {
  ArPair P{};
  const size_t half = sc.partial_cap / 2;
  P.nsides = sw ? 2 : 1;
  const int64_t rows0 = sv.rows, rows1 = sw ? sw->rows : 0;
  const size_t aux0 = aux_len(S, rows0), aux1 = sw ? aux_len(S, rows1) : 0;
  P.s[0] = make_side(sv, sc, 0, half, aux0);
  if (sw) P.s[1] = make_side(*sw, sc, 1, half, aux1);
  for (int i = 0; i < P.nsides; ++i) {
    const int64_t rows = i ? rows1 : rows0;
    P.s[i].nb_spmm = (int)nb_rows(rows);
    P.s[i].nb_upd = (int)cdiv(rows, UROWS);
    P.s[i].nb_qr = (int)nb_qr(rows);
  }
  const int64_t total = rows0 + rows1;
  const int ncols = (jb + 1) * S;
  const int nout = ncols * S;
  const double bytes_v = (double)sizeof(T) * (double)total * ncols, flops_v = 2.0 * (double)total * ncols * S;

  // U = M V_j
  set_ranges(P, nb_rows(rows0), sw ? nb_rows(rows1) : 0);
  prof_begin(sc, st);
  for (int i = 0; i < P.nsides; ++i) {
    const SideDesc &d = i ? *sw : sv;
    P.s[i].pin = d.panel[jb % 2];
    P.s[i].pout = d.panel[(jb + 1) % 2];
  }
  spmm_pair<S, T><<<total_blocks(P), TPB, 0, st>>>(P, ds);
  HIPOK(hipGetLastError());
  prof_end(sc, FAM_SPMM,
           12.0 * (sv.nnz + (sw ? sw->nnz : 0)) + 4.0 * (total + 2) + 16.0 * total * S,
           2.0 * (sv.nnz + (sw ? sw->nnz : 0)) * S, st);

  // chunking of the Gram sweeps
  const int64_t rpc0 = gram_rpc(S, rows0, total), rpc1 = sw ? gram_rpc(S, rows1, total) : 1;
  const int nch0 = (int)cdiv(rows0, rpc0), nch1 = sw ? (int)cdiv(rows1, rpc1) : 0;
  if ((size_t)nch0 * nout + aux0 > half || (size_t)nch1 * nout + aux1 > half)
    return SYLV_ERR_WORKSPACE;
  // coefficient chunk of the MFMA update in LDS (at most 64 KiB)
  const size_t lds =
      (size_t)std::min((ncols + 127) / 128 * 128, UPD_KCH<S>()) * S * sizeof(double);
  const int64_t rtiles = cdiv(nout, OPB);

  for (int pass = 1; pass <= 2; ++pass) {
    P.s[0].rpc = rpc0;
    P.s[1].rpc = rpc1;
    set_ranges(P, nch0, nch1);
    prof_begin(sc, st);
    gram_part_pair<S, T><<<total_blocks(P), TPB, 0, st>>>(P, ncols, ds);
    HIPOK(hipGetLastError());
    set_ranges(P, rtiles, sw ? rtiles : 0);
    gram_reduce_pair<<<total_blocks(P), TPB, 0, st>>>(P, S, ncols, nch0, nch1, ldh, jb * S, pass,
                                                      ds);
    HIPOK(hipGetLastError());
    prof_end(sc, FAM_GRAM, bytes_v + 8.0 * total * S + 8.0 * nout * P.nsides, flops_v, st);
    P.s[0].rpc = UROWS;
    P.s[1].rpc = UROWS;
    set_ranges(P, cdiv(rows0, UROWS), sw ? cdiv(rows1, UROWS) : 0);
    prof_begin(sc, st);
    update_mfma_pair<S, T><<<total_blocks(P), TPB, lds, st>>>(P, ncols, ds);
    HIPOK(hipGetLastError());
    if (pass == 2) {
      // U^T U partials for the first QR pass (one record per 256 rows)
      for (int i = 0; i < P.nsides; ++i) P.s[i].nb_upd = (int)nb_rows(i ? rows1 : rows0);
      set_ranges(P, nb_rows(rows0), sw ? nb_rows(rows1) : 0);
      ugram_pair<S><<<total_blocks(P), TPB, 0, st>>>(P, ds);
      HIPOK(hipGetLastError());
    }
    prof_end(sc, FAM_UPDATE, bytes_v + 16.0 * total * S + 8.0 * nout * P.nsides, flops_v, st);
  }
  // QR passes and the new block
  set_ranges(P, nb_qr(rows0), sw ? nb_qr(rows1) : 0);
  prof_begin(sc, st);
  qr2_pair<S><<<total_blocks(P), TPB, 0, st>>>(P, closure_tol, ds);
  HIPOK(hipGetLastError());
  final_pair<S, T><<<total_blocks(P), TPB, 0, st>>>(P, jb, ldh, ds);
  HIPOK(hipGetLastError());
  prof_end(sc, FAM_QR, 8.0 * total * S * 3, 6.0 * total * S * S, st);
  return 0;
}


template <int S, typename T>
int lanczos_pair_t(const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,
                   double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st) {
  ArPair P{};
  const size_t half = sc.partial_cap / 2;
  P.nsides = sw ? 2 : 1;
  const int64_t rows0 = sv.rows, rows1 = sw ? sw->rows : 0;
  const size_t aux0 = aux_len(S, rows0), aux1 = sw ? aux_len(S, rows1) : 0;
  if (aux0 > half || aux1 > half) return SYLV_ERR_WORKSPACE;
  P.s[0] = make_side(sv, sc, 0, half, aux0);
  if (sw) P.s[1] = make_side(*sw, sc, 1, half, aux1);
  for (int i = 0; i < P.nsides; ++i) {
    const SideDesc &d = i ? *sw : sv;
    const int64_t rows = i ? rows1 : rows0;
    P.s[i].nb_spmm = (int)nb_rows(rows);
    P.s[i].nb_upd = (int)nb_rows(rows);  // U^T U partials come from lz_update_pair
    P.s[i].nb_qr = (int)nb_qr(rows);
    P.s[i].pin = d.panel[jb % 2];
    P.s[i].pout = d.panel[(jb + 1) % 2];
  }
  const int64_t total = rows0 + rows1;
  set_ranges(P, nb_rows(rows0), sw ? nb_rows(rows1) : 0);
  prof_begin(sc, st);
  lz_spmm_pair<S, T><<<total_blocks(P), TPB, 0, st>>>(P, jb, ldh, ds);
  HIPOK(hipGetLastError());
  lz_update_pair<S, T><<<total_blocks(P), TPB, 0, st>>>(P, jb, ldh, ds);
  HIPOK(hipGetLastError());
  // matrix + gather V_j + read V_{j-1}, V_j + U write/read (local three-term step)
  prof_end(sc, FAM_SPMM,
           12.0 * (sv.nnz + (sw ? sw->nnz : 0)) + 4.0 * (total + 2) + 8.0 * total * S * 6,
           2.0 * (sv.nnz + (sw ? sw->nnz : 0)) * S + 8.0 * total * S * S, st);
  set_ranges(P, nb_qr(rows0), sw ? nb_qr(rows1) : 0);
  prof_begin(sc, st);
  qr2_pair<S><<<total_blocks(P), TPB, 0, st>>>(P, closure_tol, ds);
  HIPOK(hipGetLastError());
  final_pair<S, T><<<total_blocks(P), TPB, 0, st>>>(P, jb, ldh, ds);
  HIPOK(hipGetLastError());
  prof_end(sc, FAM_QR, 8.0 * total * S * 3, 6.0 * total * S * S, st);
  return 0;
}

}  // namespace

size_t arnoldi_partials_needed(int s, int64_t rows_v, int64_t rows_w, int64_t max_cols) {
  const int64_t total = rows_v + rows_w;
  const int64_t n0 = cdiv(rows_v, gram_rpc(s, rows_v, total));
  const int64_t n1 = rows_w ? cdiv(rows_w, gram_rpc(s, rows_w, total)) : 0;
  const size_t per0 = (size_t)n0 * max_cols * s + aux_len(s, rows_v);
  const size_t per1 = rows_w ? (size_t)n1 * max_cols * s + aux_len(s, rows_w) : 0;
  return 2 * std::max(per0, per1);
}

int launch_arnoldi_pair(int s, const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,
                        double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st) {
  switch (s) {
#define CASE(SS) \
  case SS:                                                                         \
    return sv.fp32 ? arnoldi_pair_t<SS, float>(sv, sw, jb, ldh, closure_tol, sc, ds, st)   \
                   : arnoldi_pair_t<SS, double>(sv, sw, jb, ldh, closure_tol, sc, ds, st);
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return SYLV_ERR_INVALID;
  }
}

int launch_lanczos_pair(int s, const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,
                        double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st) {
  switch (s) {
#define CASE(SS) \
  case SS:                                                                         \
    return sv.fp32 ? lanczos_pair_t<SS, float>(sv, sw, jb, ldh, closure_tol, sc, ds, st)   \
                   : lanczos_pair_t<SS, double>(sv, sw, jb, ldh, closure_tol, sc, ds, st);
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return SYLV_ERR_INVALID;
  }
}
