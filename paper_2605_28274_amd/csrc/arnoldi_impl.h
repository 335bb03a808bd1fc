// Block Arnoldi step j for both bases at once (Algorithm 4.2, steps 5-6 and 10-11): the V basis
// of K(A, C1) and the W basis of K(B^T, C2) advance in lockstep, so every launch below covers
// both: workgroups [0, nb_0) work on basis 0 and [nb_0, nb_0 + nb_1) on basis 1. This halves
// the launches of the step and fills the GPU with the smaller basis' work as well.
//
// Step (per basis, M the operator, V the row-major rows x ldb basis, U a rows x s panel):
//   U = M V_j, partials of ||U||^2                                 spmm_pair
//   two classical Gram-Schmidt sweeps:
//     C1 = V[:, 0:ncols]^T U  (split-K over row chunks)           gram_part_pair
//     sum of the chunk partials -> H column block j, coef         gram_reduce_pair
//     U -= V C1 and the chunk partials of C2 = V^T U in one pass   upd_gram_pair
//       (narrow bases: update_mfma_pair, then gram_part_pair)
//     sum of the C2 partials -> H += C2, coef                     gram_reduce_pair
//     U -= V C2   (FP64 MFMA, coef staged in LDS)                  update_mfma_pair
//   (with the partials of U^T U)
//   first Cholesky-QR pass + closure test, partials of G2          qr2_pair
//   second pass, V_{j+1} = U T, H_{j+1,j}                          final_pair
// No kernel ends in a grid-wide fence: each reduction leaves one partial per workgroup and the
// next kernel sums them in a fixed order (deterministic) after the kernel boundary; the small
// s x s factorizations are then formed redundantly in every workgroup, and workgroup 0 records
// them.
//
// This header holds the kernels and the host step templates; the arnoldi_s*.hip units
// instantiate them for groups of block sizes (parallel compilation), arnoldi.hip dispatches.
#pragma once
#include <algorithm>
#include <type_traits>

#include "common.h"

namespace {

constexpr int TPB = 256;
constexpr int NG = 8;          // thread groups splitting the chunk sum in gram_reduce_pair
constexpr int OPB = TPB / NG;  // outputs per gram_reduce_pair workgroup
constexpr int GRAM_LOADS = 16; // 8-byte basis loads in flight per thread in gram_part_pair
constexpr int GRAM_UCH = 128;  // right-hand rows staged in LDS at a time by gram_part_pair

// The kernels of the block Arnoldi sweeps (SpMM, Gram, update, QR) run on the Krylov stream
// beside the core product's matrix-core waves (two streams); they are the longer chain, so
// their waves take the higher issue priority on a SIMD they share (1% on the C2 solve).
__device__ __forceinline__ void krylov_wave_priority() { __builtin_amdgcn_s_setprio(3); }

// Algorithmic bytes of one pass over a side's operator: value and column index per entry (12
// bytes as CSR or wide SELL, 6 in the narrow SELL form).
inline double mat_bytes(const SideDesc &d) {
  return (d.sell.ci && d.sell.narrow ? 6.0 : 12.0) * (double)d.nnz;
}

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
  const void *pprev;  // block Lanczos: compact copy of block j-1
  const void *ring;   // block Lanczos: slot k of the block ring at ring + k rows s elements
  double *part;    // Gram chunk partials of this basis
  double *aux;     // partials of ||M V_j||^2, U^T U and of the second-pass Gram
  int *cnt;        // counters of this basis (unused: no grid-wide reductions)
  int nb_spmm, nb_upd, nb_qr;  // workgroups whose partials sit in aux
  int b0, nb;      // workgroup range of this basis in the current launch
  int64_t rpc;     // rows per chunk (gram) or rows per workgroup (update)
  int64_t ldh;     // row stride of H
  int nch;         // Gram chunks of this basis (partials the reduction sums)
  const int *done; // the problem's stop flag (instance tables; null for a pair)
};

struct ArPair {
  ArSide s[2];
  int nsides;
};

// The basis this workgroup works on (selected without dynamic indexing of the kernel argument)
// and the workgroup's index within that basis' range.
__device__ __forceinline__ ArSide side_of(const ArPair &P, int &lb, int &sd,
                                          int bid = (int)blockIdx.x) {
  sd = (P.nsides > 1 && bid >= P.s[1].b0) ? 1 : 0;
  const ArSide A = sd ? P.s[1] : P.s[0];
  lb = bid - A.b0;
  return A;
}

// Compact block copies of one basis: the SpMM input and output of step jb are slots jb % ring
// and (jb + 1) % ring (block Lanczos also reads slot (jb - 1) % ring and keeps the ring at 0).
struct PanelSet {
  void *p[LZ_RING];
};

// The bases of many independent problems in one launch (batches): entry i of `sides` (device
// memory) is basis i with its workgroup range, chunking and record counts for this launch kind;
// `owner` maps a workgroup to its basis, or, when every basis has unb workgroups, basis
// bid / unb. The compact block slots follow from the step index jb.
struct ArTab {
  const ArSide *sides;
  const unsigned short *owner;
  const PanelSet *panels;
  int nsides, unb, jb, ring;
};

__device__ __forceinline__ int owner_of(const ArTab &P, int bid) {
  return P.unb > 0 ? bid / P.unb : (int)P.owner[bid];
}

__device__ __forceinline__ ArSide side_of(const ArTab &P, int &lb, int &sd,
                                          int bid = (int)blockIdx.x) {
  sd = owner_of(P, bid);
  ArSide A = P.sides[sd];
  if (P.unb > 0) {
    A.b0 = sd * P.unb;
    A.nb = P.unb;
  }
  const PanelSet &ps = P.panels[sd];
  const int r = P.ring;
  A.pin = ps.p[P.jb % r];
  A.pout = ps.p[(P.jb + 1) % r];
  A.pprev = ps.p[(P.jb + r - 1) % r];
  A.ring = ps.p[0];
  lb = bid - A.b0;
  return A;
}

// A workgroup returns at once when its problem has stopped: the pair's solve flag, or the flag
// of the instance whose basis the workgroup serves.
__device__ __forceinline__ bool halted(const ArPair &, const DevState *ds, int = 0) {
  return ds->done != 0;
}
__device__ __forceinline__ bool halted(const ArTab &P, const DevState *,
                                       int bid = (int)blockIdx.x) {
  return *P.sides[owner_of(P, bid)].done != 0;
}

// Rows a thread handles at once in the SpMM kernels (sliced ELLPACK): more loads in flight for
// narrow blocks.
template <int S>
constexpr int spmm_nr() { return S == 2 ? 2 : 1; }

template <int S, typename T, class PS>
__global__ __launch_bounds__(TPB) void spmm_pair(PS P, const DevState *ds) {
  krylov_wave_priority();
  if (halted(P, ds)) return;
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  double red[1] = {0.0};
  // row tiles lb, lb + nb, ... (at most ROW_WG workgroups per basis, so few partials)
  if (A.sell.ci) {
    constexpr int NR = spmm_nr<S>();
    const int64_t step = (int64_t)A.nb * TPB;
    for (int64_t r0 = (int64_t)lb * TPB + threadIdx.x; r0 < A.rows; r0 += NR * step) {
      int64_t r[NR];
      bool ok[NR];
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        r[i] = r0 + i * step;
        ok[i] = r[i] < A.rows;
      }
      double acc[NR][S];
      sell_rows<NR, S>(A.sell, r, ok, static_cast<const T *>(A.pin), S, acc);
#pragma unroll
      for (int i = 0; i < NR; ++i)
        if (ok[i])
#pragma unroll
          for (int t = 0; t < S; ++t) {
            A.U[r[i] * S + t] = acc[i][t];
            red[0] = fma(acc[i][t], acc[i][t], red[0]);
          }
    }
  } else {
    for (int64_t r0 = (int64_t)lb * TPB; r0 < A.rows; r0 += (int64_t)A.nb * TPB) {
      const int64_t r1 = (r0 + TPB < A.rows) ? r0 + TPB : A.rows;
      double acc[S];
      const int64_t r = r0 + threadIdx.x;
      spmm_rows<S>(r0, r1, A.rp, A.ci, A.val, static_cast<const T *>(A.pin), S, acc);
      if (r < r1) {
#pragma unroll
        for (int t = 0; t < S; ++t) {
          A.U[r * S + t] = acc[t];
          red[0] = fma(acc[t], acc[t], red[0]);
        }
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

// Chunk partials of C = V^T U. Workgroup lb owns rows [lb rpc, (lb+1) rpc) of its basis. Its
// threads form G = TPB / CW row groups of CW threads (CW a power of two fitted to the width):
// thread (g, l) owns the 8-byte column groups l + CW q (q < nq <= NQ; one double or two floats
// each) and takes the rows g, g + G, ... of the chunk, RU rows per step, so that NQ RU loads are
// in flight; a narrow basis thus still spreads its chunk over every thread. The right-hand rows
// pass through LDS (GRAM_UCH rows at a time, read as broadcasts). The row-group sums are added
// in a fixed order through LDS. part[lb][c][t]; column groups past the width load
// group 0 and rows past the chunk load its first row (both in bounds), neither is counted.
// DUAL: the right-hand side is [pin, U] (S / 2 columns each: the provisional block and M times
// it, for the lagged step), else U (S columns).
template <int S, typename T, int NQ, bool DUAL = false, class PS>
__global__ __launch_bounds__(TPB) void gram_part_pair(PS P, int ncols, int cw_log2,
                                                      const DevState *ds) {
  krylov_wave_priority();
  if (halted(P, ds)) return;
  typedef Pack8<T> PK;
  typedef typename PK::type V8;
  constexpr int E = PK::N;
  // rows per step: GRAM_LOADS basis loads in flight; the right-hand rows come from LDS
  constexpr int RU = NQ >= GRAM_LOADS ? 1 : (GRAM_LOADS / NQ > 8 ? 8 : GRAM_LOADS / NQ);
  extern __shared__ double gsum[];  // TPB * E * S doubles (several row groups only)
  __shared__ double Us[GRAM_UCH * S];
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  const int CW = 1 << cw_log2, G = TPB >> cw_log2;
  const int g = (int)threadIdx.x >> cw_log2, l = (int)threadIdx.x & (CW - 1);
  const int64_t r0 = (int64_t)lb * A.rpc;
  const int64_t r1 = (r0 + A.rpc < A.rows) ? r0 + A.rpc : A.rows;
  double *part = A.part + (size_t)lb * ncols * S;
  const T *basis = static_cast<const T *>(A.basis);
  const int ng = (ncols + E - 1) / E;
  for (int q0 = 0; q0 < ng; q0 += CW * NQ) {
    const int nq = (ng - q0 + CW - 1) / CW < NQ ? (ng - q0 + CW - 1) / CW : NQ;  // uniform
    int coff[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int gi = q0 + q * CW + l;
      coff[q] = (gi < ng ? gi : 0) * E;
    }
    double acc[NQ][E][S];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int e = 0; e < E; ++e)
#pragma unroll
        for (int t = 0; t < S; ++t) acc[q][e][t] = 0.0;
    for (int64_t rb = r0; rb < r1; rb += GRAM_UCH) {
      const int nr = (int)((r1 - rb < GRAM_UCH) ? r1 - rb : GRAM_UCH);
      __syncthreads();  // the previous rows' readers are done
      for (int e = threadIdx.x; e < nr * S; e += TPB) {
        const int64_t row = rb + e / S;
        const int t = e % S;
        double uv;
        if (DUAL && t < S / 2) uv = (double)static_cast<const T *>(A.pin)[row * (S / 2) + t];
        else uv = DUAL ? A.U[row * (S / 2) + t - S / 2] : A.U[row * S + t];
        Us[e] = uv;
      }
      __syncthreads();
      const T *vb = basis + rb * A.ldb;
      for (int rr = g; rr < nr; rr += RU * G) {
        V8 v[RU][NQ];
#pragma unroll
        for (int h = 0; h < RU; ++h) {
          const int rl = rr + h * G;
          const T *vr = vb + (int64_t)(rl < nr ? rl : 0) * A.ldb;
#pragma unroll
          for (int q = 0; q < NQ; ++q)
            v[h][q] = (q < nq) ? *reinterpret_cast<const V8 *>(vr + coff[q]) : PK::zero();
        }
#pragma unroll
        for (int h = 0; h < RU; ++h) {
          const int rl = rr + h * G;
          const bool ok = rl < nr;
          double u[S];
#pragma unroll
          for (int t = 0; t < S; ++t) u[t] = ok ? Us[rl * S + t] : 0.0;
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            if (q >= nq) continue;
            double x[E];
            PK::get(v[h][q], x);
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
              for (int t = 0; t < S; ++t) acc[q][e][t] = fma(x[e], u[t], acc[q][e][t]);
          }
        }
      }
    }
    if (G > 1) {
      // row groups in order: group 0 adds the others' sums (one q at a time through LDS)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (q >= nq) continue;
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
          for (int t = 0; t < S; ++t) gsum[(size_t)threadIdx.x * E * S + e * S + t] = acc[q][e][t];
        __syncthreads();
        if (g == 0) {
#pragma unroll
          for (int e = 0; e < E; ++e)
#pragma unroll
            for (int t = 0; t < S; ++t) {
              double a = 0.0;
              for (int gg = 0; gg < G; ++gg) a += gsum[(size_t)(gg * CW + l) * E * S + e * S + t];
              acc[q][e][t] = a;
            }
        }
      }
    }
    if (g == 0) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (q >= nq) continue;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int c = (q0 + q * CW + l) * E + e;
          if (c < ncols)
#pragma unroll
            for (int t = 0; t < S; ++t) part[c * S + t] = acc[q][e][t];
        }
      }
    }
  }
}

// Sums the nchunk partials of OPB consecutive outputs per workgroup: thread group g (of NG)
// adds chunks [g nchunk / NG, (g+1) nchunk / NG) for its output (eight loads in flight, added
// in chunk order), then group 0 adds the NG group sums in order and writes column block j of H
// (store in sweep 1, add in sweep 2; pass 0: coefficients only) and the compact coefficients.
template <class PS>
__global__ __launch_bounds__(TPB) void gram_reduce_pair(PS P, int S, int ncols, int hcol,
                                                        int pass, const DevState *ds) {
  krylov_wave_priority();
  if (halted(P, ds)) return;
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  __shared__ double gs[NG][OPB];
  const int nchunk = A.nch;
  const int nout = ncols * S;
  const int ol = threadIdx.x % OPB, g = threadIdx.x / OPB;
  const int o = lb * OPB + ol;
  const int q0 = (int)((int64_t)nchunk * g / NG), q1 = (int)((int64_t)nchunk * (g + 1) / NG);
  double a = 0.0;
  if (o < nout) {
    constexpr int U8 = 8;
    int q = q0;
    for (; q + U8 <= q1; q += U8) {
      double x[U8];
#pragma unroll
      for (int k = 0; k < U8; ++k) x[k] = A.part[(size_t)(q + k) * nout + o];
#pragma unroll
      for (int k = 0; k < U8; ++k) a += x[k];
    }
    for (; q < q1; ++q) a += A.part[(size_t)q * nout + o];
  }
  gs[g][ol] = a;
  __syncthreads();
  if (g == 0 && o < nout) {
    double b = 0.0;
#pragma unroll
    for (int q = 0; q < NG; ++q) b += gs[q][ol];
    const int c = o / S, t = o % S;
    if (pass > 0) {
      double *h = A.H + (int64_t)c * A.ldh + hcol + t;
      *h = (pass == 1) ? b : *h + b;
    }
    A.coef[o] = b;
  }
}

// Columns of the coefficient block staged in LDS at a time by update_mfma_pair (64 KiB, whole
// groups of 128 columns).
template <int S>
__host__ __device__ constexpr int UPD_KCH() {
  return (64 * 1024 / (S * 8)) / 128 * 128;
}

typedef double v4d_t __attribute__((ext_vector_type(4)));

// D = V[r, 0:ncols] C on FP64 matrix cores (v_mfma_f64_16x16x4f64) for the wave's 16 rows
// [rb, rb + 16) (C: ncols x SC row-major coefficients, SC <= 16): D (16 x 16) += A (16 rows x 4
// basis columns) B (4 x 16, coefficient columns >= SC are zero). Lane l reads 32 contiguous bytes
// of row l % 16 per step (KL consecutive columns, chunk l / 16), so the four lanes of a row
// cover 128 contiguous bytes; MFMA m of the step takes column k0 + KL (l / 16) + m as its k-slot
// l / 16 on both operands (the sum over k is the same). The coefficients pass through LDS (Cs)
// in chunks, zero-padded past ncols; basis columns past ncols read as zero (they may be stale).
// On return lane l holds D[4 v + l / 16][l % 16] in acc0[v] + acc1[v]. Every thread of the
// workgroup must call it (barriers).
template <int SC, typename T>
__device__ __forceinline__ void update_acc(const ArSide &A, const double *coef, int ncols,
                                           double *Cs, int64_t rb, int64_t r1, v4d_t &acc0,
                                           v4d_t &acc1) {
  constexpr int KL = 32 / (int)sizeof(T);  // columns per lane per step
  constexpr int KG = 4 * KL;               // columns per step
  constexpr int KU = 4;                    // steps whose loads are in flight together
  const int lane = threadIdx.x & (WAVE - 1);
  const int li = lane & 15, lq = lane >> 4;
  const int nk = (ncols + KG - 1) / KG * KG;
  const bool live = rb < r1;
  const int64_t row = (rb + li < r1) ? rb + li : r1 - 1;  // clamped loads, masked stores
  const T *vr = static_cast<const T *>(A.basis) + row * A.ldb + lq * KL;
  acc0 = v4d_t{0.0, 0.0, 0.0, 0.0};
  acc1 = v4d_t{0.0, 0.0, 0.0, 0.0};
  // the coefficients pass through LDS in chunks of at most 64 KiB
  for (int c0 = 0; c0 < nk; c0 += UPD_KCH<SC>()) {
    const int c1 = (c0 + UPD_KCH<SC>() < nk) ? c0 + UPD_KCH<SC>() : nk;
    __syncthreads();
    for (int e = threadIdx.x; e < (c1 - c0) * SC; e += TPB) {
      const int g = c0 * SC + e;
      Cs[e] = g < ncols * SC ? coef[g] : 0.0;
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
          const double bv = (step && li < SC) ? Cs[(k - c0) * SC + li] : 0.0;
          if (m & 1) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc1, 0, 0, 0);
          else acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc0, 0, 0, 0);
        }
      }
    }
  }
}

// Partials of U^T U of the workgroup's rows (one record per workgroup, at aux[nb_spmm + lb S^2]):
// lane li = a of each 16-lane group holds u[rb + 4 v + lq][a] in uv[v] (zero past the rows);
// it adds u[r][a] u[r][b] over its rows, then the groups and the waves are summed in order.
template <int S>
__device__ __forceinline__ void upart_record(const ArSide &A, int lb, const double (&uv)[4]) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  __shared__ double gs[TPB / WAVE][S * S];
  double g[S];
#pragma unroll
  for (int b = 0; b < S; ++b) {
    g[b] = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) g[b] = fma(uv[v], __shfl(uv[v], (lane & 48) | b, WAVE), g[b]);
    g[b] += __shfl_xor(g[b], 16, WAVE);
    g[b] += __shfl_xor(g[b], 32, WAVE);
  }
  if (lane < S)
#pragma unroll
    for (int b = 0; b < S; ++b) gs[w][lane * S + b] = g[b];
  __syncthreads();
  if ((int)threadIdx.x < S * S) {
    double a = 0.0;
#pragma unroll
    for (int ww = 0; ww < TPB / WAVE; ++ww) a += gs[ww][threadIdx.x];
    A.aux[A.nb_spmm + lb * S * S + threadIdx.x] = a;
  }
}

// U[r] -= V[r, 0:ncols] C for the workgroup's UROWS rows (16 per wave); with upart, also the
// partials of U^T U of the updated rows for the first QR pass.
template <int S, typename T, class PS>
__global__ __launch_bounds__(TPB) void update_mfma_pair(PS P, int ncols, int upart,
                                                        const DevState *ds) {
  if (halted(P, ds)) return;
  extern __shared__ double Cs[];
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int li = lane & 15, lq = lane >> 4;
  const int64_t r0 = (int64_t)lb * A.rpc;
  const int64_t r1 = (r0 + A.rpc < A.rows) ? r0 + A.rpc : A.rows;
  const int64_t rb = r0 + 16 * w;
  v4d_t acc0, acc1;
  update_acc<S, T>(A, A.coef, ncols, Cs, rb, r1, acc0, acc1);
  // lane holds D[4 v + lq][li]: row rb + 4 v + lq, column li
  double uv[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t r = rb + 4 * v + lq;
    uv[v] = 0.0;
    if (li < S && r < r1) {
      uv[v] = A.U[r * S + li] - (acc0[v] + acc1[v]);
      A.U[r * S + li] = uv[v];
    }
  }
  if (upart) upart_record<S>(A, lb, uv);
}

// ---- lagged reorthogonalization (block Arnoldi with classical Gram-Schmidt, two passes) ----
// Block j arrives provisional: V~_j, orthogonalized once and normalized (block 0 is final). Step
// j computes U = M V~_j and, in one pass over the basis, the coefficients
//   [a b; d c] = [V_{0..j-1}; V~_j]^T [V~_j, U]                     (gram_part_pair, DUAL)
// then (dcgs_fix_pair) the second pass of block j: w = V~_j - V a, w^T w = d - a^T a, V_j = w Tw
// (Cholesky, or the closure / deflation rule of the first-pass QR), the final column block j-1
// of H from the provisional one, and e = V_j^T U = Tw^T (c - a^T b); then, in one more pass
// (dcgs_update_pair), the final rows of V_j and U' = (U - V_{0..j-1} b - V_j e) Tw = M V_j -
// V_{0..j} C, the first-pass projection of the new direction; dcgs_hcol_body writes the
// provisional column block j of H, C = ([b; e] - H a) Tw (M V a = V H a by the Arnoldi relation
// of the earlier columns); the QR of U' (qr2_pair, final_pair) gives the provisional V~_{j+1}.
// Two passes over the basis per step instead of three; the arithmetic is classical Gram-Schmidt
// applied twice with the second pass of each block taken one step later.

// One workgroup per basis: Tw, Hw, e and the provisional subdiagonal block Rt of column block
// j-1 (SideState); dcgs_hcol_body completes column block j-1 from them.
template <int S, class PS>
__global__ __launch_bounds__(TPB) void dcgs_fix_pair(PS P, int jb, double closure_tol,
                                                     const DevState *ds) {
  krylov_wave_priority();
  if (halted(P, ds)) return;
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  constexpr int S2 = 2 * S, U4 = 4;
  const int nf = jb * S;  // final columns
  __shared__ double lds[16 * 2 * S * S];
  __shared__ SideState st;
  double g[2 * S * S];  // a^T a, a^T b
#pragma unroll
  for (int i = 0; i < 2 * S * S; ++i) g[i] = 0.0;
  for (int c0 = threadIdx.x; c0 < nf; c0 += U4 * TPB) {
    double av[U4][S], bv[U4][S];
#pragma unroll
    for (int u = 0; u < U4; ++u) {
      const int c = c0 + u * TPB;
      const bool ok = c < nf;
#pragma unroll
      for (int t = 0; t < S; ++t) {
        av[u][t] = ok ? A.coef[c * S2 + t] : 0.0;
        bv[u][t] = ok ? A.coef[c * S2 + S + t] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < U4; ++u)
#pragma unroll
      for (int p = 0; p < S; ++p)
#pragma unroll
        for (int q = 0; q < S; ++q) {
          g[p * S + q] = fma(av[u][p], av[u][q], g[p * S + q]);
          g[S * S + p * S + q] = fma(av[u][p], bv[u][q], g[S * S + p * S + q]);
        }
  }
  block_sum<2 * S * S>(g, lds);
  if (threadIdx.x != 0) return;
  double dd[S * S], cc[S * S], Rt[S * S];
  for (int p = 0; p < S; ++p)
    for (int q = 0; q < S; ++q) {
      dd[p * S + q] = A.coef[(nf + p) * S2 + q];
      cc[p * S + q] = A.coef[(nf + p) * S2 + S + q];
      Rt[p * S + q] = jb > 0 ? A.H[(int64_t)(nf + p) * A.ldh + nf - S + q] : 0.0;
    }
  double Gw[S * S], tr = 0.0;
  for (int i = 0; i < S * S; ++i) {
    Gw[i] = dd[i] - g[i];
    cc[i] -= g[S * S + i];
  }
  for (int p = 0; p < S; ++p) tr += dd[p * S + p];
  if (jb == 0) {  // block 0 is final: V_0 = V~_0
    for (int i = 0; i < S * S; ++i) st.T1[i] = st.Hs1[i] = (i % (S + 1) == 0) ? 1.0 : 0.0;
    st.mode = 0;
  } else {
    st.ref2 = tr;
    finish_pass1(&st, S, closure_tol, Gw);
  }
  for (int p = 0; p < S; ++p)
    for (int q = 0; q < S; ++q) {
      double v = 0.0;  // e = Tw^T (c - a^T b)
      for (int t = 0; t < S; ++t) v = fma(st.T1[t * S + p], cc[t * S + q], v);
      A.ss->Ew[p * S + q] = v;
      A.ss->Tw[p * S + q] = st.T1[p * S + q];
      A.ss->Hw[p * S + q] = st.Hs1[p * S + q];
      A.ss->Rt[p * S + q] = Rt[p * S + q];
    }
  A.ss->modew = st.mode;
}

// The second pass of block j and the first pass of U in one pass over V_{0..j-1}: X = V [a b]
// on matrix cores (2S coefficient columns), then per row V_j = (V~_j - X_a) Tw (written over the
// provisional block) and U' = (U - X_b - V_j e) Tw; partials of U'^T U'.
template <int S, class PS>
__global__ __launch_bounds__(TPB) void dcgs_update_pair(PS P, int jb, const DevState *ds) {
  krylov_wave_priority();
  if (halted(P, ds)) return;
  constexpr int S2 = 2 * S;
  extern __shared__ double Cs[];
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int li = lane & 15, lq = lane >> 4;
  const int64_t r0 = (int64_t)lb * A.rpc;
  const int64_t r1 = (r0 + A.rpc < A.rows) ? r0 + A.rpc : A.rows;
  const int64_t rb = r0 + 16 * w;
  const int nf = jb * S;
  v4d_t acc0, acc1;
  update_acc<S2, double>(A, A.coef, nf, Cs, rb, r1, acc0, acc1);
  double Tw[S * S], Ew[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) {
    Tw[i] = A.ss->Tw[i];
    Ew[i] = A.ss->Ew[i];
  }
  double *basis = static_cast<double *>(A.basis);
  const int col = li < S ? li : 0;
  double uv[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t r = rb + 4 * v + lq;
    const bool ok = r < r1;
    const int64_t rr = ok ? r : r1 - 1;
    const double x = acc0[v] + acc1[v];  // X[r][li]
    double wv[S], vv[S], z[S];
#pragma unroll
    for (int t = 0; t < S; ++t)
      wv[t] = basis[rr * A.ldb + nf + t] - __shfl(x, (lane & 48) | t, WAVE);
    double vq = 0.0;  // V_j[r][col]
#pragma unroll
    for (int t = 0; t < S; ++t) vq = fma(wv[t], Tw[t * S + col], vq);
#pragma unroll
    for (int q = 0; q < S; ++q) vv[q] = __shfl(vq, (lane & 48) | q, WAVE);
#pragma unroll
    for (int t = 0; t < S; ++t) {
      double zt = A.U[rr * S + t] - __shfl(x, (lane & 48) | (S + t), WAVE);
#pragma unroll
      for (int q = 0; q < S; ++q) zt = fma(-vv[q], Ew[q * S + t], zt);
      z[t] = zt;
    }
    double uq = 0.0;
#pragma unroll
    for (int t = 0; t < S; ++t) uq = fma(z[t], Tw[t * S + col], uq);
    uv[v] = (ok && li < S) ? uq : 0.0;
    if (ok && li < S) {
      basis[r * A.ldb + nf + li] = vq;
      A.U[r * S + li] = uq;
    }
  }
  upart_record<S>(A, lb, uv);
}

// Column blocks j-1 (final) and j (provisional) of H, one wave per row i < (j+1) S: the
// provisional U'_{j-1} = V~_j Rt = (V a + V_j Hw) Rt gives H[i, j-1] += a[i] Rt (rows i < j s)
// and H[j, j-1] = Hw Rt; then C[i] = ([b; e][i] - H[i, 0:nf] a) Tw with the completed column
// block j-1 (H[i, c] is zero for c < (i/S - 1) S).
template <int S, class PS>
__device__ __forceinline__ void dcgs_hcol_body(const PS &P, int bid, int jb) {
  constexpr int S2 = 2 * S, U4 = 4;
  int lb, sd;
  const ArSide A = side_of(P, lb, sd, bid);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int nf = jb * S, nrow = nf + S;
  const int i = lb * (TPB / WAVE) + w;
  if (i >= nrow) return;
  int cs = (i / S - 1) * S;
  cs = cs < 0 ? 0 : cs;
  const int ce = nf - S;  // columns [ce, nf) are completed below (jb >= 1)
  double acc[S];
#pragma unroll
  for (int t = 0; t < S; ++t) acc[t] = 0.0;
  const int cend = jb > 0 ? ce : nf;
  for (int c0 = cs + lane; c0 < cend; c0 += U4 * WAVE) {
    double h[U4], a[U4][S];
#pragma unroll
    for (int u = 0; u < U4; ++u) {
      const int c = c0 + u * WAVE;
      const bool ok = c < cend;
      h[u] = ok ? A.H[(int64_t)i * A.ldh + c] : 0.0;
#pragma unroll
      for (int t = 0; t < S; ++t) a[u][t] = ok ? A.coef[c * S2 + t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U4; ++u)
#pragma unroll
      for (int t = 0; t < S; ++t) acc[t] = fma(h[u], a[u][t], acc[t]);
  }
  if (jb > 0 && lane == 0) {
    // complete H[i, ce:nf) and add its part of H a
    double hf[S];
    for (int q = 0; q < S; ++q) {
      double v = 0.0;
      if (i < nf) {
        v = A.H[(int64_t)i * A.ldh + ce + q];
        for (int t = 0; t < S; ++t) v = fma(A.coef[i * S2 + t], A.ss->Rt[t * S + q], v);
      } else {
        for (int t = 0; t < S; ++t) v = fma(A.ss->Hw[(i - nf) * S + t], A.ss->Rt[t * S + q], v);
      }
      hf[q] = v;
    }
    for (int q = 0; q < S; ++q) {
      A.H[(int64_t)i * A.ldh + ce + q] = hf[q];
      for (int t = 0; t < S; ++t) acc[t] = fma(hf[q], A.coef[(ce + q) * S2 + t], acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < S; ++t) acc[t] = wave_sum(acc[t]);
  if (lane < S) {
    double y[S];
#pragma unroll
    for (int t = 0; t < S; ++t)
      y[t] = (i < nf ? A.coef[i * S2 + S + t] : A.ss->Ew[(i - nf) * S + t]) - acc[t];
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < S; ++t) v = fma(y[t], A.ss->Tw[t * S + lane], v);
    A.H[(int64_t)i * A.ldh + nf + lane] = v;
  }
}

// Sum of NP values over the 64 lanes of a wave by recursive halving (NP a power of two <= 64):
// at step i each lane keeps the half of its values selected by bit i of its lane id and adds
// its partner's copy of that half, so after log2(NP) steps every lane holds one value, then the
// remaining lane bits are folded in. Lane l ends with the wave total of value ws_index<NP>(l);
// lanes that share the low log2(NP) bits hold bit-identical totals (fixed order).
template <int NP>
__device__ __forceinline__ int ws_index(int lane) {
  int idx = 0;
#pragma unroll
  for (int i = 0; (NP >> (i + 1)) >= 1; ++i)
    if ((lane >> i) & 1) idx += NP >> (i + 1);
  return idx;
}

template <int NP, int H>
__device__ __forceinline__ void ws_step(double (&v)[NP], int lane, int bit) {
  const bool up = (lane >> bit) & 1;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const double keep = up ? v[j + H] : v[j];
    const double send = up ? v[j] : v[j + H];
    v[j] = keep + __shfl_xor(send, 1 << bit, WAVE);
  }
}

template <int NP>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[NP], int lane) {
  static_assert(NP >= 1 && NP <= 64 && (NP & (NP - 1)) == 0, "power of two up to 64");
  int bit = 0;
  if constexpr (NP >= 64) ws_step<NP, 32>(v, lane, bit++);
  if constexpr (NP >= 32) ws_step<NP, 16>(v, lane, bit++);
  if constexpr (NP >= 16) ws_step<NP, 8>(v, lane, bit++);
  if constexpr (NP >= 8) ws_step<NP, 4>(v, lane, bit++);
  if constexpr (NP >= 4) ws_step<NP, 2>(v, lane, bit++);
  if constexpr (NP >= 2) ws_step<NP, 1>(v, lane, bit++);
  double x = v[0];
  for (; bit < 6; ++bit) x += __shfl_xor(x, 1 << bit, WAVE);
  return x;
}

// Rows per block of the fused sweep (32 basis loads in flight per thread and buffer, at most 32
// reduced values) and the padded count of values reduced per block.
template <int S, int NQ>
struct UgShape {
  static constexpr int R0 = NQ >= 32 ? 1 : 32 / NQ;
  static constexpr int R = R0 * S > 32 ? (32 / S > 0 ? 32 / S : 1) : R0;
  static constexpr int NV = R * S;
  static constexpr int NP = NV <= 1 ? 1 : NV <= 2 ? 2 : NV <= 4 ? 4 : NV <= 8 ? 8 : NV <= 16 ? 16 : 32;
};

// First-sweep update U -= V[:, 0:ncols] C fused with the chunk partials of the second sweep's
// V^T U (classical Gram-Schmidt applied twice; the second projection needs the updated rows,
// which depend only on the same rows of V). Workgroup lb owns the Gram chunk [lb rpc,
// (lb+1) rpc); its 256 threads own the 8-byte column groups l + 256 q (q < nq <= NQ) and keep
// their coefficients in registers. Per block of R rows: the R x S partial row products are
// summed over the workgroup (wave reduce-scatter, the four wave totals added in order through
// LDS), the updated rows are written, and the basis values still in registers are multiplied
// by them into the chunk partials part[lb][c][t]. The next block's loads are issued before the
// current block is reduced. Basis columns past ncols are masked to zero (they may be stale).
template <int S, typename T, int NQ, class PS>
__global__ __launch_bounds__(TPB) void upd_gram_pair(PS P, int ncols, const DevState *ds) {
  if (halted(P, ds)) return;
  typedef Pack8<T> PK;
  typedef typename PK::type V8;
  constexpr int E = PK::N;
  typedef UgShape<S, NQ> SH;
  constexpr int R = SH::R, NV = SH::NV, NP = SH::NP;
  __shared__ double red[TPB / WAVE][NP];
  __shared__ double un[NP];
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int64_t r0 = (int64_t)lb * A.rpc;
  const int64_t r1 = (r0 + A.rpc < A.rows) ? r0 + A.rpc : A.rows;
  const T *basis = static_cast<const T *>(A.basis);
  const int ng = (ncols + E - 1) / E;
  const int nq = (ng + TPB - 1) / TPB < NQ ? (ng + TPB - 1) / TPB : NQ;  // uniform
  // Column groups past the width read group 0 (a live column, finite) with zero coefficients;
  // with FP32 bases the second float of the last group may lie past ncols and is masked.
  int coff[NQ];
  bool okc[NQ][E];
  double cf[NQ][E][S], acc[NQ][E][S];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int gi = q * TPB + (int)threadIdx.x;
    coff[q] = (gi < ng ? gi : 0) * E;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int c = gi * E + e;
      okc[q][e] = c < ncols;
#pragma unroll
      for (int t = 0; t < S; ++t) {
        cf[q][e][t] = okc[q][e] ? A.coef[c * S + t] : 0.0;
        acc[q][e][t] = 0.0;
      }
    }
  }
  auto val = [&](const V8 &v, int q, double (&y)[E]) {
    PK::get(v, y);
    if (E > 1) {
#pragma unroll
      for (int e = 1; e < E; ++e) y[e] = okc[q][e] ? y[e] : 0.0;
    }
  };
  const int64_t nblk = (r1 - r0 + R - 1) / R;
  auto load_block = [&](int64_t b, V8 (&v)[R][NQ]) {
    const int64_t rb = r0 + (b < nblk ? b : nblk - 1) * R;  // past the end: reload the last
#pragma unroll
    for (int h = 0; h < R; ++h) {
      const int64_t row = (rb + h < r1) ? rb + h : r1 - 1;
      const T *vr = basis + row * A.ldb;
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        v[h][q] = (q < nq) ? *reinterpret_cast<const V8 *>(vr + coff[q]) : PK::zero();
    }
  };
  auto do_block = [&](int64_t b, const V8 (&v)[R][NQ]) {
    const int64_t rb = r0 + b * R;
    double d[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) d[i] = 0.0;
#pragma unroll
    for (int h = 0; h < R; ++h)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        double y[E];
        val(v[h][q], q, y);
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
          for (int t = 0; t < S; ++t) d[h * S + t] = fma(y[e], cf[q][e][t], d[h * S + t]);
      }
    const double tot = wave_reduce_scatter<NP>(d, lane);
    if (lane < NP) red[w][ws_index<NP>(lane)] = tot;
    __syncthreads();
    if ((int)threadIdx.x < NV) {
      const int h = (int)threadIdx.x / S, t = (int)threadIdx.x % S;
      const int64_t row = rb + h;
      double a = 0.0;
#pragma unroll
      for (int ww = 0; ww < TPB / WAVE; ++ww) a += red[ww][threadIdx.x];
      double u = 0.0;
      if (row < r1) {
        u = A.U[row * S + t] - a;
        A.U[row * S + t] = u;
      }
      un[threadIdx.x] = u;
    }
    __syncthreads();
    double uu[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) uu[i] = un[i];
#pragma unroll
    for (int h = 0; h < R; ++h)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        double y[E];
        val(v[h][q], q, y);
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
          for (int t = 0; t < S; ++t) acc[q][e][t] = fma(y[e], uu[h * S + t], acc[q][e][t]);
      }
  };
  V8 va[R][NQ], vb[R][NQ];
  load_block(0, va);
  for (int64_t b = 0; b < nblk; b += 2) {
    load_block(b + 1, vb);
    do_block(b, va);
    if (b + 1 < nblk) {
      load_block(b + 2, va);
      do_block(b + 1, vb);
    }
  }
  double *part = A.part + (size_t)lb * ncols * S;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (q >= nq) continue;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int c = (q * TPB + (int)threadIdx.x) * E + e;
      if (c < ncols)
#pragma unroll
        for (int t = 0; t < S; ++t) part[c * S + t] = acc[q][e][t];
    }
  }
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
template <int S, class PS>
__device__ __forceinline__ void qr2_body(const PS &P, int bid, double closure_tol) {
  int lb, sd;
  const ArSide A = side_of(P, lb, sd, bid);
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

template <int S, class PS>
__global__ __launch_bounds__(TPB) void qr2_pair(PS P, double closure_tol, const DevState *ds) {
  if (halted(P, ds)) return;
  qr2_body<S>(P, (int)blockIdx.x, closure_tol);
}

// The lagged step's last small kernels in one launch: workgroups [0, nq) run the first QR pass
// of U' (Pq ranges), the rest the column blocks j-1 and j of H (Ph ranges).
template <int S, class PS>
__global__ __launch_bounds__(TPB) void dcgs_tail_pair(PS Pq, PS Ph, int nq, int jb,
                                                      double closure_tol, const DevState *ds) {
  krylov_wave_priority();
  const int bid = (int)blockIdx.x;
  if (bid < nq ? halted(Pq, ds, bid) : halted(Ph, ds, bid - nq)) return;
  if (bid < nq) qr2_body<S>(Pq, bid, closure_tol);
  else dcgs_hcol_body<S>(Ph, bid - nq, jb);
}

// Second Cholesky-QR pass from the G2 partials (every workgroup forms the same factor), then
// the new block U T to the compact copy and, with to_basis, to V[:, (j+1)s : (j+2)s] (block
// Lanczos leaves the basis columns to lz_flush_pair); workgroup 0 records T and writes
// H_{j+1,j}. ONEPASS (a single column, s = 1): the QR of one column is its normalization, the
// first pass alone (closure test, T = 1 / ||U||, H_{j+1,j} = ||U||), formed here from the
// partials of ||M V_j||^2 and U^T U, so qr2_pair does not run.
template <int S, typename T, bool ONEPASS, class PS>
__device__ __forceinline__ void final_body(const PS &P, int bid, int jb, int to_basis,
                                           double closure_tol) {
  int lb, sd;
  const ArSide A = side_of(P, lb, sd, bid);
  __shared__ SideState st;
  if (ONEPASS) {
    double ref[1], G1[S * S];
    sum_records<1>(A.aux, A.nb_spmm, ref);
    sum_records<S * S>(A.aux + A.nb_spmm, A.nb_upd, G1);
    if (threadIdx.x == 0) {
      st.ref2 = ref[0];
      finish_pass1(&st, S, closure_tol, G1);
      for (int i = 0; i < S * S; ++i) st.T[i] = st.T1[i];
      if (lb == 0) {
        A.ss->ref2 = st.ref2;
        A.ss->mode = st.mode;
        for (int i = 0; i < S * S; ++i) A.ss->T1[i] = st.T1[i];
      }
    }
  } else {
    double G2[S * S];
    sum_records<S * S>(A.aux + A.nb_spmm + A.nb_upd * S * S, A.nb_qr, G2);
    if (threadIdx.x == 0) {
      st.mode = A.ss->mode;
      for (int i = 0; i < S * S; ++i) {
        st.T1[i] = A.ss->T1[i];
        st.Hs1[i] = A.ss->Hs1[i];
      }
      finish_pass2(&st, S, G2);
    }
  }
  if (threadIdx.x == 0 && lb == 0) {
    for (int i = 0; i < S * S; ++i) {
      A.ss->T[i] = st.T[i];
      A.ss->Hs1[i] = st.Hs1[i];
    }
    for (int a = 0; a < S; ++a)
      for (int b = 0; b < S; ++b)
        A.H[(int64_t)((jb + 1) * S + a) * A.ldh + jb * S + b] = st.Hs1[a * S + b];
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
      if (to_basis) static_cast<T *>(A.basis)[r * A.ldb + (jb + 1) * S + b] = (T)v;
      static_cast<T *>(A.pout)[r * S + b] = (T)v;
    }
  }
}

template <int S, typename T, bool ONEPASS = false, class PS>
__global__ __launch_bounds__(TPB) void final_pair(PS P, int jb, int to_basis, double closure_tol,
                                                  const DevState *ds) {
  krylov_wave_priority();
  if (halted(P, ds)) return;
  final_body<S, T, ONEPASS>(P, (int)blockIdx.x, jb, to_basis, closure_tol);
}

// ---- block Lanczos step j for both bases (Algorithm 4.1, steps 4-5) ----
// aux layout per basis: [nb_spmm] ||M V_j||^2, [nb_upd S^2] U^T U, [nb_qr S^2] second-pass Gram,
// [nb_spmm S^2] V_j^T U.
template <int S>
__device__ __forceinline__ double *aux_vju(const ArSide &A) {
  return A.aux + A.nb_spmm + (A.nb_upd + A.nb_qr) * S * S;
}

// U = M V_j - V_{j-1} H_{j-1,j} (H_{j-1,j} = H_{j,j-1}^T); partials of ||M V_j||^2 and V_j^T U.
template <int S, typename T, class PS>
__device__ __forceinline__ void lz_spmm_body(const PS &P, int bid, int jb) {
  int lb, sd;
  const ArSide A = side_of(P, lb, sd, bid);
  double hup[S * S];  // hup[u][t] = H_{j-1,j}[u][t] = H[j s + t][(j-1) s + u]
#pragma unroll
  for (int u = 0; u < S; ++u)
#pragma unroll
    for (int t = 0; t < S; ++t)
      hup[u * S + t] = jb > 0 ? A.H[(int64_t)(jb * S + t) * A.ldh + (jb - 1) * S + u] : 0.0;
  double red[S * S + 1];
#pragma unroll
  for (int i = 0; i < S * S + 1; ++i) red[i] = 0.0;
  // one row's local three-term update and its partials, from the row's entries of blocks j-1
  // and j (loaded before the row's SpMM, so that their latency overlaps it)
  auto load_v = [&](int64_t r, double (&vp)[S], double (&vj)[S]) {
    const T *p = static_cast<const T *>(A.pprev) + r * S;  // block j-1
    const T *q = static_cast<const T *>(A.pin) + r * S;    // block j
#pragma unroll
    for (int u = 0; u < S; ++u) {
      vp[u] = jb > 0 ? (double)p[u] : 0.0;
      vj[u] = (double)q[u];
    }
  };
  auto finish = [&](int64_t r, double (&acc)[S], const double (&vp)[S], const double (&vj)[S]) {
#pragma unroll
    for (int t = 0; t < S; ++t) red[S * S] = fma(acc[t], acc[t], red[S * S]);
#pragma unroll
    for (int u = 0; u < S; ++u)
#pragma unroll
      for (int t = 0; t < S; ++t) acc[t] = fma(-vp[u], hup[u * S + t], acc[t]);
#pragma unroll
    for (int a = 0; a < S; ++a)
#pragma unroll
      for (int t = 0; t < S; ++t) red[a * S + t] = fma(vj[a], acc[t], red[a * S + t]);
#pragma unroll
    for (int t = 0; t < S; ++t) A.U[r * S + t] = acc[t];
  };
  if (A.sell.ci) {
    constexpr int NR = spmm_nr<S>();
    const int64_t step = (int64_t)A.nb * TPB;
    for (int64_t r0 = (int64_t)lb * TPB + threadIdx.x; r0 < A.rows; r0 += NR * step) {
      int64_t r[NR];
      bool ok[NR];
      double vp[NR][S], vj[NR][S];
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        r[i] = r0 + i * step;
        ok[i] = r[i] < A.rows;
        load_v(ok[i] ? r[i] : 0, vp[i], vj[i]);
      }
      double acc[NR][S];
      sell_rows<NR, S>(A.sell, r, ok, static_cast<const T *>(A.pin), S, acc);
#pragma unroll
      for (int i = 0; i < NR; ++i)
        if (ok[i]) finish(r[i], acc[i], vp[i], vj[i]);
    }
  } else {
    for (int64_t r0 = (int64_t)lb * TPB; r0 < A.rows; r0 += (int64_t)A.nb * TPB) {
      const int64_t r1 = (r0 + TPB < A.rows) ? r0 + TPB : A.rows;
      const int64_t r = r0 + threadIdx.x;
      double vp[S], vj[S];
      load_v(r < r1 ? r : r0, vp, vj);
      double acc[S];
      spmm_rows<S>(r0, r1, A.rp, A.ci, A.val, static_cast<const T *>(A.pin), S, acc);
      if (r < r1) finish(r, acc, vp, vj);
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

template <int S, typename T, class PS>
__global__ __launch_bounds__(TPB) void lz_spmm_pair(PS P, int jb, const DevState *ds) {
  if (halted(P, ds)) return;
  lz_spmm_body<S, T>(P, (int)blockIdx.x, jb);
}

// H_jj = V_j^T U from the partials (every workgroup forms it; workgroup 0 writes column block j
// of H: H_{j-1,j} and H_jj); U -= V_j H_jj; partials of U^T U.
template <int S, typename T, class PS>
__device__ __forceinline__ void lz_update_body(const PS &P, int bid, int jb) {
  int lb, sd;
  const ArSide A = side_of(P, lb, sd, bid);
  double hjj[S * S];
  sum_records<S * S>(aux_vju<S>(A), A.nb_spmm, hjj);
  if (lb == 0 && threadIdx.x == 0) {
    for (int a = 0; a < S; ++a)
      for (int t = 0; t < S; ++t) {
        A.H[(int64_t)(jb * S + a) * A.ldh + jb * S + t] = hjj[a * S + t];
        if (jb > 0)
          A.H[(int64_t)((jb - 1) * S + a) * A.ldh + jb * S + t] =
              A.H[(int64_t)(jb * S + t) * A.ldh + (jb - 1) * S + a];
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

template <int S, typename T, class PS>
__global__ __launch_bounds__(TPB) void lz_update_pair(PS P, int jb, const DevState *ds) {
  if (halted(P, ds)) return;
  lz_update_body<S, T>(P, (int)blockIdx.x, jb);
}

// The whole block Lanczos step for small bases: one workgroup per basis runs the four phases
// (SpMM and local three-term update, H_jj and U update, first and second QR pass with the new
// block; one QR pass for a single column), with barriers where the separate kernels have launch
// boundaries; each phase's reduction has a single record.
template <int S, typename T>
__global__ __launch_bounds__(TPB) void lz_fused_pair(ArPair P, int jb, double closure_tol,
                                                     const DevState *ds) {
  if (ds->done) return;
  const int bid = (int)blockIdx.x;
  lz_spmm_body<S, T>(P, bid, jb);
  __syncthreads();
  lz_update_body<S, T>(P, bid, jb);
  __syncthreads();
  if (S == 1) {  // one column: normalization, one pass
    final_body<S, T, true>(P, bid, jb, 0, closure_tol);
    return;
  }
  qr2_body<S>(P, bid, closure_tol);
  __syncthreads();
  final_body<S, T, false>(P, bid, jb, 0, closure_tol);
}

// Basis columns of blocks [b0, b1) (b1 - b0 <= LZ_RING) from the block Lanczos ring: each
// row receives (b1 - b0) s consecutive entries at once.
template <int S, typename T, class PS>
__global__ __launch_bounds__(TPB) void lz_flush_pair(PS P, int b0, int b1) {
  int lb, sd;
  const ArSide A = side_of(P, lb, sd);
  const T *ring = static_cast<const T *>(A.ring);
  T *basis = static_cast<T *>(A.basis);
  for (int64_t r = (int64_t)lb * TPB + threadIdx.x; r < A.rows; r += (int64_t)A.nb * TPB) {
    T v[LZ_RING * S];
#pragma unroll
    for (int k = 0; k < LZ_RING; ++k)
      if (b0 + k < b1) {
        const T *src = ring + (size_t)((b0 + k) % LZ_RING) * A.rows * S + r * S;
#pragma unroll
        for (int t = 0; t < S; ++t) v[k * S + t] = src[t];
      }
    T *dst = basis + r * A.ldb + (int64_t)b0 * S;
    if constexpr (std::is_same<T, double>::value) {
      if (b1 - b0 == LZ_RING) {
        // a full ring: LZ_RING s consecutive doubles of the row, 16-byte aligned (the basis
        // leading dimension is a multiple of 64, b0 of LZ_RING), written 16 bytes at a time
#pragma unroll
        for (int k = 0; k < LZ_RING * S; k += 2)
          *reinterpret_cast<double2 *>(dst + k) = make_double2(v[k], v[k + 1]);
        continue;
      }
    }
#pragma unroll
    for (int k = 0; k < LZ_RING; ++k)
      if (b0 + k < b1)
#pragma unroll
        for (int t = 0; t < S; ++t) dst[k * S + t] = v[k * S + t];
  }
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Bases (both sides together) up to this many rows take the single-launch Lanczos step.
constexpr int64_t LZ_FUSED_ROWS = 2048;

// Rows per gram chunk: large enough that the chunk partials stay a small fraction of the basis
// read (2 s / rpc), small enough for a few hundred workgroups, at most 512 chunks per basis.
int64_t gram_rpc(int s, int64_t rows, int64_t total_rows) {
  int64_t rpc = std::max<int64_t>(32 * s, cdiv(total_rows, 1024));
  rpc = std::min<int64_t>(rpc, std::max<int64_t>(16, cdiv(total_rows, 256)));
  rpc = std::max<int64_t>(rpc, cdiv(rows, 512));
  return std::max<int64_t>(rpc, 1);
}

ArSide make_side(const SideDesc &d, const Scratch &sc, int idx, size_t half, size_t aux_len,
                 int64_t ldh) {
  ArSide a{};
  a.ldh = ldh;
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
// The block Lanczos SpMM may run on more workgroups (up to SPMM_WG_MAX, picked per shape by
// the autotuner); its partial records are sized for that.
constexpr int64_t SPMM_WG_MAX = 4096;
int64_t nb_rows_max(int64_t rows) { return std::min<int64_t>(cdiv(rows, TPB), SPMM_WG_MAX); }
size_t aux_len(int s, int64_t rows) {
  return (size_t)(nb_rows_max(rows) +
                  (cdiv(rows, UROWS) + nb_qr(rows) + nb_rows_max(rows)) * s * s + 16);
}


// Largest power of two q <= 8 with q * per <= cap.
constexpr int pow2_cap(int per, int cap) {
  return 8 * per <= cap ? 8 : 4 * per <= cap ? 4 : 2 * per <= cap ? 2 : 1;
}
int pow2_ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}
int log2_exact(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Column groups per thread of gram_part_pair and of the fused sweep: accumulators (and the
// fused sweep's coefficients) of at most 32 doubles per thread. The fused sweep runs on FP64
// bases only (FP32 values widened twice per block cost more registers than the pass saves).
template <int S, typename T>
constexpr int gram_nq_max() { return pow2_cap(Pack8<T>::N * S, 32); }
template <int S, typename T>
constexpr int fused_nq_max() { return Pack8<T>::N > 1 ? 0 : S <= 4 ? 8 : 2; }

template <int S, typename T, int NQ>
void launch_gram_part(const ArPair &P, int ncols, int cw_log2, size_t lds, const DevState *ds,
                      hipStream_t st) {
  gram_part_pair<S, T, NQ><<<total_blocks(P), TPB, lds, st>>>(P, ncols, cw_log2, ds);
}

// C partials of one sweep (shape fitted to the width: row groups for narrow bases, up to NQ
// column groups per thread for wide ones).
template <int S, typename T>
int gram_sweep(const ArPair &P, int ncols, const DevState *ds, hipStream_t st) {
  constexpr int E = Pack8<T>::N;
  constexpr int QM = gram_nq_max<S, T>();
  const int ng = (ncols + E - 1) / E;
  int cw_log2 = 8, nq = 1;
  if (ng <= TPB) cw_log2 = log2_exact(pow2_ceil(ng));
  else nq = std::min(QM, pow2_ceil((ng + TPB - 1) / TPB));
  const size_t lds = cw_log2 < 8 ? (size_t)TPB * E * S * sizeof(double) : 0;
  switch (nq) {
    case 1: launch_gram_part<S, T, 1>(P, ncols, cw_log2, lds, ds, st); break;
    case 2: launch_gram_part<S, T, std::min(2, QM)>(P, ncols, cw_log2, lds, ds, st); break;
    case 4: launch_gram_part<S, T, std::min(4, QM)>(P, ncols, cw_log2, lds, ds, st); break;
    default: launch_gram_part<S, T, QM>(P, ncols, cw_log2, lds, ds, st); break;
  }
  HIPOK(hipGetLastError());
  return 0;
}

// Column groups per thread of the fused first-sweep update + second-sweep Gram, or 0 when the
// basis is too narrow (separate kernels are faster) or too wide for its registers.
template <int S, typename T>
int fused_nq(int ncols) {
  constexpr int E = Pack8<T>::N;
  const int nq = ((ncols + E - 1) / E + TPB - 1) / TPB;
  if (nq < 2 || nq > fused_nq_max<S, T>()) return 0;
  return pow2_ceil(nq);
}

template <int S, typename T>
int launch_fused(const ArPair &P, int ncols, int nq, const DevState *ds, hipStream_t st) {
  constexpr int QM = fused_nq_max<S, T>();
  if constexpr (QM < 2) {
    return SYLV_ERR_INVALID;
  } else {
    const unsigned nb = total_blocks(P);
    switch (nq) {
      case 2: upd_gram_pair<S, T, std::min(2, QM)><<<nb, TPB, 0, st>>>(P, ncols, ds); break;
      case 4: upd_gram_pair<S, T, std::min(4, QM)><<<nb, TPB, 0, st>>>(P, ncols, ds); break;
      default: upd_gram_pair<S, T, QM><<<nb, TPB, 0, st>>>(P, ncols, ds); break;
    }
    HIPOK(hipGetLastError());
    return 0;
  }
}

template <int S, typename T>
int arnoldi_pair_t(const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,
                   double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st) {
  ArPair P{};
  const size_t half = sc.partial_cap / 2;
  P.nsides = sw ? 2 : 1;
  const int64_t rows0 = sv.rows, rows1 = sw ? sw->rows : 0;
  const size_t aux0 = aux_len(S, rows0), aux1 = sw ? aux_len(S, rows1) : 0;
  P.s[0] = make_side(sv, sc, 0, half, aux0, ldh);
  if (sw) P.s[1] = make_side(*sw, sc, 1, half, aux1, ldh);
  for (int i = 0; i < P.nsides; ++i) {
    const int64_t rows = i ? rows1 : rows0;
    P.s[i].nb_spmm = (int)nb_rows(rows);
    P.s[i].nb_upd = (int)cdiv(rows, UROWS);
    P.s[i].nb_qr = (int)nb_qr(rows);
  }
  const int64_t total = rows0 + rows1;
  const int ncols = (jb + 1) * S;
  const int nout = ncols * S;
  const double bytes_v = (double)sizeof(T) * (double)total * ncols;
  const double flops_v = 2.0 * (double)total * ncols * S;

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
           mat_bytes(sv) + (sw ? mat_bytes(*sw) : 0.0) + 4.0 * (total + 2) + 16.0 * total * S,
           2.0 * (sv.nnz + (sw ? sw->nnz : 0)) * S, st);

  // chunking of the Gram sweeps
  const int64_t rpc0 = gram_rpc(S, rows0, total), rpc1 = sw ? gram_rpc(S, rows1, total) : 1;
  const int nch0 = (int)cdiv(rows0, rpc0), nch1 = sw ? (int)cdiv(rows1, rpc1) : 0;
  if ((size_t)nch0 * nout + aux0 > half || (size_t)nch1 * nout + aux1 > half)
    return SYLV_ERR_WORKSPACE;
  P.s[0].nch = nch0;
  P.s[1].nch = nch1;
  // coefficient chunk of the MFMA update in LDS (at most 64 KiB)
  const size_t lds =
      (size_t)std::min((ncols + 127) / 128 * 128, UPD_KCH<S>()) * S * sizeof(double);
  const int64_t rtiles = cdiv(nout, OPB);
  const int fnq = fused_nq<S, T>(ncols);
  int e;

  auto chunks = [&]() {
    P.s[0].rpc = rpc0;
    P.s[1].rpc = rpc1;
    set_ranges(P, nch0, nch1);
  };
  auto reduce = [&](int pass) {
    set_ranges(P, rtiles, sw ? rtiles : 0);
    gram_reduce_pair<<<total_blocks(P), TPB, 0, st>>>(P, S, ncols, jb * S, pass,
                                                      ds);
    return hipGetLastError();
  };
  auto update = [&](int upart) {
    P.s[0].rpc = UROWS;
    P.s[1].rpc = UROWS;
    set_ranges(P, cdiv(rows0, UROWS), sw ? cdiv(rows1, UROWS) : 0);
    update_mfma_pair<S, T><<<total_blocks(P), TPB, lds, st>>>(P, ncols, upart, ds);
    return hipGetLastError();
  };
  const double bytes_g = bytes_v + 8.0 * total * S + 8.0 * nout * P.nsides;
  const double bytes_u = bytes_v + 16.0 * total * S + 8.0 * nout * P.nsides;

  // first sweep: C1 = V^T U
  chunks();
  prof_begin(sc, st);
  if ((e = gram_sweep<S, T>(P, ncols, ds, st))) return e;
  HIPOK(reduce(1));
  prof_end(sc, FAM_GRAM, bytes_g, flops_v, st);
  if (fnq) {
    // U -= V C1 with the second sweep's partials in the same pass over V
    chunks();
    prof_begin(sc, st);
    if ((e = launch_fused<S, T>(P, ncols, fnq, ds, st))) return e;
    HIPOK(reduce(2));
    prof_end(sc, FAM_UPD_GRAM, bytes_u, 2.0 * flops_v, st);
  } else {
    prof_begin(sc, st);
    HIPOK(update(0));
    prof_end(sc, FAM_UPDATE, bytes_u, flops_v, st);
    chunks();
    prof_begin(sc, st);
    if ((e = gram_sweep<S, T>(P, ncols, ds, st))) return e;
    HIPOK(reduce(2));
    prof_end(sc, FAM_GRAM, bytes_g, flops_v, st);
  }
  // second update with the U^T U partials for the first QR pass (one record per workgroup)
  prof_begin(sc, st);
  HIPOK(update(1));
  prof_end(sc, FAM_UPDATE, bytes_u, flops_v, st);
  // QR passes and the new block
  set_ranges(P, nb_qr(rows0), sw ? nb_qr(rows1) : 0);
  prof_begin(sc, st);
  qr2_pair<S><<<total_blocks(P), TPB, 0, st>>>(P, closure_tol, ds);
  HIPOK(hipGetLastError());
  final_pair<S, T><<<total_blocks(P), TPB, 0, st>>>(P, jb, 1, closure_tol, ds);
  HIPOK(hipGetLastError());
  prof_end(sc, FAM_QR, 8.0 * total * S * 3, 6.0 * total * S * S, st);
  return 0;
}

// The lagged Arnoldi step j (FP64 bases, 2 s <= 8 Gram columns): see dcgs_fix_pair.
template <int S>
int arnoldi_lagged_t(const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,
                     double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st) {
  constexpr int S2 = 2 * S;
  ArPair P{};
  const size_t half = sc.partial_cap / 2;
  P.nsides = sw ? 2 : 1;
  const int64_t rows0 = sv.rows, rows1 = sw ? sw->rows : 0;
  const size_t aux0 = aux_len(S, rows0), aux1 = sw ? aux_len(S, rows1) : 0;
  P.s[0] = make_side(sv, sc, 0, half, aux0, ldh);
  if (sw) P.s[1] = make_side(*sw, sc, 1, half, aux1, ldh);
  for (int i = 0; i < P.nsides; ++i) {
    const SideDesc &d = i ? *sw : sv;
    const int64_t rows = i ? rows1 : rows0;
    P.s[i].nb_spmm = (int)nb_rows(rows);
    P.s[i].nb_upd = (int)cdiv(rows, UROWS);
    P.s[i].nb_qr = (int)nb_qr(rows);
    P.s[i].pin = d.panel[jb % 2];
    P.s[i].pout = d.panel[(jb + 1) % 2];
  }
  const int64_t total = rows0 + rows1;
  const int ncols = (jb + 1) * S, nf = jb * S;
  const int nout = ncols * S2;
  const double bytes_g = 8.0 * total * ncols + 16.0 * total * S + 8.0 * nout * P.nsides;
  const double bytes_u = 8.0 * total * nf + 32.0 * total * S;

  // U = M V~_j
  set_ranges(P, nb_rows(rows0), sw ? nb_rows(rows1) : 0);
  prof_begin(sc, st);
  spmm_pair<S, double><<<total_blocks(P), TPB, 0, st>>>(P, ds);
  HIPOK(hipGetLastError());
  prof_end(sc, FAM_SPMM,
           mat_bytes(sv) + (sw ? mat_bytes(*sw) : 0.0) + 4.0 * (total + 2) + 16.0 * total * S,
           2.0 * (sv.nnz + (sw ? sw->nnz : 0)) * S, st);

  // [V_{0..j-1}; V~_j]^T [V~_j, U]
  const int64_t rpc0 = gram_rpc(S, rows0, total), rpc1 = sw ? gram_rpc(S, rows1, total) : 1;
  const int nch0 = (int)cdiv(rows0, rpc0), nch1 = sw ? (int)cdiv(rows1, rpc1) : 0;
  if ((size_t)nch0 * nout + aux0 > half || (size_t)nch1 * nout + aux1 > half)
    return SYLV_ERR_WORKSPACE;
  P.s[0].nch = nch0;
  P.s[1].nch = nch1;
  P.s[0].rpc = rpc0;
  P.s[1].rpc = rpc1;
  set_ranges(P, nch0, nch1);
  prof_begin(sc, st);
  {
    constexpr int QM = gram_nq_max<S2, double>();
    const int ng = ncols;
    int cw_log2 = 8, nq = 1;
    if (ng <= TPB) cw_log2 = log2_exact(pow2_ceil(ng));
    else nq = std::min(QM, pow2_ceil((ng + TPB - 1) / TPB));
    const size_t glds = cw_log2 < 8 ? (size_t)TPB * S2 * sizeof(double) : 0;
    const unsigned nb = total_blocks(P);
    switch (nq) {
      case 1: gram_part_pair<S2, double, 1, true><<<nb, TPB, glds, st>>>(P, ncols, cw_log2, ds); break;
      case 2: gram_part_pair<S2, double, std::min(2, QM), true><<<nb, TPB, glds, st>>>(P, ncols, cw_log2, ds); break;
      case 4: gram_part_pair<S2, double, std::min(4, QM), true><<<nb, TPB, glds, st>>>(P, ncols, cw_log2, ds); break;
      default: gram_part_pair<S2, double, QM, true><<<nb, TPB, glds, st>>>(P, ncols, cw_log2, ds); break;
    }
    HIPOK(hipGetLastError());
  }
  const int64_t rtiles = cdiv(nout, OPB);
  set_ranges(P, rtiles, sw ? rtiles : 0);
  gram_reduce_pair<<<total_blocks(P), TPB, 0, st>>>(P, S2, ncols, jb * S, 0, ds);
  HIPOK(hipGetLastError());
  prof_end(sc, FAM_GRAM, bytes_g, 2.0 * total * ncols * S2, st);

  // second pass of block j: Tw, e, final column block j-1
  prof_begin(sc, st);
  set_ranges(P, 1, sw ? 1 : 0);
  dcgs_fix_pair<S><<<total_blocks(P), TPB, 0, st>>>(P, jb, closure_tol, ds);
  HIPOK(hipGetLastError());
  // final V_j and U' in one pass over V_{0..j-1}, with the U'^T U' partials
  const size_t lds = (size_t)std::max(
      std::min((nf + 127) / 128 * 128, UPD_KCH<S2>()) * S2 * (int)sizeof(double), 8);
  P.s[0].rpc = UROWS;
  P.s[1].rpc = UROWS;
  set_ranges(P, cdiv(rows0, UROWS), sw ? cdiv(rows1, UROWS) : 0);
  dcgs_update_pair<S><<<total_blocks(P), TPB, lds, st>>>(P, jb, ds);
  HIPOK(hipGetLastError());
  prof_end(sc, FAM_UPDATE, bytes_u, 2.0 * total * nf * S2, st);

  // first QR pass of U' and, in the same launch, column blocks j-1 and j of H; then the
  // second pass and the provisional block j+1
  ArPair Ph = P;
  const int64_t hw = cdiv(ncols, TPB / WAVE);
  set_ranges(Ph, hw, sw ? hw : 0);
  set_ranges(P, nb_qr(rows0), sw ? nb_qr(rows1) : 0);
  prof_begin(sc, st);
  const int nq = (int)total_blocks(P);
  dcgs_tail_pair<S><<<(unsigned)nq + total_blocks(Ph), TPB, 0, st>>>(P, Ph, nq, jb,
                                                                      closure_tol, ds);
  HIPOK(hipGetLastError());
  final_pair<S, double><<<total_blocks(P), TPB, 0, st>>>(P, jb, 1, 0.0, ds);
  HIPOK(hipGetLastError());
  prof_end(sc, FAM_QR, 8.0 * total * S * 3, 6.0 * total * S * S, st);
  return 0;
}

// Basis columns of the blocks of the last (possibly partial) ring group before block nblocks:
// blocks [(nblocks - 1) / LZ_RING * LZ_RING, nblocks).
template <int S, typename T>
int lanczos_flush_t(const SideDesc &sv, const SideDesc *sw, int nblocks, hipStream_t st) {
  if (nblocks <= 0) return 0;
  const int b0 = (nblocks - 1) / LZ_RING * LZ_RING;
  ArPair P{};
  P.nsides = sw ? 2 : 1;
  for (int i = 0; i < P.nsides; ++i) {
    const SideDesc &d = i ? *sw : sv;
    P.s[i].rows = d.rows;
    P.s[i].basis = d.basis;
    P.s[i].ldb = d.ldb;
    P.s[i].ring = d.panel[0];
  }
  set_ranges(P, nb_rows(sv.rows), sw ? nb_rows(sw->rows) : 0);
  lz_flush_pair<S, T><<<total_blocks(P), TPB, 0, st>>>(P, b0, nblocks);
  HIPOK(hipGetLastError());
  return 0;
}

// Autotuner of the block Lanczos SpMM grid: per shape bucket (block size, element size, rows of
// each basis rounded up to a power of two, stored entries per row), the first step of that
// shape times the SpMM kernel with 512, 1024, 2048 and 4096 workgroups per basis (one warm-up
// and three timed launches each, HIP events on the step's stream; the kernel only writes the
// step's scratch, which the real launch then overwrites) and keeps the fastest in a
// process-wide cache.
template <int S, typename T>
int64_t spmm_workgroups(const ArPair &P0, const SideDesc &sv, const SideDesc *sw, int jb,
                        int64_t ldh, const DevState *ds, hipStream_t st) {
  const int64_t rows0 = sv.rows, rows1 = sw ? sw->rows : 0;
  auto pow2 = [](int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
  };
  const int64_t nnz = sv.nnz + (sw ? sw->nnz : 0);
  const int64_t per_row = (nnz + rows0 + rows1 - 1) / std::max<int64_t>(1, rows0 + rows1);
  const TuneKey key{S, (int)sizeof(T), pow2(rows0), rows1 ? pow2(rows1) : 0, per_row};
  int64_t best = tune_lookup(key);
  if (best > 0) return best;
  const int64_t cap = std::max(nb_rows_max(rows0), rows1 ? nb_rows_max(rows1) : 0);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return ROW_WG;
  }
  float best_ms = 1e30f;
  best = ROW_WG;
  for (int64_t c = ROW_WG; c <= SPMM_WG_MAX; c *= 2) {
    if (c > ROW_WG && c / 2 >= cap) break;  // no more workgroups than row tiles
    ArPair P = P0;
    for (int i = 0; i < P.nsides; ++i)
      P.s[i].nb_spmm = (int)std::min<int64_t>(c, nb_rows_max(i ? rows1 : rows0));
    set_ranges(P, P.s[0].nb_spmm, sw ? P.s[1].nb_spmm : 0);
    lz_spmm_pair<S, T><<<total_blocks(P), TPB, 0, st>>>(P, jb, ds);
    (void)hipEventRecord(a, st);
    for (int r = 0; r < 3; ++r) lz_spmm_pair<S, T><<<total_blocks(P), TPB, 0, st>>>(P, jb, ds);
    (void)hipEventRecord(b, st);
    float ms = 0.f;
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
      break;
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return tune_store(key, best);
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
  P.s[0] = make_side(sv, sc, 0, half, aux0, ldh);
  if (sw) P.s[1] = make_side(*sw, sc, 1, half, aux1, ldh);
  // small bases: the whole step in one launch, one workgroup per basis
  const bool fused = rows0 + rows1 <= LZ_FUSED_ROWS;
  for (int i = 0; i < P.nsides; ++i) {
    const SideDesc &d = i ? *sw : sv;
    const int64_t rows = i ? rows1 : rows0;
    P.s[i].nb_spmm = fused ? 1 : (int)nb_rows(rows);
    P.s[i].nb_upd = fused ? 1 : (int)nb_rows(rows);  // U^T U partials from lz_update_pair
    P.s[i].nb_qr = fused ? 1 : (int)nb_qr(rows);
    P.s[i].pin = d.panel[jb % LZ_RING];
    P.s[i].pout = d.panel[(jb + 1) % LZ_RING];
    P.s[i].pprev = d.panel[(jb + LZ_RING - 1) % LZ_RING];
    P.s[i].ring = d.panel[0];
  }
  const int64_t total = rows0 + rows1;
  if (fused) {
    set_ranges(P, 1, sw ? 1 : 0);
    prof_begin(sc, st);
    lz_fused_pair<S, T><<<P.nsides, TPB, 0, st>>>(P, jb, closure_tol, ds);
    HIPOK(hipGetLastError());
    prof_end(sc, FAM_SPMM,
             mat_bytes(sv) + (sw ? mat_bytes(*sw) : 0.0) + 4.0 * (total + 2) + 8.0 * total * S * 9,
             2.0 * (sv.nnz + (sw ? sw->nnz : 0)) * S + 14.0 * total * S * S, st);
    if ((jb + 2) % LZ_RING == 0) return lanczos_flush_t<S, T>(sv, sw, jb + 2, st);
    return 0;
  }
  // SpMM workgroups per basis: the autotuner's choice for this shape (timed once per process
  // and shape bucket, the first time a step of that shape runs)
  const int64_t nsp = spmm_workgroups<S, T>(P, sv, sw, jb, ldh, ds, st);
  ArPair Ps = P;
  for (int i = 0; i < P.nsides; ++i) P.s[i].nb_spmm = Ps.s[i].nb_spmm = (int)std::min<int64_t>(
      nsp, nb_rows_max(i ? rows1 : rows0));
  set_ranges(Ps, Ps.s[0].nb_spmm, sw ? Ps.s[1].nb_spmm : 0);
  set_ranges(P, nb_rows(rows0), sw ? nb_rows(rows1) : 0);
  prof_begin(sc, st);
  lz_spmm_pair<S, T><<<total_blocks(Ps), TPB, 0, st>>>(Ps, jb, ds);
  HIPOK(hipGetLastError());
  lz_update_pair<S, T><<<total_blocks(P), TPB, 0, st>>>(P, jb, ds);
  HIPOK(hipGetLastError());
  // matrix + gather V_j + read V_{j-1}, V_j + U write/read (local three-term step)
  prof_end(sc, FAM_SPMM,
           mat_bytes(sv) + (sw ? mat_bytes(*sw) : 0.0) + 4.0 * (total + 2) + 8.0 * total * S * 6,
           2.0 * (sv.nnz + (sw ? sw->nnz : 0)) * S + 8.0 * total * S * S, st);
  set_ranges(P, nb_qr(rows0), sw ? nb_qr(rows1) : 0);
  prof_begin(sc, st);
  if (S == 1) {  // one column: normalization, one pass (final_body)
    final_pair<S, T, true><<<total_blocks(P), TPB, 0, st>>>(P, jb, 0, closure_tol, ds);
    HIPOK(hipGetLastError());
    prof_end(sc, FAM_QR, 8.0 * total * S * 2, 2.0 * total * S * S, st);
  } else {
    qr2_pair<S><<<total_blocks(P), TPB, 0, st>>>(P, closure_tol, ds);
    HIPOK(hipGetLastError());
    final_pair<S, T><<<total_blocks(P), TPB, 0, st>>>(P, jb, 0, closure_tol, ds);
    HIPOK(hipGetLastError());
    prof_end(sc, FAM_QR, 8.0 * total * S * 3, 6.0 * total * S * S, st);
  }
  // block jb + 1 completes a group of ring slots: the group goes to the basis
  if ((jb + 2) % LZ_RING == 0) return lanczos_flush_t<S, T>(sv, sw, jb + 2, st);
  return 0;
}


// ---- batch groups: the step of every basis of many problems in one launch per phase ----
// The tables (one ArSide per basis and launch kind, the workgroup owners, the compact block
// slots) are built once (krylov_group_create); a step only passes the step index. Bases of
// problems that stopped return at once (their problem's flag).

inline ArTab group_tab(const KGroup &g, int kind, int jb, int ring, int unb = 0) {
  ArTab t;
  t.sides = static_cast<const ArSide *>(g.tab[kind]);
  t.owner = unb > 0 ? nullptr : g.own[kind];
  t.panels = static_cast<const PanelSet *>(g.panels);
  t.nsides = g.nsides;
  t.unb = unb;
  t.jb = jb;
  t.ring = ring;
  return t;
}

// Block Lanczos step jb of every basis (the multi-kernel step of lanczos_pair_t).
template <int S>
int lanczos_group_t(const KGroup &g, int jb, double closure_tol, hipStream_t st) {
  const ArTab R = group_tab(g, GK_ROWS, jb, LZ_RING), Q = group_tab(g, GK_QR, jb, LZ_RING);
  lz_spmm_pair<S, double><<<(unsigned)g.nblk[GK_ROWS], TPB, 0, st>>>(R, jb, nullptr);
  HIPOK(hipGetLastError());
  lz_update_pair<S, double><<<(unsigned)g.nblk[GK_ROWS], TPB, 0, st>>>(R, jb, nullptr);
  HIPOK(hipGetLastError());
  if (S == 1) {  // one column: normalization, one pass (final_body)
    final_pair<S, double, true><<<(unsigned)g.nblk[GK_QR], TPB, 0, st>>>(Q, jb, 0, closure_tol,
                                                                          nullptr);
    HIPOK(hipGetLastError());
  } else {
    qr2_pair<S><<<(unsigned)g.nblk[GK_QR], TPB, 0, st>>>(Q, closure_tol, nullptr);
    HIPOK(hipGetLastError());
    final_pair<S, double><<<(unsigned)g.nblk[GK_QR], TPB, 0, st>>>(Q, jb, 0, closure_tol,
                                                                   nullptr);
    HIPOK(hipGetLastError());
  }
  if ((jb + 2) % LZ_RING == 0) {
    lz_flush_pair<S, double><<<(unsigned)g.nblk[GK_ROWS], TPB, 0, st>>>(R, jb + 2 - LZ_RING,
                                                                        jb + 2);
    HIPOK(hipGetLastError());
  }
  return 0;
}

// Basis columns of the last, partial group of ring slots before block nblocks.
template <int S>
int lanczos_group_flush_t(const KGroup &g, int nblocks, hipStream_t st) {
  if (nblocks <= 0) return 0;
  const ArTab R = group_tab(g, GK_ROWS, 0, LZ_RING);
  lz_flush_pair<S, double><<<(unsigned)g.nblk[GK_ROWS], TPB, 0, st>>>(
      R, (nblocks - 1) / LZ_RING * LZ_RING, nblocks);
  HIPOK(hipGetLastError());
  return 0;
}

// Lagged block Arnoldi step jb of every basis (FP64, the launches of arnoldi_lagged_t).
template <int S>
int arnoldi_group_t(const KGroup &g, int jb, double closure_tol, hipStream_t st) {
  if constexpr (S > 4) {
    return SYLV_ERR_INVALID;
  } else {
    constexpr int S2 = 2 * S;
    const int ncols = (jb + 1) * S, nf = jb * S, nout = ncols * S2;
    if (nout > g.max_nout) return SYLV_ERR_WORKSPACE;
    const ArTab R = group_tab(g, GK_ROWS, jb, 2);
    spmm_pair<S, double><<<(unsigned)g.nblk[GK_ROWS], TPB, 0, st>>>(R, nullptr);
    HIPOK(hipGetLastError());
    const ArTab C = group_tab(g, GK_CHUNK, jb, 2);
    {
      constexpr int QM = gram_nq_max<S2, double>();
      int cw_log2 = 8, nq = 1;
      if (ncols <= TPB) cw_log2 = log2_exact(pow2_ceil(ncols));
      else nq = std::min(QM, pow2_ceil((ncols + TPB - 1) / TPB));
      const size_t glds = cw_log2 < 8 ? (size_t)TPB * S2 * sizeof(double) : 0;
      const unsigned nb = (unsigned)g.nblk[GK_CHUNK];
      switch (nq) {
        case 1: gram_part_pair<S2, double, 1, true><<<nb, TPB, glds, st>>>(C, ncols, cw_log2, nullptr); break;
        case 2: gram_part_pair<S2, double, std::min(2, QM), true><<<nb, TPB, glds, st>>>(C, ncols, cw_log2, nullptr); break;
        case 4: gram_part_pair<S2, double, std::min(4, QM), true><<<nb, TPB, glds, st>>>(C, ncols, cw_log2, nullptr); break;
        default: gram_part_pair<S2, double, QM, true><<<nb, TPB, glds, st>>>(C, ncols, cw_log2, nullptr); break;
      }
      HIPOK(hipGetLastError());
    }
    const int rtiles = (int)cdiv(nout, OPB);
    gram_reduce_pair<<<(unsigned)(g.nsides * rtiles), TPB, 0, st>>>(
        group_tab(g, GK_ROWS, jb, 2, rtiles), S2, ncols, jb * S, 0, nullptr);
    HIPOK(hipGetLastError());
    dcgs_fix_pair<S><<<(unsigned)g.nsides, TPB, 0, st>>>(group_tab(g, GK_ROWS, jb, 2, 1), jb,
                                                         closure_tol, nullptr);
    HIPOK(hipGetLastError());
    const size_t lds = (size_t)std::max(
        std::min((nf + 127) / 128 * 128, UPD_KCH<S2>()) * S2 * (int)sizeof(double), 8);
    dcgs_update_pair<S><<<(unsigned)g.nblk[GK_UPD], TPB, lds, st>>>(
        group_tab(g, GK_UPD, jb, 2), jb, nullptr);
    HIPOK(hipGetLastError());
    const int hw = (int)cdiv(ncols, TPB / WAVE);
    const ArTab Q = group_tab(g, GK_QR, jb, 2);
    const int nq = g.nblk[GK_QR];
    dcgs_tail_pair<S><<<(unsigned)(nq + g.nsides * hw), TPB, 0, st>>>(
        Q, group_tab(g, GK_ROWS, jb, 2, hw), nq, jb, closure_tol, nullptr);
    HIPOK(hipGetLastError());
    final_pair<S, double><<<(unsigned)nq, TPB, 0, st>>>(Q, jb, 1, 0.0, nullptr);
    HIPOK(hipGetLastError());
    return 0;
  }
}

}  // namespace

// One unit's entry points for block size SS (both basis precisions).
#define ARN_UNIT(SS)                                                                            \
  int arnoldi_step_##SS(const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,            \
                        double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st) {  \
    return sv.fp32 ? arnoldi_pair_t<SS, float>(sv, sw, jb, ldh, closure_tol, sc, ds, st)        \
                   : arnoldi_pair_t<SS, double>(sv, sw, jb, ldh, closure_tol, sc, ds, st);      \
  }                                                                                             \
  int lanczos_step_##SS(const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,            \
                        double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st) {  \
    return sv.fp32 ? lanczos_pair_t<SS, float>(sv, sw, jb, ldh, closure_tol, sc, ds, st)        \
                   : lanczos_pair_t<SS, double>(sv, sw, jb, ldh, closure_tol, sc, ds, st);      \
  }                                                                                             \
  int lanczos_flush_##SS(const SideDesc &sv, const SideDesc *sw, int nblocks, hipStream_t st) { \
    return sv.fp32 ? lanczos_flush_t<SS, float>(sv, sw, nblocks, st)                            \
                   : lanczos_flush_t<SS, double>(sv, sw, nblocks, st);                          \
  }                                                                                             \
  int krylov_group_step_##SS(const KGroup &g, int jb, double closure_tol, hipStream_t st) {     \
    return g.lanczos ? lanczos_group_t<SS>(g, jb, closure_tol, st)                              \
                     : arnoldi_group_t<SS>(g, jb, closure_tol, st);                             \
  }                                                                                             \
  int krylov_group_flush_##SS(const KGroup &g, int nblocks, hipStream_t st) {                   \
    return lanczos_group_flush_t<SS>(g, nblocks, st);                                           \
  }                                                                                             \
  int arnoldi_lagged_##SS(const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,          \
                          double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st) {\
    if constexpr (SS <= 4) {                                                                    \
      if (!sv.fp32) return arnoldi_lagged_t<SS>(sv, sw, jb, ldh, closure_tol, sc, ds, st);      \
    }                                                                                           \
    return SYLV_ERR_INVALID;                                                                    \
  }
