// Internal definitions shared by the HIP translation units of libsylv (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "sylv.h"

#define SYLV_MAX_S 8
#define WAVE 64

// Per-solve scalar state, resident in device memory. All recurrence scalars are FP64 and are
// produced and consumed on the device; the host only polls `done`.
struct DevState {
  double rho;        // rho_k
  double rho_next;   // rho_{k+1}
  double alpha, omega, beta;
  double normR0;     // ||R_0||_F = ||C1 C2^T||_F
  double tol;
  double relres;     // ||R_{k+1}|| / ||R_0||
  double pq;         // CG: <P_k, Q_k(1:(k+1)s, 1:(k+1)s)>
  double ts, tt;     // BiCGSTAB: <T(1:(2k+2)s,.), S>, <T, T>
  int done;          // set once the solve stopped (converged or breakdown)
  int status;        // SYLV_OK / SYLV_BREAKDOWN once done
  int iters;         // completed iterations when done
  int rho_zero;      // BiCGSTAB: rho_{k+1} == 0 (breakdown after the update)
  double eta;        // GPBiCG: second parameter of the two-term minimization (zeta in omega)
};

// State of one basis (V with H, or W with G) for the block orthonormalization of a new block.
struct SideState {
  double ref2;                          // ||M V_j||_F^2 before orthogonalization
  double g[SYLV_MAX_S * SYLV_MAX_S];    // Gram matrix of the current pass
  double T1[SYLV_MAX_S * SYLV_MAX_S];   // first-pass normalizer (U1 = U T1)
  double Hs1[SYLV_MAX_S * SYLV_MAX_S];  // first-pass subdiagonal factor (U = U1 Hs1)
  double T[SYLV_MAX_S * SYLV_MAX_S];    // combined normalizer (V_{j+1} = U T)
  int mode;                             // 0 regular, 1 closed (zero block), 2 deflated
  int pad_[3];
  // lagged reorthogonalization of the provisional block (w = V~_j - V a, V_j = w Tw)
  double Tw[SYLV_MAX_S * SYLV_MAX_S];
  double Ew[SYLV_MAX_S * SYLV_MAX_S];   // V_j^T (M V~_j)
  double Rt[SYLV_MAX_S * SYLV_MAX_S];   // provisional subdiagonal block of column block j-1
  double Hw[SYLV_MAX_S * SYLV_MAX_S];   // w = V_j Hw
  int modew;
  int padw_[3];
};

// Counter slots for the "last workgroup reduces" pattern; each kernel family owns a range.
enum {
  CNT_SPMM = 0,
  CNT_LZ1 = 8,
  CNT_UPD = 16,
  CNT_NRM = 24,
  CNT_CORE = 32,
  CNT_ELEM = 40,
  CNT_PAIR = 512,  // paired Arnoldi: 1536 counters per basis
  CNT_MAX = 4096
};

// Records the last HIP runtime error seen by the library (reported by sylv_last_error).
void note_hip_error(hipError_t e, const char *what);
// Records a library error message (reported by sylv_last_error).
void note_error(const char *msg);

#define HIPOK(x)                                      \
  do {                                                \
    hipError_t e_ = (x);                              \
    if (e_ != hipSuccess) {                           \
      note_hip_error(e_, #x);                         \
      return SYLV_ERR_HIP;                            \
    }                                                 \
  } while (0)

// ---- wave / block reductions (deterministic: fixed shuffle tree, fixed LDS order) ----

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Sum over a group of g lanes (g a power of two <= 64, groups aligned to g).
__device__ __forceinline__ double group_sum(double v, int g) {
  for (int off = g >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Block-wide sum of NV values per thread; result valid in thread 0. blockDim.x <= 1024.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds /* >= 16*NV */) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = threadIdx.x / WAVE;
  const int nw = (blockDim.x + WAVE - 1) / WAVE;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[w * NV + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double a = 0.0;
      for (int q = 0; q < nw; ++q) a += lds[q * NV + i];
      v[i] = a;
    }
  }
  __syncthreads();
}

// Returns true in every thread of the workgroup that arrives last at `counter` (grid of
// `nblocks` workgroups). Partial results written before the call are visible to it. The last
// workgroup must reset the counter (reset_counter) when done.
__device__ __forceinline__ bool last_block(int *counter, int nblocks) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    int prev = atomicAdd(counter, 1);
    s_last = (prev == nblocks - 1);
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) __threadfence();
  return last;
}

__device__ __forceinline__ void reset_counter(int *counter) {
  if (threadIdx.x == 0) atomicExch(counter, 0);
}

// Block-reduces NV values per thread, stores one partial per workgroup (index bid of nb), and
// lets the last of the nb workgroups sum the partials into out[0..NV) (shared memory of the
// caller). The final sum is spread over the workgroup in a fixed order, so results are
// deterministic. Returns true in every thread of that last workgroup (out is valid there).
template <int NV>
__device__ bool reduce_sub(double (&v)[NV], int bid, int nb, double *partials, int *counter,
                           double *out) {
  __shared__ double lds[16 * NV];
  block_sum<NV>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) partials[(size_t)bid * NV + i] = v[i];
  }
  if (!last_block(counter, nb)) return false;
  double a[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) a[i] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < NV; ++i) a[i] += partials[(size_t)b * NV + i];
  block_sum<NV>(a, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = a[i];
  __syncthreads();
  reset_counter(counter);
  return true;
}

// reduce_sub over the whole (x, y) grid.
template <int NV>
__device__ bool reduce_grid(double (&v)[NV], double *partials, int *counter, double *out) {
  return reduce_sub<NV>(v, blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y, partials,
                        counter, out);
}

// ---- CSR SpMM building block ----

constexpr int SPMM_TPB = 256;   // rows per workgroup (one per thread)
constexpr int SPMM_CAP = 2048;  // CSR entries staged in LDS per workgroup

// acc = A[r, :] X[:, 0:S] for row r = r0 + threadIdx.x (< r1), X with leading dimension ldx.
// The workgroup's CSR range rp[r0] .. rp[r1] is contiguous; when it fits SPMM_CAP it is staged
// in LDS with coalesced loads and every thread walks its row from LDS (stencil rows are short,
// so direct per-thread reads of col_idx / values would be strided across the wave). Larger
// ranges are read directly. All threads of the workgroup must call (it synchronizes).
template <int S, typename T = double>
__device__ __forceinline__ void spmm_rows(int64_t r0, int64_t r1, const int32_t *__restrict__ rp,
                                          const int32_t *__restrict__ ci,
                                          const double *__restrict__ val,
                                          const T *__restrict__ X, int64_t ldx,
                                          double (&acc)[S]) {
  __shared__ int s_ci[SPMM_CAP];
  __shared__ double s_val[SPMM_CAP];
#pragma unroll
  for (int t = 0; t < S; ++t) acc[t] = 0.0;
  const int64_t r = r0 + threadIdx.x;
  const int base = rp[r0];
  const int len = rp[r1] - base;
  const bool staged = len <= SPMM_CAP;
  if (staged) {
    for (int e = threadIdx.x; e < len; e += blockDim.x) {
      s_ci[e] = ci[base + e];
      s_val[e] = val[base + e];
    }
  }
  __syncthreads();
  if (r < r1) {
    const int b = rp[r], e = rp[r + 1];
    if (staged) {
      for (int q = b - base; q < e - base; ++q) {
        const double a = s_val[q];
        const T *x = X + (int64_t)s_ci[q] * ldx;
#pragma unroll
        for (int t = 0; t < S; ++t) acc[t] = fma(a, (double)x[t], acc[t]);
      }
    } else {
      for (int q = b; q < e; ++q) {
        const double a = val[q];
        const T *x = X + (int64_t)ci[q] * ldx;
#pragma unroll
        for (int t = 0; t < S; ++t) acc[t] = fma(a, (double)x[t], acc[t]);
      }
    }
  }
  __syncthreads();
}

// ---- sliced ELLPACK (SELL-64) ----
// Rows are grouped in slices of 64 (one wave); slice k stores width[k] = max row length entries
// per row, column-major inside the slice: entry q of row r sits at off[k] + 64 q + (r % 64).
// Short rows are padded with value 0 and their own row index as column. Every load of the
// SpMM below is then one contiguous 64-lane access, and no row pointer lies on the dependent
// path of the gathers. Narrow form (the solver's own copies of a matrix whose every value is
// exactly a float and whose every column lies within 32767 of its row): the entries are stored
// as float values and int16 column offsets from the row (6 instead of 12 bytes per entry, the
// same products bit for bit), in the regions of the wide arrays.
struct SellMat {
  int64_t rows;
  int64_t nslices;
  const int32_t *width;  // [nslices]
  const int64_t *off;    // [nslices]
  const int32_t *ci;     // [capacity] (not null whenever the copy exists)
  const double *val;     // [capacity]
  int narrow;            // entries in cd / valf instead of ci / val
  const int16_t *cd;     // [capacity] column - row (narrow)
  const float *valf;     // [capacity] (narrow)
};

// Capacity (entries) reserved for the SELL copy of a CSR matrix with nnz entries: up to 25%
// padding plus one full padded row per slice.
inline int64_t sell_capacity(int64_t rows, int64_t nnz) {
  return nnz + nnz / 4 + 64 * ((rows + 63) / 64) + 64;
}
// Bytes of a SELL buffer (widths, offsets, indices, values; 256-byte aligned parts).
inline size_t sell_bytes(int64_t rows, int64_t nnz) {
  const int64_t ns = (rows + 63) / 64, cap = sell_capacity(rows, nnz);
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  return al(ns * 4) + al(ns * 8) + al(cap * 4) + al(cap * 8);
}
inline SellMat sell_view(int64_t rows, int64_t nnz, void *buf) {
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const int64_t ns = (rows + 63) / 64, cap = sell_capacity(rows, nnz);
  char *p = reinterpret_cast<char *>(buf);
  SellMat m;
  m.rows = rows;
  m.nslices = ns;
  m.width = reinterpret_cast<const int32_t *>(p);
  p += al(ns * 4);
  m.off = reinterpret_cast<const int64_t *>(p);
  p += al(ns * 8);
  m.ci = reinterpret_cast<const int32_t *>(p);
  m.cd = reinterpret_cast<const int16_t *>(p);
  p += al(cap * 4);
  m.val = reinterpret_cast<const double *>(p);
  m.valf = reinterpret_cast<const float *>(p);
  m.narrow = 0;
  return m;
}

// Entry q of a slice at position `at` of row r: its column and value (either form).
__device__ __forceinline__ void sell_entry(const SellMat &M, int64_t at, int64_t r, bool in,
                                           int &c, double &a) {
  if (M.narrow) {
    c = in ? (int)(r + M.cd[at]) : 0;
    a = in ? (double)M.valf[at] : 0.0;
  } else {
    c = in ? M.ci[at] : 0;
    a = in ? M.val[at] : 0.0;
  }
}

// acc = A[r, :] X[:, 0:S] for one row r < rows (thread r % 64 of a wave-aligned slice). Rows
// are walked in chunks of 8 entries: all index/value loads of a chunk issue together, then all
// its gathers, so a stencil row costs two dependent memory round trips.
// Row c of X (S consecutive values at X + c ldx) as doubles. With vec (FP64, S even, X and ldx
// keeping every row 16-byte aligned) the values load two at a time, halving the gather loads;
// in == false gives zeros (the load reads row c, which the caller keeps in range).
template <int S, typename T>
__device__ __forceinline__ void gather_row(const T *__restrict__ X, int64_t c, int64_t ldx,
                                           bool vec, bool in, double (&x)[S]) {
  if constexpr (S % 2 == 0 && sizeof(T) == 8) {
    if (vec) {
      const double2 *p = reinterpret_cast<const double2 *>(X + c * ldx);
#pragma unroll
      for (int t = 0; t < S / 2; ++t) {
        const double2 v = p[t];
        x[2 * t] = in ? v.x : 0.0;
        x[2 * t + 1] = in ? v.y : 0.0;
      }
      return;
    }
  }
#pragma unroll
  for (int t = 0; t < S; ++t) x[t] = in ? (double)X[c * ldx + t] : 0.0;
}

// Whether gather_row may load pairs for this X and ldx.
template <int S, typename T>
__device__ __forceinline__ bool gather_vec(const T *X, int64_t ldx) {
  return S % 2 == 0 && sizeof(T) == 8 && ldx % 2 == 0 &&
         (reinterpret_cast<uintptr_t>(X) & 15) == 0;
}

template <int S, typename T = double>
__device__ __forceinline__ void sell_row(const SellMat &M, int64_t r,
                                         const T *__restrict__ X, int64_t ldx,
                                         double (&acc)[S]) {
#pragma unroll
  for (int t = 0; t < S; ++t) acc[t] = 0.0;
  const int64_t k = r >> 6;
  const int w = M.width[k];
  const int64_t base = M.off[k] + (r & 63);
  const bool vec = gather_vec<S>(X, ldx);
  for (int q0 = 0; q0 < w; q0 += 8) {
    int c[8];
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) sell_entry(M, base + 64 * (q0 + u), r, q0 + u < w, c[u], a[u]);
    double x[8][S];
#pragma unroll
    for (int u = 0; u < 8; ++u) gather_row<S>(X, c[u], ldx, vec, q0 + u < w, x[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int t = 0; t < S; ++t) acc[t] = fma(a[u], x[u][t], acc[t]);
  }
}

// NR rows at once (one per entry of r; rows with ok false yield zeros): the slice headers, then
// the indices and values, then the gathers of all rows are issued together, so a thread keeps
// NR times the loads of sell_row in flight.
template <int NR, int S, typename T = double>
__device__ __forceinline__ void sell_rows(const SellMat &M, const int64_t (&r)[NR],
                                          const bool (&ok)[NR], const T *__restrict__ X,
                                          int64_t ldx, double (&acc)[NR][S]) {
  int w[NR];
  int64_t base[NR];
  int wmax = 0;
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int64_t rr = ok[i] ? r[i] : 0;
    w[i] = ok[i] ? M.width[rr >> 6] : 0;
    base[i] = M.off[rr >> 6] + (rr & 63);
    wmax = w[i] > wmax ? w[i] : wmax;
#pragma unroll
    for (int t = 0; t < S; ++t) acc[i][t] = 0.0;
  }
  for (int q0 = 0; q0 < wmax; q0 += 8) {
    int c[NR][8];
    double a[NR][8];
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
      for (int u = 0; u < 8; ++u)
        sell_entry(M, base[i] + 64 * (q0 + u), ok[i] ? r[i] : 0, q0 + u < w[i], c[i][u],
                   a[i][u]);
    double x[NR][8][S];
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool in = q0 + u < w[i];
#pragma unroll
        for (int t = 0; t < S; ++t)
          x[i][u][t] = in ? (double)X[(int64_t)c[i][u] * ldx + t] : 0.0;
      }
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int t = 0; t < S; ++t) acc[i][t] = fma(a[i][u], x[i][u][t], acc[i][t]);
  }
}

// Builds the SELL copy of a CSR matrix into buf (sell_bytes(rows, nnz) bytes). Returns
// SYLV_ERR_WORKSPACE when the padded size exceeds the reserved capacity (the caller then keeps
// using CSR). Synchronizes the stream. With allow_narrow, the narrow form is built when every
// entry allows it, and *narrow (required then) tells which form was built.
int build_sell(int64_t rows, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *val,
               void *buf, hipStream_t st, bool allow_narrow = false, int *narrow = nullptr);
int launch_sell_spmm(int s, const SellMat &M, const double *X, int64_t ldx, double *Y, int64_t ldy,
                     hipStream_t st);

// ---- small dense helpers executed by one thread (s <= 8) ----

// Cholesky G = R^T R (upper R) of an s x s SPD matrix. Returns the smallest pivot ratio
// d_i / G_ii (<= 0 on failure); rows of exactly-zero diagonal are passed through as identity.
__device__ inline double chol_upper(const double *G, double *R, int s) {
  double minratio = 1.0;
  for (int i = 0; i < s * s; ++i) R[i] = 0.0;
  for (int j = 0; j < s; ++j) {
    double d = G[j * s + j];
    if (d == 0.0) {  // an exactly zero column (deflated direction)
      R[j * s + j] = 1.0;
      continue;
    }
    for (int k = 0; k < j; ++k) d -= R[k * s + j] * R[k * s + j];
    const double ratio = d / G[j * s + j];
    if (ratio < minratio) minratio = ratio;
    if (!(d > 0.0)) return ratio;
    const double rjj = sqrt(d);
    R[j * s + j] = rjj;
    for (int i = j + 1; i < s; ++i) {
      double v = G[j * s + i];
      for (int k = 0; k < j; ++k) v -= R[k * s + j] * R[k * s + i];
      R[j * s + i] = v / rjj;
    }
  }
  return minratio;
}

// Inverse of an upper-triangular s x s matrix.
__device__ inline void inv_upper(const double *R, double *Ri, int s) {
  for (int i = 0; i < s * s; ++i) Ri[i] = 0.0;
  for (int j = 0; j < s; ++j) {
    Ri[j * s + j] = 1.0 / R[j * s + j];
    for (int i = j - 1; i >= 0; --i) {
      double v = 0.0;
      for (int k = i + 1; k <= j; ++k) v += R[i * s + k] * Ri[k * s + j];
      Ri[i * s + j] = -v / R[i * s + i];
    }
  }
}

// C = A B for s x s row-major matrices (C must not alias A or B).
__device__ inline void matmul_small(const double *A, const double *B, double *C, int s) {
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) {
      double v = 0.0;
      for (int k = 0; k < s; ++k) v += A[i * s + k] * B[k * s + j];
      C[i * s + j] = v;
    }
}

// Cyclic Jacobi eigen-decomposition of a symmetric s x s matrix: G = Z diag(lam) Z^T.
__device__ inline void jacobi_eig(const double *G, double *lam, double *Z, int s) {
  double a[SYLV_MAX_S * SYLV_MAX_S];
  for (int i = 0; i < s * s; ++i) a[i] = G[i];
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) Z[i * s + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) {
        tot += a[i * s + j] * a[i * s + j];
        if (i != j) off += a[i * s + j] * a[i * s + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < s; ++p)
      for (int q = p + 1; q < s; ++q) {
        const double apq = a[p * s + q];
        if (apq == 0.0) continue;
        const double theta = (a[q * s + q] - a[p * s + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < s; ++k) {  // columns p, q
          const double akp = a[k * s + p], akq = a[k * s + q];
          a[k * s + p] = c * akp - sn * akq;
          a[k * s + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < s; ++k) {  // rows p, q
          const double apk = a[p * s + k], aqk = a[q * s + k];
          a[p * s + k] = c * apk - sn * aqk;
          a[q * s + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < s; ++k) {
          const double zkp = Z[k * s + p], zkq = Z[k * s + q];
          Z[k * s + p] = c * zkp - sn * zkq;
          Z[k * s + q] = sn * zkp + c * zkq;
        }
      }
  }
  for (int i = 0; i < s; ++i) lam[i] = a[i * s + i];
}

// Closure / rank decision after the first Cholesky-QR pass (thread 0 of the last workgroup).
// G = U^T U, ss->ref2 = ||M V_j||_F^2. Sets ss->mode, ss->T1 (U1 = U T1) and ss->Hs1 (U = U1 Hs1).
__device__ inline void finish_pass1(SideState *ss, int s, double closure_tol, const double *G) {
  double tr = 0.0;
  for (int i = 0; i < s; ++i) tr += G[i * s + i];
  for (int i = 0; i < s * s; ++i) {
    ss->T1[i] = 0.0;
    ss->Hs1[i] = 0.0;
  }
  if (!(tr > closure_tol * closure_tol * ss->ref2)) {  // Krylov space closed: zero block
    ss->mode = 1;
    return;
  }
  double R[SYLV_MAX_S * SYLV_MAX_S];
  const double minratio = chol_upper(G, R, s);
  if (minratio > 1e-14) {
    ss->mode = 0;
    inv_upper(R, ss->T1, s);
    for (int i = 0; i < s * s; ++i) ss->Hs1[i] = R[i];
    return;
  }
  // Some directions of U (nearly) vanish: orthonormalize through the eigen-decomposition of
  // G = Z diag(lam) Z^T, keeping eigenvalues above the closure threshold.
  double lam[SYLV_MAX_S], Z[SYLV_MAX_S * SYLV_MAX_S];
  jacobi_eig(G, lam, Z, s);
  double lmax = 0.0;
  for (int i = 0; i < s; ++i) lmax = fmax(lmax, lam[i]);
  const double thr = fmax(closure_tol * closure_tol * ss->ref2, 1e-14 * lmax);
  int kept = 0;
  for (int i = 0; i < s; ++i) {
    if (lam[i] > thr) {
      const double sq = sqrt(lam[i]);
      for (int a = 0; a < s; ++a) {
        ss->T1[a * s + i] = Z[a * s + i] / sq;
        ss->Hs1[i * s + a] = sq * Z[a * s + i];
      }
      ++kept;
    }
  }
  ss->mode = kept ? 2 : 1;
}

// Second Cholesky-QR pass: G2 = (U T1)^T (U T1) = R2^T R2; V_{j+1} = U T1 R2^{-1}, H_{j+1,j} = R2 Hs1.
__device__ inline void finish_pass2(SideState *ss, int s, const double *G2) {
  if (ss->mode == 1) {
    for (int i = 0; i < s * s; ++i) {
      ss->T[i] = 0.0;
      ss->Hs1[i] = 0.0;
    }
    return;
  }
  double R2[SYLV_MAX_S * SYLV_MAX_S], R2i[SYLV_MAX_S * SYLV_MAX_S], tmp[SYLV_MAX_S * SYLV_MAX_S];
  chol_upper(G2, R2, s);
  inv_upper(R2, R2i, s);
  matmul_small(ss->T1, R2i, ss->T, s);
  matmul_small(R2, ss->Hs1, tmp, s);
  for (int i = 0; i < s * s; ++i) ss->Hs1[i] = tmp[i];
}


// ---- launchers implemented in the .hip files (all return 0 or SYLV_ERR_HIP) ----

// Slots of the ring of compact block copies (block Lanczos: the basis receives LZ_RING blocks
// per row at a time instead of one block's s entries).
constexpr int LZ_RING = 8;

struct SideDesc {
  int64_t rows;            // n (V side) or m (W side)
  int64_t nnz;
  const int32_t *rp;       // CSR of the operator applied to the basis (A, or B^T)
  const int32_t *ci;
  const double *val;
  void *basis;             // rows x ldb row-major; block j occupies columns [j s, (j+1) s);
                           // double, or float when fp32 (mixed precision)
  int64_t ldb;
  double *H;               // block Hessenberg, ldc x ldc row-major
  double *U;               // rows x s work panel
  double *coef;            // compact coefficient block (ldb x s)
  SideState *ss;           // device
  void *panel[LZ_RING];    // compact rows x s copies of the newest blocks, basis type, slots
                           // contiguous: block j in panel[j % 2] (block Arnoldi) or in
                           // panel[j % LZ_RING] (block Lanczos, whose basis columns are
                           // written from the ring LZ_RING blocks at a time)
  int fp32;                // basis and panels stored in FP32
  SellMat sell;            // SELL copy of the operator (sell.ci == nullptr: use CSR)
};

struct Scratch {
  double *partials;        // reduction partials
  size_t partial_cap;      // in doubles
  int *counters;           // CNT_MAX ints, zero at rest
  void *prof;              // kernel timing recorder (null: off)
};

// Kernel families timed by the optional profiler (HIP events around each launch).
enum {
  FAM_SPMM = 0,     // M V_j (+ Lanczos local update / norms)
  FAM_GRAM,         // Arnoldi V^T U
  FAM_UPDATE,       // Arnoldi U -= V C
  FAM_QR,           // block Cholesky-QR passes and normalization
  FAM_CORE_OP,      // eq. (3.11) on dense Hessenberg cores (FP64 MFMA)
  FAM_CORE_BAND,    // eq. (3.11) on block-tridiagonal cores
  FAM_CORE_ELEM,    // core axpys, inner products and scalar updates
  FAM_UPD_GRAM,     // Arnoldi U -= V C1 fused with the second sweep's V^T U
  FAM_RES_GRAM,     // true residual: FP64 Gram blocks of the stacked factors (FP64 MFMA)
  FAM_RES_BF16,     // true residual: split-BF16 Gram blocks (BF16 MFMA; flops counted as issued)
  FAM_RES_PACK,     // true residual: column scales and the BF16 pack of a row chunk
  FAM_RES_DEFECT,   // true residual: basis defects A V - V H of a row chunk
  FAM_COUNT
};
void prof_begin(const Scratch &sc, hipStream_t st);
void prof_end(const Scratch &sc, int fam, double bytes, double flops, hipStream_t st);

int launch_spmm(int s, int64_t rows, const int32_t *rp, const int32_t *ci, const double *val,
                const double *X, int64_t ldx, double *Y, int64_t ldy, hipStream_t st);
int launch_spmm_rows(int s, int64_t r0, int64_t r1, const int32_t *rp, const int32_t *ci,
                     const double *val, const void *X, bool x_fp32, int64_t ldx, int ncols,
                     double *Y, int64_t ldy, hipStream_t st);
// D = C - V_1 R (rows x s, D compact): right-hand-side factor minus its first basis block.
int launch_qr_defect(int64_t rows, int s, const double *C, int64_t ldc, const void *V, bool v_fp32,
                     int64_t ldv, const double *R, double *D, hipStream_t st);
// dst = src widened from FP32 to FP64 (rows x cols).
int launch_widen(int64_t rows, int64_t cols, const float *src, int64_t lds, double *dst,
                 int64_t ldd, hipStream_t st);
int launch_csr_transpose(int64_t rows, int64_t nnz, const int32_t *rp, const int32_t *ci,
                         const double *val, int32_t *orp, int32_t *oci, double *oval,
                         void *scratch, hipStream_t st);
size_t csr_transpose_scratch(int64_t rows);

// Block orthonormalization steps (krylov.hip).
int launch_first_block(int s, const SideDesc &sd, const double *C, int64_t ldc_in,
                       double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st);
// Both bases' block Lanczos steps j (arnoldi.hip); sw may be null (Lyapunov).
int launch_lanczos_pair(int s, const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,
                        double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st);
// Block Lanczos keeps its newest blocks in the ring of SideDesc::panel and writes their basis
// columns a group of LZ_RING blocks at a time; this writes the last, possibly partial group of
// the first nblocks blocks (after the final step of a solve).
int launch_lanczos_flush(int s, const SideDesc &sv, const SideDesc *sw, int nblocks,
                         hipStream_t st);

// Both bases' block Arnoldi steps j (same j) in shared launches (arnoldi.hip); sw may be null
// (Lyapunov: one basis).
int launch_arnoldi_pair(int s, const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,
                        double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st,
                        bool lagged = false);
// Whether the lagged (one fewer pass over the basis) Arnoldi step exists for this block size and
// basis precision.
bool arnoldi_lagged_supported(int s, bool fp32);
// Workspace doubles the paired Arnoldi step needs in Scratch::partials.
size_t arnoldi_partials_needed(int s, int64_t rows_v, int64_t rows_w, int64_t max_cols);
// ---- batch groups: the block Krylov step of many problems of one block size per launch ----
// One basis of a group (host description of where its data and scratch live).
struct GroupSide {
  SideDesc d;
  Scratch sc;         // the problem's Krylov scratch (partials split between its two bases)
  int idx;            // 0: V basis, 1: W basis (second half of the partials)
  int64_t pair_rows;  // rows of both bases of the problem (chunking of the Gram sweeps)
  int64_t ldh;        // row stride of the basis' H (or G)
  const int *done;    // the problem's DevState::done (device)
};

// Launch kinds of a group: row tiles (SpMM, local update, ring flush), QR workgroups, Gram
// chunks, update row blocks.
enum { GK_ROWS = 0, GK_QR, GK_CHUNK, GK_UPD, GK_COUNT };

// Device tables of a group (arnoldi.hip). tab[kind] holds one basis record per basis with that
// kind's workgroup range; own[kind] maps each workgroup of the kind to its basis.
struct KGroup {
  int s = 0, lanczos = 0, nsides = 0;
  const void *tab[GK_COUNT] = {};
  const unsigned short *own[GK_COUNT] = {};
  int nblk[GK_COUNT] = {};
  const void *panels = nullptr;
  int max_nout = 0;  // Gram outputs per chunk the partial buffers of every basis hold
  int *idx = nullptr;  // device scratch of the compaction
};
// Device bytes of a group's tables; 0 if a basis does not fit its scratch.
size_t krylov_group_bytes(int s, bool lanczos, const GroupSide *sides, int n);
// Builds the tables into dev (krylov_group_bytes bytes, 256-aligned), synchronously on st: g
// covers every basis; act has room for the same tables restricted to the bases whose problem
// still runs, which launch_krylov_group_compact fills (then act.nsides = counts[0] and
// act.nblk[k] = counts[1 + k], read back by the host, make it usable).
int krylov_group_create(KGroup *g, KGroup *act, int s, bool lanczos, const GroupSide *sides, int n,
                        void *dev, size_t bytes, hipStream_t st);
int launch_krylov_group_compact(const KGroup &g, const KGroup &act, int *counts, hipStream_t st);
// Bounds for sizing before the contexts exist: bytes per basis of `rows` rows, and per group.
size_t krylov_side_bytes_bound(int64_t rows);
size_t krylov_group_bytes_fixed();
// Step jb of every basis (block Lanczos, or lagged block Arnoldi with FP64 bases, s <= 4).
int launch_krylov_group(const KGroup &g, int jb, double closure_tol, hipStream_t st);
// Block Lanczos: basis columns of the last partial group of ring slots before block nblocks.
int launch_krylov_group_flush(const KGroup &g, int nblocks, hipStream_t st);

// One problem of a batch group as the core kernels see it (device table, one entry per
// problem; the kernels take the problem from blockIdx.y). Cores as in a single solve.
struct CoreInst {
  const double *H, *G;
  double *X, *R, *P, *Q, *S, *T;
  const double *Rt;
  double *part;  // the problem's core-stream reduction partials
  DevState *ds;
  double *hist;
  int64_t ldc;
  int max_iter, pad_;
};
// The group launches take the problem of blockIdx.y from list (the problems still running,
// n of them), or all problems of tab in order when list is null.
// CG iteration k (p = (k+1) s) of every problem: P_k, <P_k, Q_k>, alpha, X, R, the stopping
// test, rho and beta (core.hip).
int launch_cg_group(int s, bool sym, int p, int k, const CoreInst *tab, const int *list, int n,
                    hipStream_t st);
// BiCGSTAB iteration k (p = (2k+1) s): which = 0: Q = op(P) on p, 1: T = op(S) on p + s
// (dense.hip); alpha and S; <T, S>, <T, T>; omega, X, R, P, the stopping test (core.hip).
int launch_core_op_group(int s, int p, int which, const CoreInst *tab, const int *list, int n,
                         hipStream_t st);
int launch_bicg_group_s(int s, int p, int k, const CoreInst *tab, const int *list, int n,
                        hipStream_t st);
int launch_bicg_group_omega(int s, int p, const CoreInst *tab, const int *list, int n,
                            hipStream_t st);
int launch_bicg_group_update(int s, int p, int k, const CoreInst *tab, const int *list, int n,
                             hipStream_t st);
// The problems of the group still running: *count (device) and their indices in list.
int launch_group_active(const CoreInst *tab, int n, int *count, int *list, hipStream_t st);

// A batch group (api.hip): problems with the same method, block size, form (Sylvester or
// Lyapunov) and iteration limit whose iterations advance in lock-step on one stream, every
// phase one launch for all of them. The host polls one small record every GROUP_SEG iterations;
// problems that stopped in between return at once through their flags, and the poll removes
// them from the launches (the tables of the running problems are compacted on the device). With
// graphs, each segment of GROUP_SEG iterations is captured once, when the group is set up, as a
// HIP graph over the full tables that every solve replays.
constexpr int GROUP_SEG = 16;
struct GroupRun {
  std::vector<void *> ctx;
  int method = 0, s = 0, sym = 0;
  hipStream_t st = nullptr;
  KGroup kg;                 // tables of every basis
  KGroup ka;                 // tables of the bases of the problems still running
  CoreInst *tab = nullptr;   // device, one entry per problem
  int *list = nullptr;       // device: the problems still running
  int *poll = nullptr;       // device: [problems running, bases running, workgroups per kind]
  int *h_poll = nullptr;     // pinned copy of poll
  int na = 0;                // problems in the launches (compacted form)
  int64_t min_ldc = 0;
  double closure_tol = 0.0;
  hipStream_t vst = nullptr; // compacted form: problems that left are finished on this stream
  bool graphs = false;       // replayed graphs over the full tables; else compacted launches
  int graph_max_iter = -1;
  std::vector<hipGraphExec_t> exec;  // per segment
};
// Whether a context can join a group: FP64 bases, no outer refinement, factored CG or the
// lagged factored BiCGSTAB, Krylov steps on the context's own stream.
bool group_eligible(void *ctx);
// Device bytes of the group's tables (0: the problems cannot form one group).
size_t group_bytes(void *const *ctxs, int n);
// With graphs, every segment of iterations up to max_iter is captured here (solves with another
// iteration limit launch the kernels instead).
int group_prepare(GroupRun &g, void *const *ctxs, int n, void *dev, size_t bytes, bool graphs,
                  int max_iter);
// One solve of every problem of the group (verified like a single solve); res[n].
int group_solve(GroupRun &g, double tol, int max_iter, sylv_result *res);
void group_release(GroupRun &g);

// Process-wide cache of the autotuner (arnoldi.hip): a launch parameter per shape bucket.
struct TuneKey {
  int s, esz;
  int64_t rows0, rows1, per_row;
};
int64_t tune_lookup(const TuneKey &k);  // 0 when the bucket has not been tuned
// Keeps the first value stored for a bucket (solves tuning the same bucket at once on other
// streams then all use it) and returns the value kept.
int64_t tune_store(const TuneKey &k, int64_t value);

// A solver context (api.hip); overlap = false keeps the Krylov steps on the caller's stream
// (batches overlap their instances instead).
int create_context(void **out, const sylv_problem *pb, const sylv_options *op, void *workspace,
                   size_t ws_bytes, void *stream, bool overlap);

// Core recurrences (core.hip).
int launch_setup_scalars(int s, const double *RL, const double *RR, double *R, double *P,
                         double *Rt, int64_t ldc, double tol, DevState *ds, hipStream_t st);
int launch_cg_pq(int s, int p, bool sym, const double *H, const double *G, const double *R,
                 const double *Pprev, double *Pk, int64_t ldc, const Scratch &sc, DevState *ds,
                 hipStream_t st);
int launch_cg_xr(int s, int p, bool sym, const double *H, const double *G, const double *Pk,
                 double *X, double *R, int64_t ldc, const Scratch &sc, DevState *ds, double *hist,
                 int k, int max_iter, hipStream_t st);
int launch_bicg_s(int s, int p, const double *Q, const double *R, double *S, const double *Rt,
                  int64_t ldc, DevState *ds, double *hist, int k, int max_iter, hipStream_t st);
int launch_bicg_omega(int s, int p, const double *T, const double *S, int64_t ldc,
                      const Scratch &sc, DevState *ds, hipStream_t st);
int launch_bicg_update(int s, int p, double *X, double *R, double *P, const double *Q,
                       const double *S, const double *T, const double *Rt, int64_t ldc,
                       const Scratch &sc, DevState *ds, double *hist, int k, int max_iter,
                       hipStream_t st);

// Further factorized methods (core_more.hip): elementwise core recurrences and scalars of CR,
// CGS and GPBiCG over q x q corners; the partials live in sc.partials.
int launch_cr_init(int q, const double *R, const double *S, double *Q, int64_t ldc,
                   const Scratch &sc, DevState *ds, hipStream_t st);
int launch_cr_xr(int q, double *X, double *R, const double *P, const double *Q, int64_t ldc,
                 const Scratch &sc, DevState *ds, double *hist, int k, int max_iter,
                 hipStream_t st);
int launch_cr_beta_pq(int q, const double *R, const double *S, double *P, double *Q,
                      int64_t ldc, const Scratch &sc, DevState *ds, double *hist, int k,
                      int max_iter, hipStream_t st);
int launch_alpha_corner(int s, const double *Rt, const double *Z, int64_t ldc, DevState *ds,
                        double *hist, int k, int max_iter, hipStream_t st);
int launch_cgs_qwx(int q, const double *U, const double *V, double *Q, double *Wk, double *X,
                   int64_t ldc, DevState *ds, hipStream_t st);
// R -= alpha Z (unless gpbicg: R was updated by launch_gp_update) with ||R||^2, the stopping
// test, rho_{k+1} and beta_k.
int launch_axpy_rho_beta(int s, int q, const double *Z, double *R, const double *Rt, int64_t ldc,
                         bool gpbicg, const Scratch &sc, DevState *ds, double *hist, int k,
                         int max_iter, hipStream_t st);
int launch_cgs_up(int q, const double *R, const double *Q, double *U, double *P, int64_t ldc,
                  DevState *ds, hipStream_t st);
int launch_gp_p(int q, const double *R, const double *U, double *P, int64_t ldc, DevState *ds,
                hipStream_t st);
int launch_gp_yt(int q, const double *Tm, const double *R, const double *Wv, const double *AP,
                 double *Y, double *T, int64_t ldc, DevState *ds, hipStream_t st);
int launch_gp_zeta(int q, const double *AT, const double *Y, const double *T, int64_t ldc,
                   bool first, const Scratch &sc, DevState *ds, double *hist, int k, int max_iter,
                   hipStream_t st);
int launch_gp_update(int q, const double *AP, const double *Tm, const double *P, const double *T,
                     const double *Y, const double *AT, double *R, double *U, double *Z,
                     double *X, int64_t ldc, const Scratch &sc, DevState *ds, hipStream_t st);
int launch_gp_w(int q, const double *AT, const double *AP, double *Wv, int64_t ldc, DevState *ds,
                hipStream_t st);

// Solution compression (compress.hip).
// Rows of M (nr x len, ldm) orthogonalized by one-sided Jacobi rotations: G M_in = M_out with G
// (nr x nr, ldg) orthogonal; info[0] = sweeps.
int launch_jacobi_rows(int nr, int64_t len, double *M, int64_t ldm, double *G, int64_t ldg,
                       int *info, hipStream_t st);
int launch_row_norms(int nr, int64_t len, const double *M, int64_t ldm, double *norms,
                     hipStream_t st);
int launch_scale_rows(int nr, int64_t len, double *M, int64_t ldm, const double *f,
                      hipStream_t st);
// ||A - B||_F (B may be null: ||A||_F) and ||A||_F to the host; partials: 1024 doubles.
int diff_norm(int64_t r, int64_t c, const double *A, int64_t lda, const double *B, int64_t ldb,
              double *partials, double *dnorm, double *anorm, hipStream_t st);
int launch_gather_cols(int64_t rows, int k, const int *idx, const double *src, int64_t lds,
                       const double *scale, double *dst, int64_t ldd, hipStream_t st);
int launch_gather_rows_t(int64_t len, int k, const int *idx, const double *src, int64_t lds,
                         const double *sig, double *dst, int64_t ldd, hipStream_t st);

// Dense FP64 GEMM C (M x N) = alpha * op(A) op(B) + beta * C with element strides:
// A(i,k) = A[i*a_rs + k*a_cs], B(k,j) = B[k*b_rs + j*b_cs], C(i,j) = C[i*ldc + j].
int launch_gemm(int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t a_rs,
                int64_t a_cs, const double *B, int64_t b_rs, int64_t b_cs, double beta, double *C,
                int64_t ldc, hipStream_t st);
// Core Sylvester operator eq. (3.11) on dense padded cores: Q = [H P, 0] + [P G^T; 0] where
// P is p x p and H, G are (p+s) x p (Hessenberg), all ldc-strided; the result is written over
// the full (p+s) region rounded up to the tile size (entries outside are exact zeros).
// Residual evaluation (dense.hip, residual.hip).
// C (+)= A^T B, A: K x M, B: K x N row-major (lda >= roundup(M, 64), ldb >= roundup(N, 64));
// `lower` computes the tiles on and below the diagonal only (M == N; launch_mirror completes).
// A and B are float (a_fp32 / b_fp32) or double; row strides multiples of 8 elements.
// part (part_cap doubles, may be null): scratch that lets launches with few output tiles split
// K over several workgroups (deterministic: slices summed in order). FP64 Grams of at least 256
// tiles of 128 x 128 run on 128 x 128 tiles when part holds their stream-K slots
// (gram_part_doubles gives a size that does for every Gram of up to that many columns).
size_t gram_part_doubles(int64_t max_cols, int64_t rows);
int launch_gram(int64_t M, int64_t N, int64_t K, const void *A, bool a_fp32, int64_t lda,
                const void *B, bool b_fp32, int64_t ldb, double beta, double *C, int64_t ldc,
                bool lower, hipStream_t st, double *part = nullptr, size_t part_cap = 0);
// C = A B (row-major, FP64 MFMA); rows of A up to roundup(M, 64) and columns of B up to
// roundup(N, 64) must be readable, lda >= roundup(K, 32), lda and ldb multiples of 8.
int launch_gemm_nn(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                   const double *B, int64_t ldb, double *C, int64_t ldc, hipStream_t st);
int launch_mirror(int64_t M, double *C, int64_t ldc, hipStream_t st);
// Tile (I, J), I >= J, of position b in the row-major order of a lower triangle of tiles.
__device__ __forceinline__ void tri_tile(int64_t b, int &I, int &J) {
  int64_t i = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > b) --i;
  while ((i + 1) * (i + 2) / 2 <= b) ++i;
  I = (int)i;
  J = (int)(b - i * (i + 1) / 2);
}

// Visiting order of the tiles: groups of eight tile rows, column by column inside a group (the
// lower form walks the triangle I >= J the same way, its diagonal block last), so the
// workgroups that run at one time on one XCD share a few row and column panels in its L2.
struct GramSeq {
  int TM, TN, lower;
  __host__ __device__ int64_t count() const {
    return lower ? (int64_t)TM * (TM + 1) / 2 : (int64_t)TM * TN;
  }
  __device__ void tile(int64_t t, int &I, int &J) const {
    int g0;  // first tile row of the group; groups start at the same positions as rows do
    int64_t idx;
    if (lower) {
      int r, c;
      tri_tile(t, r, c);
      g0 = r & ~7;
      idx = t - (int64_t)g0 * (g0 + 1) / 2;
    } else {
      g0 = (int)(t / ((int64_t)8 * TN)) * 8;
      idx = t - (int64_t)g0 * TN;
    }
    const int h = TM - g0 < 8 ? TM - g0 : 8;
    const int64_t full = (int64_t)(lower ? g0 : TN) * h;
    if (idx < full) {
      J = (int)(idx / h);
      I = g0 + (int)(idx % h);
      return;
    }
    // lower form, diagonal block: column g0 + d holds rows g0 + d .. g0 + h - 1
    int64_t e = idx - full;
    int d = 0;
    while (e >= h - d) {
      e -= h - d;
      ++d;
    }
    J = g0 + d;
    I = J + (int)e;
  }
};

// One FP64 Gram C (+)= A^T B of a job table (all jobs over the same K rows): sq.lower selects
// the lower-triangle form (M == N); sq's tile counts and t0 are filled in by the launcher.
struct GramJob {
  GramSeq sq;
  int64_t M, N;
  const double *A;
  int64_t lda;
  const double *B;
  int64_t ldb;
  double *C;
  int64_t ldc;
  int64_t t0;
};
constexpr int GRAM_JOBS_MAX = 8;
struct GramJobs {
  GramJob j[GRAM_JOBS_MAX];
  int n;
  int64_t total;
};
// 128 x 128 tiles of a Gram (the lower triangle with `lower`)
int64_t gram_wide_tiles(int64_t M, int64_t N, bool lower);
// The jobs (n <= GRAM_JOBS_MAX) as one launch on 128 x 128 tiles; returns 1 (nothing launched)
// when part cannot hold the stream-K slots or the jobs have fewer than 256 tiles, so the caller
// runs the jobs one by one; SYLV_ERR_INVALID for a leading dimension below the width or not a
// multiple of 8 (as launch_gram).
int launch_gram_jobs(const GramJob *jobs, int n, int64_t K, double beta, hipStream_t st,
                     double *part, size_t part_cap);


// Split-BF16 Grams (gram_bf16.hip). The stacked columns of one row chunk come from up to
// BF_MAX_SEGS segments: segment i supplies columns [col0, col0 + cols) from a row-major source
// (row r at ptr + r ld esz, esz 4 for float or 8 for double; row 0 is the chunk's first row).
constexpr int BF_MAX_SEGS = 16;
struct BfSeg {
  const char *ptr;
  int64_t ld, col0, cols;
  int esz, pad_;
};
struct BfSegs {
  BfSeg s[BF_MAX_SEGS];
  int count;
};
// Packed width for ctot stacked columns; bytes of the packed chunk; FP32 partial capacity that
// any Gram block of a cpad-wide pack over `rows` rows fits into.
int64_t bf16_pack_width(int64_t ctot);
size_t bf16_pack_bytes(int64_t rows, int64_t cpad);
size_t bf16_part_floats(int64_t cpad, int64_t rows);
// Column maxima, per-column power-of-two scales (cexp, cpad ints) and the hi/lo pack of the
// chunk's nr rows; cmax: cpad 64-bit words of scratch.
int launch_bf16_pack(const BfSegs &sg, int64_t nr, int64_t ctot, int64_t cpad,
                     unsigned long long *cmax, int *cexp, void *packed, hipStream_t st);
// C (M x N, ldc) (+)= A^T B over the nr packed rows, A = stacked columns [a0, a0 + M), B =
// [b0, b0 + N), in split BF16 with FP32 partials summed in FP64; `lower` as launch_gram.
int launch_gram_bf16(int64_t M, int64_t N, int64_t nr, const void *packed, int64_t cpad,
                     const int *cexp, int64_t a0, int64_t b0, double beta, double *C, int64_t ldc,
                     bool lower, hipStream_t st, float *part, size_t part_floats);
// E(0:rows, 0:p) -= V(0:rows, 0:q) H(0:q, 0:p), H block upper Hessenberg; V columns
// [q, roundup(q, 32)) must be finite.
int launch_defect_gemm(int64_t rows, int p, int q, int s, const void *V, bool v_fp32, int64_t ldv,
                       const double *H, int64_t ldh, double *E, int64_t lde, hipStream_t st);
int launch_zero_cols(int64_t rows, void *V, bool v_fp32, int64_t ldv, int c0, int c1,
                     hipStream_t st);
// E(r - r0, 0:p) = M(r, :) V(:, 0:p) - V(r, 0:q) H(0:q, 0:p) for block-tridiagonal H; `pack`
// first writes the band of H into Hb (3s x ldhb).
int launch_defect_band(int64_t r0, int64_t r1, const int32_t *rp, const int32_t *ci,
                       const double *val, const void *V, bool v_fp32, int64_t ldv, int p, int q,
                       int s,
                       const double *H, int64_t ldh, double *Hb, int64_t ldhb, bool pack,
                       double *E, int64_t lde, hipStream_t st);
// Outer refinement (refine.hip). Narrow panels: rows x q FP64 (q <= 8), row stride ldz.
int launch_gauss_fill(int64_t rows, int q, uint64_t seed, double *Z, int64_t ldz, hipStream_t st);
size_t tn_partials_needed(int64_t rows, int64_t ncols, int q);
// out (ncols x q, ldo) = V[:, 0:ncols]^T Z; part: scratch of tn_partials_needed doubles.
int launch_tn(int64_t rows, int ncols, int q, const void *V, bool v_fp32, int64_t ldv,
              const double *Z, int64_t ldz, double *out, int64_t ldo, double *part,
              size_t part_cap, hipStream_t st);
// Y = beta Y + alpha V[:, 0:ncols] Z (Z: ncols x q, ldz).
int launch_nn(int64_t rows, int ncols, int q, double alpha, const void *V, bool v_fp32,
              int64_t ldv, const double *Z, int64_t ldz, double beta, double *Y, int64_t ldy,
              hipStream_t st);
// From G = Y^T Y (q x q): T (q x k) with Y T orthonormal, info[0] = k, dinfo[0] = trace(G).
int launch_orth_small(int q, const double *G, int64_t ldg, double *T, int64_t ldt, int *info,
                      double *dinfo, hipStream_t st);
int launch_copy_block(int rows, int cols, double alpha, const double *src, int64_t lds, bool trans,
                      double *dst, int64_t ldd, hipStream_t st);
// dst (rows x cols, row stride ldd) = src (row stride lds), FP64 (refine.hip).
int launch_copy_rows(int64_t rows, int64_t cols, const double *src, int64_t lds, double *dst,
                     int64_t ldd, hipStream_t st);
int launch_diag_fill(int k, double v, double *dst, int64_t ldd, hipStream_t st);
int launch_axpy_narrow(int64_t rows, int q, double alpha, const double *F, int64_t ldf, double *Y,
                       int64_t ldy, hipStream_t st);
// part (part_cap doubles, may be null): scratch for the split-K form used when the cores span
// few 64 x 64 tiles.
int launch_core_op(int s, int p, const double *H, const double *G, const double *P, double *Q,
                   int64_t ldc, const int *done, hipStream_t st, double *part = nullptr,
                   size_t part_cap = 0);
int launch_csr_validate(int64_t rows, int64_t nnz, const int32_t *rp, const int32_t *ci, int *flag,
                        hipStream_t st);
int launch_dot(int64_t M, int64_t N, const double *A, int64_t lda, const double *B, int64_t ldb,
               double *out, const Scratch &sc, hipStream_t st);
int launch_rhat(int s, int q, const double *Lx, const double *R0, double *Rh, int64_t ldc,
                hipStream_t st);
