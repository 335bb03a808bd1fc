// Dense FP64 products on small cores and tall factors, on FP64 MFMA (v_mfma_f64_16x16x4f64).
//
// * core_op: the Sylvester operator on cores, eq. (3.11): Q = [H P, 0] + [P G^T; 0], with H, G
//   block upper Hessenberg (block Arnoldi). The K range of each output tile skips the
//   structurally zero part of H (rows of block b only meet columns of blocks >= b-1).
// * gemm: C = alpha op(A) op(B) + beta C with arbitrary element strides, used by the residual
//   evaluation (tall-skinny Grams V^T E with K = n, and small core products).
//
// Tiling: 64 x 64 output tile per 256-thread workgroup, each wave a 32 x 32 quarter (2 x 2 MFMA
// tiles); K in slabs of 32 staged through double-buffered LDS. The next slab's global loads are
// issued into registers before the MFMAs of the current slab, so one barrier per slab remains
// and the load latency overlaps the matrix-core work.
#include "common.h"

namespace {

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int LD = BM + 1;  // +1 pad: fewer bank conflicts on the transposed fills
static_assert(BM == BN, "one LDS slab shape serves both operands");

typedef double v4d __attribute__((ext_vector_type(4)));

struct WaveAcc {
  v4d c[2][2];
};

typedef double Slab[BK][LD];

struct Smem {
  Slab As[2];
  Slab Bs[2];
};

// MFMA f64 16x16x4 operand layout (wave64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator element v of lane l holds D[4 * v + l / 16][l % 16].
// All operands of the slab are read from LDS first (one wait), then the slab's 32 MFMAs issue
// back to back on four independent accumulators.
__device__ __forceinline__ void mma_slab(const Slab &As, const Slab &Bs, WaveAcc &acc, int wm,
                                         int wn) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  double a[BK / 4][2], b[BK / 4][2];
#pragma unroll
  for (int q = 0; q < BK / 4; ++q)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[q][t] = As[4 * q + lk][wm * 32 + t * 16 + li];
      b[q][t] = Bs[4 * q + lk][wn * 32 + t * 16 + li];
    }
#pragma unroll
  for (int q = 0; q < BK / 4; ++q)
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
        acc.c[ti][tj] =
            __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][ti], b[q][tj], acc.c[ti][tj], 0, 0, 0);
}

__device__ __forceinline__ void zero_acc(WaveAcc &acc) {
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) acc.c[ti][tj] = v4d{0.0, 0.0, 0.0, 0.0};
}

template <typename F>
__device__ __forceinline__ void for_each_acc(const WaveAcc &acc, int wm, int wn, F f) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        f(wm * 32 + ti * 16 + v * 4 + rq, wn * 32 + tj * 16 + col, acc.c[ti][tj][v]);
}

// ---- slab loaders for row-major operands inside ldc-strided buffers (no bounds masks) ----
// "rows" slab: 64 rows x 32 consecutive columns of a row-major matrix, stored transposed
//   (dst[k][i]); thread t loads row t/4, columns 8*(t%4) .. +7 as four 16-byte loads.
// "cols" slab: 32 rows x 64 consecutive columns, stored as is (dst[k][j]); thread t loads row
//   t/8, columns 8*(t%8) .. +7.
struct RegSlab {
  double2 v[4];
};

__device__ __forceinline__ void load_rows(const double *base, int64_t ld, RegSlab &r) {
  const int i = threadIdx.x >> 2, k = (threadIdx.x & 3) * 8;
  const double2 *p = reinterpret_cast<const double2 *>(base + (int64_t)i * ld + k);
#pragma unroll
  for (int u = 0; u < 4; ++u) r.v[u] = p[u];
}

__device__ __forceinline__ void store_rows(Slab &dst, const RegSlab &r) {
  const int i = threadIdx.x >> 2, k = (threadIdx.x & 3) * 8;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    dst[k + 2 * u][i] = r.v[u].x;
    dst[k + 2 * u + 1][i] = r.v[u].y;
  }
}

__device__ __forceinline__ void load_cols(const double *base, int64_t ld, RegSlab &r) {
  const int k = threadIdx.x >> 3, j = (threadIdx.x & 7) * 8;
  const double2 *p = reinterpret_cast<const double2 *>(base + (int64_t)k * ld + j);
#pragma unroll
  for (int u = 0; u < 4; ++u) r.v[u] = p[u];
}

__device__ __forceinline__ void store_cols(Slab &dst, const RegSlab &r) {
  const int k = threadIdx.x >> 3, j = (threadIdx.x & 7) * 8;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    dst[k][j + 2 * u] = r.v[u].x;
    dst[k][j + 2 * u + 1] = r.v[u].y;
  }
}

template <bool B_FROM_ROWS>
__device__ __forceinline__ void load_slab(const double *A, const double *B, int64_t ld, int l,
                                          RegSlab &ra, RegSlab &rb) {
  load_rows(A + l, ld, ra);
  if (B_FROM_ROWS) load_rows(B + l, ld, rb);
  else load_cols(B + (int64_t)l * ld, ld, rb);
}

template <bool B_FROM_ROWS>
__device__ __forceinline__ void store_slab(Smem &sm, int buf, const RegSlab &ra,
                                           const RegSlab &rb) {
  store_rows(sm.As[buf], ra);
  if (B_FROM_ROWS) store_rows(sm.Bs[buf], rb);
  else store_cols(sm.Bs[buf], rb);
}

// One pipelined product over K slabs [l_begin, l_end) (multiples of BK):
//   B_FROM_ROWS == false: acc += A(i0.., l) * B(l, j0..)  with B row-major (cols slab)
//   B_FROM_ROWS == true : acc += A(i0.., l) * B(j0.., l)^T (B given by its rows: rows slab)
// Global loads run two slabs ahead of the MFMAs (two register sets, the loop unrolled by two so
// they stay static); LDS is double-buffered with one barrier per slab.
template <bool B_FROM_ROWS>
__device__ __forceinline__ void pipelined(Smem &sm, WaveAcc &acc, int wm, int wn,
                                          const double *A, const double *B, int64_t ld,
                                          int l_begin, int l_end) {
  if (l_begin >= l_end) return;
  const int nsl = (l_end - l_begin) / BK;
  // Prefetches are unconditional (a slab index past the end re-reads the last slab, always in
  // bounds), so the number of loads in flight is the same on every path and the wait before an
  // LDS fill only covers the older register set.
  auto lslab = [&](int t) { return l_begin + (t < nsl ? t : nsl - 1) * BK; };
  RegSlab ra0, rb0, ra1, rb1;
  load_slab<B_FROM_ROWS>(A, B, ld, lslab(0), ra0, rb0);
  load_slab<B_FROM_ROWS>(A, B, ld, lslab(1), ra1, rb1);
  __syncthreads();  // previous users of the LDS buffers are done
  store_slab<B_FROM_ROWS>(sm, 0, ra0, rb0);
  __syncthreads();
  // invariant at slab t: LDS[t % 2] holds slab t; register set (t+1) % 2 holds slab t+1
  int t = 0;
  for (; t + 1 < nsl; t += 2) {
    load_slab<B_FROM_ROWS>(A, B, ld, lslab(t + 2), ra0, rb0);
    mma_slab(sm.As[0], sm.Bs[0], acc, wm, wn);
    store_slab<B_FROM_ROWS>(sm, 1, ra1, rb1);
    __syncthreads();
    load_slab<B_FROM_ROWS>(A, B, ld, lslab(t + 3), ra1, rb1);
    mma_slab(sm.As[1], sm.Bs[1], acc, wm, wn);
    store_slab<B_FROM_ROWS>(sm, 0, ra0, rb0);
    __syncthreads();
  }
  if (t < nsl) mma_slab(sm.As[0], sm.Bs[0], acc, wm, wn);  // odd slab count: the last slab
}

// ---- core operator (all indices < ldc; entries outside the active cores are exact zeros) ----
// The K range of output tile (I, J) has (T - I) + (T - J) slab-rows of work (T tiles per side),
// so workgroup b computes the complementary pair of tiles b and T*T - 1 - b, i.e. (I, J) and
// (T-1-I, T-1-J): every workgroup then does the same amount of matrix-core work.
__device__ __forceinline__ void core_op_tile(Smem &sm, int s, int p, const double *H,
                                             const double *G, const double *P, double *Q,
                                             int64_t ldc, int i0, int j0, int wm, int wn) {
  WaveAcc acc;
  zero_acc(acc);
  const int pk = (p + BK - 1) / BK * BK;
  // [H P, 0]: rows of H in this tile start at column block (i0/s - 1)
  if (j0 < p) {
    int ls = (i0 / s - 1) * s;
    ls = ls < 0 ? 0 : ls / BK * BK;
    pipelined<false>(sm, acc, wm, wn, H + (int64_t)i0 * ldc, P + j0, ldc, ls, pk);
  }
  // [P G^T; 0]: rows of G in this tile start at column block (j0/s - 1)
  if (i0 < p) {
    int ls = (j0 / s - 1) * s;
    ls = ls < 0 ? 0 : ls / BK * BK;
    pipelined<true>(sm, acc, wm, wn, P + (int64_t)i0 * ldc, G + (int64_t)j0 * ldc, ldc, ls, pk);
  }
  for_each_acc(acc, wm, wn, [&](int ii, int jj, double v) {
    Q[(int64_t)(i0 + ii) * ldc + j0 + jj] = v;
  });
}

__global__ __launch_bounds__(256) void core_op_kernel(int s, int p, int T,
                                                      const double *__restrict__ H,
                                                      const double *__restrict__ G,
                                                      const double *__restrict__ P,
                                                      double *__restrict__ Q, int64_t ldc,
                                                      const int *done) {
  if (done && *done) return;
  __shared__ Smem sm;
  const int w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
  const int t1 = blockIdx.x, t2 = T * T - 1 - t1;
  core_op_tile(sm, s, p, H, G, P, Q, ldc, (t1 / T) * BM, (t1 % T) * BN, wm, wn);
  if (t2 != t1) core_op_tile(sm, s, p, H, G, P, Q, ldc, (t2 / T) * BM, (t2 % T) * BN, wm, wn);
}

// ---- generic strided GEMM with bounds masks (residual Grams and core products) ----
__global__ __launch_bounds__(256) void gemm_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                   const double *__restrict__ A, int64_t a_rs,
                                                   int64_t a_cs, const double *__restrict__ B,
                                                   int64_t b_rs, int64_t b_cs, double beta,
                                                   double *__restrict__ C, int64_t ldc) {
  __shared__ Smem sm;
  const int64_t i0 = (int64_t)blockIdx.y * BM, j0 = (int64_t)blockIdx.x * BN;
  const int w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
  WaveAcc acc;
  zero_acc(acc);
  // thread mapping along each operand's unit-stride dimension (coalesced fills)
  const bool a_k_fast = (a_cs == 1);
  const bool b_j_fast = (b_cs == 1) || (b_rs != 1);
  const int64_t nslab = (K + BK - 1) / BK;
  int buf = 0;
  for (int64_t sl = 0; sl < nslab; ++sl) {
    const int64_t l0 = sl * BK;
    for (int e = threadIdx.x; e < BM * BK; e += 256) {
      int ii, kk;
      if (a_k_fast) { ii = e / BK; kk = e % BK; } else { kk = e / BM; ii = e % BM; }
      const int64_t gi = i0 + ii, gk = l0 + kk;
      sm.As[buf][kk][ii] = (gi < M && gk < K) ? A[gi * a_rs + gk * a_cs] : 0.0;
    }
    for (int e = threadIdx.x; e < BK * BN; e += 256) {
      int kk, jj;
      if (b_j_fast) { kk = e / BN; jj = e % BN; } else { jj = e / BK; kk = e % BK; }
      const int64_t gk = l0 + kk, gj = j0 + jj;
      sm.Bs[buf][kk][jj] = (gk < K && gj < N) ? B[gk * b_rs + gj * b_cs] : 0.0;
    }
    __syncthreads();
    mma_slab(sm.As[buf], sm.Bs[buf], acc, wm, wn);
    buf ^= 1;  // the other buffer is free: its last readers passed the barrier above
  }
  for_each_acc(acc, wm, wn, [&](int ii, int jj, double v) {
    const int64_t gi = i0 + ii, gj = j0 + jj;
    if (gi < M && gj < N) {
      double *c = C + gi * ldc + gj;
      *c = (beta == 0.0) ? alpha * v : fma(alpha, v, beta * *c);
    }
  });
}

}  // namespace

int launch_core_op(int s, int p, const double *H, const double *G, const double *P, double *Q,
                   int64_t ldc, const int *done, hipStream_t st) {
  const int q = p + s;
  const int T = (q + BM - 1) / BM;
  if ((int64_t)T * BM > ldc || ((p + BK - 1) / BK * BK) > ldc) return SYLV_ERR_WORKSPACE;
  core_op_kernel<<<(unsigned)((T * T + 1) / 2), 256, 0, st>>>(s, p, T, H, G, P, Q, ldc, done);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_gemm(int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t a_rs,
                int64_t a_cs, const double *B, int64_t b_rs, int64_t b_cs, double beta, double *C,
                int64_t ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return 0;
  const dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM));
  gemm_kernel<<<grid, 256, 0, st>>>(M, N, K, alpha, A, a_rs, a_cs, B, b_rs, b_cs, beta, C, ldc);
  HIPOK(hipGetLastError());
  return 0;
}
