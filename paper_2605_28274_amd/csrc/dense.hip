// Dense FP64 products on small cores and tall factors.
//
// * core_op: the Sylvester operator on cores, eq. (3.11): Q = [H P, 0] + [P G^T; 0], with H, G
//   block upper Hessenberg (block Arnoldi). The K range of each output tile skips the
//   structurally zero part of H (rows of block b only meet columns of blocks >= b-1).
// * gemm: C = alpha op(A) op(B) + beta C with arbitrary element strides, used by the residual
//   evaluation (tall-skinny Grams V^T E with K = n, and small core products).
//
// Both use 64 x 64 output tiles per 256-thread workgroup with FP64 MFMA 16x16x4 (each wave owns
// a 32 x 32 quarter = 2 x 2 MFMA tiles), K staged through LDS in slabs of 16.
#include "common.h"

namespace {

constexpr int BM = 64, BN = 64, BK = 16;

typedef double v4d __attribute__((ext_vector_type(4)));

// Register tile of one wave: 2 x 2 MFMA accumulators of 16 x 16.
struct WaveAcc {
  v4d c[2][2];
};

// LDS layout: As[k][i] (A slab transposed, i fastest) and Bs[k][j]; +1 pad on the fast dim
// breaks bank conflicts of the column-wise fills.
struct Slabs {
  double As[BK][BM + 1];
  double Bs[BK][BN + 1];
};

// MFMA f64 16x16x4 operand layout (wave64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator element v of lane l holds D[4 * v + l / 16][l % 16].
__device__ __forceinline__ void mma_slab(const Slabs &sl, WaveAcc &acc, int wm, int wn) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < BK; kk += 4) {
    double a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = sl.As[kk + lk][wm * 32 + t * 16 + li];
      b[t] = sl.Bs[kk + lk][wn * 32 + t * 16 + li];
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
        acc.c[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], acc.c[ti][tj], 0, 0, 0);
  }
}

__device__ __forceinline__ void zero_acc(WaveAcc &acc) {
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) acc.c[ti][tj] = v4d{0.0, 0.0, 0.0, 0.0};
}

// Calls f(i_local, j_local, value) for each accumulator element of this thread.
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

// ---- core operator: unmasked loads (all indices < ldc; entries outside active cores are 0) ----

__global__ __launch_bounds__(256) void core_op_kernel(int s, int p, const double *__restrict__ H,
                                                      const double *__restrict__ G,
                                                      const double *__restrict__ P,
                                                      double *__restrict__ Q, int64_t ldc,
                                                      const int *done) {
  if (done && *done) return;
  __shared__ Slabs sl;
  const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
  const int w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
  WaveAcc acc;
  zero_acc(acc);
  const int pk = (p + BK - 1) / BK * BK;
  // phase 1: H[i0:i0+64, l] P[l, j0:j0+64] for l in [lstart, p); skipped when j0 >= p
  if (j0 < p) {
    int ls = (i0 / s - 1) * s;
    ls = ls < 0 ? 0 : ls / BK * BK;
    for (int l0 = ls; l0 < pk; l0 += BK) {
      // A slab: H rows i0..i0+63, cols l0..l0+15 -> As[k][i]
      for (int e = threadIdx.x; e < BM * BK; e += 256) {
        const int ii = e / BK, kk = e % BK;
        sl.As[kk][ii] = H[(int64_t)(i0 + ii) * ldc + l0 + kk];
      }
      // B slab: P rows l0..l0+15, cols j0..j0+63 -> Bs[k][j]
      for (int e = threadIdx.x; e < BK * BN; e += 256) {
        const int kk = e / BN, jj = e % BN;
        sl.Bs[kk][jj] = P[(int64_t)(l0 + kk) * ldc + j0 + jj];
      }
      __syncthreads();
      mma_slab(sl, acc, wm, wn);
      __syncthreads();
    }
  }
  // phase 2: P[i0:i0+64, l] G[j0:j0+64, l]^T; skipped when i0 >= p
  if (i0 < p) {
    int ls = (j0 / s - 1) * s;
    ls = ls < 0 ? 0 : ls / BK * BK;
    for (int l0 = ls; l0 < pk; l0 += BK) {
      for (int e = threadIdx.x; e < BM * BK; e += 256) {
        const int ii = e / BK, kk = e % BK;
        sl.As[kk][ii] = P[(int64_t)(i0 + ii) * ldc + l0 + kk];
      }
      for (int e = threadIdx.x; e < BN * BK; e += 256) {
        const int jj = e / BK, kk = e % BK;
        sl.Bs[kk][jj] = G[(int64_t)(j0 + jj) * ldc + l0 + kk];
      }
      __syncthreads();
      mma_slab(sl, acc, wm, wn);
      __syncthreads();
    }
  }
  for_each_acc(acc, wm, wn, [&](int ii, int jj, double v) {
    Q[(int64_t)(i0 + ii) * ldc + j0 + jj] = v;
  });
}

// ---- generic strided GEMM with bounds masks ----

__global__ __launch_bounds__(256) void gemm_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                   const double *__restrict__ A, int64_t a_rs,
                                                   int64_t a_cs, const double *__restrict__ B,
                                                   int64_t b_rs, int64_t b_cs, double beta,
                                                   double *__restrict__ C, int64_t ldc) {
  __shared__ Slabs sl;
  const int64_t i0 = (int64_t)blockIdx.y * BM, j0 = (int64_t)blockIdx.x * BN;
  const int w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
  WaveAcc acc;
  zero_acc(acc);
  // A slab fill: choose the thread mapping along A's unit-stride dimension for coalescing.
  const bool a_k_fast = (a_cs == 1);
  const bool b_j_fast = (b_cs == 1) || (b_rs != 1);
  for (int64_t l0 = 0; l0 < K; l0 += BK) {
    for (int e = threadIdx.x; e < BM * BK; e += 256) {
      int ii, kk;
      if (a_k_fast) { ii = e / BK; kk = e % BK; } else { kk = e / BM; ii = e % BM; }
      const int64_t gi = i0 + ii, gk = l0 + kk;
      sl.As[kk][ii] = (gi < M && gk < K) ? A[gi * a_rs + gk * a_cs] : 0.0;
    }
    for (int e = threadIdx.x; e < BK * BN; e += 256) {
      int kk, jj;
      if (b_j_fast) { kk = e / BN; jj = e % BN; } else { jj = e / BK; kk = e % BK; }
      const int64_t gk = l0 + kk, gj = j0 + jj;
      sl.Bs[kk][jj] = (gk < K && gj < N) ? B[gk * b_rs + gj * b_cs] : 0.0;
    }
    __syncthreads();
    mma_slab(sl, acc, wm, wn);
    __syncthreads();
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
  const unsigned t = (unsigned)((q + BM - 1) / BM);
  if ((int64_t)t * BM > ldc) return SYLV_ERR_WORKSPACE;
  core_op_kernel<<<dim3(t, t), 256, 0, st>>>(s, p, H, G, P, Q, ldc, done);
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
