// Small kernels of the true-residual evaluation: the residual core R^ = [R0 0; 0 0] - L(X)
// and Frobenius inner products <A, B> = tr(A^T B) of strided matrices (deterministic two-stage
// reduction, result written to device memory).
#include "common.h"

namespace {

constexpr int TPB = 256;

__global__ __launch_bounds__(TPB) void dot_kernel(int64_t M, int64_t N, const double *__restrict__ A,
                                                  int64_t lda, const double *__restrict__ B,
                                                  int64_t ldb, double *partials, int *counter,
                                                  double *out) {
  double v = 0.0;
  for (int64_t i = blockIdx.x; i < M; i += gridDim.x)
    for (int64_t j = threadIdx.x; j < N; j += TPB) v = fma(A[i * lda + j], B[i * ldb + j], v);
  double vv[1] = {v};
  __shared__ double res[1];
  if (reduce_grid<1>(vv, partials, counter, res) && threadIdx.x == 0) *out = res[0];
}

// Rh = -Lx over (q x q); Rh[0:s, 0:s] += R0 (s x s, dense).
__global__ __launch_bounds__(TPB) void rhat_kernel(int s, int q, const double *__restrict__ Lx,
                                                   const double *__restrict__ R0,
                                                   double *__restrict__ Rh, int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= (int64_t)q * q) return;
  const int i = (int)(e / q), j = (int)(e % q);
  double v = -Lx[(int64_t)i * ldc + j];
  if (i < s && j < s) v += R0[i * s + j];
  Rh[(int64_t)i * ldc + j] = v;
}

}  // namespace

int launch_dot(int64_t M, int64_t N, const double *A, int64_t lda, const double *B, int64_t ldb,
               double *out, const Scratch &sc, hipStream_t st) {
  int64_t g = M < 1024 ? M : 1024;
  if (g < 1) g = 1;
  dot_kernel<<<(unsigned)g, TPB, 0, st>>>(M, N, A, lda, B, ldb, sc.partials,
                                          sc.counters + CNT_ELEM + 4, out);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_rhat(int s, int q, const double *Lx, const double *R0, double *Rh, int64_t ldc,
                hipStream_t st) {
  const int64_t tot = (int64_t)q * q;
  if (tot == 0) return 0;
  rhat_kernel<<<(unsigned)((tot + TPB - 1) / TPB), TPB, 0, st>>>(s, q, Lx, R0, Rh, ldc);
  HIPOK(hipGetLastError());
  return 0;
}
