// Kernels of the true-residual evaluation: the basis defect E = M V_p - V_{p+s} H for the
// block-tridiagonal H of block Lanczos (fused with the sparse product), the residual core
// R^ = [R0 0; 0 0] - L(X), and Frobenius inner products <A, B> = tr(A^T B) of strided matrices
// (deterministic two-stage reduction, result written to device memory).
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

// Hb[t][c] = H[(blk(c) - 1) s + t][c], t < 3s: the three nonzero s x s blocks of column c of a
// block-tridiagonal H, stored so that consecutive columns are consecutive in memory.
__global__ __launch_bounds__(TPB) void band_pack_kernel(int p, int q, int s,
                                                        const double *__restrict__ H, int64_t ldh,
                                                        double *__restrict__ Hb, int64_t ldhb) {
  const int c = blockIdx.x * TPB + threadIdx.x;
  if (c >= p) return;
  const int base = (c / s - 1) * s;
  for (int t = 0; t < 3 * s; ++t) {
    const int row = base + t;
    Hb[(int64_t)t * ldhb + c] = (row >= 0 && row < q) ? H[(int64_t)row * ldh + c] : 0.0;
  }
}

// E(r - r0, c) = (M V)(r, c) - sum_t V(r, base(c) + t) Hb(t, c) for c < p (one wave per row,
// lanes across columns, four columns per lane; only rows 0 <= base + t < q of the band enter).
// Every load is unconditional and in bounds (columns past p read column p - 1, band rows outside
// [0, q) read a clamped row with weight zero; only the store is guarded), so a lane's loads of
// a column chunk issue together. A row of at most DEFECT_NZ entries keeps its column indices and
// values in registers, padded with zero weights on the row itself; longer rows take the entry
// loop. SS = s (the band spans 3 SS rows).
constexpr int DEFECT_NZ = 8;

template <typename T, int SS>
__device__ __forceinline__ void defect_band_store(const T *__restrict__ vr, int j0, int lane,
                                                  int p, int q, const double *__restrict__ Hb,
                                                  int64_t ldhb, const double (&acc)[4],
                                                  double *__restrict__ er) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = j0 + u * WAVE + lane, jc = j < p ? j : p - 1;
    const int base = (jc / SS - 1) * SS;
    double v = acc[u];
#pragma unroll
    for (int t = 0; t < 3 * SS; ++t) {
      const int row = base + t;
      const bool in = row >= 0 && row < q;
      const double h = Hb[(int64_t)t * ldhb + jc];
      v = fma(-(double)vr[in ? row : 0], in ? h : 0.0, v);
    }
    if (j < p) er[j] = v;
  }
}

template <typename T, int SS>
__global__ __launch_bounds__(TPB) void defect_band_kernel(
    int64_t r0, int64_t r1, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const double *__restrict__ val, const T *__restrict__ V, int64_t ldv, int p, int q,
    const double *__restrict__ Hb, int64_t ldhb, double *__restrict__ E, int64_t lde) {
  const int64_t r = r0 + (int64_t)blockIdx.x * (TPB / WAVE) + threadIdx.x / WAVE;
  const int lane = threadIdx.x & (WAVE - 1);
  if (r >= r1) return;
  const int b = rp[r], e = rp[r + 1];
  const T *vr = V + r * ldv;
  double *er = E + (r - r0) * lde;
  auto cols = [&](int j0, int (&jc)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + u * WAVE + lane;
      jc[u] = j < p ? j : p - 1;
    }
  };
  if (e - b <= DEFECT_NZ) {
    const T *xs[DEFECT_NZ];
    double as[DEFECT_NZ];
#pragma unroll
    for (int k = 0; k < DEFECT_NZ; ++k) {
      const bool in = b + k < e;
      as[k] = in ? val[b + k] : 0.0;
      xs[k] = V + (in ? (int64_t)ci[b + k] : r) * ldv;
    }
    for (int j0 = 0; j0 < p; j0 += 4 * WAVE) {
      int jc[4];
      cols(j0, jc);
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < DEFECT_NZ; ++k)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = fma(as[k], (double)xs[k][jc[u]], acc[u]);
      defect_band_store<T, SS>(vr, j0, lane, p, q, Hb, ldhb, acc, er);
    }
    return;
  }
  for (int j0 = 0; j0 < p; j0 += 4 * WAVE) {
    int jc[4];
    cols(j0, jc);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int z = b; z < e; ++z) {
      const double a = val[z];
      const T *x = V + (int64_t)ci[z] * ldv;
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = fma(a, (double)x[jc[u]], acc[u]);
    }
    defect_band_store<T, SS>(vr, j0, lane, p, q, Hb, ldhb, acc, er);
  }
}

// dst (rows x cols, ldd) = src (float, lds), widened to FP64.
__global__ __launch_bounds__(TPB) void widen_kernel(int64_t rows, int64_t cols,
                                                    const float *__restrict__ src, int64_t lds,
                                                    double *__restrict__ dst, int64_t ldd) {
  for (int64_t i = blockIdx.x; i < rows; i += gridDim.x)
    for (int64_t j = threadIdx.x; j < cols; j += TPB) dst[i * ldd + j] = (double)src[i * lds + j];
}

// D[r][b] = C[r][b] - sum_a V[r][a] R[a][b] (r < rows, b < s; R s x s with stride s): the part of
// a right-hand-side factor that its stored first basis block V_1 R misses.
template <typename T>
__global__ __launch_bounds__(TPB) void qr_defect_kernel(int64_t rows, int s,
                                                        const double *__restrict__ C, int64_t ldc,
                                                        const T *__restrict__ V, int64_t ldv,
                                                        const double *__restrict__ R,
                                                        double *__restrict__ D) {
  const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= rows * s) return;
  const int64_t r = e / s;
  const int b = (int)(e - r * s);
  double v = C[r * ldc + b];
  for (int a = 0; a < s; ++a) v = fma(-(double)V[r * ldv + a], R[a * s + b], v);
  D[r * s + b] = v;
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

int launch_defect_band(int64_t r0, int64_t r1, const int32_t *rp, const int32_t *ci,
                       const double *val, const void *V, bool v_fp32, int64_t ldv, int p, int q,
                       int s,
                       const double *H, int64_t ldh, double *Hb, int64_t ldhb, bool pack,
                       double *E, int64_t lde, hipStream_t st) {
  if (p <= 0 || r1 <= r0) return 0;
  if (pack) {
    band_pack_kernel<<<(unsigned)((p + TPB - 1) / TPB), TPB, 0, st>>>(p, q, s, H, ldh, Hb, ldhb);
    HIPOK(hipGetLastError());
  }
  if (s < 1 || s > SYLV_MAX_S) return SYLV_ERR_INVALID;
  const int64_t nr = r1 - r0;
  const unsigned g = (unsigned)((nr + 3) / 4);
  switch (s) {
#define CASE(SS)                                                                                 \
  case SS:                                                                                       \
    if (v_fp32)                                                                                  \
      defect_band_kernel<float, SS><<<g, TPB, 0, st>>>(r0, r1, rp, ci, val,                      \
                                                       static_cast<const float *>(V), ldv, p, q, \
                                                       Hb, ldhb, E, lde);                        \
    else                                                                                         \
      defect_band_kernel<double, SS><<<g, TPB, 0, st>>>(r0, r1, rp, ci, val,                     \
                                                        static_cast<const double *>(V), ldv, p,  \
                                                        q, Hb, ldhb, E, lde);                    \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
  }
  HIPOK(hipGetLastError());
  return 0;
}

int launch_widen(int64_t rows, int64_t cols, const float *src, int64_t lds, double *dst,
                 int64_t ldd, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return 0;
  widen_kernel<<<(unsigned)std::min<int64_t>(rows, 65536), TPB, 0, st>>>(rows, cols, src, lds, dst,
                                                                         ldd);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_qr_defect(int64_t rows, int s, const double *C, int64_t ldc, const void *V, bool v_fp32,
                     int64_t ldv, const double *R, double *D, hipStream_t st) {
  const int64_t tot = rows * s;
  if (tot <= 0) return 0;
  const unsigned g = (unsigned)((tot + TPB - 1) / TPB);
  if (v_fp32)
    qr_defect_kernel<float><<<g, TPB, 0, st>>>(rows, s, C, ldc, static_cast<const float *>(V), ldv,
                                               R, D);
  else
    qr_defect_kernel<double><<<g, TPB, 0, st>>>(rows, s, C, ldc, static_cast<const double *>(V),
                                                ldv, R, D);
  HIPOK(hipGetLastError());
  return 0;
}
