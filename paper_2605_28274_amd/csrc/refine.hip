// Kernels of the outer refinement around the mixed-precision solve: products of the factored
// residual with narrow panels (sketch R Omega and R^T P), the orthonormalization of the sketch,
// and the Gaussian test matrix.
//
// Narrow panels are rows x q FP64 arrays (q <= 8) with a row stride of NLD doubles; bases are
// rows x ldb arrays of T (double, or float when the bases are stored in FP32).
#include "common.h"

namespace {

constexpr int TPB = 256;

// SplitMix64 finalizer (Steele, Lea, Flood 2014) of a 64-bit counter.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Z[i][t] ~ N(0, 1) for i < rows, t < q: Box-Muller on two uniforms drawn from the counter
// (seed, i, t); deterministic for a given seed.
__global__ __launch_bounds__(TPB) void gauss_fill_kernel(int64_t rows, int q, uint64_t seed,
                                                         double *__restrict__ Z, int64_t ldz) {
  const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= rows * q) return;
  const int64_t i = e / q;
  const int t = (int)(e - i * q);
  const uint64_t c = seed * 0x100000001B3ull + (uint64_t)e * 2;
  const double u1 = ((double)(splitmix64(c) >> 11) + 0.5) * 0x1.0p-53;  // (0, 1)
  const double u2 = (double)(splitmix64(c + 1) >> 11) * 0x1.0p-53;      // [0, 1)
  Z[i * ldz + t] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Chunk partials of out = V[:, 0:ncols]^T Z (ncols x Q): workgroup lb owns rows
// [lb rpc, (lb+1) rpc), thread t the columns t + 256 k; Z rows staged in LDS.
template <int Q, typename T>
__global__ __launch_bounds__(TPB) void tn_part_kernel(int64_t rows, int ncols, const T *__restrict__ V,
                                                      int64_t ldv, const double *__restrict__ Z,
                                                      int64_t ldz, int64_t rpc,
                                                      double *__restrict__ part) {
  constexpr int CH = 128;
  __shared__ double Zs[CH * Q];
  const int64_t r0 = (int64_t)blockIdx.x * rpc;
  const int64_t r1 = (r0 + rpc < rows) ? r0 + rpc : rows;
  double *pp = part + (size_t)blockIdx.x * ncols * Q;
  for (int c0 = 0; c0 < ncols; c0 += TPB) {
    const int c = c0 + threadIdx.x;
    double acc[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t) acc[t] = 0.0;
    for (int64_t rb = r0; rb < r1; rb += CH) {
      const int nr = (int)((r1 - rb < CH) ? r1 - rb : CH);
      __syncthreads();
      for (int e = threadIdx.x; e < nr * Q; e += TPB) Zs[e] = Z[(rb + e / Q) * ldz + e % Q];
      __syncthreads();
      if (c < ncols)
        for (int r = 0; r < nr; ++r) {
          const double v = (double)V[(rb + r) * ldv + c];
#pragma unroll
          for (int t = 0; t < Q; ++t) acc[t] = fma(v, Zs[r * Q + t], acc[t]);
        }
    }
    if (c < ncols)
#pragma unroll
      for (int t = 0; t < Q; ++t) pp[c * Q + t] = acc[t];
  }
}

// out[c][t] (row stride ldo) = sum over chunks of the partials, in chunk order.
__global__ __launch_bounds__(TPB) void tn_reduce_kernel(int nchunk, int nout, int q,
                                                        const double *__restrict__ part,
                                                        double *__restrict__ out, int64_t ldo) {
  const int o = blockIdx.x * TPB + threadIdx.x;
  if (o >= nout) return;
  double a = 0.0;
  for (int k = 0; k < nchunk; ++k) a += part[(size_t)k * nout + o];
  out[(int64_t)(o / q) * ldo + o % q] = a;
}

// Y[r][t] = beta Y[r][t] + alpha sum_c V[r][c] Z[c][t] (Z: ncols x Q, row stride ldz, staged in
// LDS); one wave per row, lanes across columns.
template <int Q, typename T>
__global__ __launch_bounds__(TPB) void nn_kernel(int64_t rows, int ncols, double alpha,
                                                 const T *__restrict__ V, int64_t ldv,
                                                 const double *__restrict__ Z, int64_t ldz,
                                                 double beta, double *__restrict__ Y,
                                                 int64_t ldy) {
  extern __shared__ double Zs[];
  for (int e = threadIdx.x; e < ncols * Q; e += TPB) Zs[e] = Z[(int64_t)(e / Q) * ldz + e % Q];
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t r = (int64_t)blockIdx.x * (TPB / WAVE) + threadIdx.x / WAVE;
  if (r >= rows) return;
  double acc[Q];
#pragma unroll
  for (int t = 0; t < Q; ++t) acc[t] = 0.0;
  const T *v = V + r * ldv;
  for (int c = lane; c < ncols; c += WAVE) {
    const double x = (double)v[c];
#pragma unroll
    for (int t = 0; t < Q; ++t) acc[t] = fma(x, Zs[c * Q + t], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < Q; ++t) acc[t] = wave_sum(acc[t]);
  if (lane < Q) {
    double a = 0.0;
#pragma unroll
    for (int t = 0; t < Q; ++t)
      if (t == lane) a = acc[t];
    double *y = Y + r * ldy + lane;
    *y = (beta == 0.0) ? alpha * a : fma(alpha, a, beta * *y);
  }
}

// Orthonormalizer of a q-column panel from its Gram G = Y^T Y (one thread): G = Z diag(lam) Z^T,
// T = Z_k diag(lam_k)^(-1/2) over the eigenvalues above 1e-12 lam_max (largest first), so Y T
// has k orthonormal columns. info[0] = k; dinfo[0] = trace(G).
__global__ void orth_small_kernel(int q, const double *__restrict__ G, int64_t ldg,
                                  double *__restrict__ T, int64_t ldt, int *info, double *dinfo) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double g[SYLV_MAX_S * SYLV_MAX_S], lam[SYLV_MAX_S], Z[SYLV_MAX_S * SYLV_MAX_S];
  double tr = 0.0;
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) g[i * q + j] = 0.5 * (G[i * ldg + j] + G[j * ldg + i]);
  for (int i = 0; i < q; ++i) tr += g[i * q + i];
  jacobi_eig(g, lam, Z, q);
  double lmax = 0.0;
  for (int i = 0; i < q; ++i) lmax = fmax(lmax, lam[i]);
  bool used[SYLV_MAX_S] = {};
  int k = 0;
  for (int pass = 0; pass < q; ++pass) {  // selection by decreasing eigenvalue
    int best = -1;
    for (int i = 0; i < q; ++i)
      if (!used[i] && (best < 0 || lam[i] > lam[best])) best = i;
    used[best] = true;
    if (!(lam[best] > 1e-12 * lmax) || !(lam[best] > 0.0)) break;
    const double is = 1.0 / sqrt(lam[best]);
    for (int a = 0; a < q; ++a) T[a * ldt + k] = Z[a * q + best] * is;
    ++k;
  }
  for (int a = 0; a < q; ++a)
    for (int j = k; j < q; ++j) T[a * ldt + j] = 0.0;
  info[0] = k;
  dinfo[0] = tr;
}

// dst (rows x cols, ldd) = alpha src (transposed when trans) for a block of the residual
// coefficient matrix.
__global__ __launch_bounds__(TPB) void copy_block_kernel(int rows, int cols, double alpha,
                                                         const double *__restrict__ src,
                                                         int64_t lds, int trans,
                                                         double *__restrict__ dst, int64_t ldd) {
  for (int i = blockIdx.x; i < rows; i += gridDim.x)
    for (int j = threadIdx.x; j < cols; j += TPB)
      dst[(int64_t)i * ldd + j] =
          alpha * (trans ? src[(int64_t)j * lds + i] : src[(int64_t)i * lds + j]);
}

// dst (rows x cols, ldd) = src (lds): rows strided over the workgroups, each thread CR
// elements of a row at a time (their loads issued together).
constexpr int CR = 8;
__global__ __launch_bounds__(TPB) void copy_rows_kernel(int64_t rows, int64_t cols,
                                                        const double *__restrict__ src,
                                                        int64_t lds, double *__restrict__ dst,
                                                        int64_t ldd) {
  for (int64_t i = blockIdx.x; i < rows; i += gridDim.x) {
    const double *a = src + i * lds;
    double *b = dst + i * ldd;
    for (int64_t j0 = threadIdx.x; j0 < cols; j0 += CR * TPB) {
      double v[CR];
#pragma unroll
      for (int u = 0; u < CR; ++u) {
        const int64_t j = j0 + u * TPB;
        v[u] = a[j < cols ? j : 0];
      }
#pragma unroll
      for (int u = 0; u < CR; ++u) {
        const int64_t j = j0 + u * TPB;
        if (j < cols) b[j] = v[u];
      }
    }
  }
}

__global__ __launch_bounds__(TPB) void diag_fill_kernel(int k, double v, double *dst, int64_t ldd) {
  const int i = threadIdx.x;
  if (i < k) dst[(int64_t)i * ldd + i] = v;
}

// Y[r][t] += alpha F[r][t] for a narrow panel.
__global__ __launch_bounds__(TPB) void axpy_narrow_kernel(int64_t rows, int q, double alpha,
                                                          const double *__restrict__ F,
                                                          int64_t ldf, double *__restrict__ Y,
                                                          int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= rows * q) return;
  const int64_t i = e / q;
  const int t = (int)(e - i * q);
  Y[i * ldy + t] = fma(alpha, F[i * ldf + t], Y[i * ldy + t]);
}

}  // namespace

int launch_gauss_fill(int64_t rows, int q, uint64_t seed, double *Z, int64_t ldz, hipStream_t st) {
  const int64_t tot = rows * q;
  if (tot <= 0) return 0;
  gauss_fill_kernel<<<(unsigned)((tot + TPB - 1) / TPB), TPB, 0, st>>>(rows, q, seed, Z, ldz);
  HIPOK(hipGetLastError());
  return 0;
}

size_t tn_partials_needed(int64_t rows, int64_t ncols, int q) {
  const int64_t nch = std::min<int64_t>((rows + 255) / 256, 1024);
  return (size_t)nch * ncols * q;
}

int launch_tn(int64_t rows, int ncols, int q, const void *V, bool v_fp32, int64_t ldv,
              const double *Z, int64_t ldz, double *out, int64_t ldo, double *part,
              size_t part_cap, hipStream_t st) {
  if (ncols <= 0) return 0;
  if (q < 1 || q > SYLV_MAX_S) return SYLV_ERR_INVALID;
  if (rows <= 0) {
    HIPOK(hipMemset2DAsync(out, ldo * 8, 0, q * 8, ncols, st));
    return 0;
  }
  int64_t nch = std::min<int64_t>((rows + 255) / 256, 1024);
  const int64_t rpc = (rows + nch - 1) / nch;
  nch = (rows + rpc - 1) / rpc;
  if ((size_t)nch * ncols * q > part_cap) return SYLV_ERR_WORKSPACE;
  switch (q) {
#define CASE(QQ)                                                                               \
  case QQ:                                                                                     \
    if (v_fp32)                                                                                \
      tn_part_kernel<QQ, float><<<(unsigned)nch, TPB, 0, st>>>(                                \
          rows, ncols, static_cast<const float *>(V), ldv, Z, ldz, rpc, part);                 \
    else                                                                                       \
      tn_part_kernel<QQ, double><<<(unsigned)nch, TPB, 0, st>>>(                               \
          rows, ncols, static_cast<const double *>(V), ldv, Z, ldz, rpc, part);                \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
  }
  HIPOK(hipGetLastError());
  const int nout = ncols * q;
  tn_reduce_kernel<<<(unsigned)((nout + TPB - 1) / TPB), TPB, 0, st>>>((int)nch, nout, q, part,
                                                                        out, ldo);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_nn(int64_t rows, int ncols, int q, double alpha, const void *V, bool v_fp32,
              int64_t ldv, const double *Z, int64_t ldz, double beta, double *Y, int64_t ldy,
              hipStream_t st) {
  if (rows <= 0) return 0;
  if (q < 1 || q > SYLV_MAX_S) return SYLV_ERR_INVALID;
  if (ncols <= 0) {
    // Y = beta Y
    if (beta == 0.0) HIPOK(hipMemset2DAsync(Y, ldy * 8, 0, q * 8, rows, st));
    else if (beta != 1.0) return SYLV_ERR_INVALID;
    return 0;
  }
  // columns in chunks whose coefficients fit in 64 KiB of LDS; later chunks accumulate
  const int chunk = (int)(64 * 1024 / ((size_t)q * sizeof(double)));
  const unsigned g = (unsigned)((rows + TPB / WAVE - 1) / (TPB / WAVE));
  const size_t esz = v_fp32 ? 4 : 8;
  for (int c0 = 0; c0 < ncols; c0 += chunk) {
    const int nc = ncols - c0 < chunk ? ncols - c0 : chunk;
    const size_t lds = (size_t)nc * q * sizeof(double);
    const void *Vc = static_cast<const char *>(V) + (size_t)c0 * esz;
    const double *Zc = Z + (int64_t)c0 * ldz;
    const double bc = c0 == 0 ? beta : 1.0;
    switch (q) {
#define CASE(QQ)                                                                               \
  case QQ:                                                                                     \
    if (v_fp32)                                                                                \
      nn_kernel<QQ, float><<<g, TPB, lds, st>>>(rows, nc, alpha, static_cast<const float *>(Vc), \
                                                ldv, Zc, ldz, bc, Y, ldy);                     \
    else                                                                                       \
      nn_kernel<QQ, double><<<g, TPB, lds, st>>>(rows, nc, alpha,                              \
                                                 static_cast<const double *>(Vc), ldv, Zc,     \
                                                 ldz, bc, Y, ldy);                             \
    break;
      CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    }
    HIPOK(hipGetLastError());
  }
  return 0;
}

int launch_orth_small(int q, const double *G, int64_t ldg, double *T, int64_t ldt, int *info,
                      double *dinfo, hipStream_t st) {
  orth_small_kernel<<<1, 64, 0, st>>>(q, G, ldg, T, ldt, info, dinfo);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_copy_block(int rows, int cols, double alpha, const double *src, int64_t lds, bool trans,
                      double *dst, int64_t ldd, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return 0;
  copy_block_kernel<<<(unsigned)std::min(rows, 2048), TPB, 0, st>>>(rows, cols, alpha, src, lds,
                                                                    trans ? 1 : 0, dst, ldd);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_copy_rows(int64_t rows, int64_t cols, const double *src, int64_t lds, double *dst,
                     int64_t ldd, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return 0;
  copy_rows_kernel<<<(unsigned)std::min<int64_t>(rows, 16384), TPB, 0, st>>>(rows, cols, src, lds,
                                                                             dst, ldd);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_diag_fill(int k, double v, double *dst, int64_t ldd, hipStream_t st) {
  if (k <= 0) return 0;
  diag_fill_kernel<<<1, 64, 0, st>>>(k, v, dst, ldd);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_axpy_narrow(int64_t rows, int q, double alpha, const double *F, int64_t ldf, double *Y,
                       int64_t ldy, hipStream_t st) {
  const int64_t tot = rows * q;
  if (tot <= 0) return 0;
  axpy_narrow_kernel<<<(unsigned)((tot + TPB - 1) / TPB), TPB, 0, st>>>(rows, q, alpha, F, ldf, Y,
                                                                        ldy);
  HIPOK(hipGetLastError());
  return 0;
}
