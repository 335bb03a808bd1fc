// Low-rank compression of the factored solution X = V Xc W^T (Corollary 3.3): a truncated SVD
// of the FP64 core Xc (r x r) and tall products with the bases, X ~= (V U_k) diag(sigma) (W Y_k)^T.
//
// The core's SVD is formed from a randomized range: Y = Xc Omega (Gaussian Omega, l columns),
// one power step Y = Xc Xc^T Q, Q an orthonormal basis of Y, then the small matrix B = Q^T Xc
// (l x r) is decomposed exactly by one-sided Jacobi rotations (Hestenes), G B = D with D's rows
// orthogonal: B = G^T diag(sigma) Yh^T, so Xc ~= (Q G^T) diag(sigma) Yh^T. The truncation rank
// is the smallest k whose singular-value tail is within the tolerance; the error of the rank-k
// core ||Xc - U_k diag(sigma_k) Y_k^T||_F is then evaluated directly (no cancellation), and l
// doubles while it misses the tolerance. One-sided Jacobi keeps high relative accuracy for
// the small singular values, which a Gram eigen-decomposition would lose.
#include <algorithm>
#include <vector>

#include "common.h"

namespace {

constexpr int JT = 1024;  // threads of the one-workgroup Jacobi kernel

// Orthogonalizes the rows of M (nr x len, row stride ldm) by plane rotations of row pairs in
// round-robin order (every pair once per sweep, the pairs of a round disjoint, one wave per
// pair), accumulating the rotations in G (nr x nr, starts as the identity), until a sweep finds
// every pair orthogonal to tol or max_sweeps ran: G M_in = M_out. info[0] = sweeps.
__global__ __launch_bounds__(JT) void jacobi_rows_kernel(int nr, int64_t len, double *M,
                                                         int64_t ldm, double *G, int64_t ldg,
                                                         double tol, int max_sweeps, int *info) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = JT / 64;
  for (int e = tid; e < nr * nr; e += JT) G[(int64_t)(e / nr) * ldg + e % nr] = (e / nr == e % nr);
  __shared__ int rotated;
  const int np = nr + (nr & 1);
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      for (int k = wv; k < np / 2; k += nw) {
        const int a = (k == 0) ? 0 : (k - 1 + round) % (np - 1) + 1;
        const int b = (np - 2 - k + round) % (np - 1) + 1;
        if (a >= nr || b >= nr) continue;
        double *ma = M + (int64_t)a * ldm, *mb = M + (int64_t)b * ldm;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int64_t x = lane; x < len; x += 64) {
          const double u = ma[x], v = mb[x];
          al = fma(u, u, al);
          be = fma(v, v, be);
          ga = fma(u, v, ga);
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (ga == 0.0 || fabs(ga) <= tol * sqrt(al * be)) continue;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int64_t x = lane; x < len; x += 64) {
          const double u = ma[x], v = mb[x];
          ma[x] = c * u - s * v;
          mb[x] = s * u + c * v;
        }
        double *ga_ = G + (int64_t)a * ldg, *gb_ = G + (int64_t)b * ldg;
        for (int x = lane; x < nr; x += 64) {
          const double u = ga_[x], v = gb_[x];
          ga_[x] = c * u - s * v;
          gb_[x] = s * u + c * v;
        }
        if (lane == 0) atomicAdd(&rotated, 1);
      }
      __syncthreads();
    }
    const int r = rotated;
    __syncthreads();
    if (r == 0) break;
  }
  if (tid == 0) info[0] = sweep;
}

// norms[i] = ||M(i, :)||_2, one wave per row.
__global__ __launch_bounds__(256) void row_norms_kernel(int nr, int64_t len, const double *M,
                                                        int64_t ldm, double *norms) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= nr) return;
  double v = 0.0;
  for (int64_t x = lane; x < len; x += 64) v = fma(M[row * ldm + x], M[row * ldm + x], v);
  v = wave_sum(v);
  if (lane == 0) norms[row] = sqrt(v);
}

// M(i, :) *= f[i] (rows whose factor is zero are cleared).
__global__ __launch_bounds__(256) void scale_rows_kernel(int nr, int64_t len, double *M,
                                                         int64_t ldm, const double *f) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)nr * len) return;
  const int64_t i = e / len;
  M[i * ldm + (e - i * len)] *= f[i];
}

// Partials of ||A - B||_F^2 and ||A||_F^2 over r x c (B may be null).
__global__ __launch_bounds__(256) void diff_norm_kernel(int64_t r, int64_t c, const double *A,
                                                        int64_t lda, const double *B, int64_t ldb,
                                                        double *partials) {
  double v[2] = {0.0, 0.0};
  for (int64_t i = blockIdx.x; i < r; i += gridDim.x)
    for (int64_t j = threadIdx.x; j < c; j += 256) {
      const double a = A[i * lda + j];
      const double d = B ? a - B[i * ldb + j] : a;
      v[0] = fma(d, d, v[0]);
      v[1] = fma(a, a, v[1]);
    }
  __shared__ double lds[32];
  block_sum<2>(v, lds);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = v[0];
    partials[2 * blockIdx.x + 1] = v[1];
  }
}

// dst(:, t) = src(:, idx[t]) * (scale ? scale[idx[t]] : 1) for t < k (rows x k).
__global__ __launch_bounds__(256) void gather_cols_kernel(int64_t rows, int k, const int *idx,
                                                          const double *src, int64_t lds,
                                                          const double *scale, double *dst,
                                                          int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * k) return;
  const int64_t i = e / k;
  const int t = (int)(e - i * k);
  const double f = scale ? scale[idx[t]] : 1.0;
  dst[i * ldd + t] = src[i * lds + idx[t]] * f;
}

// dst(:, t) = src(idx[t], :)^T / sig[idx[t]] for t < k (rows of the orthogonalized B become the
// right singular vectors), len x k.
__global__ __launch_bounds__(256) void gather_rows_t_kernel(int64_t len, int k, const int *idx,
                                                            const double *src, int64_t lds,
                                                            const double *sig, double *dst,
                                                            int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= len * k) return;
  const int64_t i = e / k;
  const int t = (int)(e - i * k);
  const double s = sig[idx[t]];
  dst[i * ldd + t] = s > 0.0 ? src[(int64_t)idx[t] * lds + i] / s : 0.0;
}

unsigned grid1(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int launch_jacobi_rows(int nr, int64_t len, double *M, int64_t ldm, double *G, int64_t ldg,
                       int *info, hipStream_t st) {
  if (nr <= 0) return 0;
  jacobi_rows_kernel<<<1, JT, 0, st>>>(nr, len, M, ldm, G, ldg, 1e-15, 40, info);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_row_norms(int nr, int64_t len, const double *M, int64_t ldm, double *norms,
                     hipStream_t st) {
  if (nr <= 0) return 0;
  row_norms_kernel<<<(unsigned)((nr + 3) / 4), 256, 0, st>>>(nr, len, M, ldm, norms);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_scale_rows(int nr, int64_t len, double *M, int64_t ldm, const double *f,
                      hipStream_t st) {
  if (nr <= 0 || len <= 0) return 0;
  scale_rows_kernel<<<grid1((int64_t)nr * len), 256, 0, st>>>(nr, len, M, ldm, f);
  HIPOK(hipGetLastError());
  return 0;
}

// ||A - B||_F and ||A||_F (host), B may be null; partials: 2 * 512 doubles of scratch.
int diff_norm(int64_t r, int64_t c, const double *A, int64_t lda, const double *B, int64_t ldb,
              double *partials, double *dnorm, double *anorm, hipStream_t st) {
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(r, 512));
  diff_norm_kernel<<<g, 256, 0, st>>>(r, c, A, lda, B, ldb, partials);
  HIPOK(hipGetLastError());
  std::vector<double> h(2 * g);
  HIPOK(hipMemcpyAsync(h.data(), partials, sizeof(double) * 2 * g, hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  double d = 0.0, a = 0.0;
  for (unsigned b = 0; b < g; ++b) {
    d += h[2 * b];
    a += h[2 * b + 1];
  }
  if (dnorm) *dnorm = std::sqrt(d);
  if (anorm) *anorm = std::sqrt(a);
  return 0;
}

int launch_gather_cols(int64_t rows, int k, const int *idx, const double *src, int64_t lds,
                       const double *scale, double *dst, int64_t ldd, hipStream_t st) {
  if (rows <= 0 || k <= 0) return 0;
  gather_cols_kernel<<<grid1(rows * k), 256, 0, st>>>(rows, k, idx, src, lds, scale, dst, ldd);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_gather_rows_t(int64_t len, int k, const int *idx, const double *src, int64_t lds,
                         const double *sig, double *dst, int64_t ldd, hipStream_t st) {
  if (len <= 0 || k <= 0) return 0;
  gather_rows_t_kernel<<<grid1(len * k), 256, 0, st>>>(len, k, idx, src, lds, sig, dst, ldd);
  HIPOK(hipGetLastError());
  return 0;
}
