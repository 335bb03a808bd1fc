// CSR kernels: SpMM with tall-skinny panels (the sparse products of the block Lanczos /
// Arnoldi step, eq. (3.8)), the wide SpMM of the residual evaluation, CSR validation and an
// exact CSR transpose (B^T for the W basis).
#include <mutex>
#include <vector>

#include "common.h"

namespace {

// Y[r, 0:S] = sum_q A[r, c_q] X[c_q, 0:S]; one thread per row, CSR range staged in LDS.
template <int S>
__global__ __launch_bounds__(SPMM_TPB) void spmm_kernel(int64_t rows,
                                                        const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci,
                                                        const double *__restrict__ val,
                                                        const double *__restrict__ X, int64_t ldx,
                                                        double *__restrict__ Y, int64_t ldy) {
  const int64_t r0 = (int64_t)blockIdx.x * SPMM_TPB;
  const int64_t r1 = (r0 + SPMM_TPB < rows) ? r0 + SPMM_TPB : rows;
  double acc[S];
  spmm_rows<S>(r0, r1, rp, ci, val, X, ldx, acc);
  const int64_t r = r0 + threadIdx.x;
  if (r < r1) {
    double *y = Y + r * ldy;
#pragma unroll
    for (int t = 0; t < S; ++t) y[t] = acc[t];
  }
}

// Wide SpMM for rows [r0, r1): Y[r - r0, 0:ncols] = A[r, :] X[:, 0:ncols]; one wave per row,
// lanes across columns (coalesced reads of X rows and writes of Y rows).
template <typename T>
__global__ __launch_bounds__(256) void spmm_wide_kernel(int64_t r0, int64_t r1,
                                                        const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci,
                                                        const double *__restrict__ val,
                                                        const T *__restrict__ X, int64_t ldx,
                                                        int ncols, double *__restrict__ Y,
                                                        int64_t ldy) {
  const int64_t r = r0 + (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  const int lane = threadIdx.x & (WAVE - 1);
  if (r >= r1) return;
  const int b = rp[r], e = rp[r + 1];
  double *y = Y + (r - r0) * ldy;
  for (int j0 = 0; j0 < ncols; j0 += 4 * WAVE) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = b; q < e; ++q) {
      const double a = val[q];
      const T *x = X + (int64_t)ci[q] * ldx;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + u * WAVE + lane;
        if (j < ncols) acc[u] = fma(a, (double)x[j], acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + u * WAVE + lane;
      if (j < ncols) y[j] = acc[u];
    }
  }
}

__global__ void csr_count_kernel(int64_t nnz, const int32_t *__restrict__ ci, int *cnt) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nnz) atomicAdd(&cnt[ci[q] + 1], 1);
}

// Exclusive scan of cnt[0..rows] (cnt[0] = 0) into out[0..rows]; one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void scan_kernel(int64_t len, const int *__restrict__ cnt,
                                                    int32_t *__restrict__ out) {
  __shared__ int buf[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < len; base += 1024) {
    const int64_t i = base + threadIdx.x;
    int v = (i < len) ? cnt[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // Hillis-Steele inclusive scan
      int t = ((int)threadIdx.x >= off) ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < len) out[i] = carry + buf[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
}

__global__ void csr_scatter_kernel(int64_t rows, const int32_t *__restrict__ rp,
                                   const int32_t *__restrict__ ci, const double *__restrict__ val,
                                   int *cursor, int32_t *__restrict__ oci,
                                   double *__restrict__ oval) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  for (int q = rp[r]; q < rp[r + 1]; ++q) {
    const int c = ci[q];
    const int pos = atomicAdd(&cursor[c], 1);
    oci[pos] = (int32_t)r;
    oval[pos] = val[q];
  }
}

// Sorts each row of the transposed matrix by column (insertion sort; rows are short).
__global__ void csr_sort_rows_kernel(int64_t rows, const int32_t *__restrict__ rp,
                                     int32_t *__restrict__ ci, double *__restrict__ val) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int b = rp[r], e = rp[r + 1];
  for (int i = b + 1; i < e; ++i) {
    const int32_t c = ci[i];
    const double v = val[i];
    int j = i - 1;
    while (j >= b && ci[j] > c) {
      ci[j + 1] = ci[j];
      val[j + 1] = val[j];
      --j;
    }
    ci[j + 1] = c;
    val[j + 1] = v;
  }
}

}  // namespace

int launch_spmm(int s, int64_t rows, const int32_t *rp, const int32_t *ci, const double *val,
                const double *X, int64_t ldx, double *Y, int64_t ldy, hipStream_t st) {
  if (rows <= 0) return 0;
  const dim3 grid((unsigned)((rows + SPMM_TPB - 1) / SPMM_TPB)), block(SPMM_TPB);
  switch (s) {
#define CASE(SS) \
  case SS: spmm_kernel<SS><<<grid, block, 0, st>>>(rows, rp, ci, val, X, ldx, Y, ldy); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return SYLV_ERR_INVALID;
  }
  HIPOK(hipGetLastError());
  return 0;
}

int launch_spmm_rows(int s, int64_t r0, int64_t r1, const int32_t *rp, const int32_t *ci,
                     const double *val, const void *X, bool x_fp32, int64_t ldx, int ncols,
                     double *Y, int64_t ldy, hipStream_t st) {
  (void)s;
  if (r1 <= r0 || ncols <= 0) return 0;
  const int64_t nr = r1 - r0;
  const unsigned g = (unsigned)((nr + 3) / 4);
  if (x_fp32)
    spmm_wide_kernel<float><<<g, 256, 0, st>>>(r0, r1, rp, ci, val, static_cast<const float *>(X),
                                               ldx, ncols, Y, ldy);
  else
    spmm_wide_kernel<double><<<g, 256, 0, st>>>(r0, r1, rp, ci, val,
                                                static_cast<const double *>(X), ldx, ncols, Y, ldy);
  HIPOK(hipGetLastError());
  return 0;
}

size_t csr_transpose_scratch(int64_t rows) {
  if (rows < 0 || rows > INT32_MAX) return 0;  // int32 row pointers
  return (size_t)(rows + 2) * 2 * sizeof(int) + 256;
}

namespace {
__global__ void fill_int_kernel(int64_t len, int *__restrict__ dst, int v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) dst[i] = v;
}

__global__ void copy_int_kernel(int64_t len, const int32_t *__restrict__ src, int *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) dst[i] = src[i];
}
}  // namespace

// Only kernels are enqueued (no memset or memcpy nodes), so the sequence may be captured into a
// HIP graph; the scratch counters are cleared by a fill kernel.
int launch_csr_transpose(int64_t rows, int64_t nnz, const int32_t *rp, const int32_t *ci,
                         const double *val, int32_t *orp, int32_t *oci, double *oval,
                         void *scratch, hipStream_t st) {
  int *cnt = reinterpret_cast<int *>(scratch);
  int *cursor = cnt + (rows + 2);
  fill_int_kernel<<<(unsigned)((rows + 1 + 255) / 256), 256, 0, st>>>(rows + 1, cnt, 0);
  HIPOK(hipGetLastError());
  if (nnz > 0)
    csr_count_kernel<<<(unsigned)((nnz + 255) / 256), 256, 0, st>>>(nnz, ci, cnt);
  HIPOK(hipGetLastError());
  scan_kernel<<<1, 1024, 0, st>>>(rows + 1, cnt, orp);
  HIPOK(hipGetLastError());
  // cursor[c] = orp[c]; the +1 shift of cnt makes the inclusive scan of cnt the row starts
  const unsigned g = (unsigned)((rows + 255) / 256);
  copy_int_kernel<<<g, 256, 0, st>>>(rows, orp, cursor);
  HIPOK(hipGetLastError());
  csr_scatter_kernel<<<g, 256, 0, st>>>(rows, rp, ci, val, cursor, oci, oval);
  HIPOK(hipGetLastError());
  csr_sort_rows_kernel<<<g, 256, 0, st>>>(rows, orp, oci, oval);
  HIPOK(hipGetLastError());
  return 0;
}

namespace {
// Flags malformed CSR: bit 1 row_ptr[0] != 0, bit 2 row_ptr[rows] != nnz, bit 4 a row range
// outside [0, nnz] or decreasing, bit 8 a column index out of range or not strictly increasing.
__global__ void csr_validate_kernel(int64_t rows, int64_t nnz, const int32_t *__restrict__ rp,
                                    const int32_t *__restrict__ ci, int *flag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  if (r == 0 && rp[0] != 0) atomicOr(flag, 1);
  if (r == rows - 1 && (int64_t)rp[rows] != nnz) atomicOr(flag, 2);
  const int64_t b = rp[r], e = rp[r + 1];
  if (b < 0 || e < b || e > nnz) {
    atomicOr(flag, 4);
    return;
  }
  int prev = -1;
  for (int64_t q = b; q < e; ++q) {
    const int c = ci[q];
    if (c < 0 || c >= rows || c <= prev) atomicOr(flag, 8);
    prev = c;
  }
}
}  // namespace

int launch_csr_validate(int64_t rows, int64_t nnz, const int32_t *rp, const int32_t *ci, int *flag,
                        hipStream_t st) {
  if (rows <= 0) return 0;
  csr_validate_kernel<<<(unsigned)((rows + 255) / 256), 256, 0, st>>>(rows, nnz, rp, ci, flag);
  HIPOK(hipGetLastError());
  return 0;
}

namespace {

__global__ void sell_width_kernel(int64_t rows, int64_t nslices, const int32_t *__restrict__ rp,
                                  int32_t *__restrict__ width) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nslices) return;
  int w = 0;
  const int64_t r1 = (k * 64 + 64 < rows) ? k * 64 + 64 : rows;
  for (int64_t r = k * 64; r < r1; ++r) {
    const int len = rp[r + 1] - rp[r];
    w = len > w ? len : w;
  }
  width[k] = w;
}

__global__ void sell_fill_kernel(int64_t rows, const int32_t *__restrict__ rp,
                                 const int32_t *__restrict__ ci, const double *__restrict__ val,
                                 const int32_t *__restrict__ width, const int64_t *__restrict__ off,
                                 int32_t *__restrict__ sci, double *__restrict__ sval) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int64_t k = r >> 6;
  const int w = width[k];
  const int64_t base = off[k] + (r & 63);
  const int b = rp[r], len = rp[r + 1] - b;
  for (int q = 0; q < w; ++q) {
    const bool in = q < len;
    sci[base + 64 * q] = in ? ci[b + q] : (int32_t)r;
    sval[base + 64 * q] = in ? val[b + q] : 0.0;
  }
}

// flag |= 1 when an entry of row r does not fit the narrow form (its value is not exactly a
// float, or its column is more than 32767 away from the row)
__global__ void sell_narrow_check_kernel(int64_t rows, const int32_t *__restrict__ rp,
                                         const int32_t *__restrict__ ci,
                                         const double *__restrict__ val, int *flag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  bool ok = true;
  for (int64_t q = rp[r]; q < rp[r + 1]; ++q) {
    const double v = val[q];
    const int64_t d = (int64_t)ci[q] - r;
    ok = ok && (double)(float)v == v && d >= -32767 && d <= 32767;
  }
  if (!ok) atomicOr(flag, 1);
}

__global__ void sell_fill_narrow_kernel(int64_t rows, const int32_t *__restrict__ rp,
                                        const int32_t *__restrict__ ci,
                                        const double *__restrict__ val,
                                        const int32_t *__restrict__ width,
                                        const int64_t *__restrict__ off, int16_t *__restrict__ cd,
                                        float *__restrict__ valf) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int64_t k = r >> 6;
  const int w = width[k];
  const int64_t base = off[k] + (r & 63);
  const int b = rp[r], len = rp[r + 1] - b;
  for (int q = 0; q < w; ++q) {
    const bool in = q < len;
    cd[base + 64 * q] = in ? (int16_t)(ci[b + q] - r) : (int16_t)0;
    valf[base + 64 * q] = in ? (float)val[b + q] : 0.0f;
  }
}

// NR rows per thread, from NR consecutive blocks of 256 rows (each block read by whole slices);
// NR > 1 keeps NR rows of loads in flight per thread and divides the workgroups of a launch over
// a large operator by NR.
template <int S, int NR>
__global__ __launch_bounds__(256) void sell_spmm_kernel(SellMat M, const double *__restrict__ X,
                                                        int64_t ldx, double *__restrict__ Y,
                                                        int64_t ldy) {
  if (NR == 1) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= M.rows) return;
    double acc[S];
    sell_row<S>(M, r, X, ldx, acc);
    double *y = Y + r * ldy;
#pragma unroll
    for (int t = 0; t < S; ++t) y[t] = acc[t];
    return;
  }
  int64_t r[NR];
  bool ok[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    r[i] = ((int64_t)blockIdx.x * NR + i) * 256 + threadIdx.x;
    ok[i] = r[i] < M.rows;
  }
  if (!ok[0]) return;
  double acc[NR][S];
  sell_rows<NR, S>(M, r, ok, X, ldx, acc);
#pragma unroll
  for (int i = 0; i < NR; ++i)
    if (ok[i])
#pragma unroll
      for (int t = 0; t < S; ++t) Y[r[i] * ldy + t] = acc[i][t];
}

}  // namespace

int build_sell(int64_t rows, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *val,
               void *buf, hipStream_t st, bool allow_narrow, int *narrow) {
  SellMat m = sell_view(rows, nnz, buf);
  const int64_t ns = m.nslices;
  int32_t *width = const_cast<int32_t *>(m.width);
  int64_t *off = const_cast<int64_t *>(m.off);
  const unsigned gr = (unsigned)((rows + 255) / 256);
  sell_width_kernel<<<(unsigned)((ns + 255) / 256), 256, 0, st>>>(rows, ns, rp, width);
  HIPOK(hipGetLastError());
  // the narrow-form flag lives in the offsets' first word until the offsets are written
  int *flag = reinterpret_cast<int *>(off);
  if (allow_narrow) {
    fill_int_kernel<<<1, 64, 0, st>>>(1, flag, 0);
    HIPOK(hipGetLastError());
    sell_narrow_check_kernel<<<gr, 256, 0, st>>>(rows, rp, ci, val, flag);
    HIPOK(hipGetLastError());
  }
  std::vector<int32_t> hw(ns);
  std::vector<int64_t> ho(ns);
  int hflag = 1;
  HIPOK(hipMemcpyAsync(hw.data(), width, ns * 4, hipMemcpyDeviceToHost, st));
  if (allow_narrow) HIPOK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  int64_t tot = 0;
  for (int64_t k = 0; k < ns; ++k) {
    ho[k] = tot;
    tot += 64 * (int64_t)hw[k];
  }
  if (tot > sell_capacity(rows, nnz)) return SYLV_ERR_WORKSPACE;
  const bool nar = allow_narrow && hflag == 0;
  HIPOK(hipMemcpyAsync(off, ho.data(), ns * 8, hipMemcpyHostToDevice, st));
  if (nar)
    sell_fill_narrow_kernel<<<gr, 256, 0, st>>>(rows, rp, ci, val, width, off,
                                                const_cast<int16_t *>(m.cd),
                                                const_cast<float *>(m.valf));
  else
    sell_fill_kernel<<<gr, 256, 0, st>>>(rows, rp, ci, val, width, off,
                                         const_cast<int32_t *>(m.ci), const_cast<double *>(m.val));
  HIPOK(hipGetLastError());
  HIPOK(hipStreamSynchronize(st));
  if (narrow) *narrow = nar ? 1 : 0;
  return 0;
}

int launch_sell_spmm(int s, const SellMat &M, const double *X, int64_t ldx, double *Y, int64_t ldy,
                     hipStream_t st) {
  if (M.rows <= 0) return 0;
  // two rows per thread (one column) where one row per thread would take more than the 2048
  // workgroups the GPU holds at once (eight per CU)
  const bool two = s == 1 && M.rows > (int64_t)2048 * 256;
  const unsigned g = (unsigned)((M.rows + (two ? 511 : 255)) / (two ? 512 : 256));
  if (two) {
    sell_spmm_kernel<1, 2><<<g, 256, 0, st>>>(M, X, ldx, Y, ldy);
    HIPOK(hipGetLastError());
    return 0;
  }
  switch (s) {
#define CASE(SS) \
  case SS: sell_spmm_kernel<SS, 1><<<g, 256, 0, st>>>(M, X, ldx, Y, ldy); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return SYLV_ERR_INVALID;
  }
  HIPOK(hipGetLastError());
  return 0;
}

// ---- CSR transpose for callers that cannot allocate ----
//
// The transpose's scratch (column counts and scatter cursors, 2 (rows + 2) ints) lives in a
// file-scope device array instead of a caller buffer. Each GPU holds its own copy for the
// life of the process; its device address is looked up once per device and kept, and only that
// address is handed to kernels (the array's name is not a device address in host code).
namespace {

constexpr int64_t NOALLOC_MAX_ROWS = SYLV_NOALLOC_TRANSPOSE_MAX_ROWS;
constexpr size_t NOALLOC_SCRATCH_INTS = 2 * (size_t)(NOALLOC_MAX_ROWS + 2) + 64;
static_assert(NOALLOC_SCRATCH_INTS * sizeof(int) >= (size_t)(NOALLOC_MAX_ROWS + 2) * 2 * sizeof(int) + 256,
              "scratch array smaller than the transpose needs at the row limit");

__device__ __align__(256) int scratch[NOALLOC_SCRATCH_INTS];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array (looked up on the first call per device, with
// that device current).
int scratch_address(void **out) {
  int dev = -1;
  HIPOK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return SYLV_ERR_INVALID;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIPOK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return SYLV_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

}  // namespace

extern "C" int sylv_csr_transpose_noalloc(const sylv_csr *A, int32_t *out_row_ptr,
                                          int32_t *out_col_idx, double *out_values,
                                          void *stream) {
  if (!A || !out_row_ptr || A->rows <= 0 || A->nnz < 0 || A->nnz >= ((int64_t)1 << 31) ||
      !A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->values || !out_col_idx || !out_values)))
    return SYLV_ERR_INVALID;
  if (A->rows > NOALLOC_MAX_ROWS) {
    note_error("sylv_csr_transpose_noalloc: rows exceed SYLV_NOALLOC_TRANSPOSE_MAX_ROWS");
    return SYLV_ERR_WORKSPACE;
  }
  void *scr = nullptr;
  int e = scratch_address(&scr);
  if (e) return e;
  return launch_csr_transpose(A->rows, A->nnz, A->row_ptr, A->col_idx, A->values, out_row_ptr,
                              out_col_idx, out_values, scr, reinterpret_cast<hipStream_t>(stream));
}
