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
constexpr int GRAM_STREAM_WG = 512;  // stream-K Gram: two workgroups per CU
constexpr int LD = BM + 1;  // +1 pad: fewer bank conflicts on the transposed fills
static_assert(BM == BN, "one LDS slab shape serves both operands");

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

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

// Eight consecutive elements (32-byte aligned for float, 64-byte for double) as doubles.
__device__ __forceinline__ void load8(const double *p, RegSlab &r) {
  const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
  for (int u = 0; u < 4; ++u) r.v[u] = q[u];
}
__device__ __forceinline__ void load8(const float *p, RegSlab &r) {
  const float4 *q = reinterpret_cast<const float4 *>(p);
  const float4 a = q[0], b = q[1];
  r.v[0] = double2{(double)a.x, (double)a.y};
  r.v[1] = double2{(double)a.z, (double)a.w};
  r.v[2] = double2{(double)b.x, (double)b.y};
  r.v[3] = double2{(double)b.z, (double)b.w};
}

template <typename T>
__device__ __forceinline__ void load_rows(const T *base, int64_t ld, RegSlab &r) {
  const int i = threadIdx.x >> 2, k = (threadIdx.x & 3) * 8;
  load8(base + (int64_t)i * ld + k, r);
}

__device__ __forceinline__ void store_rows(Slab &dst, const RegSlab &r) {
  const int i = threadIdx.x >> 2, k = (threadIdx.x & 3) * 8;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    dst[k + 2 * u][i] = r.v[u].x;
    dst[k + 2 * u + 1][i] = r.v[u].y;
  }
}

template <typename T>
__device__ __forceinline__ void load_cols(const T *base, int64_t ld, RegSlab &r) {
  const int k = threadIdx.x >> 3, j = (threadIdx.x & 7) * 8;
  load8(base + (int64_t)k * ld + j, r);
}

__device__ __forceinline__ void store_cols(Slab &dst, const RegSlab &r) {
  const int k = threadIdx.x >> 3, j = (threadIdx.x & 7) * 8;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    dst[k][j + 2 * u] = r.v[u].x;
    dst[k][j + 2 * u + 1] = r.v[u].y;
  }
}

// Operand slabs: A(i, l) is A[i * lda + l] ("rows", A_T = false) or A[l * lda + i] (A_T = true,
// a K x M row-major matrix read transposed); B(l, j) is B[l * ldb + j] ("cols", B_ROWS = false)
// or B[j * ldb + l] (B_ROWS = true).
template <bool A_T, bool B_ROWS, typename TA, typename TB>
__device__ __forceinline__ void load_slab(const TA *A, int64_t lda, const TB *B, int64_t ldb,
                                          int64_t l, RegSlab &ra, RegSlab &rb) {
  if (A_T) load_cols(A + l * lda, lda, ra);
  else load_rows(A + l, lda, ra);
  if (B_ROWS) load_rows(B + l, ldb, rb);
  else load_cols(B + l * ldb, ldb, rb);
}

// Zeroes the elements of a "rows" slab at slab column lim and beyond (a select, so whatever was
// read there is dropped).
__device__ __forceinline__ void mask_rows(RegSlab &r, int lim) {
  const int k = (threadIdx.x & 3) * 8;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (k + 2 * u >= lim) r.v[u].x = 0.0;
    if (k + 2 * u + 1 >= lim) r.v[u].y = 0.0;
  }
}

// lim: the K columns of the row-form operands from the slab start that are used (>= BK: all);
// the rest are stored as zeros.
template <bool A_T, bool B_ROWS>
__device__ __forceinline__ void store_slab(Smem &sm, int buf, RegSlab &ra, RegSlab &rb,
                                           int64_t lim) {
  if (lim < BK) {
    if (!A_T) mask_rows(ra, (int)lim);
    if (B_ROWS) mask_rows(rb, (int)lim);
  }
  if (A_T) store_cols(sm.As[buf], ra);
  else store_rows(sm.As[buf], ra);
  if (B_ROWS) store_rows(sm.Bs[buf], rb);
  else store_cols(sm.Bs[buf], rb);
}

// One pipelined product over K slabs [l_begin, l_end) (multiples of BK): acc += A(i0.., l) B(l, j0..)
// with the operand forms above (A, B point at row/column i0 and j0). Global loads run two slabs
// ahead of the MFMAs (two register sets, the loop unrolled by two so they stay static); LDS is
// double-buffered with one barrier per slab. Row-form operands enter with their K columns at
// kmax and beyond as zeros (applied when a slab is stored to LDS, after its loads have landed).
template <bool A_T, bool B_ROWS, typename TA = double, typename TB = double>
__device__ __forceinline__ void pipelined(Smem &sm, WaveAcc &acc, int wm, int wn, const TA *A,
                                          int64_t lda, const TB *B, int64_t ldb,
                                          int64_t l_begin, int64_t l_end,
                                          int64_t kmax = INT64_MAX) {
  if (l_begin >= l_end) return;
  const int64_t nsl = (l_end - l_begin) / BK;
  // Prefetches are unconditional (a slab index past the end re-reads the last slab, always in
  // bounds), so the number of loads in flight is the same on every path and the wait before an
  // LDS fill only covers the older register set.
  auto lslab = [&](int64_t t) { return l_begin + (t < nsl ? t : nsl - 1) * BK; };
  auto lim = [&](int64_t t) { return kmax - lslab(t); };
  RegSlab ra0, rb0, ra1, rb1;
  load_slab<A_T, B_ROWS, TA, TB>(A, lda, B, ldb, lslab(0), ra0, rb0);
  load_slab<A_T, B_ROWS, TA, TB>(A, lda, B, ldb, lslab(1), ra1, rb1);
  __syncthreads();  // previous users of the LDS buffers are done
  store_slab<A_T, B_ROWS>(sm, 0, ra0, rb0, lim(0));
  __syncthreads();
  // invariant at slab t: LDS[t % 2] holds slab t; register set (t+1) % 2 holds slab t+1
  int64_t t = 0;
  for (; t + 1 < nsl; t += 2) {
    load_slab<A_T, B_ROWS, TA, TB>(A, lda, B, ldb, lslab(t + 2), ra0, rb0);
    mma_slab(sm.As[0], sm.Bs[0], acc, wm, wn);
    store_slab<A_T, B_ROWS>(sm, 1, ra1, rb1, lim(t + 1));
    __syncthreads();
    load_slab<A_T, B_ROWS, TA, TB>(A, lda, B, ldb, lslab(t + 3), ra1, rb1);
    mma_slab(sm.As[1], sm.Bs[1], acc, wm, wn);
    store_slab<A_T, B_ROWS>(sm, 0, ra0, rb0, lim(t + 2));
    __syncthreads();
  }
  if (t < nsl) mma_slab(sm.As[0], sm.Bs[0], acc, wm, wn);  // odd slab count: the last slab
}

// ---- core operator (all indices < ldc; entries outside the active cores are exact zeros) ----
// Output tile (I, J) (64 x 64, T tiles per side) is the slab sequence of its two products:
// H P over K slabs [lsH(I), pk) (columns J < Tp only, Tp = ceil(p / 64)), then P G^T over
// [lsG(J), pk) (rows I < Tp only); lsH and lsG skip the structurally zero part of the block
// Hessenberg factors (rows of block b only meet columns of blocks >= b - 1).
__host__ __device__ inline int core_start(int s, int idx) {  // first K of tile row / column idx
  int ls = (idx * BM / s - 1) * s;
  return ls < 0 ? 0 : ls / BK * BK;
}

// Per-launch table of the slab counts (passed by value): ns[i] slabs of tile row / column i,
// colpre / rowpre prefix sums of ns and of the row lengths. Tile (I, J) has nH = ns[I] H P slabs
// (J < Tp) and ns[J] P G^T slabs (I < Tp).
constexpr int CT_MAX = 32;  // tiles per side of the stream-K form
struct CoreTab {
  int T, Tp, pk, p;
  int ns[CT_MAX], colpre[CT_MAX + 1], rowpre[CT_MAX + 1];
  __host__ __device__ int nh(int I, int J) const { return J < Tp ? ns[I] : 0; }
  __host__ __device__ int len(int I, int J) const { return nh(I, J) + (I < Tp ? ns[J] : 0); }
  __host__ __device__ int offset(int I, int J) const {
    return rowpre[I] + (J < Tp ? J : Tp) * ns[I] + (I < Tp ? colpre[J] : 0);
  }
  __host__ __device__ int total() const { return rowpre[T]; }
};

CoreTab make_core_tab(int s, int p, int T) {
  CoreTab t{};
  t.T = T;
  t.Tp = (p + BM - 1) / BM;
  t.pk = (p + BK - 1) / BK * BK;
  t.p = p;
  for (int i = 0; i < T; ++i) t.ns[i] = (t.pk - core_start(s, i)) / BK;
  for (int i = 0; i < T; ++i) t.colpre[i + 1] = t.colpre[i] + t.ns[i];
  for (int i = 0; i < T; ++i)
    t.rowpre[i + 1] = t.rowpre[i] + t.Tp * t.ns[i] + (i < t.Tp ? t.colpre[T] : 0);
  return t;
}

// Slabs [a, b) of tile (I, J)'s sequence (nH H P slabs from K = lsH, then P G^T slabs from lsG)
// into acc. Columns of H and G at or past p are stored to LDS as zeros: they belong to Krylov
// steps that may be writing them on the other stream (they meet the exact-zero rows of P, but a
// provisional non-finite value would still reach the sum through a product with zero).
__device__ __forceinline__ void core_tile_part(Smem &sm, WaveAcc &acc, const double *H,
                                               const double *G, const double *P, int64_t ldc,
                                               int p, int I, int J, int nH, int lsH, int lsG,
                                               int a, int b, int wm, int wn) {
  const int i0 = I * BM, j0 = J * BN;
  const int ha = a < nH ? a : nH, hb = b < nH ? b : nH;
  if (hb > ha)
    pipelined<false, false>(sm, acc, wm, wn, H + (int64_t)i0 * ldc, ldc, P + j0, ldc,
                            lsH + ha * BK, lsH + hb * BK, p);
  const int ga = (a > nH ? a : nH) - nH, gb = (b > nH ? b : nH) - nH;
  if (gb > ga)
    pipelined<false, true>(sm, acc, wm, wn, P + (int64_t)i0 * ldc, ldc, G + (int64_t)j0 * ldc,
                           ldc, lsG + ga * BK, lsG + gb * BK, p);
}

// One workgroup per complementary pair of tiles b and T*T - 1 - b, i.e. (I, J) and
// (T-1-I, T-1-J): their sequences add up to the same length for every b.
__device__ __forceinline__ void core_op_body(int s, int p, int T, const double *__restrict__ H,
                                             const double *__restrict__ G,
                                             const double *__restrict__ P,
                                             double *__restrict__ Q, int64_t ldc,
                                             const int *done) {
  if (done && *done) return;
  __shared__ Smem sm;
  const int w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
  const int pk = (p + BK - 1) / BK * BK;
  const int t1 = blockIdx.x, t2 = T * T - 1 - t1;
  for (int t = t1;; t = t2) {
    const int I = t / T, J = t % T;
    const int lsH = core_start(s, I), lsG = core_start(s, J);
    const int nH = J * BN < p ? (pk - lsH) / BK : 0;
    const int nG = I * BM < p ? (pk - lsG) / BK : 0;
    WaveAcc acc;
    zero_acc(acc);
    core_tile_part(sm, acc, H, G, P, ldc, p, I, J, nH, lsH, lsG, 0, nH + nG, wm, wn);
    for_each_acc(acc, wm, wn, [&](int ii, int jj, double v) {
      Q[(int64_t)(I * BM + ii) * ldc + J * BN + jj] = v;
    });
    if (t == t2) break;
  }
}

__global__ __launch_bounds__(256, 2) void core_op_kernel(int s, int p, int T, const double *H,
                                                         const double *G, const double *P,
                                                         double *Q, int64_t ldc,
                                                         const int *done) {
  core_op_body(s, p, T, H, G, P, Q, ldc, done);
}

// The core operator of every problem of a batch group (blockIdx.y): Q = op(P) (which = 0) or
// T = op(S) (which = 1).
__global__ __launch_bounds__(256, 2) void core_op_group(const CoreInst *tab, const int *list,
                                                        int s, int p, int T, int which) {
  const CoreInst &c = tab[list ? list[blockIdx.y] : blockIdx.y];
  core_op_body(s, p, T, c.H, c.G, which ? c.S : c.P, which ? c.T : c.Q, c.ldc, &c.ds->done);
}

// Stream-K form: the concatenated sequence of all tiles (row-major) is cut into chunks of c
// slabs, chunk w for workgroup w, so every workgroup does the same matrix-core work whatever
// the tile lengths. Workgroup w stores its part of tile t as partial tile t + w (distinct for
// all pieces); core_op_reduce sums a tile's pieces in chunk order (deterministic). Chunks are
// numbered so that XCD x (workgroups b with b % 8 == x) runs a contiguous eighth of the
// sequence: its tiles share their H and P row panels in its L2.
__global__ __launch_bounds__(256, 2) void core_op_stream_kernel(const CoreTab tab, int c,
                                                                int nchunks,
                                                                const double *__restrict__ H,
                                                                const double *__restrict__ G,
                                                                const double *__restrict__ P,
                                                                int64_t ldc, const int *done,
                                                                double *__restrict__ part) {
  if (done && *done) return;
  const int per = (int)(gridDim.x >> 3);
  const int w = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (w >= nchunks) return;
  __shared__ Smem sm;
  const int T = tab.T;
  const int total = tab.total();
  const int c0 = w * c, c1 = (c0 + c < total) ? c0 + c : total;
  const int wv = threadIdx.x >> 6, wm = wv >> 1, wn = wv & 1;
  // locate the tile holding position c0
  int I = 0;
  while (I + 1 < T && tab.rowpre[I + 1] <= c0) ++I;
  int J = 0;
  int off = tab.rowpre[I];
  while (off + tab.len(I, J) <= c0) off += tab.len(I, J++);
  int pos = c0;
  while (pos < c1 && I < T) {
    const int l = tab.len(I, J);
    if (l > 0) {
      const int a = pos - off;
      const int b = (c1 < off + l ? c1 : off + l) - off;
      WaveAcc acc;
      zero_acc(acc);
      core_tile_part(sm, acc, H, G, P, ldc, tab.p, I, J, tab.nh(I, J), tab.pk - tab.ns[I] * BK,
                     tab.pk - tab.ns[J] * BK, a, b, wm, wn);
      double *pt = part + (size_t)(I * T + J + w) * (BM * BN);
      for_each_acc(acc, wm, wn, [&](int ii, int jj, double v) { pt[ii * BN + jj] = v; });
      pos = off + b;
    }
    off += l;
    if (++J == T) {
      J = 0;
      ++I;
    }
  }
}

// Q tile t = sum of its pieces t + w over the chunks w that cover it, in chunk order (zero for
// tiles with an empty sequence). 16 workgroups per tile, one element per thread.
__global__ __launch_bounds__(256) void core_op_reduce_kernel(const CoreTab tab, int c,
                                                             const double *__restrict__ part,
                                                             double *__restrict__ Q, int64_t ldc,
                                                             const int *done) {
  if (done && *done) return;
  const int T = tab.T;
  const int t = blockIdx.x / 16, sub = blockIdx.x % 16;
  const int I = t / T, J = t % T;
  const int l = tab.len(I, J);
  const int e = sub * 256 + threadIdx.x;
  double v = 0.0;
  if (l > 0) {
    const int off = tab.offset(I, J);
    const int w0 = off / c, w1 = (off + l - 1) / c;
    for (int w = w0; w <= w1; ++w) v += part[(size_t)(t + w) * (BM * BN) + e];
  }
  Q[(int64_t)(I * BM + e / BN) * ldc + J * BN + e % BN] = v;
}

// ---- tall-skinny Gram C (+)= A^T B over K rows (residual evaluation) ----
// A: K x M and B: K x N row-major with row strides lda, ldb; columns up to the next multiple of
// 64 of M (N) must lie inside the rows (lda >= roundup(M, 64)); K is a multiple of BK. With
// `lower`, only tiles I >= J are computed (symmetric A^T A; mirror_kernel fills the rest).
// With part != nullptr the K range is split: workgroup b computes tile b % ntiles over rows
// [kz kchunk, (kz+1) kchunk), kz = b / ntiles, and stores the whole tile to part; gram_reduce
// sums the slices in order.
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void gram_kernel(int64_t M, int64_t N, int64_t K,
                                                   const TA *__restrict__ A, int64_t lda,
                                                   const TB *__restrict__ B, int64_t ldb,
                                                   double beta, double *__restrict__ C,
                                                   int64_t ldc, int tiles_n, int lower, int ntiles,
                                                   int64_t kchunk, double *__restrict__ part) {
  __shared__ Smem sm;
  const int tile = (int)(blockIdx.x % ntiles), kz = (int)(blockIdx.x / ntiles);
  int I, J;
  if (lower) tri_tile(tile, I, J);
  else {
    I = tile / tiles_n;
    J = tile % tiles_n;
  }
  const int64_t i0 = (int64_t)I * BM, j0 = (int64_t)J * BN;
  const int w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
  WaveAcc acc;
  zero_acc(acc);
  const int64_t k0 = (int64_t)kz * kchunk, k1 = (k0 + kchunk < K) ? k0 + kchunk : K;
  const int64_t kb = k0 + (k1 - k0) / BK * BK;
  pipelined<true, false, TA, TB>(sm, acc, wm, wn, A + i0, lda, B + j0, ldb, k0, kb);
  if (k1 > kb) {
    // last k1 - kb < BK rows, zero-filled past k1
    __syncthreads();
    for (int e = threadIdx.x; e < BK * BM; e += 256) {
      const int kk = e / BM, ii = e % BM;
      sm.As[0][kk][ii] = (kb + kk < k1) ? (double)A[(kb + kk) * lda + i0 + ii] : 0.0;
      sm.Bs[0][kk][ii] = (kb + kk < k1) ? (double)B[(kb + kk) * ldb + j0 + ii] : 0.0;
    }
    __syncthreads();
    mma_slab(sm.As[0], sm.Bs[0], acc, wm, wn);
  }
  if (part) {
    double *pt = part + ((size_t)kz * ntiles + tile) * (BM * BN);
    for_each_acc(acc, wm, wn, [&](int ii, int jj, double v) { pt[ii * BN + jj] = v; });
    return;
  }
  for_each_acc(acc, wm, wn, [&](int ii, int jj, double v) {
    const int64_t gi = i0 + ii, gj = j0 + jj;
    if (gi < M && gj < N) {
      double *c = C + gi * ldc + gj;
      *c = (beta == 0.0) ? v : *c + v;
    }
  });
}

// C tile (beta C +) sum over the nk K-slices of the tile's partials, in slice order; 16
// workgroups per tile.
__global__ __launch_bounds__(256) void gram_reduce_kernel(int64_t M, int64_t N, int tiles_n,
                                                          int lower, int ntiles, int nk,
                                                          const double *__restrict__ part,
                                                          double beta, double *__restrict__ C,
                                                          int64_t ldc) {
  const int tile = blockIdx.x / 16, sub = blockIdx.x % 16;
  int I, J;
  if (lower) tri_tile(tile, I, J);
  else {
    I = tile / tiles_n;
    J = tile % tiles_n;
  }
  {
    const int e = sub * 256 + threadIdx.x;
    double v = 0.0;
    for (int kz = 0; kz < nk; ++kz) v += part[((size_t)kz * ntiles + tile) * (BM * BN) + e];
    const int64_t gi = (int64_t)I * BM + e / BN, gj = (int64_t)J * BN + e % BN;
    if (gi < M && gj < N) {
      double *c = C + gi * ldc + gj;
      *c = (beta == 0.0) ? v : *c + v;
    }
  }
}

// ---- stream-K form of the tall-skinny Gram (launches with many output tiles) ----
// Schedule over G workgroups (G a multiple of 8; workgroup b is worker w = (b % 8) G/8 + b / 8,
// so XCD x runs workers [x G/8, (x+1) G/8)):
// * whole tiles first: worker w computes tiles w, w + G, ... below dp = floor(T / G) G. The
//   workers of one XCD then hold 64 consecutive tiles of the visiting order (eight tile rows by
//   eight columns) and walk K in step, so their row and column panels are shared in its L2;
// * then the remaining tiles [dp, T) in stream-K form: their slab sequences (nsl slabs each, the
//   last one zero-filled past K when K % BK != 0) are concatenated and cut into chunks of c
//   slabs, chunk w for worker w. A tile inside one chunk goes to C directly; a tile cut by chunk
//   boundaries leaves its piece of chunk w in partial slot 2w (the chunk's first tile) or 2w + 1
//   (its last tile), and gram_stream_fix_kernel sums the pieces in chunk order.
// Whole tiles write C = acc (C += acc when beta != 0). Every worker does the same matrix-core
// work, whatever the number of tiles.
template <typename TA, typename TB>
__device__ __forceinline__ void gram_piece(Smem &sm, WaveAcc &acc, int64_t i0, int64_t j0,
                                           int64_t K, const TA *__restrict__ A, int64_t lda,
                                           const TB *__restrict__ B, int64_t ldb, int64_t a,
                                           int64_t b, int wm, int wn) {
  const int64_t nfull = K / BK;
  const int64_t bf = b < nfull ? b : nfull;
  if (bf > a)
    pipelined<true, false, TA, TB>(sm, acc, wm, wn, A + i0, lda, B + j0, ldb, a * BK, bf * BK);
  if (b > nfull) {
    // the last K % BK rows, zero-filled past K
    const int64_t kb = nfull * BK;
    __syncthreads();
    for (int e = threadIdx.x; e < BK * BM; e += 256) {
      const int kk = e / BM, ii = e % BM;
      sm.As[0][kk][ii] = (kb + kk < K) ? (double)A[(kb + kk) * lda + i0 + ii] : 0.0;
      sm.Bs[0][kk][ii] = (kb + kk < K) ? (double)B[(kb + kk) * ldb + j0 + ii] : 0.0;
    }
    __syncthreads();
    mma_slab(sm.As[0], sm.Bs[0], acc, wm, wn);
  }
}

__device__ __forceinline__ void gram_store(const WaveAcc &acc, int64_t i0, int64_t j0, int64_t M,
                                           int64_t N, double beta, double *__restrict__ C,
                                           int64_t ldc, int wm, int wn) {
  for_each_acc(acc, wm, wn, [&](int ii, int jj, double v) {
    const int64_t gi = i0 + ii, gj = j0 + jj;
    if (gi < M && gj < N) {
      double *cp = C + gi * ldc + gj;
      *cp = (beta == 0.0) ? v : *cp + v;
    }
  });
}

template <typename TA, typename TB>
__global__ __launch_bounds__(256, 2) void gram_stream_kernel(
    const GramSeq sq, int64_t M, int64_t N, int64_t K, const TA *__restrict__ A, int64_t lda,
    const TB *__restrict__ B, int64_t ldb, double beta, double *__restrict__ C, int64_t ldc,
    int64_t nsl, int64_t dp, int64_t c, int nchunks, double *__restrict__ part) {
  const int G = (int)gridDim.x, per = G >> 3;
  const int w = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  __shared__ Smem sm;
  const int wv = threadIdx.x >> 6, wm = wv >> 1, wn = wv & 1;
  for (int64_t t = w; t < dp; t += G) {
    int I, J;
    sq.tile(t, I, J);
    const int64_t i0 = (int64_t)I * BM, j0 = (int64_t)J * BN;
    WaveAcc acc;
    zero_acc(acc);
    gram_piece<TA, TB>(sm, acc, i0, j0, K, A, lda, B, ldb, 0, nsl, wm, wn);
    gram_store(acc, i0, j0, M, N, beta, C, ldc, wm, wn);
  }
  if (w >= nchunks) return;
  const int64_t total = (sq.count() - dp) * nsl;
  const int64_t c0 = (int64_t)w * c, c1 = (c0 + c < total) ? c0 + c : total;
  for (int64_t pos = c0; pos < c1;) {
    const int64_t tr = pos / nsl, ts = tr * nsl;
    const int64_t a = pos - ts, b = ((c1 < ts + nsl) ? c1 : ts + nsl) - ts;
    int I, J;
    sq.tile(dp + tr, I, J);
    const int64_t i0 = (int64_t)I * BM, j0 = (int64_t)J * BN;
    WaveAcc acc;
    zero_acc(acc);
    gram_piece<TA, TB>(sm, acc, i0, j0, K, A, lda, B, ldb, a, b, wm, wn);
    if (a == 0 && b == nsl) {
      gram_store(acc, i0, j0, M, N, beta, C, ldc, wm, wn);
    } else {
      double *pt = part + (size_t)(2 * w + (pos == c0 ? 0 : 1)) * (BM * BN);
      for_each_acc(acc, wm, wn, [&](int ii, int jj, double v) { pt[ii * BN + jj] = v; });
    }
    pos = ts + b;
  }
}

// The remaining tiles cut by chunk boundaries: boundary wb (between chunks wb and wb + 1)
// handles the tile it falls in unless an earlier boundary falls in the same tile; TW * TW / 256
// workgroups per boundary (TW the tile width), one element per thread. Tile indices count from
// dp.
template <int TW>
__global__ __launch_bounds__(256) void gram_stream_fix_kernel(const GramSeq sq, int64_t M,
                                                              int64_t N, int64_t nsl, int64_t dp,
                                                              int64_t c,
                                                              const double *__restrict__ part,
                                                              double beta, double *__restrict__ C,
                                                              int64_t ldc) {
  constexpr int SUBS = TW * TW / 256;
  const int wb = (int)(blockIdx.x / SUBS), sub = (int)(blockIdx.x % SUBS);
  const int64_t pb = (int64_t)(wb + 1) * c, total = (sq.count() - dp) * nsl;
  if (pb >= total || pb % nsl == 0) return;
  const int64_t tr = pb / nsl, ts = tr * nsl;
  if ((int64_t)wb * c > ts) return;
  const int w0 = (int)(ts / c), w1 = (int)((ts + nsl - 1) / c);
  const int e = sub * 256 + threadIdx.x;
  double v = 0.0;
  for (int w = w0; w <= w1; ++w) {
    const int slot = 2 * w + ((int64_t)w * c / nsl == tr ? 0 : 1);
    v += part[(size_t)slot * (TW * TW) + e];
  }
  int I, J;
  sq.tile(dp + tr, I, J);
  const int64_t gi = (int64_t)I * TW + e / TW, gj = (int64_t)J * TW + e % TW;
  if (gi < M && gj < N) {
    double *cp = C + gi * ldc + gj;
    *cp = (beta == 0.0) ? v : *cp + v;
  }
}

// ---- 128 x 128 tiles: the large FP64 Grams ----
// Each 256-thread workgroup owns a 128 x 128 output tile, each wave a 64 x 64 quarter (4 x 4
// MFMA tiles, sixteen accumulators), two workgroups per CU. K runs in slabs of 16 rows through
// two LDS buffers: at slab t, after one barrier, the waves run the first 16 of the slab's 64
// MFMAs per wave on the current buffer, store slab t + 1 (loaded into registers during slab
// t - 1) into the free buffer, issue the global loads of slab t + 2, and run the other 48. Per
// flop this reads half the LDS and L2 bytes of the 64 x 64 tiles and meets a barrier half as
// often. FP64 operands only.
constexpr int TW2 = 128, BK2 = 16;
constexpr int LW2 = TW2 + 16;  // slab row of 128 doubles, padded by 32 banks: the two rows
                               // that one LDS pass of an MFMA operand read meets do not collide
constexpr int GRAM_WIDE_WG = 512;  // two workgroups per CU (72 KB of LDS each)

struct Smem2 {
  double A[2][BK2][LW2];
  double B[2][BK2][LW2];
};

struct Acc2 {
  v4d c[4][4];
};

// MFMA operand layout as in mma_slab; each step of 4 rows reads its operands, then runs its 16
// MFMAs (the other workgroup on the CU covers the LDS latency). Steps [Q0, Q1) of the slab.
template <int Q0 = 0, int Q1 = BK2 / 4>
__device__ __forceinline__ void mma2(const double (&As)[BK2][LW2], const double (&Bs)[BK2][LW2],
                                     Acc2 &acc, int wm, int wn) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const double *pa = &As[lk][wm * 64 + li], *pb = &Bs[lk][wn * 64 + li];
#pragma unroll
  for (int q = Q0; q < Q1; ++q) {
    double a[4], b[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      a[t] = pa[q * 4 * LW2 + t * 16];
      b[t] = pb[q * 4 * LW2 + t * 16];
    }
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
        acc.c[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], acc.c[ti][tj], 0, 0, 0);
  }
}

__device__ __forceinline__ void zero_acc2(Acc2 &acc) {
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc.c[ti][tj] = v4d{0.0, 0.0, 0.0, 0.0};
}

template <typename F>
__device__ __forceinline__ void for_each_acc2(const Acc2 &acc, int wm, int wn, F f) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        f(wm * 64 + ti * 16 + v * 4 + rq, wn * 64 + tj * 16 + col, acc.c[ti][tj][v]);
}

// acc += A(:, i0 ..)^T B(:, j0 ..) over K slabs [a, b) of tile (i0, j0); the slab past the last
// full one holds the last K % BK2 rows, zero-filled past K.
__device__ __forceinline__ void gram_piece2(Smem2 &sm, Acc2 &acc, int64_t i0, int64_t j0,
                                            int64_t K, const double *__restrict__ A, int64_t lda,
                                            const double *__restrict__ B, int64_t ldb, int64_t a,
                                            int64_t b, int wm, int wn) {
  const int64_t nfull = K / BK2;
  const int64_t bf = b < nfull ? b : nfull;
  if (bf > a) {
    // one thread's share of a slab: rows threadIdx.x / 64 + 4 u, the column pair
    // 2 (threadIdx.x % 64) (a wave reads whole 1 KB slab rows). A column pair at or past the
    // leading dimension reads column 0 instead: in bounds, and it only feeds outputs that are
    // not stored.
    const int kr = threadIdx.x >> 6, c = 2 * (threadIdx.x & 63);
    const double *pa = A + (i0 + c < lda ? i0 + c : 0) + kr * lda;
    const double *pb = B + (j0 + c < ldb ? j0 + c : 0) + kr * ldb;
    v2d ra[BK2 / 4], rb[BK2 / 4];
    auto load = [&](int64_t l) {
#pragma unroll
      for (int u = 0; u < BK2 / 4; ++u) {
        ra[u] = *reinterpret_cast<const v2d *>(pa + (l + 4 * u) * lda);
        rb[u] = *reinterpret_cast<const v2d *>(pb + (l + 4 * u) * ldb);
      }
    };
    auto store = [&](int buf) {
#pragma unroll
      for (int u = 0; u < BK2 / 4; ++u) {
        *reinterpret_cast<v2d *>(&sm.A[buf][kr + 4 * u][c]) = ra[u];
        *reinterpret_cast<v2d *>(&sm.B[buf][kr + 4 * u][c]) = rb[u];
      }
    };
    const int64_t nsl = bf - a;
    load(a * BK2);
    __syncthreads();  // earlier users of both buffers are done
    store(0);
    load((a + (nsl > 1 ? 1 : 0)) * BK2);
    for (int64_t t = 0; t < nsl; ++t) {
      __syncthreads();  // slab t is in buffer t % 2 for every wave; the other buffer is free
      const int cur = (int)(t & 1);
      // the slab's MFMAs at a raised priority: the co-resident workgroup's stores and loads take
      // the issue slots they leave. The first step's MFMAs go before this wave's own store of
      // slab t + 1, whose wait for the loads issued a slab ago comes that much later.
      __builtin_amdgcn_s_setprio(1);
      mma2<0, 1>(sm.A[cur], sm.B[cur], acc, wm, wn);
      __builtin_amdgcn_s_setprio(0);
      if (t + 1 < nsl) {
        store(cur ^ 1);
        load((a + (t + 2 < nsl ? t + 2 : nsl - 1)) * BK2);
      }
      __builtin_amdgcn_s_setprio(1);
      mma2<1, BK2 / 4>(sm.A[cur], sm.B[cur], acc, wm, wn);
      __builtin_amdgcn_s_setprio(0);
    }
  }
  if (b > nfull) {
    const int64_t kb = nfull * BK2;
    __syncthreads();
    for (int e = threadIdx.x; e < BK2 * TW2; e += 256) {
      const int kk = e / TW2, ii = e % TW2;
      const bool in = kb + kk < K;
      sm.A[0][kk][ii] = (in && i0 + ii < lda) ? A[(kb + kk) * lda + i0 + ii] : 0.0;
      sm.B[0][kk][ii] = (in && j0 + ii < ldb) ? B[(kb + kk) * ldb + j0 + ii] : 0.0;
    }
    __syncthreads();
    mma2(sm.A[0], sm.B[0], acc, wm, wn);
  }
}

// Stream-K schedule as gram_stream_kernel's, over 128 x 128 tiles (partial slots of 128 x 128),
// for a table of Gram products that share K: the tiles of all jobs form one sequence (job q's
// tiles from jobs.j[q].t0 on, each job in its own visiting order), so several products of one
// row chunk run as one launch with whole-tile rounds across all of them.
__device__ __forceinline__ const GramJob &job_of(const GramJobs &jobs, int64_t t, int64_t &lt) {
  int q = 0;
  while (q + 1 < jobs.n && jobs.j[q + 1].t0 <= t) ++q;
  lt = t - jobs.j[q].t0;
  return jobs.j[q];
}

__global__ __launch_bounds__(256, 2) void gram_wide_kernel(const GramJobs jobs, int64_t K,
                                                           double beta, int64_t nsl, int64_t dp,
                                                           int64_t c, int nchunks,
                                                           double *__restrict__ part) {
  const int G = (int)gridDim.x, per = G >> 3;
  const int w = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  __shared__ Smem2 sm;
  const int wv = threadIdx.x >> 6, wm = wv >> 1, wn = wv & 1;
  auto store_c = [&](const Acc2 &acc, const GramJob &jb, int64_t i0, int64_t j0) {
    for_each_acc2(acc, wm, wn, [&](int ii, int jj, double v) {
      const int64_t gi = i0 + ii, gj = j0 + jj;
      if (gi < jb.M && gj < jb.N) {
        double *cp = jb.C + gi * jb.ldc + gj;
        *cp = (beta == 0.0) ? v : *cp + v;
      }
    });
  };
  for (int64_t t = w; t < dp; t += G) {
    int64_t lt;
    const GramJob &jb = job_of(jobs, t, lt);
    int I, J;
    jb.sq.tile(lt, I, J);
    const int64_t i0 = (int64_t)I * TW2, j0 = (int64_t)J * TW2;
    Acc2 acc;
    zero_acc2(acc);
    gram_piece2(sm, acc, i0, j0, K, jb.A, jb.lda, jb.B, jb.ldb, 0, nsl, wm, wn);
    store_c(acc, jb, i0, j0);
  }
  if (w >= nchunks) return;
  const int64_t total = (jobs.total - dp) * nsl;
  const int64_t c0 = (int64_t)w * c, c1 = (c0 + c < total) ? c0 + c : total;
  for (int64_t pos = c0; pos < c1;) {
    const int64_t tr = pos / nsl, ts = tr * nsl;
    const int64_t a = pos - ts, b = ((c1 < ts + nsl) ? c1 : ts + nsl) - ts;
    int64_t lt;
    const GramJob &jb = job_of(jobs, dp + tr, lt);
    int I, J;
    jb.sq.tile(lt, I, J);
    const int64_t i0 = (int64_t)I * TW2, j0 = (int64_t)J * TW2;
    Acc2 acc;
    zero_acc2(acc);
    gram_piece2(sm, acc, i0, j0, K, jb.A, jb.lda, jb.B, jb.ldb, a, b, wm, wn);
    if (a == 0 && b == nsl) {
      store_c(acc, jb, i0, j0);
    } else {
      double *pt = part + (size_t)(2 * w + (pos == c0 ? 0 : 1)) * (TW2 * TW2);
      for_each_acc2(acc, wm, wn, [&](int ii, int jj, double v) { pt[ii * TW2 + jj] = v; });
    }
    pos = ts + b;
  }
}

// The tiles of a job table cut by stream-K chunk boundaries (as gram_stream_fix_kernel<128>).
__global__ __launch_bounds__(256) void gram_wide_fix_kernel(const GramJobs jobs, int64_t nsl,
                                                            int64_t dp, int64_t c,
                                                            const double *__restrict__ part,
                                                            double beta) {
  constexpr int SUBS = TW2 * TW2 / 256;
  const int wb = (int)(blockIdx.x / SUBS), sub = (int)(blockIdx.x % SUBS);
  const int64_t pb = (int64_t)(wb + 1) * c, total = (jobs.total - dp) * nsl;
  if (pb >= total || pb % nsl == 0) return;
  const int64_t tr = pb / nsl, ts = tr * nsl;
  if ((int64_t)wb * c > ts) return;
  const int w0 = (int)(ts / c), w1 = (int)((ts + nsl - 1) / c);
  const int e = sub * 256 + threadIdx.x;
  double v = 0.0;
  for (int w = w0; w <= w1; ++w) {
    const int slot = 2 * w + ((int64_t)w * c / nsl == tr ? 0 : 1);
    v += part[(size_t)slot * (TW2 * TW2) + e];
  }
  int64_t lt;
  const GramJob &jb = job_of(jobs, dp + tr, lt);
  int I, J;
  jb.sq.tile(lt, I, J);
  const int64_t gi = (int64_t)I * TW2 + e / TW2, gj = (int64_t)J * TW2 + e % TW2;
  if (gi < jb.M && gj < jb.N) {
    double *cp = jb.C + gi * jb.ldc + gj;
    *cp = (beta == 0.0) ? v : *cp + v;
  }
}

// C[i][j] = C[j][i] for i < j < M (upper from lower).
__global__ __launch_bounds__(256) void mirror_kernel(int64_t M, double *__restrict__ C,
                                                     int64_t ldc) {
  for (int64_t i = blockIdx.x; i < M; i += gridDim.x)
    for (int64_t j = i + 1 + threadIdx.x; j < M; j += 256) C[i * ldc + j] = C[j * ldc + i];
}

// Basis defect rows: E(i, 0:p) -= V(i, 0:q) H(0:q, 0:p) for i < rows, with H block upper
// Hessenberg (H(l, c) = 0 when block(l) > block(c) + 1), so output tile J only needs
// l < (block(j0 + 63) + 2) s. V columns in [q, roundup(q, BK)) must be finite (they meet zero
// rows of H); V rows past `rows` are never read (row index clamped, results masked).
template <typename T>
__global__ __launch_bounds__(256) void defect_gemm_kernel(int64_t rows, int p, int q, int s,
                                                          const T *__restrict__ V, int64_t ldv,
                                                          const double *__restrict__ H,
                                                          int64_t ldh, double *__restrict__ E,
                                                          int64_t lde) {
  __shared__ Smem sm;
  const int64_t i0 = (int64_t)blockIdx.y * BM;
  const int j0 = blockIdx.x * BN;
  const int w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
  const int jl = (j0 + BN - 1 < p - 1) ? j0 + BN - 1 : p - 1;
  int le = (jl / s + 2) * s;
  le = le < q ? le : q;
  le = (le + BK - 1) / BK * BK;
  WaveAcc acc;
  zero_acc(acc);
  if (i0 + BM <= rows) {
    pipelined<false, false, T, double>(sm, acc, wm, wn, V + i0 * ldv, ldv, H + j0, ldh, 0, le);
  } else {
    // last row tile: stage through a clamped copy of the row pointer range
    const int64_t last = rows - 1;
    for (int64_t l0 = 0; l0 < le; l0 += BK) {
      for (int e = threadIdx.x; e < BM * BK; e += 256) {
        const int ii = e / BK, kk = e % BK;
        const int64_t gi = i0 + ii < last ? i0 + ii : last;
        sm.As[0][kk][ii] = (double)V[gi * ldv + l0 + kk];
      }
      for (int e = threadIdx.x; e < BK * BN; e += 256) {
        const int kk = e / BN, jj = e % BN;
        sm.Bs[0][kk][jj] = H[(l0 + kk) * ldh + j0 + jj];
      }
      __syncthreads();
      mma_slab(sm.As[0], sm.Bs[0], acc, wm, wn);
      __syncthreads();
    }
  }
  for_each_acc(acc, wm, wn, [&](int ii, int jj, double v) {
    const int64_t gi = i0 + ii;
    const int gj = j0 + jj;
    if (gi < rows && gj < p) E[gi * lde + gj] -= v;
  });
}

// V(i, c0:c1) = 0 for all rows (finite padding columns before defect_gemm_kernel).
template <typename T>
__global__ __launch_bounds__(256) void zero_cols_kernel(int64_t rows, T *V, int64_t ldv, int c0,
                                                        int c1) {
  const int w = c1 - c0;
  const int64_t total = rows * w;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / w;
    V[i * ldv + c0 + (e - i * w)] = (T)0;
  }
}

// ---- C = A B for row-major operands on the pipelined slabs (one 64 x 64 tile per workgroup) ----
// A: M x K (lda), B: K x N (ldb); rows of A up to roundup(M, 64) and columns of B up to
// roundup(N, 64) must be readable (their products only reach masked outputs); K runs in full
// slabs, the last K % BK entries zero-filled, so nothing past K is read.
__global__ __launch_bounds__(256, 2) void gemm_nn_kernel(int64_t M, int64_t N, int64_t K,
                                                         const double *__restrict__ A, int64_t lda,
                                                         const double *__restrict__ B, int64_t ldb,
                                                         double *__restrict__ C, int64_t ldc,
                                                         int tiles_n) {
  __shared__ Smem sm;
  const int64_t i0 = (int64_t)(blockIdx.x / tiles_n) * BM, j0 = (int64_t)(blockIdx.x % tiles_n) * BN;
  const int w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
  WaveAcc acc;
  zero_acc(acc);
  const int64_t kb = K / BK * BK;
  pipelined<false, false>(sm, acc, wm, wn, A + i0 * lda, lda, B + j0, ldb, 0, kb);
  if (K > kb) {
    __syncthreads();
    for (int e = threadIdx.x; e < BK * BM; e += 256) {
      const int kk = e / BM, ii = e % BM;
      sm.As[0][kk][ii] = (kb + kk < K) ? A[(i0 + ii) * lda + kb + kk] : 0.0;
      sm.Bs[0][kk][ii] = (kb + kk < K) ? B[(kb + kk) * ldb + j0 + ii] : 0.0;
    }
    __syncthreads();
    mma_slab(sm.As[0], sm.Bs[0], acc, wm, wn);
  }
  for_each_acc(acc, wm, wn, [&](int ii, int jj, double v) {
    const int64_t gi = i0 + ii, gj = j0 + jj;
    if (gi < M && gj < N) C[gi * ldc + gj] = v;
  });
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
                   int64_t ldc, const int *done, hipStream_t st, double *part, size_t part_cap) {
  const int q = p + s;
  const int T = (q + BM - 1) / BM;
  if ((int64_t)T * BM > ldc || ((p + BK - 1) / BK * BK) > ldc) return SYLV_ERR_WORKSPACE;
  const int tiles = T * T;
  // stream-K over up to 256 workgroups (one per CU: the Krylov steps of the next iteration run
  // beside it), chunks of at least two slabs, as long as the partial tiles (one per tile plus
  // one per chunk) fit in part; otherwise tile pairs
  if (part && T <= CT_MAX) {
    const CoreTab tab = make_core_tab(s, p, T);
    const int total = tab.total();
    constexpr int NWG = 256;
    const int c = std::max(2, (total + NWG - 1) / NWG);
    const int nchunks = (total + c - 1) / c;
    if (total > 0 && (size_t)(tiles + nchunks) * BM * BN <= part_cap) {
      const int per = (nchunks + 7) / 8;
      core_op_stream_kernel<<<(unsigned)(8 * per), 256, 0, st>>>(tab, c, nchunks, H, G, P, ldc,
                                                                  done, part);
      HIPOK(hipGetLastError());
      core_op_reduce_kernel<<<(unsigned)(tiles * 16), 256, 0, st>>>(tab, c, part, Q, ldc, done);
      HIPOK(hipGetLastError());
      return 0;
    }
  }
  core_op_kernel<<<(unsigned)((tiles + 1) / 2), 256, 0, st>>>(s, p, T, H, G, P, Q, ldc, done);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_core_op_group(int s, int p, int which, const CoreInst *tab, const int *list, int n,
                         hipStream_t st) {
  if (n < 1) return 0;  // no problem in the launches
  const int T = (p + s + BM - 1) / BM;
  core_op_group<<<dim3((unsigned)((T * T + 1) / 2), (unsigned)n), 256, 0, st>>>(tab, list, s, p,
                                                                                 T, which);
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

int launch_gemm_nn(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                   const double *B, int64_t ldb, double *C, int64_t ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return 0;
  if (lda % 8 || ldb % 8 || lda < (K + BK - 1) / BK * BK || ldb < (N + BN - 1) / BN * BN)
    return SYLV_ERR_INVALID;
  const int64_t TM = (M + BM - 1) / BM, TN = (N + BN - 1) / BN;
  gemm_nn_kernel<<<(unsigned)(TM * TN), 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc, (int)TN);
  HIPOK(hipGetLastError());
  return 0;
}

// FP64 Grams of at least this many 128 x 128 tiles take gram_wide_kernel
constexpr int64_t GRAM_WIDE_MIN_TILES = 256;

// Stream-K launch of gram_wide_kernel over a job table when its partial slots fit (two per
// stream-K chunk, one chunk per workgroup); returns 1 when it did not launch.
static int launch_gram_wide(GramJobs &jobs, int64_t K, double beta, hipStream_t st, double *part,
                            size_t part_cap) {
  jobs.total = 0;
  for (int q = 0; q < jobs.n; ++q) {
    GramJob &jb = jobs.j[q];
    const int TM = (int)((jb.M + TW2 - 1) / TW2), TN = (int)((jb.N + TW2 - 1) / TW2);
    jb.sq = GramSeq{TM, TN, jb.sq.lower};
    jb.t0 = jobs.total;
    jobs.total += jb.sq.count();
  }
  const int64_t G = GRAM_WIDE_WG, nsl = (K + BK2 - 1) / BK2, dp = jobs.total / G * G;
  const int64_t total = (jobs.total - dp) * nsl;
  const int64_t c = std::max<int64_t>((total + G - 1) / G, 4);
  const int64_t nchunks = (total + c - 1) / c;
  if ((size_t)(2 * nchunks) * (TW2 * TW2) > part_cap) return 1;
  gram_wide_kernel<<<(unsigned)G, 256, 0, st>>>(jobs, K, beta, nsl, dp, c, (int)nchunks, part);
  HIPOK(hipGetLastError());
  if (nchunks > 1) {
    gram_wide_fix_kernel<<<(unsigned)(nchunks - 1) * (TW2 * TW2 / 256), 256, 0, st>>>(
        jobs, nsl, dp, c, part, beta);
    HIPOK(hipGetLastError());
  }
  return 0;
}

int64_t gram_wide_tiles(int64_t M, int64_t N, bool lower) {
  const int64_t TM = (M + TW2 - 1) / TW2, TN = (N + TW2 - 1) / TW2;
  return lower ? TM * (TM + 1) / 2 : TM * TN;
}

int launch_gram_jobs(const GramJob *jobs, int n, int64_t K, double beta, hipStream_t st,
                     double *part, size_t part_cap) {
  if (n < 1 || n > GRAM_JOBS_MAX || K <= 0 || !part) return 1;
  GramJobs t{};
  t.n = 0;
  for (int q = 0; q < n; ++q) {
    const GramJob &jb = jobs[q];
    if (jb.M <= 0 || jb.N <= 0) continue;
    if ((jb.sq.lower && jb.M != jb.N) || jb.lda % 8 || jb.ldb % 8 || jb.lda < jb.M ||
        jb.ldb < jb.N)
      return SYLV_ERR_INVALID;
    t.j[t.n++] = jb;
  }
  if (t.n == 0) return 0;
  int64_t tiles = 0;
  for (int q = 0; q < t.n; ++q) tiles += gram_wide_tiles(t.j[q].M, t.j[q].N, t.j[q].sq.lower);
  if (tiles < GRAM_WIDE_MIN_TILES) return 1;
  return launch_gram_wide(t, K, beta, st, part, part_cap);
}


size_t gram_part_doubles(int64_t max_cols, int64_t rows) {
  // the wide form's slots for a full round of workgroups where its Grams can occur
  return (max_cols >= 2048 && rows >= 4096) ? (size_t)2 * GRAM_WIDE_WG * TW2 * TW2
                                            : (size_t)1024 * BM * BN;
}

int launch_gram(int64_t M, int64_t N, int64_t K, const void *A, bool a_fp32, int64_t lda,
                const void *B, bool b_fp32, int64_t ldb, double beta, double *C, int64_t ldc,
                bool lower, hipStream_t st, double *part, size_t part_cap) {
  if (M <= 0 || N <= 0) return 0;
  if (lower && M != N) return SYLV_ERR_INVALID;
  const int64_t TM = (M + BM - 1) / BM, TN = (N + BN - 1) / BN;
  if (lda < TM * BM || ldb < TN * BN || lda % 8 || ldb % 8) return SYLV_ERR_INVALID;
  if (K <= 0) return 0;
  const int64_t tiles = lower ? TM * (TM + 1) / 2 : TM * TN;
  if (!a_fp32 && !b_fp32 && part && gram_wide_tiles(M, N, lower) >= GRAM_WIDE_MIN_TILES) {
    GramJobs t{};
    t.n = 1;
    t.j[0] = GramJob{GramSeq{0, 0, lower ? 1 : 0}, M, N, static_cast<const double *>(A), lda,
                     static_cast<const double *>(B), ldb, C, ldc, 0};
    const int e = launch_gram_wide(t, K, beta, st, part, part_cap);
    if (e <= 0) return e;  // launched, or an error; 1: the slots do not fit
  }
  // many tiles: whole tiles in rounds of 512 workgroups (two per CU), the rest in stream-K
  // form, when the partial slots fit
  if (part && tiles >= 64) {
    const GramSeq sq{(int)TM, (int)TN, lower ? 1 : 0};
    const int64_t G = GRAM_STREAM_WG;
    const int64_t nsl = (K + BK - 1) / BK, dp = tiles / G * G, total = (tiles - dp) * nsl;
    const int64_t c = std::max<int64_t>((total + G - 1) / G, 4);
    const int64_t nchunks = (total + c - 1) / c;
    if ((size_t)(2 * nchunks) * (BM * BN) <= part_cap) {
#define GRAM_SK(TA, TB)                                                                         \
  gram_stream_kernel<TA, TB><<<(unsigned)G, 256, 0, st>>>(                                      \
      sq, M, N, K, static_cast<const TA *>(A), lda, static_cast<const TB *>(B), ldb, beta, C, \
      ldc, nsl, dp, c, (int)nchunks, part)
      if (a_fp32 && b_fp32) GRAM_SK(float, float);
      else if (a_fp32) GRAM_SK(float, double);
      else if (b_fp32) GRAM_SK(double, float);
      else GRAM_SK(double, double);
#undef GRAM_SK
      HIPOK(hipGetLastError());
      if (nchunks > 1) {
        gram_stream_fix_kernel<BM><<<(unsigned)(nchunks - 1) * (BM * BN / 256), 256, 0, st>>>(
            sq, M, N, nsl, dp, c, part, beta, C, ldc);
        HIPOK(hipGetLastError());
      }
      return 0;
    }
  }
  // few tiles over a long K: split K so that about 512 workgroups run (partials in part)
  int64_t nk = 1;
  if (part && tiles < 64 && K >= 4 * 1024) {
    nk = std::min<int64_t>({(256 + tiles - 1) / tiles, K / 1024, 64,
                            (int64_t)(part_cap / ((size_t)tiles * BM * BN))});
    if (nk < 2) nk = 1;
  }
  int64_t kchunk = K;
  if (nk > 1) {
    kchunk = ((K + nk - 1) / nk + BK - 1) / BK * BK;
    nk = (K + kchunk - 1) / kchunk;
  }
  double *pp = nk > 1 ? part : nullptr;
  const unsigned grid = (unsigned)(tiles * nk);
#define GRAM(TA, TB)                                                                           \
  gram_kernel<TA, TB><<<grid, 256, 0, st>>>(M, N, K, static_cast<const TA *>(A), lda,          \
                                            static_cast<const TB *>(B), ldb, beta, C, ldc,     \
                                            (int)TN, lower ? 1 : 0, (int)tiles, kchunk, pp)
  if (a_fp32 && b_fp32) GRAM(float, float);
  else if (a_fp32) GRAM(float, double);
  else if (b_fp32) GRAM(double, float);
  else GRAM(double, double);
#undef GRAM
  HIPOK(hipGetLastError());
  if (pp) {
    gram_reduce_kernel<<<(unsigned)tiles * 16, 256, 0, st>>>(M, N, (int)TN, lower ? 1 : 0,
                                                             (int)tiles, (int)nk, pp, beta, C, ldc);
    HIPOK(hipGetLastError());
  }
  return 0;
}

int launch_mirror(int64_t M, double *C, int64_t ldc, hipStream_t st) {
  if (M <= 1) return 0;
  mirror_kernel<<<(unsigned)std::min<int64_t>(M, 1024), 256, 0, st>>>(M, C, ldc);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_defect_gemm(int64_t rows, int p, int q, int s, const void *V, bool v_fp32, int64_t ldv,
                       const double *H, int64_t ldh, double *E, int64_t lde, hipStream_t st) {
  if (rows <= 0 || p <= 0) return 0;
  const int qk = (q + BK - 1) / BK * BK;
  const int pn = (p + BN - 1) / BN * BN;
  if (ldv < qk || ldh < pn || ldv % 8) return SYLV_ERR_INVALID;
  const dim3 grid((unsigned)(pn / BN), (unsigned)((rows + BM - 1) / BM));
  if (v_fp32)
    defect_gemm_kernel<float><<<grid, 256, 0, st>>>(rows, p, q, s, static_cast<const float *>(V),
                                                    ldv, H, ldh, E, lde);
  else
    defect_gemm_kernel<double><<<grid, 256, 0, st>>>(rows, p, q, s,
                                                     static_cast<const double *>(V), ldv, H, ldh,
                                                     E, lde);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_zero_cols(int64_t rows, void *V, bool v_fp32, int64_t ldv, int c0, int c1,
                     hipStream_t st) {
  if (rows <= 0 || c1 <= c0) return 0;
  const int64_t total = rows * (c1 - c0);
  const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
  if (v_fp32) zero_cols_kernel<float><<<g, 256, 0, st>>>(rows, static_cast<float *>(V), ldv, c0, c1);
  else zero_cols_kernel<double><<<g, 256, 0, st>>>(rows, static_cast<double *>(V), ldv, c0, c1);
  HIPOK(hipGetLastError());
  return 0;
}
