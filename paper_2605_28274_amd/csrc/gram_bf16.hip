// Split-BF16 Gram products on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16), for the Gram
// blocks of the true-residual evaluation that may run below FP64.
//
// Every operand value x is scaled by a power of two per column (so the column's largest entry
// lies in [1/2, 1); scaling is exact) and split as x = hi + lo + d with hi = bf16(x),
// lo = bf16(x - hi), |d| <= 2^-17 |x|. A product is formed as hi_a hi_b + hi_a lo_b + lo_a hi_b
// (the dropped lo_a lo_b term is below 2^-16 of it) with FP32 accumulation over at most 4096
// rows per partial; partials are summed, and unscaled, in FP64. The relative error of a Gram
// entry is therefore of order 1e-5 of the sum of the absolute products, against 1e-16 for the
// FP64 Grams: this path is for blocks whose contribution to the residual norm is small (the
// basis defects A V - V H, which are at rounding level) or where that accuracy suffices.
//
// Operands are packed per row chunk: slab t (32 consecutive rows) and stacked column c hold one
// 128-byte record, hi[0..31] then lo[0..31], so a lane's eight K values of one column are one
// 16-byte load and the records of 16 neighbouring columns are 2 KB of contiguous memory.
#include <algorithm>

#include "common.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int PT = 128;      // output tile per workgroup (four waves of 64 x 64)
constexpr int SLAB = 32;     // rows per packed record (one MFMA K step)
constexpr int REC = 128;     // bytes per packed record (32 hi + 32 lo bf16)
constexpr int KS_SLABS = 128;  // slabs (4096 rows) per FP32 partial

__device__ __forceinline__ double seg_load(const BfSeg &sg, int64_t r, int64_t c) {
  const char *p = sg.ptr + (r * sg.ld + c) * sg.esz;
  return sg.esz == 4 ? (double)*reinterpret_cast<const float *>(p)
                     : *reinterpret_cast<const double *>(p);
}

__device__ __forceinline__ int seg_of(const BfSegs &sg, int64_t c) {
  for (int i = 0; i < sg.count; ++i)
    if (c >= sg.s[i].col0 && c < sg.s[i].col0 + sg.s[i].cols) return i;
  return -1;
}

__global__ __launch_bounds__(256) void fill_u64_kernel(int64_t len, unsigned long long *p) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < len) p[i] = 0ull;
}

// Column maxima of |x| over the chunk (rows [0, nr)): thread = column, workgroup row = a block
// of 256 rows; the bit patterns of non-negative doubles order like the values, so an integer
// atomic maximum gives the exact maximum in any order.
__global__ __launch_bounds__(256) void colmax_kernel(const BfSegs sg, int64_t nr, int64_t ctot,
                                                     unsigned long long *cmax) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= ctot) return;
  const int si = seg_of(sg, c);
  if (si < 0) return;
  const BfSeg &s = sg.s[si];
  const int64_t cc = c - s.col0;
  const int64_t r0 = (int64_t)blockIdx.y * 256, r1 = r0 + 256 < nr ? r0 + 256 : nr;
  double m = 0.0;
  for (int64_t r = r0; r < r1; ++r) m = fmax(m, fabs(seg_load(s, r, cc)));
  if (m > 0.0) atomicMax(&cmax[c], (unsigned long long)__double_as_longlong(m));
}

// Packs slab t of every column c < cpad: scaled by 2^-e_c (e_c from the column maximum; 0 for
// zero or padding columns), split into hi and lo, rows past nr and columns past the segments
// zero. Writes e_c for the reduction.
__global__ __launch_bounds__(256) void pack_kernel(const BfSegs sg, int64_t nr, int64_t cpad,
                                                   const unsigned long long *cmax, int *cexp,
                                                   char *out) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t t = blockIdx.y;
  if (c >= cpad) return;
  const int si = seg_of(sg, c);
  int e = 0;
  double scale = 1.0;
  if (si >= 0) {
    const double mx = __longlong_as_double((long long)cmax[c]);
    if (mx > 0.0 && isfinite(mx)) {
      frexp(mx, &e);
      scale = ldexp(1.0, -e);
    }
  }
  if (t == 0) cexp[c] = e;
  bf16x8 hi[4], lo[4];
#pragma unroll
  for (int k = 0; k < SLAB; ++k) {
    const int64_t r = t * SLAB + k;
    double x = 0.0;
    if (si >= 0 && r < nr) x = seg_load(sg.s[si], r, c - sg.s[si].col0) * scale;
    const __bf16 h = (__bf16)(float)x;
    hi[k >> 3][k & 7] = h;
    lo[k >> 3][k & 7] = (__bf16)(float)(x - (double)(float)h);
  }
  bf16x8 *dst = reinterpret_cast<bf16x8 *>(out + ((size_t)t * cpad + c) * REC);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    dst[u] = hi[u];
    dst[4 + u] = lo[u];
  }
}

struct Frag {
  bf16x8 ah[4], al[4], bh[4], bl[4];
};

// Lane l supplies row (column of the tall operand) l % 16 of a 16-row MFMA operand block and
// K values 8 (l / 16) .. +7 of the slab (the same K subset for both operands).
__device__ __forceinline__ void load_frag(const char *slab, int64_t ca, int64_t cb, int g,
                                          Frag &f) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const char *pa = slab + (ca + 16 * u) * REC + 16 * g;
    const char *pb = slab + (cb + 16 * u) * REC + 16 * g;
    f.ah[u] = *reinterpret_cast<const bf16x8 *>(pa);
    f.al[u] = *reinterpret_cast<const bf16x8 *>(pa + 64);
    f.bh[u] = *reinterpret_cast<const bf16x8 *>(pb);
    f.bl[u] = *reinterpret_cast<const bf16x8 *>(pb + 64);
  }
}

// The three partial products of a slab, each pass over all 16 accumulators before the next,
// so that dependent matrix-core operations are 16 apart.
__device__ __forceinline__ void mma_frag(const Frag &f, f32x4 (&acc)[4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.al[i], f.bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ah[i], f.bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ah[i], f.bh[j], acc[i][j], 0, 0, 0);
}

// Worker w (of nw = ntiles * nk) computes tile number w % ntiles of the grouped visiting order
// (GramSeq) over slabs [kz KS, (kz+1) KS) of the chunk, kz = w / ntiles, and stores its FP32
// 128 x 128 partial to part[kz][tile]. Workers map to XCDs in contiguous ranges (workgroup b
// runs worker (b % 8) G/8 + b / 8 of a grid of G, a multiple of 8), so the workgroups resident
// on one XCD hold neighbouring tiles of one K range and share their row and column panels in
// its L2. Each wave loads its operand fragments straight into registers, one slab ahead (the
// loads of slab t + 1 are in flight during slab t's matrix-core work; the prefetch past the end
// re-reads the last slab). Staging the slabs in LDS (one coalesced fill per workgroup, padded
// records) and a third register set were both slower. Columns a0 + I*128 .. +127 and b0 + J*128 .. +127 must
// lie inside the packed width.
__global__ __launch_bounds__(256, 2) void gram_bf16_kernel(const char *__restrict__ pk,
                                                           int64_t cpad, int64_t a0, int64_t b0,
                                                           const GramSeq sq, int ntiles, int nw,
                                                           int nsl, int ks,
                                                           float *__restrict__ part) {
  const int G = (int)gridDim.x;
  const int w = (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3);
  if (w >= nw) return;
  const int tile = w % ntiles, kz = w / ntiles;
  int I, J;
  sq.tile(tile, I, J);
  const int wv = threadIdx.x >> 6, wm = wv >> 1, wn = wv & 1;
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int64_t ca = a0 + (int64_t)I * PT + wm * 64 + li;
  const int64_t cb = b0 + (int64_t)J * PT + wn * 64 + li;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int t0 = kz * ks, t1 = (t0 + ks < nsl) ? t0 + ks : nsl;
  const size_t sstride = (size_t)cpad * REC;
  auto slab = [&](int t) { return pk + (size_t)(t < t1 ? t : t1 - 1) * sstride; };
  Frag f0, f1;
  load_frag(slab(t0), ca, cb, g, f0);
  int t = t0;
  // matrix-core work at a raised wave priority: the co-resident waves' load issue takes the
  // slots it leaves
  for (; t + 1 < t1; t += 2) {
    load_frag(slab(t + 1), ca, cb, g, f1);
    __builtin_amdgcn_s_setprio(1);
    mma_frag(f0, acc);
    __builtin_amdgcn_s_setprio(0);
    load_frag(slab(t + 2), ca, cb, g, f0);
    __builtin_amdgcn_s_setprio(1);
    mma_frag(f1, acc);
    __builtin_amdgcn_s_setprio(0);
  }
  if (t < t1) mma_frag(f0, acc);
  float *pt = part + ((size_t)kz * ntiles + tile) * (PT * PT);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        pt[(wm * 64 + i * 16 + 4 * g + v) * PT + wn * 64 + j * 16 + li] = acc[i][j][v];
}

// C(i, j) = beta C(i, j) + 2^(e_a(i) + e_b(j)) sum over kz of the partials, in FP64 and in kz
// order (deterministic); 64 workgroups per tile, one element per thread.
__global__ __launch_bounds__(256) void gram_bf16_reduce_kernel(int64_t M, int64_t N,
                                                               const GramSeq sq, int ntiles, int nk,
                                                               const float *__restrict__ part,
                                                               const int *__restrict__ cexp,
                                                               int64_t a0, int64_t b0, double beta,
                                                               double *__restrict__ C,
                                                               int64_t ldc) {
  const int tile = (int)(blockIdx.x / 64), sub = (int)(blockIdx.x % 64);
  int I, J;
  sq.tile(tile, I, J);
  const int e = sub * 256 + threadIdx.x;
  const int64_t gi = (int64_t)I * PT + e / PT, gj = (int64_t)J * PT + e % PT;
  if (gi >= M || gj >= N) return;
  double v = 0.0;
  for (int kz = 0; kz < nk; ++kz) v += (double)part[((size_t)kz * ntiles + tile) * (PT * PT) + e];
  v = ldexp(v, cexp[a0 + gi] + cexp[b0 + gj]);
  double *cp = C + gi * ldc + gj;
  *cp = (beta == 0.0) ? v : *cp + v;
}

}  // namespace

size_t bf16_pack_bytes(int64_t rows, int64_t cpad) {
  return (size_t)((rows + SLAB - 1) / SLAB) * (size_t)cpad * REC;
}

int64_t bf16_pack_width(int64_t ctot) { return (ctot + 2 * PT - 1) / PT * PT + PT; }

size_t bf16_part_floats(int64_t cpad, int64_t rows) {
  const int64_t T = cpad / PT;
  const int64_t nk = ((rows + SLAB - 1) / SLAB + KS_SLABS - 1) / KS_SLABS;
  return (size_t)(T * (T + 1) / 2) * (size_t)std::max<int64_t>(nk, 1) * PT * PT;
}

int launch_bf16_pack(const BfSegs &sg, int64_t nr, int64_t ctot, int64_t cpad,
                     unsigned long long *cmax, int *cexp, void *packed, hipStream_t st) {
  if (nr <= 0) return 0;
  if (ctot + PT > cpad || sg.count > BF_MAX_SEGS) return SYLV_ERR_INVALID;
  fill_u64_kernel<<<(unsigned)((cpad + 255) / 256), 256, 0, st>>>(cpad, cmax);
  HIPOK(hipGetLastError());
  colmax_kernel<<<dim3((unsigned)((ctot + 255) / 256), (unsigned)((nr + 255) / 256)), 256, 0,
                  st>>>(sg, nr, ctot, cmax);
  HIPOK(hipGetLastError());
  const int64_t nsl = (nr + SLAB - 1) / SLAB;
  pack_kernel<<<dim3((unsigned)((cpad + 255) / 256), (unsigned)nsl), 256, 0, st>>>(
      sg, nr, cpad, cmax, cexp, static_cast<char *>(packed));
  HIPOK(hipGetLastError());
  return 0;
}

int launch_gram_bf16(int64_t M, int64_t N, int64_t nr, const void *packed, int64_t cpad,
                     const int *cexp, int64_t a0, int64_t b0, double beta, double *C, int64_t ldc,
                     bool lower, hipStream_t st, float *part, size_t part_floats) {
  if (M <= 0 || N <= 0 || nr <= 0) return 0;
  if (lower && (M != N || a0 != b0)) return SYLV_ERR_INVALID;
  const int64_t TM = (M + PT - 1) / PT, TN = (N + PT - 1) / PT;
  if (a0 + TM * PT > cpad || b0 + TN * PT > cpad) return SYLV_ERR_INVALID;
  const int64_t tiles = lower ? TM * (TM + 1) / 2 : TM * TN;
  const int64_t nsl = (nr + SLAB - 1) / SLAB;
  int64_t ks = KS_SLABS;
  int64_t nk = (nsl + ks - 1) / ks;
  while ((size_t)(tiles * nk) * PT * PT > part_floats && ks < nsl) {
    ks *= 2;
    nk = (nsl + ks - 1) / ks;
  }
  if ((size_t)(tiles * nk) * PT * PT > part_floats) return SYLV_ERR_WORKSPACE;
  const GramSeq sq{(int)TM, (int)TN, lower ? 1 : 0};
  const int64_t nw = tiles * nk, G = (nw + 7) / 8 * 8;
  gram_bf16_kernel<<<(unsigned)G, 256, 0, st>>>(static_cast<const char *>(packed), cpad, a0, b0,
                                                 sq, (int)tiles, (int)nw, (int)nsl, (int)ks,
                                                 part);
  HIPOK(hipGetLastError());
  gram_bf16_reduce_kernel<<<(unsigned)(tiles * 64), 256, 0, st>>>(
      M, N, sq, (int)tiles, (int)nk, part, cexp, a0, b0, beta, C, ldc);
  HIPOK(hipGetLastError());
  return 0;
}
