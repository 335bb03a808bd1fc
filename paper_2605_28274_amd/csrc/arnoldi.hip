// Dispatch of the paired block Arnoldi / Lanczos steps to the per-block-size units, and the
// partial-buffer size they need.
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "arnoldi_impl.h"

#define ARN_DECL(SS)                                                                          \
  int arnoldi_step_##SS(const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,          \
                        double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st); \
  int lanczos_step_##SS(const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,          \
                        double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st); \
  int arnoldi_lagged_##SS(const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,        \
                          double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st); \
  int lanczos_flush_##SS(const SideDesc &sv, const SideDesc *sw, int nblocks, hipStream_t st); \
  int krylov_group_step_##SS(const KGroup &g, int jb, double closure_tol, hipStream_t st);     \
  int krylov_group_flush_##SS(const KGroup &g, int nblocks, hipStream_t st);
ARN_DECL(1) ARN_DECL(2) ARN_DECL(3) ARN_DECL(4) ARN_DECL(5) ARN_DECL(6) ARN_DECL(7) ARN_DECL(8)
#undef ARN_DECL

size_t arnoldi_partials_needed(int s, int64_t rows_v, int64_t rows_w, int64_t max_cols) {
  const int64_t total = rows_v + rows_w;
  const int64_t n0 = cdiv(rows_v, gram_rpc(s, rows_v, total));
  const int64_t n1 = rows_w ? cdiv(rows_w, gram_rpc(s, rows_w, total)) : 0;
  // 2 s Gram columns per basis column (the lagged step's [V~_j, M V~_j])
  const size_t per0 = (size_t)n0 * max_cols * 2 * s + aux_len(s, rows_v);
  const size_t per1 = rows_w ? (size_t)n1 * max_cols * 2 * s + aux_len(s, rows_w) : 0;
  return 2 * std::max(per0, per1);
}

bool arnoldi_lagged_supported(int s, bool fp32) { return !fp32 && s >= 1 && s <= 4; }

namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int64_t, int64_t, int64_t>, int64_t> g_tune;
std::tuple<int, int, int64_t, int64_t, int64_t> tkey(const TuneKey &k) {
  return {k.s, k.esz, k.rows0, k.rows1, k.per_row};
}
}  // namespace

int64_t tune_lookup(const TuneKey &k) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(tkey(k));
  return it == g_tune.end() ? 0 : it->second;
}

int64_t tune_store(const TuneKey &k, int64_t value) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  return g_tune.emplace(tkey(k), value).first->second;
}

int launch_arnoldi_pair(int s, const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,
                        double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st,
                        bool lagged) {
  switch (s) {
#define CASE(SS)                                                                  \
  case SS:                                                                        \
    return lagged ? arnoldi_lagged_##SS(sv, sw, jb, ldh, closure_tol, sc, ds, st) \
                  : arnoldi_step_##SS(sv, sw, jb, ldh, closure_tol, sc, ds, st);
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return SYLV_ERR_INVALID;
  }
}

int launch_lanczos_pair(int s, const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,
                        double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st) {
  switch (s) {
#define CASE(SS) \
  case SS: return lanczos_step_##SS(sv, sw, jb, ldh, closure_tol, sc, ds, st);
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return SYLV_ERR_INVALID;
  }
}

int launch_lanczos_flush(int s, const SideDesc &sv, const SideDesc *sw, int nblocks,
                         hipStream_t st) {
  switch (s) {
#define CASE(SS) \
  case SS: return lanczos_flush_##SS(sv, sw, nblocks, st);
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return SYLV_ERR_INVALID;
  }
}

// ---- batch group tables ----
namespace {

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Per-basis records of every launch kind, their owners and the compact block slots (host).
struct GroupTables {
  std::vector<ArSide> tab[GK_COUNT];
  std::vector<unsigned short> own[GK_COUNT];
  std::vector<PanelSet> panels;
  int max_nout = 0;
};

int build_tables(int s, bool lanczos, const GroupSide *sides, int n, GroupTables &t) {
  if (n < 1 || n > 65535 || s < 1 || s > SYLV_MAX_S) return SYLV_ERR_INVALID;
  if (!lanczos && s > 4) return SYLV_ERR_INVALID;
  t.max_nout = 1 << 30;
  for (int i = 0; i < n; ++i) {
    const GroupSide &g = sides[i];
    const int64_t rows = g.d.rows;
    const size_t half = g.sc.partial_cap / 2, aux = aux_len(s, rows);
    if (rows < 1 || aux > half || g.d.fp32) return SYLV_ERR_WORKSPACE;
    ArSide a = make_side(g.d, g.sc, g.idx, half, aux, g.ldh);
    a.done = g.done;
    a.nb_spmm = (int)nb_rows(rows);
    a.nb_upd = lanczos ? (int)nb_rows(rows) : (int)cdiv(rows, UROWS);
    a.nb_qr = (int)nb_qr(rows);
    const int64_t rpc = gram_rpc(s, rows, g.pair_rows);
    a.nch = (int)cdiv(rows, rpc);
    if (!lanczos)
      t.max_nout = std::min<int64_t>(t.max_nout, (int64_t)((half - aux) / (size_t)a.nch));
    const int64_t nb[GK_COUNT] = {nb_rows(rows), nb_qr(rows), lanczos ? 0 : a.nch,
                                  lanczos ? 0 : cdiv(rows, UROWS)};
    const int64_t rp[GK_COUNT] = {0, 0, rpc, UROWS};
    for (int k = 0; k < GK_COUNT; ++k) {
      ArSide e = a;
      e.b0 = (int)t.own[k].size();
      e.nb = (int)nb[k];
      e.rpc = rp[k];
      t.tab[k].push_back(e);
      t.own[k].insert(t.own[k].end(), (size_t)nb[k], (unsigned short)i);
    }
    PanelSet ps{};
    for (int k = 0; k < LZ_RING; ++k) ps.p[k] = g.d.panel[k];
    t.panels.push_back(ps);
  }
  if (lanczos) t.max_nout = 0;
  return 0;
}

// The full tables, then a second copy of the same size for the running bases (compaction),
// then n ints of index scratch.
size_t tables_bytes(const GroupTables &t, int n) {
  size_t b = 0;
  for (int k = 0; k < GK_COUNT; ++k)
    b += align256(sizeof(ArSide) * n) + align256(sizeof(unsigned short) * (t.own[k].size() + 1));
  b += align256(sizeof(PanelSet) * n);
  return 2 * b + align256(sizeof(int) * n);
}

// Arguments of the compaction kernel.
struct CompactArgs {
  const ArSide *tab[GK_COUNT];
  ArSide *atab[GK_COUNT];
  unsigned short *aown[GK_COUNT];
  const PanelSet *panels;
  PanelSet *apanels;
  int *idx;     // n ints
  int *counts;  // [bases still running, workgroups of each kind]
  int n;
};

// One workgroup: the records of the bases whose problem still runs, in basis order, into the
// active tables with their workgroup ranges packed, their owners and compact block slots;
// counts[0] = those bases, counts[1 + k] = workgroups of kind k.
__global__ __launch_bounds__(1024) void krylov_compact_kernel(CompactArgs a) {
  __shared__ int na;
  if (threadIdx.x == 0) {
    int c = 0;
    for (int i = 0; i < a.n; ++i)
      if (*a.tab[0][i].done == 0) a.idx[c++] = i;
    na = c;
    a.counts[0] = c;
  }
  __syncthreads();
  if (threadIdx.x < GK_COUNT) {
    const int k = threadIdx.x;
    int b0 = 0;
    for (int j = 0; j < na; ++j) {
      ArSide e = a.tab[k][a.idx[j]];
      e.b0 = b0;
      b0 += e.nb;
      a.atab[k][j] = e;
    }
    a.counts[1 + k] = b0;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < na; j += blockDim.x) {
    a.apanels[j] = a.panels[a.idx[j]];
    for (int k = 0; k < GK_COUNT; ++k) {
      const ArSide &e = a.atab[k][j];
      for (int t = 0; t < e.nb; ++t) a.aown[k][e.b0 + t] = (unsigned short)j;
    }
  }
}

}  // namespace

size_t krylov_group_bytes(int s, bool lanczos, const GroupSide *sides, int n) {
  GroupTables t;
  if (build_tables(s, lanczos, sides, n, t)) return 0;
  return tables_bytes(t, n);
}

int krylov_group_create(KGroup *g, KGroup *act, int s, bool lanczos, const GroupSide *sides, int n,
                        void *dev, size_t bytes, hipStream_t st) {
  if (!g || !act) return SYLV_ERR_INVALID;
  GroupTables t;
  if (int e = build_tables(s, lanczos, sides, n, t)) return e;
  if (!dev || (reinterpret_cast<uintptr_t>(dev) & 255) || bytes < tables_bytes(t, n))
    return SYLV_ERR_WORKSPACE;
  char *p = static_cast<char *>(dev);
  *g = KGroup{};
  g->s = s;
  g->lanczos = lanczos ? 1 : 0;
  g->nsides = n;
  g->max_nout = t.max_nout;
  for (int k = 0; k < GK_COUNT; ++k) {
    HIPOK(hipMemcpyAsync(p, t.tab[k].data(), sizeof(ArSide) * n, hipMemcpyHostToDevice, st));
    g->tab[k] = p;
    p += align256(sizeof(ArSide) * n);
    if (!t.own[k].empty())
      HIPOK(hipMemcpyAsync(p, t.own[k].data(), sizeof(unsigned short) * t.own[k].size(),
                           hipMemcpyHostToDevice, st));
    g->own[k] = reinterpret_cast<const unsigned short *>(p);
    g->nblk[k] = (int)t.own[k].size();
    p += align256(sizeof(unsigned short) * (t.own[k].size() + 1));
  }
  HIPOK(hipMemcpyAsync(p, t.panels.data(), sizeof(PanelSet) * n, hipMemcpyHostToDevice, st));
  g->panels = p;
  p += align256(sizeof(PanelSet) * n);
  // the active copy: same layout, filled by launch_krylov_group_compact
  *act = *g;
  for (int k = 0; k < GK_COUNT; ++k) {
    act->tab[k] = p;
    p += align256(sizeof(ArSide) * n);
    act->own[k] = reinterpret_cast<const unsigned short *>(p);
    p += align256(sizeof(unsigned short) * (t.own[k].size() + 1));
  }
  act->panels = p;
  p += align256(sizeof(PanelSet) * n);
  g->idx = act->idx = reinterpret_cast<int *>(p);
  HIPOK(hipStreamSynchronize(st));  // the host tables go out of scope
  return 0;
}

int launch_krylov_group_compact(const KGroup &g, const KGroup &act, int *counts, hipStream_t st) {
  CompactArgs a{};
  for (int k = 0; k < GK_COUNT; ++k) {
    a.tab[k] = static_cast<const ArSide *>(g.tab[k]);
    a.atab[k] = const_cast<ArSide *>(static_cast<const ArSide *>(act.tab[k]));
    a.aown[k] = const_cast<unsigned short *>(act.own[k]);
  }
  a.panels = static_cast<const PanelSet *>(g.panels);
  a.apanels = const_cast<PanelSet *>(static_cast<const PanelSet *>(act.panels));
  a.idx = g.idx;
  a.counts = counts;
  a.n = g.nsides;
  krylov_compact_kernel<<<1, 1024, 0, st>>>(a);
  HIPOK(hipGetLastError());
  return 0;
}

int launch_krylov_group(const KGroup &g, int jb, double closure_tol, hipStream_t st) {
  if (g.nsides < 1) return 0;  // no basis in the launches
  switch (g.s) {
#define CASE(SS) \
  case SS: return krylov_group_step_##SS(g, jb, closure_tol, st);
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return SYLV_ERR_INVALID;
  }
}

int launch_krylov_group_flush(const KGroup &g, int nblocks, hipStream_t st) {
  if (!g.lanczos || g.nsides < 1) return 0;
  switch (g.s) {
#define CASE(SS) \
  case SS: return krylov_group_flush_##SS(g, nblocks, st);
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return SYLV_ERR_INVALID;
  }
}

size_t krylov_side_bytes_bound(int64_t rows) {
  const int64_t own = 2 * cdiv(rows, TPB) + std::min<int64_t>(rows, 512) + cdiv(rows, UROWS);
  return 2 * (GK_COUNT * sizeof(ArSide) + sizeof(PanelSet) + sizeof(unsigned short) * (size_t)own) +
         sizeof(int);
}

size_t krylov_group_bytes_fixed() { return (size_t)(4 * GK_COUNT + 3) * 256 + 64; }
