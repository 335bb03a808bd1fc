// Dispatch of the paired block Arnoldi / Lanczos steps to the per-block-size units, and the
// partial-buffer size they need.
#include <map>
#include <mutex>
#include <tuple>

#include "arnoldi_impl.h"

#define ARN_DECL(SS)                                                                          \
  int arnoldi_step_##SS(const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,          \
                        double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st); \
  int lanczos_step_##SS(const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,          \
                        double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st); \
  int arnoldi_lagged_##SS(const SideDesc &sv, const SideDesc *sw, int jb, int64_t ldh,        \
                          double closure_tol, const Scratch &sc, DevState *ds, hipStream_t st); \
  int lanczos_flush_##SS(const SideDesc &sv, const SideDesc *sw, int nblocks, hipStream_t st);
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
