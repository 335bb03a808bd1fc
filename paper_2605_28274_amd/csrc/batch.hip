// Batches of independent problems on one GPU: every instance gets its own context (carved from
// one workspace) and is assigned to one of a few HIP streams; one host thread per stream drives
// its instances' solves, so the small launches of different instances overlap on the device and
// the host-side enqueue work runs in parallel.
#include <algorithm>
#include <new>
#include <thread>
#include <vector>

#include "common.h"

namespace {

constexpr size_t BALIGN = 256;

struct Batch {
  int count = 0, device = 0;
  std::vector<hipStream_t> streams;
  std::vector<void *> ctx;
  std::vector<int> method, max_iter;
  std::vector<std::vector<int>> plan;  // instance indices per stream
};

size_t align_up(size_t b) { return (b + BALIGN - 1) / BALIGN * BALIGN; }

// Relative cost of one instance: the Krylov bases' traffic and the core work both grow with the
// rank, so (n + m) s iterations plus the core size is a fair ordering key.
double cost_estimate(const sylv_problem &p, const sylv_options &o) {
  const bool one = o.method == SYLV_METHOD_CG || o.method == SYLV_METHOD_CR;
  const double r = (double)o.max_iter * p.s * (one ? 1.0 : 2.0);
  return (double)(p.n + p.m) * r + r * r * (one ? 1.0 : r / 64.0);
}

void destroy_batch(Batch *b) {
  for (void *c : b->ctx)
    if (c) sylv_destroy(c);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  delete b;
}

}  // namespace

extern "C" {

size_t sylv_batch_workspace_bytes(int count, const sylv_problem *probs, const sylv_options *opts) {
  if (count < 1 || !probs || !opts) return 0;
  size_t tot = BALIGN;
  for (int i = 0; i < count; ++i) {
    const size_t b = sylv_workspace_bytes(&probs[i], &opts[i]);
    if (b == 0) return 0;
    tot += align_up(b);
  }
  return tot;
}

int sylv_batch_create(void **out, int count, const sylv_problem *probs, const sylv_options *opts,
                      void *workspace, size_t ws_bytes, int nstreams) {
  if (!out) return SYLV_ERR_INVALID;
  *out = nullptr;
  if (count < 1 || !probs || !opts || nstreams < 1 || nstreams > 64) return SYLV_ERR_INVALID;
  const size_t need = sylv_batch_workspace_bytes(count, probs, opts);
  if (need == 0) return SYLV_ERR_INVALID;
  if (!workspace || ws_bytes < need) return SYLV_ERR_WORKSPACE;
  Batch *b = new (std::nothrow) Batch();
  if (!b) return SYLV_ERR_INVALID;
  b->count = count;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return SYLV_ERR_HIP;
  }
  nstreams = std::min(nstreams, count);
  for (int k = 0; k < nstreams; ++k) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      destroy_batch(b);
      return SYLV_ERR_HIP;
    }
    b->streams.push_back(s);
  }
  // longest-processing-time assignment of instances to streams
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int x, int y) {
    return cost_estimate(probs[x], opts[x]) > cost_estimate(probs[y], opts[y]);
  });
  std::vector<double> load(nstreams, 0.0);
  b->plan.assign(nstreams, {});
  for (int i : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[k] += cost_estimate(probs[i], opts[i]);
    b->plan[k].push_back(i);
  }
  // contexts: consecutive slices of the workspace, created on their streams (one thread each)
  b->ctx.assign(count, nullptr);
  b->method.resize(count);
  b->max_iter.resize(count);
  std::vector<char *> base(count);
  char *p = reinterpret_cast<char *>(
      (reinterpret_cast<uintptr_t>(workspace) + BALIGN - 1) / BALIGN * BALIGN);
  std::vector<size_t> bytes(count);
  for (int i = 0; i < count; ++i) {
    bytes[i] = align_up(sylv_workspace_bytes(&probs[i], &opts[i]));
    base[i] = p;
    p += bytes[i];
    b->method[i] = opts[i].method;
    b->max_iter[i] = opts[i].max_iter;
  }
  std::vector<int> err(nstreams, 0);
  std::vector<std::thread> th;
  for (int k = 0; k < nstreams; ++k)
    th.emplace_back([&, k] {
      if (hipSetDevice(b->device) != hipSuccess) {
        err[k] = SYLV_ERR_HIP;
        return;
      }
      for (int i : b->plan[k]) {
        const int e = create_context(&b->ctx[i], &probs[i], &opts[i], base[i], bytes[i],
                                     b->streams[k], false);
        if (e) {
          err[k] = e;
          return;
        }
      }
    });
  for (auto &t : th) t.join();
  for (int k = 0; k < nstreams; ++k)
    if (err[k]) {
      destroy_batch(b);
      return err[k];
    }
  *out = b;
  return 0;
}

int sylv_batch_solve(void *batch, double tol, sylv_result *res) {
  Batch *b = reinterpret_cast<Batch *>(batch);
  if (!b || !res) return SYLV_ERR_INVALID;
  const int ns = (int)b->streams.size();
  std::vector<int> err(ns, 0);
  std::vector<std::thread> th;
  for (int k = 0; k < ns; ++k)
    th.emplace_back([&, k] {
      if (hipSetDevice(b->device) != hipSuccess) {
        err[k] = SYLV_ERR_HIP;
        return;
      }
      for (int i : b->plan[k]) {
        int (*solve)(void *, double, int, sylv_result *) = sylv_factored_bicgstab;
        switch (b->method[i]) {
          case SYLV_METHOD_CG: solve = sylv_factored_cg; break;
          case SYLV_METHOD_CR: solve = sylv_factored_cr; break;
          case SYLV_METHOD_CGS: solve = sylv_factored_cgs; break;
          case SYLV_METHOD_GPBICG: solve = sylv_factored_gpbicg; break;
          default: break;
        }
        const int e = solve(b->ctx[i], tol, b->max_iter[i], &res[i]);
        if (e < 0) {
          err[k] = e;
          return;
        }
      }
    });
  for (auto &t : th) t.join();
  int worst = 0;
  for (int k = 0; k < ns; ++k)
    if (err[k]) return err[k];
  for (int i = 0; i < b->count; ++i) worst = std::max(worst, res[i].status);
  return worst;
}

void *sylv_batch_context(void *batch, int i) {
  Batch *b = reinterpret_cast<Batch *>(batch);
  if (!b || i < 0 || i >= b->count) return nullptr;
  return b->ctx[i];
}

void sylv_batch_destroy(void *batch) {
  Batch *b = reinterpret_cast<Batch *>(batch);
  if (b) destroy_batch(b);
}

}  // extern "C"
