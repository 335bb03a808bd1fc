// Batches of independent problems on one GPU. Every instance gets its own context, carved from
// one workspace. Two execution forms:
//  * streams: instances are assigned to a few HIP streams; one host thread per stream drives its
//    instances' solves one after another, so the small launches of different instances overlap
//    on the device (results are bit-identical to solving each instance alone);
//  * grouped: instances with the same method, block size, form and iteration limit form a
//    group whose iterations advance in lock-step, every phase of an iteration one launch over
//    the group's instance table (per-instance stop flags let finished instances drop out), one
//    stream and host thread per group; optionally each segment of iterations is captured once
//    as a HIP graph and replayed by later solves. Instances that cannot join a group (mixed
//    precision, refinement, other methods) run in the streams form beside the groups.
#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "common.h"

namespace {

constexpr size_t BALIGN = 256;

struct Batch {
  int count = 0, device = 0, form = SYLV_BATCH_STREAMS;
  std::vector<hipStream_t> streams;
  std::vector<void *> ctx;
  std::vector<int> method, max_iter;
  std::vector<std::vector<int>> plan;     // streams form: instance indices per stream
  std::vector<int> plan_stream;           // stream of each plan
  std::vector<std::vector<int>> members;  // grouped form: instance indices per group
  std::vector<GroupRun> groups;
};

size_t align_up(size_t b) { return (b + BALIGN - 1) / BALIGN * BALIGN; }

// Relative cost of one instance: the Krylov bases' traffic and the core work both grow with the
// rank, so (n + m) s iterations plus the core size is a fair ordering key.
double cost_estimate(const sylv_problem &p, const sylv_options &o) {
  const bool one = o.method == SYLV_METHOD_CG || o.method == SYLV_METHOD_CR;
  const double r = (double)o.max_iter * p.s * (one ? 1.0 : 2.0);
  return (double)(p.n + p.m) * r + r * r * (one ? 1.0 : r / 64.0);
}

// Instances that can advance in lock-step with others (the conditions of group_eligible, read
// from the options), and the key that groups them.
bool groupable(const sylv_problem &p, const sylv_options &o) {
  if (o.precision != SYLV_FP64 || o.refine_max > 0) return false;
  if (o.method == SYLV_METHOD_CG) return true;
  return o.method == SYLV_METHOD_BICGSTAB && o.reorth != 1 && p.s <= 4;
}
typedef std::tuple<int, int64_t, int, int, double> GroupKey;
GroupKey group_key(const sylv_problem &p, const sylv_options &o) {
  return GroupKey{o.method, p.s, p.lyapunov ? 1 : 0, o.max_iter, o.closure_tol};
}

// Upper bound of the device bytes of the group tables of a batch (every instance may form a
// group of its own).
size_t group_tables_bound(int count, const sylv_problem *probs) {
  size_t b = 0;
  for (int i = 0; i < count; ++i) {
    b += krylov_side_bytes_bound(probs[i].n);
    if (!probs[i].lyapunov) b += krylov_side_bytes_bound(probs[i].m);
    b += sizeof(CoreInst) + krylov_group_bytes_fixed() + 3 * BALIGN;
  }
  return b;
}

void destroy_batch(Batch *b) {
  for (GroupRun &g : b->groups) group_release(g);
  for (void *c : b->ctx)
    if (c) sylv_destroy(c);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  delete b;
}

int solve_one(Batch *b, int i, double tol, sylv_result *res) {
  int (*solve)(void *, double, int, sylv_result *) = sylv_factored_bicgstab;
  switch (b->method[i]) {
    case SYLV_METHOD_CG: solve = sylv_factored_cg; break;
    case SYLV_METHOD_CR: solve = sylv_factored_cr; break;
    case SYLV_METHOD_CGS: solve = sylv_factored_cgs; break;
    case SYLV_METHOD_GPBICG: solve = sylv_factored_gpbicg; break;
    default: break;
  }
  return solve(b->ctx[i], tol, b->max_iter[i], res);
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
  return tot + align_up(group_tables_bound(count, probs));
}

int sylv_batch_create_ex(void **out, int count, const sylv_problem *probs,
                         const sylv_options *opts, void *workspace, size_t ws_bytes, int nstreams,
                         int form) {
  if (!out) return SYLV_ERR_INVALID;
  *out = nullptr;
  if (count < 1 || !probs || !opts || nstreams < 1 || nstreams > 64) return SYLV_ERR_INVALID;
  if (form != SYLV_BATCH_STREAMS && form != SYLV_BATCH_GROUPED && form != SYLV_BATCH_GRAPH)
    return SYLV_ERR_INVALID;
  const size_t need = sylv_batch_workspace_bytes(count, probs, opts);
  if (need == 0) return SYLV_ERR_INVALID;
  if (!workspace || ws_bytes < need) return SYLV_ERR_WORKSPACE;
  Batch *b = new (std::nothrow) Batch();
  if (!b) return SYLV_ERR_INVALID;
  b->count = count;
  b->form = form;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return SYLV_ERR_HIP;
  }
  // groups (grouped forms), in order of first appearance
  std::vector<int> loose;
  if (form != SYLV_BATCH_STREAMS) {
    std::map<GroupKey, int> gid;
    for (int i = 0; i < count; ++i) {
      if (!groupable(probs[i], opts[i])) {
        loose.push_back(i);
        continue;
      }
      auto it = gid.emplace(group_key(probs[i], opts[i]), (int)b->members.size()).first;
      if (it->second == (int)b->members.size()) b->members.emplace_back();
      b->members[it->second].push_back(i);
    }
  } else {
    for (int i = 0; i < count; ++i) loose.push_back(i);
  }
  const int ngroups = (int)b->members.size();
  const int nloose_streams = loose.empty() ? 0 : std::min<int>(nstreams, (int)loose.size());
  for (int k = 0; k < ngroups + nloose_streams; ++k) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      destroy_batch(b);
      return SYLV_ERR_HIP;
    }
    b->streams.push_back(s);
  }
  // instances outside groups: longest-processing-time assignment to the remaining streams
  std::sort(loose.begin(), loose.end(), [&](int x, int y) {
    return cost_estimate(probs[x], opts[x]) > cost_estimate(probs[y], opts[y]);
  });
  std::vector<double> load(nloose_streams, 0.0);
  b->plan.assign(nloose_streams, {});
  for (int k = 0; k < nloose_streams; ++k) b->plan_stream.push_back(ngroups + k);
  for (int i : loose) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[k] += cost_estimate(probs[i], opts[i]);
    b->plan[k].push_back(i);
  }
  // contexts: consecutive slices of the workspace, created on their stream (one thread each)
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
  std::vector<std::vector<int>> by_stream(b->streams.size());
  for (int g = 0; g < ngroups; ++g) by_stream[g] = b->members[g];
  for (int k = 0; k < nloose_streams; ++k) by_stream[ngroups + k] = b->plan[k];
  std::vector<int> err(by_stream.size(), 0);
  std::vector<std::thread> th;
  for (size_t k = 0; k < by_stream.size(); ++k) {
    auto make = [&, k] {
      if (hipSetDevice(b->device) != hipSuccess) {
        err[k] = SYLV_ERR_HIP;
        return;
      }
      for (int i : by_stream[k]) {
        const int e = create_context(&b->ctx[i], &probs[i], &opts[i], base[i], bytes[i],
                                     b->streams[k], false);
        if (e) {
          err[k] = e;
          return;
        }
      }
    };
    if (by_stream.size() == 1) make();  // one stream: on the calling thread
    else th.emplace_back(make);
  }
  for (auto &t : th) t.join();
  for (int e : err)
    if (e) {
      destroy_batch(b);
      return e;
    }
  // group tables after the contexts' slices
  const char *end = static_cast<const char *>(workspace) + ws_bytes;
  b->groups.resize(ngroups);
  for (int g = 0; g < ngroups; ++g) {
    std::vector<void *> cs;
    for (int i : b->members[g]) cs.push_back(b->ctx[i]);
    const size_t gb = align_up(group_bytes(cs.data(), (int)cs.size()));
    int e = gb == 0 ? SYLV_ERR_INVALID : 0;
    if (!e && p + gb > end) e = SYLV_ERR_WORKSPACE;
    if (!e) e = group_prepare(b->groups[g], cs.data(), (int)cs.size(), p, gb,
                              form == SYLV_BATCH_GRAPH, b->max_iter[b->members[g][0]]);
    if (e) {
      destroy_batch(b);
      return e;
    }
    p += gb;
  }
  *out = b;
  return 0;
}

int sylv_batch_create(void **out, int count, const sylv_problem *probs, const sylv_options *opts,
                      void *workspace, size_t ws_bytes, int nstreams) {
  return sylv_batch_create_ex(out, count, probs, opts, workspace, ws_bytes, nstreams,
                              SYLV_BATCH_STREAMS);
}

int sylv_batch_solve(void *batch, double tol, sylv_result *res) {
  Batch *b = reinterpret_cast<Batch *>(batch);
  if (!b || !res) return SYLV_ERR_INVALID;
  const int ng = (int)b->groups.size(), nl = (int)b->plan.size();
  std::vector<int> err(ng + nl, 0);
  std::vector<std::string> msg(ng + nl);  // the workers' error text (thread-local otherwise)
  std::vector<std::thread> th;
  // one worker (one group, or one stream of instances): it runs on the calling thread
  const bool inline_one = ng + nl == 1;
  auto spawn = [&](auto &&fn) {
    if (inline_one) fn();
    else th.emplace_back(fn);
  };
  for (int g = 0; g < ng; ++g)
    spawn([&, g] {
      if (hipSetDevice(b->device) != hipSuccess) {
        err[g] = SYLV_ERR_HIP;
        return;
      }
      const std::vector<int> &mem = b->members[g];
      std::vector<sylv_result> r(mem.size());
      const int e = group_solve(b->groups[g], tol, b->max_iter[mem[0]], r.data());
      if (e < 0) {
        err[g] = e;
        msg[g] = sylv_last_error();
        return;
      }
      for (size_t j = 0; j < mem.size(); ++j) res[mem[j]] = r[j];
    });
  for (int k = 0; k < nl; ++k)
    spawn([&, k] {
      if (hipSetDevice(b->device) != hipSuccess) {
        err[ng + k] = SYLV_ERR_HIP;
        return;
      }
      for (int i : b->plan[k]) {
        const int e = solve_one(b, i, tol, &res[i]);
        if (e < 0) {
          err[ng + k] = e;
          msg[ng + k] = sylv_last_error();
          return;
        }
      }
    });
  for (auto &t : th) t.join();
  for (size_t k = 0; k < err.size(); ++k)
    if (err[k]) {
      note_error(msg[k].c_str());
      return err[k];
    }
  int worst = 0;
  for (int i = 0; i < b->count; ++i) worst = std::max(worst, res[i].status);
  return worst;
}

void *sylv_batch_context(void *batch, int i) {
  Batch *b = reinterpret_cast<Batch *>(batch);
  if (!b || i < 0 || i >= b->count) return nullptr;
  return b->ctx[i];
}

int sylv_batch_groups(void *batch) {
  Batch *b = reinterpret_cast<Batch *>(batch);
  return b ? (int)b->groups.size() : SYLV_ERR_INVALID;
}

void sylv_batch_destroy(void *batch) {
  Batch *b = reinterpret_cast<Batch *>(batch);
  if (b) destroy_batch(b);
}

}  // extern "C"
