#!/usr/bin/env python3
"""Benchmark of the factored Krylov hot path on one MI355X.

Default workload (`--workload c5cg`): Lyapunov factored CG, FP64, A = 2D Laplacian on a
1024 x 1024 grid (n = m = 1,048,576), B = A^T, s = 1, C1 ~ N(0, 1) (seed 1005), tol 1e-8, the
largest single-GPU configuration. Other workloads (same JSON line):
  c1    factored CG, FP64, 1D Laplacians (n+1)^2 tridiag, n = 256, m = 192, s = 1, 200 iterations
  c2    factored BiCGSTAB, FP64, 2D CD 128^2 (Pe = 10) x 1D CD m = 8192 (Pe = 10), s = 2
  c3    factored BiCGSTAB, FP64, 3D CD 64^3 x 2D CD 256^2 (Pe = 10), s = 4
  c5bi  Lyapunov factored BiCGSTAB, FP64, 2D CD 1024^2 (Pe = 1), s = 1, 200-iteration window
  batch64  64 independent instances (2D A with n in [1024, 32768]; 1D or 2D B with m in [512,
        16384]; s in {1, 2, 4}; CG on Laplacians and BiCGSTAB on Pe = 10 alternately), solved as
        one batch in the grouped form (instances of one method and block size advance in
        lock-step, one launch per phase over the group's instance table), beside the streams
        form, the grouped form replaying captured HIP graphs, and the same instances one after
        another

One step = one pass of the whole path over resident inputs: sylv_create (CSR validation, B^T,
sliced-ELLPACK copies, QR of C1 and C2), the factored solve with the verified stopping rule (the
recursive test ||R|| <= tol ||R0||, then the true residual ||A X + X B - C1 C2^T||_F, which must
meet tol too), sylv_get_factors into device buffers and sylv_residual_norm (returns the verified
figure). `value` is factored iterations per second over whole steps; ms_per_step is the time to
a verified solution including setup.

Precision of the default line: FP64 everywhere ("FP64 plain"). `comparisons` times the mixed
and batched forms of the same and of the other workloads beside their FP64-plain runs (two steps
after one warm-up each): split-BF16 Gram products for the true residual (gram_precision 2), FP32
bases with outer refinement, and the 64-instance batch against the same instances solved one
after another.

After the timed region one more (untimed) solve runs with per-kernel HIP-event timing on the
solver's stream, for the roofline fraction of the dominant kernel family; the CPU oracle is
timed on a bounded sample of the same workload for `cpu_baseline`.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0     # MI355X HBM3E
PEAK_FP64_TFS = 78.6      # MI355X FP64 (vector and MFMA)
PEAK_BF16_TFS = 2500.0    # MI355X dense BF16 MFMA
METRIC = "time-to-1e-8 rel. residual + factored iters/s; mixed/batched vs FP64 plain"

# kernel families bound by the matrix cores (peak TFLOP/s); the others are bound by HBM
MFMA_FAMILIES = {"core_op": PEAK_FP64_TFS, "res_gram": PEAK_FP64_TFS,
                 "res_gram_bf16": PEAK_BF16_TFS}


def workload(name, max_iter=0):
    from workloads import configs
    if name == "c1":
        return configs.c1_cg_1d(), "cg"
    if name == "c2":
        return configs.c2_bicgstab(max_iter=max_iter or 800), "bicgstab"
    if name == "c3":
        return configs.c3_bicgstab(max_iter=max_iter or 400), "bicgstab"
    if name == "c5cg":
        return configs.c5_lyap("cg", max_iter=max_iter or 4000), "cg"
    if name == "c5bi":
        return configs.c5_lyap("bicgstab", max_iter=max_iter or 200), "bicgstab"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(p, method, iters, iters_1t):
    """The oracle as it stands on the host cores: its first `iters` factored iterations of the
    same workload with the BLAS threads the host gives it, and its first `iters_1t` iterations
    on one thread (cost per iteration grows with the rank, so an early sample understates the
    full-solve time per iteration)."""
    from oracle import factored
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threadpool_limits, cores = None, os.cpu_count() or 1
    fn = factored.factored_cg if method == "cg" else factored.factored_bicgstab

    def sample(k):
        t0 = time.perf_counter()
        _, _, _, info = fn(p.A, p.B, p.C1, p.C2, tol=0.0, max_iter=k, lyapunov=p.lyapunov)
        return info["iters"], time.perf_counter() - t0

    it, dt = sample(iters)
    one = None
    if threadpool_limits is not None and iters_1t > 0:
        with threadpool_limits(limits=1):
            it1, dt1 = sample(iters_1t)
        one = {"value": round(it1 / dt1, 3), "cores": 1,
               "sample": f"first {it1} iterations ({dt1:.1f} s, one BLAS thread)"}
    name = "CG" if method == "cg" else "BiCGSTAB"
    return {"value": it / dt, "unit": "iters/s", "cores": int(cores), "kind": "oracle",
            "sample": f"first {it} factored {name} iterations of the same workload "
                      f"({dt:.1f} s on the host; SciPy's sparse products use one thread)",
            "one_thread": one}


class DeviceProblem:
    """Device copies of one problem and its sylv_problem record."""

    def __init__(self, sylv, torch, p):
        dev = "cuda"
        self.p = p
        self.rpA, self.ciA, self.vaA = sylv.csr_tensors(p.A, dev)
        self.C1 = torch.as_tensor(p.C1, device=dev)
        if p.lyapunov:
            csrB, self.C2 = sylv.make_csr(p.m, self.rpA, self.ciA, self.vaA), self.C1
        else:
            self.B = sylv.csr_tensors(p.B, dev)
            csrB = sylv.make_csr(p.m, *self.B)
            self.C2 = torch.as_tensor(p.C2, device=dev)
        self.prob = sylv.sylv_problem(p.n, p.m, p.s, sylv.make_csr(p.n, self.rpA, self.ciA,
                                                                     self.vaA), csrB,
                                      1 if p.lyapunov else 0, self.C1.data_ptr(), p.s,
                                      self.C2.data_ptr(), p.s)


def run_config(sylv, torch, np, p, method, cfg, steps, warmup, measure=False):
    """Times `steps` whole steps (after `warmup`) of one configuration: cfg holds precision
    ('fp64' or 'fp32' bases), gram_precision, refine, check_every, streams, reorth."""
    cg = method == "cg"
    dp = DeviceProblem(sylv, torch, p)
    mixed = cfg.get("precision", "fp64") == "fp32"
    refine = cfg.get("refine", 3 if mixed else 0)
    opts = sylv.default_options(sylv.SYLV_METHOD_CG if cg else sylv.SYLV_METHOD_BICGSTAB,
                                p.max_iter, check_every=cfg.get("check_every", 16),
                                precision=sylv.SYLV_MIXED_FP32 if mixed else sylv.SYLV_FP64,
                                refine_max=refine, refine_max_iter=100,
                                streams=cfg.get("streams", 0), reorth=cfg.get("reorth", 0),
                                gram_precision=cfg.get("gram_precision", 0), verify=1)
    ws = torch.empty(sylv.sylv_workspace_bytes(dp.prob, opts), dtype=torch.uint8, device="cuda")
    rmax = (p.max_iter + 1 if cg else 2 * p.max_iter + 1) * p.s
    if refine > 0:  # the summed iterate stacks the corrections' bases
        rmax += refine * (101 if cg else 201) * 8
    V = torch.empty((p.n, rmax), dtype=torch.float64, device="cuda")
    W = V if p.lyapunov else torch.empty((p.m, rmax), dtype=torch.float64, device="cuda")
    Xc = torch.empty((rmax, rmax), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    solve = sylv.sylv_factored_cg if cg else sylv.sylv_factored_bicgstab

    def step():
        ctx = sylv.sylv_create(dp.prob, opts, ws, stream.cuda_stream)
        res = solve(ctx, p.tol, p.max_iter)
        rv, rw = res.rank_v, res.rank_w
        sylv.sylv_get_factors(ctx, V[:, :rv], Xc[:rv, :rw], None if p.lyapunov else W[:, :rw])
        _, rel = sylv.sylv_residual_norm(ctx)
        sylv.sylv_destroy(ctx)
        return res, rel

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    iters, rels, statuses, outer = 0, [], [], 0
    t0 = time.perf_counter()
    for _ in range(steps):
        res, rel = step()
        iters += res.iters
        rels.append(rel)
        statuses.append(res.status)
        outer = res.outer_steps
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"ms_per_step": 1000.0 * dt / steps, "iters_per_step": iters // steps,
           "iters_per_s": iters / dt, "true_rel_res": float(np.max(rels)),
           "statuses": sorted(set(int(s) for s in statuses)), "outer_steps": int(outer),
           "rank": int(res.rank_v)}
    if measure:
        # untimed measurement pass: per-family kernel times with HIP events on the solver's
        # stream (the solve and the true residual of its verification)
        ctx = sylv.sylv_create(dp.prob, opts, ws, stream.cuda_stream)
        sylv.sylv_set_profiling(ctx, True)
        t1 = time.perf_counter()
        solve(ctx, p.tol, p.max_iter)
        out["profiled_solve_ms"] = 1000.0 * (time.perf_counter() - t1)
        out["stats"] = sylv.sylv_get_kernel_stats(ctx)
        sylv.sylv_destroy(ctx)
    del V, W, Xc, ws, dp
    torch.cuda.empty_cache()
    return out


def roofline_of(stats, workload, precision):
    tot = sum(s["ms"] for s in stats) or 1.0
    dom = max(stats, key=lambda s: s["ms"])
    fam = dom["family"]
    if fam in MFMA_FAMILIES:
        bound, unit, peak = "mfma", "TFLOP/s", MFMA_FAMILIES[fam]
        achieved = dom["flops"] / (dom["ms"] * 1e-3) / 1e12
    else:
        bound, unit, peak = "hbm", "GB/s", PEAK_HBM_GBS
        achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
    return {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4),
            "traffic": measured_traffic(workload, fam, precision),
            "kernel": fam, "launches": dom["launches"],
            "avg_launch_us": round(1000 * dom["ms"] / max(dom["launches"], 1), 3),
            "share_of_kernel_time": round(dom["ms"] / tot, 3)}


def breakdown_of(stats):
    return {s["family"]: {"ms": round(s["ms"], 3), "launches": s["launches"],
                          "GB/s": round(s["bytes"] / max(s["ms"], 1e-9) / 1e6, 1),
                          "TFLOP/s": round(s["flops"] / max(s["ms"], 1e-9) / 1e9, 3)}
            for s in stats if s["launches"]}


def summary(r):
    return {"time_to_1e-8_ms": round(r["ms_per_step"], 3), "iters": r["iters_per_step"],
            "iters_per_s": round(r["iters_per_s"], 2), "true_rel_res": r["true_rel_res"],
            "statuses": r["statuses"], "outer_steps": r["outer_steps"], "rank": r["rank"]}


def comparisons(sylv, torch, np, main_name, main_res):
    """Mixed and batched forms beside FP64 plain (two steps after one warm-up each)."""
    out = {}
    plans = {
        "c5cg": [("fp64_plain", {}), ("mixed_bf16_grams", {"gram_precision": 2})],
        "c2": [("fp64_plain", {}), ("mixed_bf16_grams", {"gram_precision": 2})],
        "c3": [("fp64_plain", {}), ("mixed_bf16_grams", {"gram_precision": 2}),
               ("mixed_fp32_bases_refined", {"precision": "fp32", "gram_precision": 2})],
    }
    for name, plan in plans.items():
        p, method = workload(name)
        rows = {}
        for label, cfg in plan:
            if name == main_name and label == "fp64_plain":
                rows[label] = summary(main_res)
                continue
            rows[label] = summary(run_config(sylv, torch, np, p, method, cfg, 2, 1))
        base = rows["fp64_plain"]["time_to_1e-8_ms"]
        for label, r in rows.items():
            r["speedup_vs_fp64_plain"] = round(base / r["time_to_1e-8_ms"], 3)
        out[name] = {"workload": p.meta["workload"], **rows}
    out["batch64"] = run_batch_compare(sylv, torch, np, steps=2, warmup=1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5cg",
                    choices=["c1", "c2", "c3", "c5cg", "c5bi", "batch64"])
    ap.add_argument("--streams", type=int, default=8, help="streams of the batched run")
    ap.add_argument("--batch-group", default=None,
                    help="METHOD:S, e.g. cg:4: time only that group of the 64-instance batch in "
                         "the grouped form, without verification (one group runs on the calling "
                         "thread; for kernel traces)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the mixed / batched comparisons")
    ap.add_argument("--check-every", type=int, default=16,
                    help="iterations between the host's looks at the convergence flag")
    ap.add_argument("--streams-solve", type=int, default=0, choices=[0, 1, 2],
                    help="sylv_options.streams (0 automatic)")
    ap.add_argument("--reorth", type=int, default=0, choices=[0, 1, 2],
                    help="sylv_options.reorth (0 automatic)")
    ap.add_argument("--cpu-iters", type=int, default=600)
    ap.add_argument("--cpu-iters-1t", type=int, default=200)
    ap.add_argument("--max-iter", type=int, default=0)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                    help="storage of the Krylov bases (fp32: mixed precision)")
    ap.add_argument("--gram-precision", type=int, default=0, choices=[0, 1, 2],
                    help="sylv_options.gram_precision of the true-residual Grams")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="one step only (for hardware-counter runs of rocprofv3 --pmc)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="device copies of 512 MiB (counter calibration) and exit")
    ap.add_argument("--spmm-only", action="store_true",
                    help="only the standalone SpMM measurement (for counter runs) and exit")
    ap.add_argument("--refine", type=int, default=-1,
                    help="correction solves of the outer refinement (default: 3 with fp32 "
                         "bases, 0 with fp64)")
    args = ap.parse_args()
    if args.refine < 0:
        args.refine = 3 if args.precision == "fp32" else 0
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU (a multi-GPU form would split "
                                   "the basis rows over the GPUs and sum the Gram partials "
                                   "across them); --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2605_28274_amd import sylv

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": src.numel() * 8, "copies": 3}), flush=True)
        return
    if args.spmm_only:
        print(json.dumps({"spmm_hbm": spmm_hbm(sylv, torch)}), flush=True)
        return
    if args.batch_group:
        print(json.dumps(run_batch_group(sylv, torch, args.batch_group, args.steps, args.warmup)),
              flush=True)
        return
    if args.workload == "batch64":
        r = run_batch_compare(sylv, torch, np, args.steps, args.warmup, args.streams)
        out = {"metric": METRIC, "value": r["batched"]["iters_per_s"], "unit": "iters/s",
               "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": r["batched"]["time_to_1e-8_ms"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": r["workload"], **r}}
        print(json.dumps(out), flush=True)
        return
    p, method = workload(args.workload, args.max_iter)
    cfg = {"precision": args.precision, "gram_precision": args.gram_precision,
           "refine": args.refine, "check_every": args.check_every,
           "streams": args.streams_solve, "reorth": args.reorth}
    if args.pmc_pass:
        r = run_config(sylv, torch, np, p, method, cfg, args.steps, 0)
        print(json.dumps({"pmc_pass": args.workload, "iters": r["iters_per_step"]}), flush=True)
        return
    r = run_config(sylv, torch, np, p, method, cfg, args.steps, args.warmup, measure=True)
    stats = r.pop("stats")
    mixed = args.precision == "fp32" or args.gram_precision > 0
    dtype = "f64"
    if args.precision == "fp32":
        dtype = "f32-basis/f64"
    if args.gram_precision > 0:
        dtype += "+bf16x3-grams"
    out = {
        "metric": METRIC, "value": round(r["iters_per_s"], 2), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": p.meta["workload"] + f", tol {p.tol:g}, seeded N(0,1) C1/C2",
                   "n": p.n, "m": p.m, "s": p.s, "lyapunov": bool(p.lyapunov),
                   "method": "factored CG" if method == "cg" else "factored BiCGSTAB",
                   "max_iter": p.max_iter, "iters_per_solve": r["iters_per_step"],
                   "basis_precision": args.precision, "gram_precision": args.gram_precision,
                   "refine_max": args.refine, "outer_steps": r["outer_steps"],
                   "rank": r["rank"], "time_to_solution_ms": round(r["ms_per_step"], 3),
                   "profiled_solve_ms": round(r["profiled_solve_ms"], 3),
                   "true_rel_res": r["true_rel_res"], "statuses": r["statuses"],
                   "stopping_rule": "recursive ||R|| <= tol ||R0||, then the true residual "
                                    "<= tol (verified)"},
        "roofline": roofline_of(stats, args.workload, "mixed" if mixed else "fp64"),
        "kernel_breakdown": breakdown_of(stats),
    }
    if not args.no_compare and not mixed:
        out["comparisons"] = comparisons(sylv, torch, np, args.workload, r)
        out["spmm_hbm"] = spmm_hbm(sylv, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, method, args.cpu_iters, args.cpu_iters_1t)
    print(json.dumps(out), flush=True)


# Kernel sources whose family the hardware-counter traffic in profiles/ was taken for.
FAMILY_SOURCES = {"core_op": "dense.hip", "gram": "arnoldi_impl.h", "update": "arnoldi_impl.h",
                  "upd_gram": "arnoldi_impl.h", "spmm": "arnoldi_impl.h",
                  "block_qr": "arnoldi_impl.h", "core_elem": "core.hip", "core_band": "core.hip",
                  "res_gram": "dense.hip", "res_gram_bf16": "gram_bf16.hip"}


def measured_traffic(workload, family, precision):
    """HBM bytes per launch of `family` from the committed counter summary
    profiles/traffic_<workload>.md (FETCH_SIZE + WRITE_SIZE over the family's kernels, scaled by
    a copy kernel of known size), or None when there is none or the kernel source changed since
    (its SHA-256 is recorded beside the figure)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    src = FAMILY_SOURCES.get(family)
    if precision != "fp64" or not src or not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2605_28274_amd", "csrc", src),
                              "rb").read()).hexdigest()
    for line in open(path):
        if line.startswith("TRAFFIC "):
            rec = json.loads(line[len("TRAFFIC "):])
            if rec.get("family") == family and rec.get("source_sha256") == sha:
                return rec["bytes_per_launch"]
    return None


def spmm_hbm(sylv, torch):
    """SpMM (sliced ELLPACK, FP64) on three large operators (the last, 336 MB, larger than the
    256 MB last-level cache): algorithmic bytes 12 nnz + 4 (rows + 1) + 16 rows s per call over
    its HIP-event time. Warm: 20 launches back to back
    between two events (the library's SpMM call only enqueues), per launch. Cold: one launch
    right after a 512 MiB read that evicts the caches (a read, so that no dirty lines are left
    to write back); the read keeps the stream busy while the launch is enqueued, so the events
    bracket the kernel and not the host call."""
    import numpy as np
    from workloads import stencils
    out = {}
    flush = torch.ones(64 * 2 ** 20, dtype=torch.float64, device="cuda")
    batch = 20
    for name, M, s in (("2D 1024^2 (n = 1048576), s = 1", stencils.cd2d(1024, 1024, 0.0), 1),
                       ("3D 64^3 (n = 262144), s = 4", stencils.cd3d(64, 64, 64, 10.0), 4),
                       ("2D 2048^2 (n = 4194304), s = 1", stencils.cd2d(2048, 2048, 0.0), 1)):
        rp, ci, va = sylv.csr_tensors(M)
        csr = sylv.make_csr(M.shape[0], rp, ci, va)
        buf = torch.empty(sylv.sylv_sell_bytes(csr), dtype=torch.uint8, device="cuda")
        sylv.sylv_sell_build(csr, buf)
        X = torch.randn(M.shape[0], s, dtype=torch.float64, device="cuda")
        Y = torch.empty_like(X)
        nbytes = 12 * M.nnz + 4 * (M.shape[0] + 1) + 16 * M.shape[0] * s
        res = {}
        for mode in ("warm", "cold"):
            ts = []
            for _ in range(5 if mode == "warm" else 10):
                k = batch if mode == "warm" else 1
                if mode == "cold":
                    flush.sum()
                else:
                    sylv.sylv_sell_spmm(csr, buf, s, X, Y)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(k):
                    sylv.sylv_sell_spmm(csr, buf, s, X, Y)
                b.record()
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b) / k)
            t = float(np.median(ts)) * 1e-3
            res[mode] = {"us": round(t * 1e6, 2), "GB/s": round(nbytes / t / 1e9, 1),
                         "frac": round(nbytes / t / 1e9 / PEAK_HBM_GBS, 3)}
        out[name] = {"bytes": nbytes, **res}
    return out


def run_batch_group(sylv, torch, spec, steps, warmup):
    """One group of the 64-instance batch (method and block size), grouped form, recursive
    stopping test only: wall time per solve (a breakdown of the batch's time)."""
    from workloads import configs
    method, s = spec.split(":")
    probs = [p for p in configs.batch64() if p.method == method and p.s == int(s)]
    for p in probs:
        p.max_iter = 1500 if p.method == "cg" else 600
    b = sylv.Batch(probs, nstreams=1, form=sylv.SYLV_BATCH_GROUPED, verify=0)
    for _ in range(warmup):
        b.solve(1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = b.solve(1e-8)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    b.close()
    return {"batch_group": spec, "instances": len(probs), "groups": 1,
            "ms_per_solve": round(1000 * dt, 3), "iters": [r.iters for r in res]}


def run_batch_compare(sylv, torch, np, steps, warmup, nstreams=8):
    """The 64-instance batch: wall time of sylv_batch_solve over all instances (every instance
    verified against its true residual) in the grouped form, in the streams form (instances spread
    over `nstreams` streams, one host thread each), in the grouped form with HIP-graph segments,
    and the same instances solved one after another on one stream (FP64 plain, one context at a
    time)."""
    from workloads import configs
    probs = configs.batch64()
    for p in probs:  # workspace sized for the instances' needs (CG up to ~1000 iterations)
        p.max_iter = 1500 if p.method == "cg" else 600

    def timed(ns, nsteps, form=None):
        b = sylv.Batch(probs, nstreams=ns, form=sylv.SYLV_BATCH_STREAMS if form is None else form)
        for _ in range(warmup):
            b.solve(1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            res = b.solve(1e-8)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / nsteps
        rels = [sylv.sylv_residual_norm(b.context(i))[1] for i in range(len(probs))]
        b.close()
        del b
        torch.cuda.empty_cache()
        return dt, res, rels

    def row(dt, res, rels):
        iters = sum(r.iters for r in res)
        return {"time_to_1e-8_ms": round(1000 * dt, 3), "iters": iters,
                "iters_per_s": round(iters / dt, 2), "max_true_rel_res": float(max(rels)),
                "statuses": sorted(set(int(r.status) for r in res))}

    dt, res, rels = timed(nstreams, steps, sylv.SYLV_BATCH_GROUPED)
    dtg, res_g, rels_g = timed(nstreams, steps, sylv.SYLV_BATCH_GRAPH)
    dtm, res_m, rels_m = timed(nstreams, steps, sylv.SYLV_BATCH_STREAMS)
    dts, res_s, rels_s = timed(1, 1)
    return {"workload": "batch of 64 seeded instances (2D A, n 1024-32768; 1D/2D B, m 512-16384; "
                        "s in {1,2,4}; CG/BiCGSTAB alternating), tol 1e-8",
            "instances": len(probs), "streams": nstreams,
            "batched": {"form": "grouped", **row(dt, res, rels)},
            "batched_graph": {"form": "grouped, HIP-graph segments", **row(dtg, res_g, rels_g)},
            "batched_streams": {"form": "streams", **row(dtm, res_m, rels_m)},
            "sequential_fp64_plain": row(dts, res_s, rels_s),
            "speedup_vs_sequential": round(dts / dt, 3),
            "speedup_vs_streams": round(dtm / dt, 3)}


if __name__ == "__main__":
    main()
