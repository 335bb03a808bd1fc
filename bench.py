#!/usr/bin/env python3
"""Benchmark of the factored Krylov hot path on one MI355X.

Default workload (`--workload c2`): factored BiCGSTAB, FP64, A = 2D convection-diffusion
128 x 128 (Pe = 10), B = 1D convection-diffusion m = 8192 (Pe = 10), s = 2, C1, C2 ~ N(0, 1)
(seed 1002), tol 1e-8. Other workloads (same JSON line, used for measurements and profiles):
  c1    factored CG, FP64, 1D Laplacians (n+1)^2 tridiag, n = 256, m = 192, s = 1, 200 iterations
  c3    factored BiCGSTAB, FP64, 3D CD 64^3 x 2D CD 256^2 (Pe = 10), s = 4
  c5cg  Lyapunov factored CG, FP64, 2D Laplacian 1024^2, s = 1
  c5bi  Lyapunov factored BiCGSTAB, FP64, 2D CD 1024^2 (Pe = 1), s = 1, 200-iteration window
  batch64  64 independent instances (2D A with n in [1024, 32768]; 1D or 2D B with m in [512,
        16384]; s in {1, 2, 4}; CG on Laplacians and BiCGSTAB on Pe = 10 alternately), solved as
        one batch over --streams streams; the same instances solved one after another on one
        stream are timed beside it (`sequential_ms`)

One step = one pass of the whole path over resident inputs: sylv_create (CSR validation, B^T,
sliced-ELLPACK copies, QR of C1 and C2), the factored solve to ||R|| <= tol ||R0|| (or the
iteration cap), sylv_get_factors into device buffers and sylv_residual_norm (FP64 true
residual). `value` is factored iterations per second over whole steps; ms_per_step is the time
to the solution including setup and the residual check.

After the timed region one more (untimed) solve runs with per-kernel HIP-event timing on the
solver's stream to report the roofline fraction of the dominant kernel family; the CPU oracle
is timed on a bounded sample for `cpu_baseline`.
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
METRIC = "time-to-1e-8 rel. residual + factored iters/s; mixed/batched vs FP64 plain"


def workload(name, max_iter):
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


def cpu_baseline(p, method, iters):
    """The oracle as it stands on the host cores: its first `iters` factored iterations of the
    same workload (cost per iteration grows with the rank, so this understates the full-solve
    time per iteration)."""
    from oracle import factored
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    fn = factored.factored_cg if method == "cg" else factored.factored_bicgstab
    t0 = time.perf_counter()
    _, _, _, info = fn(p.A, p.B, p.C1, p.C2, tol=0.0, max_iter=iters, lyapunov=p.lyapunov)
    dt = time.perf_counter() - t0
    name = "CG" if method == "cg" else "BiCGSTAB"
    return {"value": info["iters"] / dt, "unit": "iters/s", "cores": int(cores), "kind": "oracle",
            "sample": f"first {info['iters']} factored {name} iterations of the same workload "
                      f"({dt:.1f} s on the host)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2",
                    choices=["c1", "c2", "c3", "c5cg", "c5bi", "batch64"])
    ap.add_argument("--streams", type=int, default=8, help="streams of the batched run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check-every", type=int, default=16,
                    help="iterations between the host's looks at the convergence flag")
    ap.add_argument("--streams-solve", type=int, default=0, choices=[0, 1, 2],
                    help="sylv_options.streams (0 automatic)")
    ap.add_argument("--reorth", type=int, default=0, choices=[0, 1, 2],
                    help="sylv_options.reorth (0 automatic)")
    ap.add_argument("--cpu-iters", type=int, default=200)
    ap.add_argument("--max-iter", type=int, default=0)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                    help="storage of the Krylov bases (fp32: mixed precision)")
    ap.add_argument("--gram-precision", type=int, default=0, choices=[0, 1, 2],
                    help="sylv_options.gram_precision of the true-residual Grams")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="one step only (for hardware-counter runs of rocprofv3 --pmc)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="device copies of 512 MiB (counter calibration) and exit")
    ap.add_argument("--refine", type=int, default=-1,
                    help="correction solves of the outer refinement (default: 3 with fp32 "
                         "bases, 0 with fp64)")
    args = ap.parse_args()
    if args.refine < 0:
        args.refine = 3 if args.precision == "fp32" else 0
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs one solve on one GPU; --gpus must be 1"}))
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
    if args.workload == "batch64":
        return run_batch(args, sylv, torch, np)
    p, method = workload(args.workload, args.max_iter)
    cg = method == "cg"
    dev = "cuda"
    rpA, ciA, vaA = sylv.csr_tensors(p.A, dev)
    C1 = torch.as_tensor(p.C1, device=dev)
    if p.lyapunov:
        csrB, C2 = sylv.make_csr(p.m, rpA, ciA, vaA), C1
    else:
        rpB, ciB, vaB = sylv.csr_tensors(p.B, dev)
        csrB, C2 = sylv.make_csr(p.m, rpB, ciB, vaB), torch.as_tensor(p.C2, device=dev)
    prob = sylv.sylv_problem(p.n, p.m, p.s, sylv.make_csr(p.n, rpA, ciA, vaA), csrB,
                             1 if p.lyapunov else 0, C1.data_ptr(), p.s, C2.data_ptr(), p.s)
    mixed = args.precision == "fp32"
    opts = sylv.default_options(sylv.SYLV_METHOD_CG if cg else sylv.SYLV_METHOD_BICGSTAB,
                                p.max_iter, check_every=args.check_every,
                                precision=sylv.SYLV_MIXED_FP32 if mixed else sylv.SYLV_FP64,
                                refine_max=args.refine, refine_max_iter=100,
                                streams=args.streams_solve, reorth=args.reorth,
                                gram_precision=args.gram_precision)
    ws = torch.empty(sylv.sylv_workspace_bytes(prob, opts), dtype=torch.uint8, device=dev)
    rmax = (p.max_iter + 1 if cg else 2 * p.max_iter + 1) * p.s
    if args.refine > 0:  # the summed iterate stacks the corrections' bases
        rmax += args.refine * (101 if cg else 201) * 8
    V = torch.empty((p.n, rmax), dtype=torch.float64, device=dev)
    W = V if p.lyapunov else torch.empty((p.m, rmax), dtype=torch.float64, device=dev)
    Xc = torch.empty((rmax, rmax), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    solve = sylv.sylv_factored_cg if cg else sylv.sylv_factored_bicgstab

    def step():
        ctx = sylv.sylv_create(prob, opts, ws, stream.cuda_stream)
        res = solve(ctx, p.tol, p.max_iter)
        rv, rw = res.rank_v, res.rank_w
        sylv.sylv_get_factors(ctx, V[:, :rv], Xc[:rv, :rw], None if p.lyapunov else W[:, :rw])
        _, rel = sylv.sylv_residual_norm(ctx)
        sylv.sylv_destroy(ctx)
        return res, rel

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    iters, rels, statuses = 0, [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res, rel = step()
        iters += res.iters
        rels.append(rel)
        statuses.append(res.status)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1000.0 * dt / args.steps
    if args.pmc_pass:
        print(json.dumps({"pmc_pass": args.workload, "iters": iters}), flush=True)
        return

    # untimed measurement pass: per-family kernel times with HIP events on the solver's stream
    ctx = sylv.sylv_create(prob, opts, ws, stream.cuda_stream)
    sylv.sylv_set_profiling(ctx, True)
    t1 = time.perf_counter()
    res = solve(ctx, p.tol, p.max_iter)
    solve_ms = 1000.0 * (time.perf_counter() - t1)
    stats = sylv.sylv_get_kernel_stats(ctx)
    sylv.sylv_destroy(ctx)
    tot = sum(s["ms"] for s in stats) or 1.0
    dom = max(stats, key=lambda s: s["ms"])
    if dom["family"] == "core_op":
        bound, unit = "mfma", "TFLOP/s"
        achieved = dom["flops"] / (dom["ms"] * 1e-3) / 1e12
        peak = PEAK_FP64_TFS
    else:
        bound, unit = "hbm", "GB/s"
        achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
        peak = PEAK_HBM_GBS
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4),
                "traffic": measured_traffic(args.workload, dom["family"], args.precision),
                "kernel": dom["family"], "launches": dom["launches"],
                "avg_launch_us": round(1000 * dom["ms"] / max(dom["launches"], 1), 3),
                "share_of_kernel_time": round(dom["ms"] / tot, 3)}
    breakdown = {s["family"]: {"ms": round(s["ms"], 3), "launches": s["launches"],
                               "GB/s": round(s["bytes"] / max(s["ms"], 1e-9) / 1e6, 1),
                               "TFLOP/s": round(s["flops"] / max(s["ms"], 1e-9) / 1e9, 3)}
                 for s in stats if s["launches"]}

    out = {
        "metric": METRIC, "value": round(iters / dt, 2), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-basis/f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": p.meta["workload"] + f", tol {p.tol:g}, seeded N(0,1) C1/C2",
                   "n": p.n, "m": p.m, "s": p.s, "lyapunov": bool(p.lyapunov),
                   "method": "factored CG" if cg else "factored BiCGSTAB",
                   "max_iter": p.max_iter, "iters_per_solve": iters // args.steps,
                   "basis_precision": args.precision, "refine_max": args.refine,
                   "outer_steps": int(res.outer_steps),
                   "rank": int(res.rank_v), "time_to_solution_ms": round(ms_per_step, 3),
                   "profiled_solve_ms": round(solve_ms, 3),
                   "true_rel_res": float(np.max(rels)), "statuses": sorted(set(statuses))},
        "roofline": roofline,
        "kernel_breakdown": breakdown,
        "spmm_hbm": spmm_hbm(sylv, torch) if args.workload == "c2" and not mixed else None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, method, args.cpu_iters)
    print(json.dumps(out), flush=True)


# Kernel sources whose family the hardware-counter traffic in profiles/ was taken for.
FAMILY_SOURCES = {"core_op": "dense.hip", "gram": "arnoldi_impl.h", "update": "arnoldi_impl.h",
                  "upd_gram": "arnoldi_impl.h", "spmm": "arnoldi_impl.h",
                  "block_qr": "arnoldi_impl.h", "core_elem": "core.hip", "core_band": "core.hip"}


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
    """SpMM (sliced ELLPACK, FP64) on two large operators: algorithmic bytes 12 nnz +
    4 (rows + 1) + 16 rows s per call over its HIP-event time. Warm: 20 launches back to back
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
                       ("3D 64^3 (n = 262144), s = 4", stencils.cd3d(64, 64, 64, 10.0), 4)):
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


def run_batch(args, sylv, torch, np):
    """The 64-instance batch: wall time of sylv_batch_solve over all instances (after one
    untimed warm-up solve), then the same instances solved sequentially on one stream."""
    from workloads import configs
    probs = configs.batch64()
    for p in probs:  # workspace sized for the instances' needs (CG up to ~1000 iterations)
        p.max_iter = 1500 if p.method == "cg" else 600
    mixed = args.precision == "fp32"
    prec = sylv.SYLV_MIXED_FP32 if mixed else sylv.SYLV_FP64

    def timed(nstreams, steps):
        b = sylv.Batch(probs, nstreams=nstreams, precision=prec)
        for _ in range(args.warmup):
            b.solve(1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = b.solve(1e-8)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        rels = []
        for i in range(len(probs)):
            _, rel = sylv.sylv_residual_norm(b.context(i))
            rels.append(rel)
        b.close()
        del b
        torch.cuda.empty_cache()
        return dt, res, rels

    dt, res, rels = timed(args.streams, args.steps)
    dts, res_s, _ = timed(1, 1)
    iters = sum(r.iters for r in res)
    out = {
        "metric": METRIC, "value": round(iters / dt, 2), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1000 * dt, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-basis/f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": "batch of 64 seeded instances (2D A, n 1024-32768; 1D/2D B, "
                               "m 512-16384; s in {1,2,4}; CG/BiCGSTAB alternating), tol 1e-8",
                   "instances": len(probs), "streams": args.streams,
                   "total_iters": iters, "time_to_1e-8_all_ms": round(1000 * dt, 3),
                   "sequential_ms": round(1000 * dts, 3),
                   "speedup_vs_sequential": round(dts / dt, 3),
                   "statuses": sorted(set(int(r.status) for r in res)),
                   "max_true_rel_res": float(max(rels)),
                   "sequential_iters": sum(r.iters for r in res_s)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
