"""Writes the stored oracle results the GPU parity tests compare against.

Calls only the CPU oracle (``oracle/``) and the seeded input generators (``workloads/``):
    python tests/golden/make_golden.py [c2] [c2_spread] [c5_window] [c3_window]

* ``c2``         full factored BiCGSTAB run of the 2D 128^2 x 1D 8192 workload (s = 2).
* ``c2_spread``  the same run with C1 perturbed at the level of its last bit (four seeds): how
                 far the oracle's own iteration counts move under rounding-size changes of the
                 input, the yardstick for comparing counts of differently rounded solvers.
* ``c5_window``  first 100 iterations of factored CG on the 1024^2 Lyapunov workload (s = 1),
                 plus a perturbed rerun giving the per-iteration rounding sensitivity.
* ``c3_window``  first 20 iterations of factored BiCGSTAB on the 3D 64^3 x 2D 256^2 workload
                 (s = 4), plus a perturbed rerun.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import factored, residual  # noqa: E402
from workloads import configs  # noqa: E402
from workloads.stencils import Problem  # noqa: E402


def perturbed(p, seed):
    """Copy of p with every entry of C1 moved by about one unit in its last place (C2 follows
    C1 for a Lyapunov problem)."""
    z = np.random.default_rng(seed).standard_normal(p.C1.shape)
    C1 = p.C1 + np.spacing(np.abs(p.C1)) * z
    C2 = C1.copy() if p.lyapunov else p.C2
    return Problem(p.name + f"_pert{seed}", p.A, p.B, C1, C2, lyapunov=p.lyapunov,
                   method=p.method, tol=p.tol, max_iter=p.max_iter, meta=p.meta)


def first_below(relres, level):
    rr = np.asarray(relres)
    hit = np.nonzero(rr <= level)[0]
    return int(hit[0]) + 1 if hit.size else -1


def sketch_rows(p, q=4, seed=7, count=64):
    Om = np.random.default_rng(seed).standard_normal((p.m, q))
    rows = np.sort(np.random.default_rng(seed + 1).choice(p.n, count, replace=False))
    return Om, rows


def dump(name, out):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)


def c2():
    p = configs.c2_bicgstab()
    t0 = time.time()
    V, X, W, info = factored.solve(p)
    secs = time.time() - t0
    _, true_rel = residual.factored_residual(p.A, p.B, p.C1, p.C2, V, X, W)
    q, seed = 4, 7
    Om = np.random.default_rng(seed).standard_normal((p.m, q))
    rows = np.sort(np.random.default_rng(8).choice(p.n, 64, replace=False))
    sk = V[rows] @ (X @ (W.T @ Om))
    out = {
        "workload": p.meta["workload"], "tol": p.tol, "seed": 1002,
        "status": info["status"], "iters": info["iters"], "rank": int(X.shape[0]),
        "alpha": info["alpha"][:40], "omega": info["omega"][:40], "beta": info["beta"][:40],
        "relres": [float(v) for v in info["relres"]], "true_relres": float(true_rel),
        "sketch_seed": seed, "sketch_q": q, "sketch_rows": rows.tolist(), "sketch": sk.tolist(),
        "oracle_seconds": secs,
    }
    dump("c2_bicgstab_oracle.json", out)
    print("c2", info["status"], info["iters"], true_rel, secs)


def _c2_one(seed):
    p = perturbed(configs.c2_bicgstab(), seed)
    _, _, _, info = factored.solve(p)
    return {"seed": seed, "status": info["status"], "iters": info["iters"],
            "k6": first_below(info["relres"], 1e-6), "k8": first_below(info["relres"], 1e-8),
            "alpha12": info["alpha"][:12]}


def c2_spread(seeds=(11, 12, 13, 14)):
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(len(seeds)) as ex:
        runs = list(ex.map(_c2_one, seeds))
    with open(os.path.join(HERE, "c2_bicgstab_oracle.json")) as f:
        base = json.load(f)
    out = {
        "workload": base["workload"],
        "what": "oracle reruns of the 2D 128^2 x 1D 8192 BiCGSTAB workload with every entry of "
                "C1 moved by about one unit in the last place (seeded Gaussian multiples of "
                "numpy.spacing); iteration counts to relative residual 1e-6 (k6) and to the "
                "tolerance 1e-8 (k8 = iters)",
        "base": {"iters": base["iters"], "k6": first_below(base["relres"], 1e-6),
                 "k8": first_below(base["relres"], 1e-8)},
        "runs": runs,
    }
    dump("c2_bicgstab_spread.json", out)
    print("c2_spread", out["base"], [(r["k6"], r["k8"]) for r in runs])


def _window(p, method, iters, tag):
    t0 = time.time()
    V, X, W, info = factored.solve(p, method=method, tol=1e-300, max_iter=iters)
    secs = time.time() - t0
    Om, rows = sketch_rows(p)
    sk = V[rows] @ (X @ (W.T @ Om))
    pv, px, pw, pinfo = factored.solve(perturbed(p, 21), method=method, tol=1e-300,
                                       max_iter=iters)
    psk = pv[rows] @ (px @ (pw.T @ Om))
    spread = {}
    for key in ("alpha", "beta", "omega", "relres"):
        a, b = np.asarray(info.get(key, [])), np.asarray(pinfo.get(key, []))
        if a.size:
            spread[key] = (np.abs(a - b) / np.abs(a)).tolist()
    out = {
        "workload": p.meta["workload"], "seed_problem": p.name, "window": iters,
        "status": info["status"], "iters": info["iters"], "rank": int(X.shape[0]),
        "alpha": [float(v) for v in info["alpha"]], "beta": [float(v) for v in info["beta"]],
        "omega": [float(v) for v in info.get("omega", [])],
        "relres": [float(v) for v in info["relres"]],
        "sketch_seed": 7, "sketch_q": int(Om.shape[1]), "sketch_rows": rows.tolist(),
        "sketch": sk.tolist(),
        "perturbed_sketch_rel": float(np.linalg.norm(psk - sk) / np.linalg.norm(sk)),
        "perturbed_rel_diff": spread,
        "oracle_seconds": secs,
    }
    dump(tag, out)
    print(tag, info["iters"], info["relres"][-1], secs, out["perturbed_sketch_rel"])


def c5_window():
    _window(configs.c5_lyap("cg"), "cg", 100, "c5_lyap_cg_window.json")


def c3_window():
    _window(configs.c3_bicgstab(), "bicgstab", 20, "c3_bicgstab_window.json")


if __name__ == "__main__":
    jobs = {"c2": c2, "c2_spread": c2_spread, "c5_window": c5_window, "c3_window": c3_window}
    for name in (sys.argv[1:] or ["c2"]):
        jobs[name]()
