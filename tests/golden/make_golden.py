"""Writes the stored oracle results the GPU parity tests compare against.

Calls only the CPU oracle (``oracle/``) and the seeded input generators (``workloads/``):
    python tests/golden/make_golden.py
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
    with open(os.path.join(HERE, "c2_bicgstab_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("c2", info["status"], info["iters"], true_rel, secs)


if __name__ == "__main__":
    c2()
