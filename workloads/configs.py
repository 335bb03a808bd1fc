"""The named synthetic workloads (shapes, seeds and stencils), built from :mod:`workloads.stencils`.

* ``c1_cg_1d``      - factored CG, FP64: A = (n+1)^2 tridiag(-1,2,-1), n = 256; B the same with
                      m = 192; s = 1; seed 1001; at most 200 iterations.
* ``c2_bicgstab``   - factored BiCGSTAB, FP64: A = 2D convection-diffusion 128 x 128 (Pe = 10),
                      B = 1D convection-diffusion m = 8192 (Pe = 10), s = 2, seed 1002.
* ``c3_bicgstab``   - factored BiCGSTAB at scale: A = 3D 64^3 (Pe = 10), B = 2D 256 x 256 (Pe = 10),
                      s = 4, seed 1003.
* ``c5_lyap_cg`` / ``c5_lyap_bicgstab`` - Lyapunov B = A^T on a 1024 x 1024 grid, s = 1,
                      seed 1005; Pe = 0 for CG (SPD), Pe = 1 for BiCGSTAB.
* ``batch64``       - 64 independent instances drawn from ``default_rng(4242)``.

C1 uses the physical 1/h^2 scaling it is stated with; the others use unit-coefficient stencils
(each operator multiplied by its own h^2).
"""
from __future__ import annotations

import numpy as np

from .stencils import Problem, cd1d, cd2d, cd3d, make_problem


def c1_cg_1d() -> Problem:
    A = cd1d(256, 0.0, "physical")
    B = cd1d(192, 0.0, "physical")
    return make_problem("c1_cg_1d", A, B, 1, 1001, method="cg", tol=1e-8, max_iter=200,
                        meta={"workload": "factored CG FP64, 1D Laplacian n=256 x m=192, s=1"})


def c2_bicgstab(max_iter: int = 800) -> Problem:
    A = cd2d(128, 128, 10.0)
    B = cd1d(8192, 10.0)
    return make_problem("c2_bicgstab", A, B, 2, 1002, method="bicgstab", tol=1e-8,
                        max_iter=max_iter,
                        meta={"workload": "factored BiCGSTAB FP64, 2D CD 128x128 (Pe=10) x 1D CD "
                                          "m=8192 (Pe=10), s=2"})


def c3_bicgstab(max_iter: int = 400) -> Problem:
    A = cd3d(64, 64, 64, 10.0)
    B = cd2d(256, 256, 10.0)
    return make_problem("c3_bicgstab", A, B, 4, 1003, method="bicgstab", tol=1e-8,
                        max_iter=max_iter,
                        meta={"workload": "factored BiCGSTAB, 3D CD 64^3 (Pe=10) x 2D CD 256^2 "
                                          "(Pe=10), s=4"})


def c5_lyap(method: str = "cg", max_iter: int = 4000) -> Problem:
    pe = 0.0 if method == "cg" else 1.0
    A = cd2d(1024, 1024, pe)
    return make_problem(f"c5_lyap_{method}", A, None, 1, 1005, lyapunov=True, method=method,
                        tol=1e-8, max_iter=max_iter,
                        meta={"workload": f"Lyapunov {method}, 2D CD 1024^2 (Pe={pe}), s=1"})


def batch64(count: int = 64, max_iter: int = 2000) -> list[Problem]:
    """Instances i = 0..count-1: even i -> CG on Laplacians, odd i -> BiCGSTAB on Pe = 10.
    A is 2D with n = Nx*Ny in [1024, 32768]; B is 1D (m in [512, 16384]) or 2D
    (Mx*My in [512, 16384]) with probability 1/2 each; s in {1, 2, 4}."""
    rng = np.random.default_rng(4242)
    out = []
    for i in range(count):
        cg = (i % 2 == 0)
        pe = 0.0 if cg else 10.0
        while True:
            nx = int(rng.integers(32, 182))
            lo = max(1, -(-1024 // nx))
            hi = 32768 // nx
            if lo <= hi:
                ny = int(rng.integers(lo, hi + 1))
                break
        A = cd2d(nx, ny, pe)
        if rng.random() < 0.5:
            m = int(rng.integers(512, 16385))
            B = cd1d(m, pe)
            bdesc = f"1D {m}"
        else:
            mx = int(rng.integers(16, 129))
            lo = max(1, -(-512 // mx))
            hi = 16384 // mx
            my = int(rng.integers(lo, hi + 1))
            B = cd2d(mx, my, pe)
            bdesc = f"2D {mx}x{my}"
        s = int(rng.choice([1, 2, 4]))
        p = make_problem(f"batch{i:02d}", A, B, s, 5000 + i,
                         method="cg" if cg else "bicgstab", tol=1e-8, max_iter=max_iter,
                         meta={"A": f"2D {nx}x{ny}", "B": bdesc, "pe": pe})
        out.append(p)
    return out


def tiny_sylvester(n=12, m=9, s=2, seed=7, pe=0.0, method="cg", max_iter=400, tol=1e-12):
    """Small 1D x 1D problem for exact-solve comparisons."""
    A = cd1d(n, pe)
    B = cd1d(m, pe)
    return make_problem(f"tiny_{method}_{n}x{m}s{s}", A, B, s, seed, method=method, tol=tol,
                        max_iter=max_iter)


CONFIGS = {
    "c1_cg_1d": c1_cg_1d,
    "c2_bicgstab": c2_bicgstab,
    "c3_bicgstab": c3_bicgstab,
}
