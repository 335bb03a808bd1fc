"""GPU checks of the FP32-basis (mixed precision) solves and of the outer refinement, through the
C ABI.

The FP32 bases limit the true residual to a floor of roughly the FP32 unit roundoff times the
conditioning; the refinement must bring the FP64 true residual of the summed iterate below the
tolerance. Every reported true residual is checked against the dense residual of the exported
factors (X = V Xc W^T formed on the host in FP64), and the refined solution against the FP64
oracle's."""
import json
import os

import numpy as np
import pytest

from oracle import factored
from workloads import configs, stencils

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def sylv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_28274_amd import sylv as _s
    return _s


def solve(sylv, p, method, tol, max_iter, **kw):
    code = sylv.SYLV_METHOD_CG if method == "cg" else sylv.SYLV_METHOD_BICGSTAB
    slv = sylv.Solver(p.A, p.B, p.C1, p.C2, lyapunov=p.lyapunov, method=code, max_iter=max_iter,
                      **kw)
    res = slv.factored_cg(tol) if method == "cg" else slv.factored_bicgstab(tol)
    V, X, W = (t.cpu().numpy() for t in slv.get_factors())
    _, rr = slv.residual_norm()
    slv.close()
    return res, V, X, W, rr


def dense_rel(p, V, X, W):
    Xf = V @ X @ W.T
    C = p.C1 @ p.C2.T
    return np.linalg.norm(C - p.A @ Xf - (p.B.T @ Xf.T).T) / np.linalg.norm(C), Xf


def tiny(kind):
    if kind == "bicgstab":
        A, B = stencils.cd2d(24, 20, 10.0), stencils.cd1d(300, 10.0)
        return stencils.make_problem("tb", A, B, 2, 11, method="bicgstab"), "bicgstab"
    if kind == "cg":
        A, B = stencils.cd2d(24, 20, 0.0), stencils.cd1d(300, 0.0)
        return stencils.make_problem("tc", A, B, 2, 12, method="cg"), "cg"
    A = stencils.cd2d(24, 20, 1.0)
    return stencils.make_problem("tl", A, None, 1, 13, lyapunov=True, method="bicgstab"), "bicgstab"


def test_fp32_bases_reach_their_floor(sylv):
    p, method = tiny("bicgstab")
    # verify = 0: the recursive stopping rule alone (a verified solve would not report this
    # floor as converged)
    res, V, X, W, rr = solve(sylv, p, method, 1e-10, 400, precision=sylv.SYLV_MIXED_FP32,
                             verify=0)
    assert res.status == sylv.SYLV_OK and res.rel_res_true < 0 and res.outer_steps == 0
    d, _ = dense_rel(p, V, X, W)
    # the FP64 true residual (with the right-hand side's QR defect) equals the dense one
    assert abs(rr - d) <= 1e-6 * d
    # above the recursive residual, at the FP32 level
    assert res.rel_res_recursive <= 1e-10 < d < 1e-6


@pytest.mark.parametrize("kind", ["bicgstab", "cg", "lyapunov"])
def test_refinement_reaches_tol(sylv, kind):
    p, method = tiny(kind)
    tol = 1e-10
    res, V, X, W, rr = solve(sylv, p, method, tol, 400, precision=sylv.SYLV_MIXED_FP32,
                             refine_max=3, refine_max_iter=100)
    assert res.status == sylv.SYLV_OK
    assert 1 <= res.outer_steps <= 3
    assert 0 < res.rel_res_true <= tol
    d, Xf = dense_rel(p, V, X, W)
    assert abs(rr - res.rel_res_true) <= 1e-12 * max(rr, 1e-300) + 1e-18
    assert abs(d - rr) <= 1e-3 * d
    # the refined solution is the FP64 solution (both within their residuals)
    Vo, Xo, Wo, info = factored.solve(p, tol=tol, max_iter=400)
    Xr = Vo @ Xo @ Wo.T
    assert np.linalg.norm(Xf - Xr) / np.linalg.norm(Xr) < 1e-6


def test_refinement_fp64_and_rank_checks(sylv):
    # refinement also runs on FP64 bases (the FP64 solve stops at a recursive residual just
    # below tol, so the sketch may still ask for one correction)
    p, method = tiny("bicgstab")
    res, V, X, W, rr = solve(sylv, p, method, 1e-9, 400, refine_max=2)
    assert res.status == sylv.SYLV_OK and res.outer_steps <= 2 and res.rel_res_true <= 1e-9
    d, _ = dense_rel(p, V, X, W)
    assert abs(d - rr) <= 1e-6 * d


def test_c2_mixed_refined_against_oracle(sylv):
    with open(os.path.join(GOLDEN, "c2_bicgstab_oracle.json")) as f:
        gold = json.load(f)
    p = configs.c2_bicgstab()
    code = sylv.SYLV_METHOD_BICGSTAB
    slv = sylv.Solver(p.A, p.B, p.C1, p.C2, method=code, max_iter=p.max_iter,
                      precision=sylv.SYLV_MIXED_FP32, refine_max=3, refine_max_iter=100)
    res = slv.factored_bicgstab(p.tol)
    assert res.status == sylv.SYLV_OK and res.rel_res_true <= p.tol
    _, rr = slv.residual_norm()
    assert abs(rr - res.rel_res_true) <= 1e-3 * rr
    V, X, W = (t.cpu().numpy() for t in slv.get_factors())
    slv.close()
    Om = np.random.default_rng(gold["sketch_seed"]).standard_normal((p.m, gold["sketch_q"]))
    rows = np.asarray(gold["sketch_rows"])
    Sg = V[rows] @ (X @ (W.T @ Om))
    So = np.asarray(gold["sketch"])
    assert np.linalg.norm(Sg - So) / np.linalg.norm(So) < 1e-4
