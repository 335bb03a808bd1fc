"""GPU parity of the further factorized methods (CR, CGS, GPBiCG; Section 4's remark and
Section 6) against the CPU oracle's factored forms (oracle/factored_more.py, pinned against
SciPy's CGS and MINRES, BiCGSTAB and exact solves), through the C ABI.

Tolerances as for CG and BiCGSTAB: early scalars to 1e-10 (both FP64, different summation
orders and orthogonalization schemes); CR (symmetric, Lanczos) keeps its count within one;
CGS and GPBiCG, like BiCGSTAB, amplify rounding differences late, so their counts are compared
within max(3, 15%) and their solutions within the conditioning times the tolerance."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import direct, factored, factored_more, residual
from workloads import stencils

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sylv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_28274_amd import sylv as _s
    return _s


def gpu_solve(sylv, p, method, tol, max_iter, **kw):
    slv = sylv.Solver(p.A, p.B, p.C1, p.C2, lyapunov=p.lyapunov,
                      method=sylv.METHOD_CODES[method], max_iter=max_iter, **kw)
    res = slv.solve(tol)
    V, X, W = (t.cpu().numpy() for t in slv.get_factors())
    return res, V, X, W, slv


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


SCALARS = {"cr": ("alpha", "beta", "relres"), "cgs": ("alpha", "beta", "relres"),
           "gpbicg": ("alpha", "beta", "relres")}


@pytest.mark.parametrize("method", ["cr", "cgs", "gpbicg"])
@pytest.mark.parametrize("s", [1, 2, 3])
def test_closed_form(sylv, method, s):
    n, m, a, b = 30, 20, 3.0, 1.5
    A = stencils._canonical(sp.csr_matrix(a * np.eye(n)))
    B = stencils._canonical(sp.csr_matrix(b * np.eye(m)))
    C1, C2 = stencils.gaussian_rhs(n, m, s, 5)
    p = stencils.Problem("cf", A, B, C1, C2)
    res, V, X, W, slv = gpu_solve(sylv, p, method, 1e-12, 5)
    assert res.status == sylv.SYLV_OK and res.iters == 1
    assert rel(V @ X @ W.T, C1 @ C2.T / (a + b)) < 1e-13
    slv.close()


@pytest.mark.parametrize("method,s", [("cr", 1), ("cr", 2), ("cgs", 2), ("cgs", 3),
                                      ("gpbicg", 1), ("gpbicg", 2)])
def test_tiny_vs_oracle_and_direct(sylv, method, s):
    pe = 0.0 if method == "cr" else 12.0
    p = stencils.make_problem("t", stencils.cd1d(14, pe), stencils.cd1d(11, pe), s, 41 + s,
                              method=method)
    res, V, X, W, slv = gpu_solve(sylv, p, method, 1e-12, 300)
    Vo, Xo, Wo, info = factored_more.METHODS[method](p.A, p.B, p.C1, p.C2, tol=1e-12, max_iter=300)
    assert res.status == sylv.SYLV_OK and info["status"] == factored.CONVERGED
    assert abs(res.iters - info["iters"]) <= (1 if method == "cr" else 2)
    h = slv.get_history()
    k = min(8, info["iters"] - 1)
    for key in SCALARS[method]:
        a, b = np.asarray(h[key][:k]), np.asarray(info[key][:k])
        assert np.max(np.abs(a - b) / np.abs(b)) < 1e-10, key
    if method == "gpbicg":
        a, b = np.asarray(h["omega"][:k]), np.asarray(info["zeta"][:k])
        assert np.max(np.abs(a - b) / np.abs(b)) < 1e-10
    Xd = direct.kron_solve(p.A, p.B, p.C1, p.C2)
    kappa = np.linalg.cond(direct.kron_matrix(p.A, p.B))
    assert rel(V @ X @ W.T, Xd) <= 10 * kappa * 1e-12
    slv.close()


@pytest.mark.parametrize("method", ["cr", "cgs", "gpbicg"])
@pytest.mark.parametrize("lyap", [False, True])
def test_medium_vs_oracle(sylv, method, lyap):
    """2D 40 x 36 (x 1D 600) with s = 2: multi-tile cores and multi-kernel basis steps."""
    pe = 0.0 if method == "cr" else 8.0
    A = stencils.cd2d(40, 36, pe)
    B = None if lyap else stencils.cd1d(600, pe)
    p = stencils.make_problem("m", A, B, 2, 51, lyapunov=lyap, method=method)
    tol = 1e-8
    res, V, X, W, slv = gpu_solve(sylv, p, method, tol, 400)
    Vo, Xo, Wo, info = factored_more.METHODS[method](p.A, p.B, p.C1, p.C2, tol=tol, max_iter=400,
                                                    lyapunov=lyap)
    assert res.status == sylv.SYLV_OK and info["status"] == factored.CONVERGED
    band = 1 if method == "cr" else max(3, round(0.15 * info["iters"]))
    assert abs(res.iters - info["iters"]) <= band, (res.iters, info["iters"])
    h = slv.get_history()
    for key in ("alpha", "relres"):
        a, b = np.asarray(h[key][:6]), np.asarray(info[key][:6])
        assert np.max(np.abs(a - b) / np.abs(b)) < 1e-10, key
    Om = residual.sketch_matrix(p.m, 8, 7)
    assert rel(residual.sketch(V, X, W, Om), residual.sketch(Vo, Xo, Wo, Om)) < 1e-5
    assert 0 < res.rel_res_true <= tol
    _, dense = residual.dense_residual(p.A, p.B, p.C1, p.C2, V, X, W)
    assert abs(dense - res.rel_res_true) <= 1e-6 * tol
    if lyap:
        Xf = V @ X @ W.T
        assert rel(Xf, Xf.T) < 1e-8
    slv.close()


def test_method_must_match_the_workspace(sylv):
    p = stencils.make_problem("w", stencils.cd1d(20), stencils.cd1d(15), 1, 3, method="cg")
    slv = sylv.Solver(p.A, p.B, p.C1, p.C2, method=sylv.SYLV_METHOD_CG, max_iter=20)
    with pytest.raises(sylv.SylvError) as ei:
        sylv.sylv_factored_gpbicg(slv.ctx, 1e-8, 20)
    assert ei.value.code == sylv.SYLV_ERR_WORKSPACE
    slv.close()
