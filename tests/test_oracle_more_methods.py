"""Pins for the oracle's further factorized Krylov methods (CR, CGS, GPBiCG).

* The matrix-oriented forms against independent implementations: SciPy's CGS and MINRES
  (MINRES and CR minimize the same residual norm over the same Krylov space, so their iterates
  coincide in exact arithmetic) on the Kronecker form eq. (1.2), and GPBiCG with its second
  parameter fixed at zero against the pinned BiCGSTAB (Algorithm 2.2 / 4.2).
* The factored forms against the matrix-oriented ones iterate by iterate (Section 5.1's
  equivalence of factored and unfactored methods), the Lyapunov form against the Sylvester one
  with B = A^T, and convergence to the exact solution of a tiny problem.
* Internal consistency: the recursive residual equals C - A X - X B of the returned iterate.
* Planted mistakes (a wrong sign in GPBiCG's two-term minimization, a dropped beta term in CGS)
  must fail these pins.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import direct, factored, factored_more, matrix_oriented
from workloads import stencils


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def _problem(method, s=2, seed=31, lyapunov=False):
    pe = 0.0 if method == "cr" else 10.0
    A = stencils.cd2d(7, 6, pe)
    B = None if lyapunov else stencils.cd1d(9, pe)
    return stencils.make_problem(f"more_{method}", A, B, s, seed, lyapunov=lyapunov,
                                 method=method)


def _kron(p):
    F = sp.csr_matrix(direct.kron_matrix(p.A, p.B))
    c = (p.C1 @ p.C2.T).reshape(-1, order="F")
    return F, c


def _vec(X):
    return X.reshape(-1, order="F")


MATRIX = {"cr": matrix_oriented.matrix_cr, "cgs": matrix_oriented.matrix_cgs,
          "gpbicg": matrix_oriented.matrix_gpbicg}


def _iterates(fn, p, k):
    """Matrix-oriented iterates X_1 .. X_k (k separate runs capped at 1..k iterations)."""
    return [fn(p.A, p.B, p.C1, p.C2, 0.0, j)[0] for j in range(1, k + 1)]


def test_matrix_cgs_matches_scipy_cgs():
    p = _problem("cgs")
    F, c = _kron(p)
    xs = []
    spla.cgs(F, c, x0=np.zeros_like(c), rtol=1e-300, maxiter=10, callback=lambda x: xs.append(x.copy()))
    mine = _iterates(matrix_oriented.matrix_cgs, p, len(xs))
    for x, X in zip(xs, mine):
        assert _rel(_vec(X), x) < 1e-10


def test_matrix_cr_matches_scipy_minres():
    p = _problem("cr")
    F, c = _kron(p)
    xs = []
    spla.minres(F, c, x0=np.zeros_like(c), rtol=1e-300, maxiter=12,
                callback=lambda x: xs.append(x.copy()))
    mine = _iterates(matrix_oriented.matrix_cr, p, len(xs))
    for x, X in zip(xs, mine):
        assert _rel(_vec(X), x) < 1e-8


def test_gpbicg_with_eta_zero_is_bicgstab():
    p = _problem("gpbicg")
    Xg, gi = matrix_oriented.matrix_gpbicg(p.A, p.B, p.C1, p.C2, 1e-10, 40, eta_zero=True)
    Xb, bi = matrix_oriented.matrix_bicgstab(p.A, p.B, p.C1, p.C2, 1e-10, 40)
    assert gi["iters"] == bi["iters"]
    k = min(15, gi["iters"])
    assert np.allclose(gi["alpha"][:k], bi["alpha"][:k], rtol=1e-10, atol=0)
    assert np.allclose(gi["zeta"][:k], bi["omega"][:k], rtol=1e-10, atol=0)
    assert _rel(Xg, Xb) < 1e-10
    Vf, Xf, Wf, fi = factored_more.factored_gpbicg(p.A, p.B, p.C1, p.C2, tol=1e-10, max_iter=40,
                                                   eta_zero=True)
    Vb, Xbf, Wb, fb = factored.factored_bicgstab(p.A, p.B, p.C1, p.C2, tol=1e-10, max_iter=40)
    assert fi["iters"] == fb["iters"]
    assert _rel(Vf @ Xf @ Wf.T, Vb @ Xbf @ Wb.T) < 1e-10


@pytest.mark.parametrize("method", ["cr", "cgs", "gpbicg"])
def test_factored_equals_matrix_oriented(method):
    p = _problem(method)
    Xm, mi = MATRIX[method](p.A, p.B, p.C1, p.C2, 1e-10, 60)
    V, X, W, fi = factored_more.METHODS[method](p.A, p.B, p.C1, p.C2, tol=1e-10, max_iter=60)
    assert fi["status"] == mi["status"] == factored.CONVERGED
    assert fi["iters"] == mi["iters"]
    keys = ["alpha", "beta", "relres"] + (["zeta", "eta"] if method == "gpbicg" else [])
    k = min(12, fi["iters"] - 1)
    for key in keys:
        a, b = np.asarray(fi[key][:k]), np.asarray(mi[key][:k])
        nz = np.abs(b) > 0
        assert np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz])) < 1e-9, key
    assert _rel(V @ X @ W.T, Xm) < 1e-8


@pytest.mark.parametrize("method", ["cr", "cgs", "gpbicg"])
def test_factored_reaches_the_exact_solution(method):
    p = _problem(method, s=1, seed=33)
    V, X, W, info = factored_more.METHODS[method](p.A, p.B, p.C1, p.C2, tol=1e-12, max_iter=200)
    assert info["status"] == factored.CONVERGED
    Xd = direct.kron_solve(p.A, p.B, p.C1, p.C2)
    kappa = np.linalg.cond(direct.kron_matrix(p.A, p.B))
    assert _rel(V @ X @ W.T, Xd) <= 10 * kappa * 1e-12


@pytest.mark.parametrize("method", ["cr", "cgs", "gpbicg"])
def test_recursive_residual_is_the_true_residual(method):
    """For the first iterations (rounding still negligible) the recursive residual of each
    method equals ||C - A X - X B|| / ||C|| of its iterate: this ties the iterate's update (x,
    z, u recurrences) to the residual's."""
    p = _problem(method)
    C = p.C1 @ p.C2.T
    for k in (1, 2, 5, 8):
        V, X, W, info = factored_more.METHODS[method](p.A, p.B, p.C1, p.C2, tol=0.0, max_iter=k)
        Xf = V @ X @ W.T
        true = np.linalg.norm(C - p.A @ Xf - (p.B.T @ Xf.T).T) / np.linalg.norm(C)
        assert abs(true - info["relres"][-1]) <= 1e-10 * max(true, 1e-3), (k, true)


@pytest.mark.parametrize("method", ["cr", "cgs", "gpbicg"])
def test_lyapunov_equals_sylvester(method):
    pl = _problem(method, s=2, seed=35, lyapunov=True)
    ps = stencils.Problem("sy", pl.A, pl.B, pl.C1, pl.C2, lyapunov=False, method=method)
    fn = factored_more.METHODS[method]
    V1, X1, W1, i1 = fn(pl.A, pl.B, pl.C1, pl.C2, tol=1e-10, max_iter=80, lyapunov=True)
    V2, X2, W2, i2 = fn(ps.A, ps.B, ps.C1, ps.C2, tol=1e-10, max_iter=80)
    assert i1["iters"] == i2["iters"]
    Xa, Xb = V1 @ X1 @ W1.T, V2 @ X2 @ W2.T
    assert _rel(Xa, Xb) < 1e-10 and _rel(Xa, Xa.T) < 1e-10


def test_planted_mistakes_fail(monkeypatch):
    p = _problem("gpbicg")
    _, mi = matrix_oriented.matrix_gpbicg(p.A, p.B, p.C1, p.C2, 1e-10, 60)
    real = matrix_oriented.gpbicg_zeta_eta

    def wrong_sign(tt, yy, ty, yt, ts):
        z, e = real(tt, yy, ty, yt, ts)
        return z, -e

    monkeypatch.setattr(factored_more, "gpbicg_zeta_eta", wrong_sign)
    V, X, W, fi = factored_more.factored_gpbicg(p.A, p.B, p.C1, p.C2, tol=0.0, max_iter=6)
    C = p.C1 @ p.C2.T
    Xf = V @ X @ W.T
    true = np.linalg.norm(C - p.A @ Xf - (p.B.T @ Xf.T).T) / np.linalg.norm(C)
    # the residual recurrence and the iterate disagree, or the scalars leave the pinned ones
    assert (abs(true - fi["relres"][-1]) > 1e-8 * true
            or abs(fi["eta"][2] - mi["eta"][2]) > 1e-6 * abs(mi["eta"][2]))
    monkeypatch.setattr(factored_more, "gpbicg_zeta_eta", real)

    pc = _problem("cgs")
    F, c = _kron(pc)
    xs = []
    spla.cgs(F, c, x0=np.zeros_like(c), rtol=1e-300, maxiter=4, callback=lambda x: xs.append(x.copy()))

    def cgs_dropped_beta(A, B, C1, C2, tol, max_iter):   # P = U + beta Q (beta^2 P term lost)
        C = C1 @ C2.T
        X = np.zeros_like(C)
        R = C.copy()
        U, P, Rt = R.copy(), R.copy(), R.copy()
        rho = matrix_oriented.inner(Rt, R)
        for _ in range(max_iter):
            Vv = matrix_oriented.sylvester_op(A, B, P)
            alpha = rho / matrix_oriented.inner(Rt, Vv)
            Q = U - alpha * Vv
            X = X + alpha * (U + Q)
            R = R - alpha * matrix_oriented.sylvester_op(A, B, U + Q)
            rho_new = matrix_oriented.inner(Rt, R)
            beta = rho_new / rho
            U = R + beta * Q
            P = U + beta * Q
            rho = rho_new
        return X, {}

    bad = cgs_dropped_beta(pc.A, pc.B, pc.C1, pc.C2, 0.0, 3)[0]
    assert _rel(_vec(bad), xs[2]) > 1e-6
