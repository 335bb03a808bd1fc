"""Pins for the truncated CG and BiCGSTAB oracle (Algorithms A.1 and A.2, oracle/truncated.py).

* The low-rank arithmetic against dense arithmetic (sum, operator, inner product) and the
  truncation operator against the dense truncated SVD.
* With a truncation threshold at rounding level the truncated methods are the matrix-oriented
  CG and BiCGSTAB (Algorithms 2.1, 2.2; Section 5.2 notes they are mathematically equivalent to
  the factorized ones except for the truncation): same scalars and residuals over the first
  iterations.
* With the paper's thresholds they converge to the tolerance in about as many iterations as the
  factorized methods (Examples 5.3 and 5.4 observe comparable counts)."""
import numpy as np
import pytest

from oracle import factored, matrix_oriented, truncated
from workloads import stencils


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _random_lr(n, m, r, seed):
    rng = np.random.default_rng(seed)
    return truncated.LowRank(rng.standard_normal((n, r)), rng.standard_normal((r, r)),
                             rng.standard_normal((m, r)))


def test_low_rank_arithmetic_matches_dense():
    A = stencils.cd2d(6, 5, 4.0)
    B = stencils.cd1d(8, 4.0)
    Z1, Z2 = _random_lr(30, 8, 3, 1), _random_lr(30, 8, 2, 2)
    S = truncated.lr_comb((0.7, Z1), (-1.3, Z2))
    assert _rel(S.dense(), 0.7 * Z1.dense() - 1.3 * Z2.dense()) < 1e-14
    F = truncated.lr_op(A, B, Z1)
    assert _rel(F.dense(), A @ Z1.dense() + Z1.dense() @ B.toarray()) < 1e-14
    assert abs(truncated.lr_inner(Z1, Z2) - np.sum(Z1.dense() * Z2.dense())) < 1e-12 * (
        np.linalg.norm(Z1.dense()) * np.linalg.norm(Z2.dense()))
    assert abs(truncated.lr_norm(S) - np.linalg.norm(S.dense())) < 1e-13 * np.linalg.norm(S.dense())


@pytest.mark.parametrize("eps", [3e-3, 3e-7])
def test_truncation_is_the_dense_truncated_svd(eps):
    rng = np.random.default_rng(3)
    # a rank-12 matrix with decaying singular values, given with redundant factors (rank 20)
    U, _ = np.linalg.qr(rng.standard_normal((40, 12)))
    Y, _ = np.linalg.qr(rng.standard_normal((25, 12)))
    s = 10.0 ** -np.arange(12)
    Z = truncated.LowRank(np.hstack([U, U[:, :8]]), np.diag(np.concatenate([s, np.zeros(8)])),
                          np.hstack([Y, Y[:, :8]]))
    Tz = truncated.lr_truncate(Z, eps)
    k = int(np.sum(s > eps * s[0]))
    assert Tz.rank == k
    Ud, sd, Ytd = np.linalg.svd(Z.dense())
    assert _rel(Tz.dense(), (Ud[:, :k] * sd[:k]) @ Ytd[:k]) < 1e-10


def test_truncated_cg_without_truncation_is_matrix_cg():
    p = stencils.make_problem("tc", stencils.cd2d(8, 7), stencils.cd1d(9), 2, 17, method="cg")
    Xm, mi = matrix_oriented.matrix_cg(p.A, p.B, p.C1, p.C2, 1e-10, 60)
    X, ti = truncated.truncated_cg(p.A, p.B, p.C1, p.C2, 1e-10, 60, 1e-15)
    k = 12
    assert np.allclose(ti["alpha"][:k], mi["alpha"][:k], rtol=1e-7)
    assert np.allclose(ti["relres"][:k], mi["relres"][:k], rtol=1e-7)
    assert ti["status"] == truncated.CONVERGED and abs(ti["iters"] - mi["iters"]) <= 1
    assert _rel(X.dense(), Xm) < 1e-8


@pytest.mark.parametrize("variant", [1, 2])
def test_truncated_bicgstab_without_truncation_is_matrix_bicgstab(variant):
    p = stencils.make_problem("tb", stencils.cd2d(8, 7, 10.0), stencils.cd1d(9, 10.0), 2, 18,
                              method="bicgstab")
    Xm, mi = matrix_oriented.matrix_bicgstab(p.A, p.B, p.C1, p.C2, 1e-10, 60)
    X, ti = truncated.truncated_bicgstab(p.A, p.B, p.C1, p.C2, 1e-10, 60, 1e-15, variant=variant)
    k = 8
    assert np.allclose(ti["alpha"][:k], mi["alpha"][:k], rtol=1e-7)
    assert np.allclose(ti["omega"][:k], mi["omega"][:k], rtol=1e-7)
    assert np.allclose(ti["relres"][:k], mi["relres"][:k], rtol=1e-6)
    assert ti["status"] == truncated.CONVERGED
    assert _rel(X.dense(), Xm) < 1e-7


@pytest.mark.parametrize("method", ["cg", "bicgstab"])
@pytest.mark.parametrize("eps", [1e-8, 1e-12])
def test_truncated_counts_close_to_factored(method, eps):
    pe = 0.0 if method == "cg" else 10.0
    A = stencils.cd2d(20, 20, pe)
    if method == "cg":
        p = stencils.make_problem("lc", A, None, 2, 19, lyapunov=True, method="cg")
        X, ti = truncated.truncated_cg(p.A, p.B, p.C1, p.C2, 1e-6, 300, eps)
    else:
        p = stencils.make_problem("lb", A, stencils.cd1d(300, pe), 2, 20, method="bicgstab")
        X, ti = truncated.truncated_bicgstab(p.A, p.B, p.C1, p.C2, 1e-6, 300, eps)
    V, Xc, W, fi = factored.solve(p, method=method, tol=1e-6, max_iter=300)
    assert ti["status"] == truncated.CONVERGED
    assert abs(ti["iters"] - fi["iters"]) <= max(3, round(0.15 * fi["iters"]))
    C = p.C1 @ p.C2.T
    Xd = X.dense()
    true = np.linalg.norm(C - p.A @ Xd - (p.B.T @ Xd.T).T) / np.linalg.norm(C)
    assert true <= 1e-6 * 1.5
