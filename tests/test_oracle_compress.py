"""Pins for the oracle's solution compression (oracle/compress.py): the factored truncation
must equal the truncated SVD of the dense solution X = V Xc W^T (Eckart-Young), whose
singular values are the core's when V and W have orthonormal columns (Corollary 3.3)."""
import numpy as np
import pytest

from oracle import compress, factored
from workloads import configs, stencils


def _solution(kind):
    if kind == "c1":
        p = configs.c1_cg_1d()
        V, X, W, _ = factored.solve(p)
    else:
        p = stencils.make_problem("cb", stencils.cd2d(20, 18, 8.0), stencils.cd1d(150, 8.0), 2, 9,
                                  method="bicgstab")
        V, X, W, _ = factored.solve(p, tol=1e-10, max_iter=200)
    return V, X, W


@pytest.mark.parametrize("kind", ["c1", "bicgstab"])
@pytest.mark.parametrize("rel_tol", [1e-4, 1e-8])
def test_compression_equals_dense_truncated_svd(kind, rel_tol):
    V, X, W = _solution(kind)
    Xd = V @ X @ W.T
    U, sd, Yt = np.linalg.svd(Xd, full_matrices=False)
    Z1, sig, Z2, err = compress.compress(V, X, W, rel_tol)
    k = sig.size
    # the core's singular values are X's (orthonormal bases, to their orthogonality level)
    assert np.allclose(sig, sd[:k], rtol=1e-8, atol=1e-12 * sd[0])
    # same rank as the dense rule, and the same truncated matrix
    assert k == compress.truncation_rank(sd, rel_tol)
    Xk = (Z1 * sig) @ Z2.T
    Xd_k = (U[:, :k] * sd[:k]) @ Yt[:k]
    assert np.linalg.norm(Xk - Xd_k) <= 1e-8 * np.linalg.norm(Xd)
    # the Frobenius error is the singular-value tail and meets the tolerance
    assert abs(np.linalg.norm(Xd - Xk) - err) <= 1e-9 * np.linalg.norm(Xd)
    assert err <= rel_tol * np.linalg.norm(Xd) * (1 + 1e-9)


def test_truncation_rank_rule():
    s = np.array([10.0, 1.0, 0.1, 0.01])
    total = np.sqrt(np.sum(s ** 2))
    assert compress.truncation_rank(s, 0.0) == 4
    assert compress.truncation_rank(s, 1.0) == 0
    assert compress.truncation_rank(s, 0.011 / total) == 3
    assert compress.truncation_rank(s, 0.0099 / total) == 4
    assert compress.truncation_rank(s, 0.2 / total, max_rank=1) == 1
