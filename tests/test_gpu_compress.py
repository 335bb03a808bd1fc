"""GPU solution compression (sylv_compress / sylv_get_compressed) against the dense truncated SVD
of the same factored solution (Eckart-Young; the oracle's rule in oracle/compress.py)."""
import numpy as np
import pytest

from oracle import compress
from workloads import stencils

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sylv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_28274_amd import sylv as _s
    return _s


def _solved(sylv, case):
    if case == "sylv_cg":
        p = stencils.make_problem("c", stencils.cd2d(24, 20), stencils.cd1d(300), 2, 81,
                                  method="cg")
        code, tol = sylv.SYLV_METHOD_CG, 1e-10
    elif case == "bicgstab":
        p = stencils.make_problem("b", stencils.cd2d(24, 20, 8.0), stencils.cd1d(300, 8.0), 2, 82,
                                  method="bicgstab")
        code, tol = sylv.SYLV_METHOD_BICGSTAB, 1e-10
    else:
        p = stencils.make_problem("l", stencils.cd2d(40, 40), None, 1, 83, lyapunov=True,
                                  method="cg")
        code, tol = sylv.SYLV_METHOD_CG, 1e-10
    slv = sylv.Solver(p.A, p.B, p.C1, p.C2, lyapunov=p.lyapunov, method=code, max_iter=400)
    res = slv.solve(tol)
    assert res.status == sylv.SYLV_OK
    return p, slv


@pytest.mark.parametrize("case", ["sylv_cg", "bicgstab", "lyap_cg"])
@pytest.mark.parametrize("rel_tol", [1e-3, 1e-6, 1e-9])
def test_compression_matches_dense_truncated_svd(sylv, case, rel_tol):
    p, slv = _solved(sylv, case)
    V, X, W = (t.cpu().numpy() for t in slv.get_factors())
    Xd = V @ X @ W.T
    sd = np.linalg.svd(Xd, compute_uv=False)
    st, Z1, sig, Z2, err = slv.compress(rel_tol)
    assert st == sylv.SYLV_OK
    Z1, sig, Z2 = Z1.cpu().numpy(), sig.cpu().numpy(), Z2.cpu().numpy()
    k = sig.size
    assert abs(k - compress.truncation_rank(sd, rel_tol)) <= 1, (k, rel_tol)
    assert np.all(np.diff(sig) <= 0)
    assert np.allclose(sig, sd[:k], rtol=1e-7, atol=1e-10 * sd[0])
    Xk = (Z1 * sig) @ Z2.T
    true_err = np.linalg.norm(Xd - Xk) / np.linalg.norm(Xd)
    assert true_err <= rel_tol * (1 + 1e-6)
    assert abs(true_err - err) <= 1e-6 * max(err, 1e-12) + 1e-13
    slv.close()


def test_rank_cap_and_states(sylv):
    p, slv = _solved(sylv, "sylv_cg")
    st, Z1, sig, Z2, err = slv.compress(1e-12, max_rank=3)
    assert st == sylv.SYLV_NOT_CONVERGED and sig.numel() == 3 and err > 1e-12
    V, X, W = (t.cpu().numpy() for t in slv.get_factors())
    sd = np.linalg.svd(V @ X @ W.T, compute_uv=False)
    assert np.allclose(sig.cpu().numpy(), sd[:3], rtol=1e-9)
    slv.solve(1e-10)  # a new solve discards the compression
    with pytest.raises(sylv.SylvError) as ei:
        sylv.sylv_get_compressed(slv.ctx)
    assert ei.value.code == sylv.SYLV_ERR_STATE
    slv.close()
