"""GPU parity against the CPU FP64 oracle on the code paths that the large workloads run.

* Bases of more than 2048 rows take the block Lanczos step as separate kernels (SpMM with the
  local three-term update, CholQR2, the ring of compact blocks and its flush into the basis)
  instead of the one-launch step of small problems; bases of 16384+ rows in total also move the
  Krylov steps to a second stream one iteration ahead of the core recurrences.
* Full-size windows: the first 100 iterations of factored CG on the 1024^2 Lyapunov workload
  and the first 20 iterations of factored BiCGSTAB on the 3D 64^3 x 2D 256^2 workload (s = 4),
  against oracle runs stored by tests/golden/make_golden.py.

Tolerances. Both sides are FP64 but round differently (CholQR2 against Householder QR, CGS2
against MGS2, other summation orders). The yardstick is the oracle's own sensitivity to
rounding: the stored windows hold the relative change of every scalar when each entry of C1 is
moved by about one unit in its last place. A GPU scalar must agree with the oracle to
max(1e-10, 1e3 x that change): the GPU injects rounding-size differences at every operation
rather than once in the input, and the factor 1e3 allows for that. CG (symmetric Lanczos) is
insensitive (the change stays near 1e-15 for 100 iterations, so 1e-10 applies throughout);
BiCGSTAB amplifies it about tenfold per iteration after the first few (Section 5.1, Example 2
observes the same late divergence between two implementations).
"""
import json
import os

import numpy as np
import pytest

from oracle import factored, residual
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


def gpu_solve(sylv, p, method, tol, max_iter, **kw):
    code = sylv.SYLV_METHOD_CG if method == "cg" else sylv.SYLV_METHOD_BICGSTAB
    slv = sylv.Solver(p.A, p.B, p.C1, p.C2, lyapunov=p.lyapunov, method=code, max_iter=max_iter,
                      **kw)
    res = slv.factored_cg(tol) if method == "cg" else slv.factored_bicgstab(tol)
    return res, slv


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def relmax(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b) / np.abs(b)))


def sketch_of(slv, rows, Om):
    V, X, W = slv.get_factors()
    Omt = torch.as_tensor(Om, device=V.device)
    return (V[torch.as_tensor(rows, device=V.device)] @ (X @ (W.T @ Omt))).cpu().numpy()


def lap2d_extremes(nx, ny):
    """Smallest and largest eigenvalue of the unit-coefficient 2D Dirichlet Laplacian on an
    nx x ny grid (sums of the 1D eigenvalues 2 - 2 cos(j pi / (N + 1)))."""
    e = lambda N, j: 2.0 - 2.0 * np.cos(j * np.pi / (N + 1))  # noqa: E731
    return e(nx, 1) + e(ny, 1), e(nx, nx) + e(ny, ny)


def kappa_sum(ea, eb):
    """Condition number of I (x) A + B^T (x) I for symmetric positive definite A, B with
    extreme eigenvalues ea, eb: the ratio of the extreme eigenvalues lambda_i + mu_j."""
    return (ea[1] + eb[1]) / (ea[0] + eb[0])


@pytest.mark.parametrize("case", ["lyapunov_64x64_s2", "sylvester_64x64_112x112_s2"])
def test_large_basis_cg_vs_oracle(sylv, case):
    """Factored CG (Algorithm 4.1) on bases of 4096 rows (Lyapunov, Section 4.3) and of
    4096 + 12544 rows (Sylvester; the Krylov steps then run on the second stream)."""
    A = stencils.cd2d(64, 64)
    if case.startswith("lyapunov"):
        p = stencils.make_problem("ly64", A, None, 2, 61, lyapunov=True, method="cg")
        kap = kappa_sum(lap2d_extremes(64, 64), lap2d_extremes(64, 64))
    else:
        p = stencils.make_problem("sy64", A, stencils.cd2d(112, 112), 2, 62, method="cg")
        kap = kappa_sum(lap2d_extremes(64, 64), lap2d_extremes(112, 112))
    tol, cap = 1e-8, 600
    res, slv = gpu_solve(sylv, p, "cg", tol, cap)
    Vo, Xo, Wo, info = factored.solve(p, tol=tol, max_iter=cap)
    assert res.status == sylv.SYLV_OK and info["status"] == factored.CONVERGED
    # CG's histories are stable under rounding here (Lanczos on both sides): counts within one
    assert abs(res.iters - info["iters"]) <= 1, (res.iters, info["iters"])
    h = slv.get_history()
    for key in ("alpha", "beta", "relres"):
        assert relmax(h[key][:30], info[key][:30]) < 1e-10, key
    k = min(res.iters, info["iters"])
    assert np.max(np.abs(np.log(h["relres"][:k] / np.asarray(info["relres"][:k])))) < 0.05
    # solutions: both satisfy ||R|| <= tol ||C|| up to the recursive/true gap, so they differ
    # by at most about 2 kappa tol relative
    V, X, W = (t.cpu().numpy() for t in slv.get_factors())
    Om = residual.sketch_matrix(p.m, 8, 7)
    Sg, So = residual.sketch(V, X, W, Om), residual.sketch(Vo, Xo, Wo, Om)
    assert rel(Sg, So) <= 2 * kap * tol, (rel(Sg, So), kap)
    _, rr = slv.residual_norm()
    _, ro = residual.factored_residual(p.A, p.B, p.C1, p.C2, Vo, Xo, Wo)
    assert rr <= 1.1 * tol and abs(rr - ro) <= 0.5 * tol, (rr, ro)
    slv.close()


def test_s4_bicgstab_vs_oracle(sylv):
    """Factored BiCGSTAB (Algorithm 4.2) with s = 4 on a 2D 48^2 x 1D 2000 convection-diffusion
    problem: the multi-kernel block Arnoldi sweeps with four-column blocks."""
    A, B = stencils.cd2d(48, 48, 10.0), stencils.cd1d(2000, 10.0)
    p = stencils.make_problem("s4", A, B, 4, 63, method="bicgstab")
    tol, cap = 1e-8, 300
    res, slv = gpu_solve(sylv, p, "bicgstab", tol, cap)
    Vo, Xo, Wo, info = factored.solve(p, tol=tol, max_iter=cap)
    assert res.status == sylv.SYLV_OK and info["status"] == factored.CONVERGED
    h = slv.get_history()
    for key in ("alpha", "omega", "relres"):
        assert relmax(h[key][:6], info[key][:6]) < 1e-10, key
    assert abs(res.iters - info["iters"]) <= max(3, round(0.15 * info["iters"]))
    Om = residual.sketch_matrix(p.m, 8, 7)
    V, X, W = (t.cpu().numpy() for t in slv.get_factors())
    assert rel(residual.sketch(V, X, W, Om), residual.sketch(Vo, Xo, Wo, Om)) < 1e-5
    _, rr = slv.residual_norm()
    assert rr <= 1.1 * tol
    slv.close()


def _window(sylv, p, method, gold, keys):
    iters = gold["window"]
    res, slv = gpu_solve(sylv, p, method, 1e-300, iters)
    assert res.status == sylv.SYLV_NOT_CONVERGED and res.iters == iters
    assert res.rank_v == gold["rank"]
    h = slv.get_history()
    spread = gold["perturbed_rel_diff"]
    for key in keys:
        g, o = np.asarray(h[key][:iters]), np.asarray(gold[key][:iters])
        if key == "beta":  # beta of the last iteration is formed only when the solve goes on
            g, o = g[:iters - 1], o[:iters - 1]
        bound = np.maximum(1e-10, 1e3 * np.asarray(spread[key][:g.size]))
        err = np.abs(g - o) / np.abs(o)
        bad = np.nonzero(err > bound)[0]
        assert bad.size == 0, (key, bad[:5].tolist(), err[bad[:5]].tolist())
    Om = np.random.default_rng(gold["sketch_seed"]).standard_normal((p.m, gold["sketch_q"]))
    Sg = sketch_of(slv, np.asarray(gold["sketch_rows"]), Om)
    err = rel(Sg, np.asarray(gold["sketch"]))
    assert err <= max(1e-10, 1e3 * gold["perturbed_sketch_rel"]), err
    slv.close()


def test_c5_lyapunov_cg_window_vs_oracle(sylv):
    """First 100 iterations of factored CG on the 1024^2 Lyapunov workload (n = 1,048,576)."""
    with open(os.path.join(GOLDEN, "c5_lyap_cg_window.json")) as f:
        gold = json.load(f)
    _window(sylv, configs.c5_lyap("cg"), "cg", gold, ("alpha", "beta", "relres"))


def test_c3_bicgstab_window_vs_oracle(sylv):
    """First 20 iterations of factored BiCGSTAB, s = 4, 3D 64^3 x 2D 256^2 (n = 262144,
    m = 65536)."""
    with open(os.path.join(GOLDEN, "c3_bicgstab_window.json")) as f:
        gold = json.load(f)
    _window(sylv, configs.c3_bicgstab(), "bicgstab", gold, ("alpha", "omega", "beta", "relres"))


@pytest.mark.parametrize("nx", [32767, 32768])
def test_narrow_sell_limit_vs_oracle(sylv, nx):
    """The solver's SELL copy of an operator whose values are all exact floats and whose columns
    lie within 32767 of their rows is stored narrow (float values, 16-bit column offsets); one
    column further it is stored wide. A Laplacian on an nx x 2 grid (column offsets +-1 and
    +-nx) sits on both sides of that limit; the first iterations of factored CG (Alg. 4.1)
    against the oracle to 1e-10, and the two forms give the same products bit for bit where
    both apply (the values are exact)."""
    A = stencils.cd2d(nx, 2)
    B = stencils.cd1d(300)
    p = stencils.make_problem("nl", A, B, 1, 81, method="cg")
    iters = 12
    res, slv = gpu_solve(sylv, p, "cg", 1e-300, iters)
    assert res.status == sylv.SYLV_NOT_CONVERGED and res.iters == iters
    _, _, _, info = factored.solve(p, tol=1e-300, max_iter=iters)
    h = slv.get_history()
    for key in ("alpha", "relres"):
        assert relmax(h[key][:iters], info[key][:iters]) < 1e-10, key
    assert relmax(h["beta"][:iters - 1], info["beta"][:iters - 1]) < 1e-10
    slv.close()
