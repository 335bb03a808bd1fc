"""The true-residual evaluation with its Gram blocks in split BF16 (gram_precision 1: blocks
with a basis-defect operand; 2: every block) against the FP64 evaluation of the same iterate and
against a dense evaluation, and the verified stopping rule (verify = 1): a converged solve
reports its true residual, and a solve whose true residual misses the tolerance is not reported
as converged."""
import numpy as np
import pytest

from workloads import stencils

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sylv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_28274_amd import sylv as _s
    return _s


def dense_rel_residual(p, Xf):
    C = p.C1 @ p.C2.T
    return np.linalg.norm(C - p.A @ Xf - (p.B.T @ Xf.T).T) / np.linalg.norm(C)


def _problem(case):
    if case == "lyap_cg":
        return stencils.make_problem("ly", stencils.cd2d(48, 40), None, 2, 71, lyapunov=True,
                                     method="cg"), "cg", 1e-9, 400
    if case == "sylv_cg":
        return stencils.make_problem("sc", stencils.cd2d(40, 36), stencils.cd1d(900), 3, 72,
                                     method="cg"), "cg", 1e-9, 400
    if case == "sylv_bicgstab":
        return stencils.make_problem("sb", stencils.cd2d(36, 30, 10.0),
                                     stencils.cd1d(1500, 10.0), 2, 73,
                                     method="bicgstab"), "bicgstab", 1e-9, 200
    if case == "large":
        # 1500 iterations of Lyapunov CG on 30000 rows (two row chunks): the FP64 blocks of the
        # stacked Gram (1501 and 1502 columns: 300 tiles of 128 x 128) run as one launch per
        # chunk over a table of the three products
        return stencils.make_problem("lg", stencils.cd1d(30000), None, 1, 76, lyapunov=True,
                                     method="cg"), "cg", 1e-300, 1500
    # unconverged: residual far above rounding, hundreds of stacked columns
    return stencils.make_problem("un", stencils.cd1d(2500), None, 2, 74, lyapunov=True,
                                 method="cg"), "cg", 1e-14, 250


@pytest.mark.parametrize("case", ["lyap_cg", "sylv_cg", "sylv_bicgstab", "unconverged", "large"])
def test_split_bf16_residual_grams(sylv, case):
    p, method, tol, cap = _problem(case)
    code = sylv.SYLV_METHOD_CG if method == "cg" else sylv.SYLV_METHOD_BICGSTAB
    rels = {}
    for gp in (0, 1, 2):
        slv = sylv.Solver(p.A, p.B, p.C1, p.C2, lyapunov=p.lyapunov, method=code, max_iter=cap,
                          gram_precision=gp, verify=0)
        res = slv.factored_cg(tol) if method == "cg" else slv.factored_bicgstab(tol)
        rels[gp] = slv.residual_norm()[1]
        if gp == 0:
            dense = None
            if p.n <= 5000:  # the dense residual of the large case would take 7 GB
                V, X, W = (t.cpu().numpy() for t in slv.get_factors())
                dense = dense_rel_residual(p, V @ X @ W.T)
            iters = res.iters
        else:
            assert res.iters == iters  # the solve itself is the same
        slv.close()
    if dense is not None:
        assert abs(rels[0] - dense) <= 1e-6 * dense + 1e-14, (rels[0], dense)
    # defect blocks in split BF16: their share of ||R||^2 is tiny, so the norm stays FP64-close
    assert abs(rels[1] - rels[0]) <= 1e-6 * rels[0], (rels[1], rels[0])
    # every block in split BF16: about 1e-5 relative per Gram entry
    assert abs(rels[2] - rels[0]) <= 1e-4 * rels[0], (rels[2], rels[0])


def test_verified_solve_reports_true_residual(sylv):
    p = stencils.make_problem("vf", stencils.cd2d(30, 30), stencils.cd1d(400), 2, 75,
                              method="cg")
    slv = sylv.Solver(p.A, p.B, p.C1, p.C2, method=sylv.SYLV_METHOD_CG, max_iter=300)
    res = slv.factored_cg(1e-8)
    assert res.status == sylv.SYLV_OK
    assert 0 < res.rel_res_true <= 1e-8
    assert slv.residual_norm()[1] == res.rel_res_true
    V, X, W = (t.cpu().numpy() for t in slv.get_factors())
    assert abs(dense_rel_residual(p, V @ X @ W.T) - res.rel_res_true) <= 1e-6 * 1e-8
    slv.close()


def test_verified_solve_rejects_a_true_residual_above_tol(sylv):
    """FP32 bases without refinement: the recursive residual reaches the tolerance, but the true
    residual stays at the FP32 floor above it, so the verified solve must not report success."""
    p = stencils.make_problem("fl", stencils.cd2d(40, 40, 10.0), stencils.cd1d(800, 10.0), 2, 76,
                              method="bicgstab")
    tol = 1e-11
    slv = sylv.Solver(p.A, p.B, p.C1, p.C2, method=sylv.SYLV_METHOD_BICGSTAB, max_iter=300,
                      precision=sylv.SYLV_MIXED_FP32, verify=1)
    res = slv.factored_bicgstab(tol)
    rel = slv.residual_norm()[1]
    if res.status == sylv.SYLV_OK:
        assert res.rel_res_true <= tol and rel <= tol
    else:
        assert res.status == sylv.SYLV_NOT_CONVERGED
        assert rel > tol and res.rel_res_true == rel
    slv.close()
    slv = sylv.Solver(p.A, p.B, p.C1, p.C2, method=sylv.SYLV_METHOD_BICGSTAB, max_iter=300,
                      precision=sylv.SYLV_MIXED_FP32, verify=0)
    res0 = slv.factored_bicgstab(tol)
    # without verification the recursive test alone decides, and the true residual misses tol
    assert res0.status == sylv.SYLV_OK and res0.rel_res_true < 0
    assert slv.residual_norm()[1] > tol
    slv.close()


def test_bf16split_precision_equals_split_grams(sylv):
    """precision = SYLV_MIXED_BF16SPLIT is FP64 bases with the split-BF16 residual Grams of
    gram_precision 1: the same solve and the same residual norm, bit for bit."""
    p, method, tol, cap = _problem("sylv_cg")
    out = []
    for kw in (dict(precision=sylv.SYLV_MIXED_BF16SPLIT), dict(gram_precision=1)):
        slv = sylv.Solver(p.A, p.B, p.C1, p.C2, lyapunov=p.lyapunov, method=sylv.SYLV_METHOD_CG,
                          max_iter=cap, verify=0, **kw)
        res = slv.factored_cg(tol)
        out.append((res.status, res.iters, slv.residual_norm()[1]))
        slv.close()
    assert out[0] == out[1]
