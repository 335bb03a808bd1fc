"""GPU checks of batched solves (sylv_batch_*): every instance of a batch, solved over several
streams by several host threads, gives exactly what it gives when solved alone (same kernels,
same order of arithmetic), and meets the stopping rule of its method."""
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


def instances():
    out = []
    rng = np.random.default_rng(99)
    for i in range(7):
        cg = i % 2 == 0
        pe = 0.0 if cg else 8.0
        A = stencils.cd2d(int(rng.integers(12, 30)), int(rng.integers(12, 30)), pe)
        B = stencils.cd1d(int(rng.integers(40, 300)), pe) if i % 3 else \
            stencils.cd2d(int(rng.integers(8, 16)), int(rng.integers(8, 16)), pe)
        s = int(rng.choice([1, 2, 4]))
        lyap = i == 5
        p = stencils.make_problem(f"b{i}", A, None if lyap else B, s, 300 + i, lyapunov=lyap,
                                  method="cg" if cg else "bicgstab", max_iter=300)
        out.append(p)
    return out


def test_batch_matches_single_solves(sylv):
    probs = instances()
    b = sylv.Batch(probs, nstreams=3)
    res = b.solve(1e-9)
    for i, p in enumerate(probs):
        code = sylv.SYLV_METHOD_CG if p.method == "cg" else sylv.SYLV_METHOD_BICGSTAB
        one = sylv.Solver(p.A, p.B, p.C1, p.C2, lyapunov=p.lyapunov, method=code,
                          max_iter=p.max_iter)
        r1 = one.factored_cg(1e-9) if p.method == "cg" else one.factored_bicgstab(1e-9)
        assert res[i].status == r1.status == sylv.SYLV_OK, p.name
        assert res[i].iters == r1.iters and res[i].rank_v == r1.rank_v
        assert res[i].rel_res_recursive == r1.rel_res_recursive
        # factors of the batch's context equal the single solve's, bit for bit
        rv, rw = sylv.sylv_get_factors(b.context(i))
        Vb = torch.empty((p.n, rv), dtype=torch.float64, device="cuda")
        Xb = torch.empty((rv, rw), dtype=torch.float64, device="cuda")
        Wb = torch.empty((p.m, rw), dtype=torch.float64, device="cuda")
        sylv.sylv_get_factors(b.context(i), Vb, Xb, None if p.lyapunov else Wb)
        V1, X1, W1 = one.get_factors()
        assert torch.equal(Vb, V1) and torch.equal(Xb, X1)
        _, rel = sylv.sylv_residual_norm(b.context(i))
        assert rel <= 1.05e-9
        one.close()
    b.close()


def test_batch_argument_errors(sylv):
    probs = instances()[:2]
    b = sylv.Batch(probs, nstreams=64)  # more streams than instances: clamped
    res = b.solve(1e-9)
    assert all(r.status == sylv.SYLV_OK for r in res)
    b.close()
    with pytest.raises(sylv.SylvError):
        sylv.Batch(probs, nstreams=0)
