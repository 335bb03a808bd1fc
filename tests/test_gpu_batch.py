"""GPU checks of batched solves (sylv_batch_*).

* Streams form: every instance, solved over several streams by several host threads, gives
  exactly what it gives when solved alone (same kernels, same order of arithmetic).
* Every form (streams, grouped lock-step launches over instance tables, the same with HIP-graph
  segments): each instance against the CPU oracle's solve of the same problem (Algorithms 4.1,
  4.2), and the true residual of the returned iterate.
* Grouped forms: graph replays are bit-identical to the launched group (same kernels, same
  arguments), at sizes whose bases span many workgroups; instances that cannot join a group run
  beside the groups."""
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


FORMS = {"streams": lambda s: s.SYLV_BATCH_STREAMS, "grouped": lambda s: s.SYLV_BATCH_GROUPED,
         "graph": lambda s: s.SYLV_BATCH_GRAPH}


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


@pytest.mark.parametrize("form", ["streams", "grouped", "graph"])
def test_batch_instances_match_the_oracle(sylv, form):
    """Every instance of a batch against the CPU oracle's solve of the same problem
    (Algorithms 4.1 / 4.2): same iteration count (CG within one; BiCGSTAB within its rounding
    band), the oracle's early scalars to 1e-10, and the same solution, compared through the
    sketch X Omega (both factors, so W of the Lyapunov instance is covered too)."""
    from oracle import factored, residual
    probs = instances()
    tol = 1e-9
    b = sylv.Batch(probs, nstreams=3, form=FORMS[form](sylv))
    if form != "streams":
        assert b.groups() >= 2
    res = b.solve(tol)
    if form == "graph":  # the second solve replays the captured segments
        res = b.solve(tol)
    for i, p in enumerate(probs):
        Vo, Xo, Wo, info = factored.solve(p, tol=tol, max_iter=p.max_iter)
        assert res[i].status == sylv.SYLV_OK and info["status"] == factored.CONVERGED, p.name
        band = 1 if p.method == "cg" else max(3, round(0.15 * info["iters"]))
        assert abs(res[i].iters - info["iters"]) <= band, (p.name, res[i].iters, info["iters"])
        ctx = b.context(i)
        hist = sylv.sylv_get_history(ctx, p.max_iter)
        k = min(5, info["iters"])
        a, o = np.asarray(hist["alpha"][:k]), np.asarray(info["alpha"][:k])
        assert np.max(np.abs(a - o) / np.abs(o)) < 1e-10, p.name
        rv, rw = sylv.sylv_get_factors(ctx)
        Vb = torch.empty((p.n, rv), dtype=torch.float64, device="cuda")
        Xb = torch.empty((rv, rw), dtype=torch.float64, device="cuda")
        Wb = torch.empty((p.m, rw), dtype=torch.float64, device="cuda")
        sylv.sylv_get_factors(ctx, Vb, Xb, Wb)
        V, X, W = Vb.cpu().numpy(), Xb.cpu().numpy(), Wb.cpu().numpy()
        if p.lyapunov:
            assert np.array_equal(V, W)
        Om = residual.sketch_matrix(p.m, 8, 7)
        Sg, So = residual.sketch(V, X, W, Om), residual.sketch(Vo, Xo, Wo, Om)
        # both iterates meet ||R|| <= tol ||C||; these small operators have condition numbers
        # of at most a few thousand, so the solutions agree to about kappa * tol
        assert np.linalg.norm(Sg - So) / np.linalg.norm(So) < 1e-5, p.name
        _, rel = sylv.sylv_residual_norm(ctx)
        _, ro = residual.dense_residual(p.A, p.B, p.C1, p.C2, V, X, W)
        assert rel <= 1.05 * tol and abs(rel - ro) <= 1e-3 * tol, (p.name, rel, ro)
    b.close()


def medium_instances():
    """Instances whose bases span several hundred workgroups (rows 4000-20000), two per group
    key, CG and BiCGSTAB, s = 1, 2, 4, plus a Lyapunov CG pair."""
    out = []
    rng = np.random.default_rng(123)
    for i, (method, s) in enumerate([("cg", 1), ("cg", 1), ("cg", 2), ("cg", 2), ("bicgstab", 1),
                                     ("bicgstab", 1), ("bicgstab", 4), ("bicgstab", 4)]):
        pe = 0.0 if method == "cg" else 8.0
        A = stencils.cd2d(int(rng.integers(64, 140)), int(rng.integers(64, 140)), pe)
        B = stencils.cd1d(int(rng.integers(2000, 6000)), pe)
        out.append(stencils.make_problem(f"m{i}", A, B, s, 700 + i, method=method,
                                         max_iter=1500 if method == "cg" else 600))
    for i in range(2):
        A = stencils.cd2d(int(rng.integers(50, 80)), int(rng.integers(50, 80)), 0.0)
        out.append(stencils.make_problem(f"ml{i}", A, None, 1, 720 + i, lyapunov=True,
                                         method="cg", max_iter=1500))
    return out


def _factors(sylv, ctx, p):
    rv, rw = sylv.sylv_get_factors(ctx)
    V = torch.empty((p.n, rv), dtype=torch.float64, device="cuda")
    X = torch.empty((rv, rw), dtype=torch.float64, device="cuda")
    W = torch.empty((p.m, rw), dtype=torch.float64, device="cuda")
    sylv.sylv_get_factors(ctx, V, X, None if p.lyapunov else W)
    return V, X, W


def test_graph_replays_equal_the_launched_group(sylv):
    """Three graph solves (the first captures, the next two replay, with eager work on the
    device between them) against the grouped form launched kernel by kernel: identical
    iteration counts, recursive residuals and factors, bit for bit; and the streams form (single
    solves) to the same iteration count within one (CG) or its rounding band (BiCGSTAB) and the
    same true-residual bound."""
    probs = medium_instances()
    tol = 1e-8
    g = sylv.Batch(probs, nstreams=2, form=sylv.SYLV_BATCH_GROUPED)
    assert g.groups() == 5
    rg = g.solve(tol)
    ref = [_factors(sylv, g.context(i), p) for i, p in enumerate(probs)]
    gr = sylv.Batch(probs, nstreams=2, form=sylv.SYLV_BATCH_GRAPH)
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        torch.cuda.synchronize()
        rr = gr.solve(tol)
        del junk
        for i, p in enumerate(probs):
            assert rr[i].status == rg[i].status == sylv.SYLV_OK, (rep, p.name)
            assert rr[i].iters == rg[i].iters, (rep, p.name)
            assert rr[i].rel_res_recursive == rg[i].rel_res_recursive, (rep, p.name)
            V, X, W = _factors(sylv, gr.context(i), p)
            assert torch.equal(V, ref[i][0]) and torch.equal(X, ref[i][1]), (rep, p.name)
            if not p.lyapunov:
                assert torch.equal(W, ref[i][2]), (rep, p.name)
    st = sylv.Batch(probs, nstreams=4, form=sylv.SYLV_BATCH_STREAMS)
    rs = st.solve(tol)
    for i, p in enumerate(probs):
        band = 1 if p.method == "cg" else max(3, round(0.15 * rs[i].iters))
        assert abs(rs[i].iters - rg[i].iters) <= band, (p.name, rs[i].iters, rg[i].iters)
        _, rel = sylv.sylv_residual_norm(g.context(i))
        assert rel <= tol, (p.name, rel)
        assert rg[i].rel_res_true == pytest.approx(rel, rel=1e-12)
    for b in (g, gr, st):
        b.close()


def test_grouped_batch_runs_loose_instances_beside_groups(sylv):
    """Instances that cannot join a group (here factored CR and CGS) run in the streams form
    beside the groups and give exactly their single-solve result."""
    probs = instances()[:4]
    A = stencils.cd2d(14, 13, 0.0)
    B = stencils.cd1d(90, 0.0)
    probs.append(stencils.make_problem("loose_cr", A, B, 2, 401, method="cr", max_iter=300))
    A = stencils.cd2d(15, 12, 8.0)
    B = stencils.cd1d(80, 8.0)
    probs.append(stencils.make_problem("loose_cgs", A, B, 1, 402, method="cgs", max_iter=300))
    b = sylv.Batch(probs, nstreams=2, form=sylv.SYLV_BATCH_GRAPH)
    res = b.solve(1e-9)
    assert all(r.status == sylv.SYLV_OK for r in res)
    for i in (4, 5):
        p = probs[i]
        one = sylv.Solver(p.A, p.B, p.C1, p.C2, method=sylv.METHOD_CODES[p.method],
                          max_iter=p.max_iter)
        r1 = one.solve(1e-9)
        assert res[i].iters == r1.iters and res[i].rel_res_recursive == r1.rel_res_recursive
        one.close()
    b.close()
