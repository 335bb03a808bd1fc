"""The oracle's own rounding sensitivity on the 2D 128^2 x 1D 8192 BiCGSTAB workload.

Section 5.1 (Example 2) observes that two BiCGSTAB runs of the same problem agree early and
part later as their rounding errors propagate differently. The GPU parity test for this
workload compares iteration counts within 1.5 times the spread the oracle itself shows when
every entry of C1 is moved by about one unit in its last place. That spread is stored in
tests/golden/c2_bicgstab_spread.json (four seeds, written by make_golden.py with two BLAS
threads per run); this test checks that the stored spread is real (rounding-size input changes
move the count to 1e-6 by more than a few iterations while the early scalars still agree to
1e-10) and reruns one seed on the CPU: the rerun's counts must fall inside the band the GPU test
allows. The rerun need not repeat the stored counts exactly: the oracle's dense products are
summed in an order that depends on the BLAS thread count, which is itself a rounding-size
change of the same kind."""
import json
import os

import numpy as np
import pytest

from oracle import factored
from workloads import configs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load():
    with open(os.path.join(GOLDEN, "c2_bicgstab_spread.json")) as f:
        return json.load(f)


def test_stored_spread_is_consistent():
    sp = _load()
    with open(os.path.join(GOLDEN, "c2_bicgstab_oracle.json")) as f:
        base = json.load(f)
    rr = np.asarray(base["relres"])
    assert sp["base"]["k8"] == base["iters"] == len(rr)
    assert sp["base"]["k6"] == int(np.argmax(rr <= 1e-6)) + 1
    d6 = [abs(r["k6"] - sp["base"]["k6"]) for r in sp["runs"]]
    d8 = [abs(r["k8"] - sp["base"]["k8"]) for r in sp["runs"]]
    assert max(d6) >= 5 and max(d8) >= 1
    for r in sp["runs"]:
        assert r["status"] == factored.CONVERGED and r["k8"] == r["iters"]
        a, b = np.asarray(r["alpha12"]), np.asarray(base["alpha"][:12])
        assert np.max(np.abs(a - b) / np.abs(b)) < 1e-10


@pytest.mark.slow
def test_perturbed_rerun_reproduces_stored_spread():
    sp = _load()
    run = sp["runs"][0]
    p = configs.c2_bicgstab()
    z = np.random.default_rng(run["seed"]).standard_normal(p.C1.shape)
    C1 = p.C1 + np.spacing(np.abs(p.C1)) * z
    assert 0 < np.max(np.abs(C1 - p.C1) / np.abs(p.C1)) < 1e-14
    _, _, _, info = factored.factored_bicgstab(p.A, p.B, C1, p.C2, tol=p.tol,
                                               max_iter=p.max_iter)
    rr = np.asarray(info["relres"])
    base = sp["base"]
    d6 = max(abs(r["k6"] - base["k6"]) for r in sp["runs"])
    d8 = max(abs(r["k8"] - base["k8"]) for r in sp["runs"])
    k6 = int(np.argmax(rr <= 1e-6)) + 1
    assert info["status"] == factored.CONVERGED
    assert abs(k6 - base["k6"]) <= int(np.ceil(1.5 * d6)), (k6, base["k6"], d6)
    assert abs(info["iters"] - base["k8"]) <= int(np.ceil(1.5 * d8)), (info["iters"], d8)
    a, b = np.asarray(info["alpha"][:12]), np.asarray(run["alpha12"])
    assert np.max(np.abs(a - b) / np.abs(b)) < 1e-10
