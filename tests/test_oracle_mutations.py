"""Planted mistakes in the oracle must fail its pins.

Each mutation is a plausible slip (a transposed operand, a dropped term, a wrong sign) applied to
a copy of the oracle's arithmetic on the CPU; the test asserts that the pin it belongs to catches it.
"""
import numpy as np

from oracle import factored, matrix_oriented
from tests.test_oracle_pins import _eq311_error, _equiv_problem


def _core_transposed_G(P, H, G):
    p, q = P.shape[0], H.shape[0]
    Q = np.zeros((q, q))
    Q[:, :p] += H @ P
    Q[:p, :] += P @ G.T[:p, :].T.T if False else (P.T @ G.T)  # P^T instead of P
    return Q


def _core_dropped_term(P, H, G):
    p, q = P.shape[0], H.shape[0]
    Q = np.zeros((q, q))
    Q[:, :p] += H @ P
    return Q


def _core_H_transposed(P, H, G):
    p, q = P.shape[0], H.shape[0]
    Q = np.zeros((q, q))
    Q[:p, :p] += H[:p, :p].T @ P
    Q[:p, :] += P @ G.T
    return Q


def test_mutations_fail_eq311():
    assert _eq311_error(factored.sylvester_core) < 1e-13
    for bad in (_core_transposed_G, _core_dropped_term, _core_H_transposed):
        assert _eq311_error(bad) > 1e-3


def test_mutation_fails_equivalence(monkeypatch):
    p = _equiv_problem("bicgstab")
    _, mi = matrix_oriented.matrix_bicgstab(p.A, p.B, p.C1, p.C2, 1e-8, 50)
    monkeypatch.setattr(factored, "sylvester_core", _core_transposed_G)
    _, _, _, fi = factored.factored_bicgstab(p.A, p.B, p.C1, p.C2, tol=1e-8, max_iter=5)
    assert abs(fi["alpha"][1] - mi["alpha"][1]) > 1e-6 * abs(mi["alpha"][1])


def test_mutation_wrong_pad_sign_fails_equivalence(monkeypatch):
    p = _equiv_problem("cg")
    _, mi = matrix_oriented.matrix_cg(p.A, p.B, p.C1, p.C2, 1e-8, 50)
    real_pad = factored.pad

    def bad_pad(Z, size):   # shifts the old core one block down instead of the upper-left corner
        out = np.zeros((size, size))
        k = Z.shape[0]
        out[size - k:, size - k:] = Z
        return out

    monkeypatch.setattr(factored, "pad", bad_pad)
    _, _, _, fi = factored.factored_cg(p.A, p.B, p.C1, p.C2, tol=1e-8, max_iter=4)
    monkeypatch.setattr(factored, "pad", real_pad)
    assert np.max(np.abs(np.array(fi["alpha"][1:4]) - np.array(mi["alpha"][1:4]))) > 1e-6
