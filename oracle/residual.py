"""Residual norms and sketches of factored solutions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* :func:`dense_residual` forms ``X = V Xc W^T`` and evaluates ``||A X + X B - C1 C2^T||_F``
  (problem statement eq. (1.1)); only for n*m that fits in memory.
* :func:`factored_residual` evaluates the same norm without forming X. The residual is written as
  one product ``L M N^T`` with ``L = [C1, A V, V]``, ``N = [C2, W, B^T W]`` and
  ``M = blkdiag(I, -Xc, -Xc)``; with thin QRs ``L = Q_L R_L``, ``N = Q_N R_N`` its Frobenius norm
  is ``||R_L M R_N^T||_F``.
* :func:`sketch` returns ``X @ Omega = V (Xc (W^T Omega))`` for a seeded Gaussian m x q Omega.
"""
from __future__ import annotations

import numpy as np


def reconstruct(V, Xc, W):
    return V @ Xc @ W.T


def dense_residual(A, B, C1, C2, V, Xc, W):
    """Returns (absolute, relative) Frobenius residual."""
    X = reconstruct(V, Xc, W)
    C = C1 @ C2.T
    Rm = C - A @ X - (B.T @ X.T).T
    a = np.linalg.norm(Rm)
    return a, a / np.linalg.norm(C)


def factored_residual(A, B, C1, C2, V, Xc, W):
    """Returns (absolute, relative) Frobenius residual without forming the n x m solution."""
    s, r = C1.shape[1], Xc.shape[0]
    L = np.hstack([C1, A @ V, V])
    N = np.hstack([C2, B.T @ W, W])
    # L M N^T = C1 C2^T - (A V) Xc W^T - V Xc (B^T W)^T
    M = np.zeros((s + 2 * r, s + 2 * r))
    M[:s, :s] = np.eye(s)
    M[s:s + r, s + r:] = -Xc           # (A V) Xc W^T
    M[s + r:, s:s + r] = -Xc           # V Xc (B^T W)^T
    _, RL = np.linalg.qr(L, mode="reduced")
    _, RN = np.linalg.qr(N, mode="reduced")
    a = np.linalg.norm(RL @ M @ RN.T)
    _, Rc1 = np.linalg.qr(C1, mode="reduced")
    _, Rc2 = np.linalg.qr(C2, mode="reduced")
    c = np.linalg.norm(Rc1 @ Rc2.T)
    return a, a / c


def sketch_matrix(m, q=8, seed=7):
    return np.random.default_rng(seed).standard_normal((m, q))


def sketch(V, Xc, W, Omega):
    return V @ (Xc @ (W.T @ Omega))
