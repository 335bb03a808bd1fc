"""Matrix-oriented CG and BiCGSTAB on the full n x m iterate (Section 2, Algorithms 2.1 and 2.2).

TEST INFRASTRUCTURE ONLY (see the package docstring). FP64, zero initial guess, R~0 = R0.

The vec correspondences of Section 2 give the three operations: addition of n x m matrices,
the trace inner product ``<X, Y> = tr(X^T Y)`` and the Sylvester operator ``X -> A X + X B``.
"""
from __future__ import annotations

import numpy as np


def sylvester_op(A, B, X):
    """``A X + X B`` for sparse A (n x n), B (m x m) and dense X (n x m)."""
    return A @ X + (B.T @ X.T).T


def inner(X, Y) -> float:
    """``<X, Y> = tr(X^T Y)`` (Section 2, inner product)."""
    return float(np.sum(X * Y))


def matrix_cg(A, B, C1, C2, tol, max_iter):
    """Algorithm 2.1 with X0 = 0. Returns (X, info) where info holds the per-iteration alpha,
    beta, rho and relative residual ||R_{k+1}|| / ||R_0||."""
    C = C1 @ C2.T
    X = np.zeros_like(C)
    R = C.copy()  # R0 = C - A X0 - X0 B with X0 = 0
    P = R.copy()
    rho = inner(R, R)
    nr0 = np.sqrt(rho)
    info = {"alpha": [], "beta": [], "rho": [rho], "relres": [], "status": 1, "iters": 0}
    for k in range(max_iter):
        Q = sylvester_op(A, B, P)
        alpha = rho / inner(P, Q)
        X = X + alpha * P
        R = R - alpha * Q
        rel = np.linalg.norm(R) / nr0
        info["alpha"].append(alpha)
        info["relres"].append(rel)
        info["iters"] = k + 1
        if rel <= tol:
            info["status"] = 0
            break
        rho_new = inner(R, R)
        beta = rho_new / rho
        info["beta"].append(beta)
        info["rho"].append(rho_new)
        P = R + beta * P
        rho = rho_new
    return X, info


def matrix_bicgstab(A, B, C1, C2, tol, max_iter):
    """Algorithm 2.2 with X0 = 0 and R~0 = R0. Returns (X, info) with alpha, omega, beta, rho and
    the relative residual per iteration."""
    C = C1 @ C2.T
    X = np.zeros_like(C)
    R = C.copy()
    Rt = R.copy()
    P = R.copy()
    rho = inner(R, Rt)
    nr0 = np.linalg.norm(R)
    info = {"alpha": [], "omega": [], "beta": [], "rho": [rho], "relres": [], "status": 1,
            "iters": 0}
    for k in range(max_iter):
        Q = sylvester_op(A, B, P)
        alpha = rho / inner(Rt, Q)
        S = R - alpha * Q
        T = sylvester_op(A, B, S)
        omega = inner(T, S) / inner(T, T)
        X = X + alpha * P + omega * S
        R = S - omega * T
        rel = np.linalg.norm(R) / nr0
        info["alpha"].append(alpha)
        info["omega"].append(omega)
        info["relres"].append(rel)
        info["iters"] = k + 1
        if rel <= tol:
            info["status"] = 0
            break
        rho_new = inner(R, Rt)
        beta = (alpha / omega) * (rho_new / rho)
        info["beta"].append(beta)
        info["rho"].append(rho_new)
        P = R + beta * (P - omega * Q)
        rho = rho_new
    return X, info
