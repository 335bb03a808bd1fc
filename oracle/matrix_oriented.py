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


# ---- other Krylov methods in matrix-oriented form (Section 4's remark that the factorization
# applies to further Krylov methods, and Section 6). Same conventions: X0 = 0, R~0 = R0, the
# stopping test ||R_{k+1}|| <= tol ||R0||, info lists per iteration.

def matrix_cr(A, B, C1, C2, tol, max_iter):
    """Conjugate residual method (Stiefel) for a symmetric operator F: with S = F(R) and
    Q = F(P) kept by recurrence, alpha = <R, S> / <Q, Q>, X += alpha P, R -= alpha Q,
    beta = <R_new, S_new> / <R, S>, P = R + beta P, Q = S + beta Q. It minimizes the residual
    norm over the Krylov space, like MINRES."""
    C = C1 @ C2.T
    X = np.zeros_like(C)
    R = C.copy()
    S = sylvester_op(A, B, R)
    P, Q = R.copy(), S.copy()
    rho = inner(R, S)
    nr0 = np.linalg.norm(R)
    info = {"alpha": [], "beta": [], "rho": [rho], "relres": [], "status": 1, "iters": 0}
    for k in range(max_iter):
        qq = inner(Q, Q)
        if qq == 0.0 or rho == 0.0:
            info["status"] = 2
            break
        alpha = rho / qq
        X = X + alpha * P
        R = R - alpha * Q
        rel = np.linalg.norm(R) / nr0
        info["alpha"].append(alpha)
        info["relres"].append(rel)
        info["iters"] = k + 1
        if rel <= tol:
            info["status"] = 0
            break
        S = sylvester_op(A, B, R)
        rho_new = inner(R, S)
        beta = rho_new / rho
        info["beta"].append(beta)
        info["rho"].append(rho_new)
        P = R + beta * P
        Q = S + beta * Q
        rho = rho_new
    return X, info


def matrix_cgs(A, B, C1, C2, tol, max_iter):
    """Conjugate gradient squared (Sonneveld), two operator applications per iteration:
    V = F(P), alpha = rho / <R~0, V>, Q = U - alpha V, X += alpha (U + Q), R -= alpha F(U + Q),
    beta = rho_new / rho, U = R + beta Q, P = U + beta (Q + beta P)."""
    C = C1 @ C2.T
    X = np.zeros_like(C)
    R = C.copy()
    Rt = R.copy()
    U, P = R.copy(), R.copy()
    rho = inner(Rt, R)
    nr0 = np.linalg.norm(R)
    info = {"alpha": [], "beta": [], "rho": [rho], "relres": [], "status": 1, "iters": 0}
    for k in range(max_iter):
        V = sylvester_op(A, B, P)
        den = inner(Rt, V)
        if den == 0.0 or rho == 0.0:
            info["status"] = 2
            break
        alpha = rho / den
        Q = U - alpha * V
        Wm = U + Q
        X = X + alpha * Wm
        R = R - alpha * sylvester_op(A, B, Wm)
        rel = np.linalg.norm(R) / nr0
        info["alpha"].append(alpha)
        info["relres"].append(rel)
        info["iters"] = k + 1
        if rel <= tol:
            info["status"] = 0
            break
        rho_new = inner(Rt, R)
        beta = rho_new / rho
        info["beta"].append(beta)
        info["rho"].append(rho_new)
        U = R + beta * Q
        P = U + beta * (Q + beta * P)
        rho = rho_new
    return X, info


def gpbicg_zeta_eta(tt, yy, ty, yt, ts):
    """The two-term minimization of GPBiCG: zeta, eta minimize ||T - eta Y - zeta F(T)|| over the
    pair, from the inner products tt = <FT, FT>, yy = <Y, Y>, ty = <FT, Y>, yt = <Y, T>,
    ts = <FT, T> (T the intermediate residual t_n, FT = F(t_n))."""
    den = tt * yy - ty * ty
    zeta = (yy * ts - yt * ty) / den
    eta = (tt * yt - ty * ts) / den
    return zeta, eta


def matrix_gpbicg(A, B, C1, C2, tol, max_iter, eta_zero=False):
    """Generalized product-type BiCG (Zhang): residual r_{n+1} = t_n - eta_n y_n - zeta_n F(t_n)
    with a two-parameter minimization per step (eta_n = 0 and zeta_n = <Ft, t>/<Ft, Ft> on the
    first step, or throughout with eta_zero, which gives BiCGSTAB)."""
    C = C1 @ C2.T
    X = np.zeros_like(C)
    R = C.copy()
    Rt = R.copy()
    nr0 = np.linalg.norm(R)
    rho = inner(Rt, R)
    Z = np.zeros_like(C)
    Pm = np.zeros_like(C)   # p_{n-1}
    Um = np.zeros_like(C)   # u_{n-1}
    Tm = np.zeros_like(C)   # t_{n-1}
    Wm = np.zeros_like(C)   # w_{n-1}
    beta = 0.0
    info = {"alpha": [], "zeta": [], "eta": [], "beta": [], "relres": [], "status": 1,
            "iters": 0}
    for k in range(max_iter):
        P = R + beta * (Pm - Um)
        AP = sylvester_op(A, B, P)
        den = inner(Rt, AP)
        if den == 0.0 or rho == 0.0:
            info["status"] = 2
            break
        alpha = rho / den
        Y = Tm - R - alpha * Wm + alpha * AP
        T = R - alpha * AP
        AT = sylvester_op(A, B, T)
        tt, ts = inner(AT, AT), inner(AT, T)
        if k == 0 or eta_zero:
            if tt == 0.0:
                info["status"] = 2
                break
            zeta, eta = ts / tt, 0.0
        else:
            zeta, eta = gpbicg_zeta_eta(tt, inner(Y, Y), inner(AT, Y), inner(Y, T), ts)
        if zeta == 0.0 or not np.isfinite(zeta) or not np.isfinite(eta):
            info["status"] = 2
            break
        U = zeta * AP + eta * (Tm - R + beta * Um)
        Z = zeta * R + eta * Z - alpha * U
        X = X + alpha * P + Z
        Rn = T - eta * Y - zeta * AT
        rel = np.linalg.norm(Rn) / nr0
        info["alpha"].append(alpha)
        info["zeta"].append(zeta)
        info["eta"].append(eta)
        info["relres"].append(rel)
        info["iters"] = k + 1
        if rel <= tol:
            info["status"] = 0
            break
        rho_new = inner(Rt, Rn)
        beta = (alpha / zeta) * (rho_new / rho)
        info["beta"].append(beta)
        Wm = AT + beta * AP
        Pm, Um, Tm, R, rho = P, U, T, Rn, rho_new
    return X, info
