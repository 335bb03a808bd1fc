"""Further factorized Krylov methods for ``A X + X B = C1 C2^T`` in FP64 on the CPU: conjugate
residual (CR), conjugate gradient squared (CGS) and generalized product-type BiCG (GPBiCG).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4 notes that the factorization carries over to other Krylov methods and Section 6 names
CR, CGS and GPBiCG among them. Each method here is its matrix-oriented form (``matrix_oriented``)
with every iterate kept as ``Z = V Zc W^T`` (Corollary 3.3): sums act on the cores (eq. (3.9),
the zero padding of smaller cores implicit), inner products are core inner products
(eq. (3.10)) and each operator application is the core product of eq. (3.11), which needs one
more block of each basis. CR needs a symmetric operator and uses the block Lanczos bases of
Algorithm 4.1; CGS and GPBiCG apply the operator twice per iteration and use the block Arnoldi
bases of Algorithm 4.2. The same readings as in ``factored`` hold (block QR with
``diag(R) >= 0``, closure rule, zero initial guess, ``R~0 = R0``, stopping test
``||R_{k+1}|| <= tol ||R_0||``, last iterate kept at a breakdown or at ``max_iter``).
"""
from __future__ import annotations

import numpy as np

from .factored import BREAKDOWN, CONVERGED, NOT_CONVERGED, _bases, inner, pad, sylvester_core
from .matrix_oriented import gpbicg_zeta_eta


def _out(V, W, X, s, A, B):
    nb = X.shape[0] // s
    return (V.basis(nb) if nb else np.zeros((A.shape[0], 0)), X,
            W.basis(nb) if nb else np.zeros((B.shape[0], 0)))


class _Side:
    """Both bases grown together (one basis for a Lyapunov problem)."""

    def __init__(self, V, W, lyapunov):
        self.V, self.W, self.lyapunov = V, W, lyapunov

    def step(self):
        self.V.step()
        if not self.lyapunov:
            self.W.step()

    def op(self, Z):
        """eq. (3.11) on a core of size p (= its rows): (p+s) x (p+s), stepping the bases when
        they have fewer than p + s columns."""
        p = Z.shape[0]
        s = self.V.s
        while self.V.nblocks * s < p + s:
            self.step()
        return sylvester_core(Z, self.V.H(p + s, p), self.W.H(p + s, p))


def factored_cr(A, B, C1, C2, tol=1e-8, max_iter=200, lyapunov=False, delta=1e-12):
    """Factorized conjugate residual method (symmetric A and B): Lanczos bases, S = F(R) by
    eq. (3.11) each iteration, Q = F(P) by recurrence. Returns ``(V, Xc, W, info)``; after k+1
    iterations Xc is (k+1)s square, like Algorithm 4.1."""
    s = C1.shape[1]
    V, W = _bases(A, B, C1, C2, "lanczos", lyapunov, delta)
    sd = _Side(V, W, lyapunov)
    R = V.R @ W.R.T
    nr0 = np.linalg.norm(R)
    S = sd.op(R)
    P, Q = R.copy(), S.copy()
    rho = inner(pad(R, S.shape[0]), S)
    X = np.zeros((0, 0))
    info = {"alpha": [], "beta": [], "rho": [rho], "relres": [], "status": NOT_CONVERGED,
            "iters": 0, "normR0": nr0}
    for k in range(max_iter):
        qq = inner(Q, Q)
        if qq == 0.0 or rho == 0.0 or not np.isfinite(qq):
            info["status"] = BREAKDOWN
            break
        alpha = rho / qq
        p = (k + 1) * s
        X = pad(X, p) + alpha * P
        R = pad(R, p + s) - alpha * Q
        rel = np.linalg.norm(R) / nr0
        info["alpha"].append(alpha)
        info["relres"].append(rel)
        info["iters"] = k + 1
        if rel <= tol:
            info["status"] = CONVERGED
            break
        S = sd.op(R)
        rho_new = inner(pad(R, p + 2 * s), S)
        beta = rho_new / rho
        info["beta"].append(beta)
        info["rho"].append(rho_new)
        P = R + beta * pad(P, p + s)
        Q = S + beta * pad(Q, p + 2 * s)
        rho = rho_new
    return (*_out(V, W, X, s, A, B), info)


def factored_cgs(A, B, C1, C2, tol=1e-8, max_iter=200, lyapunov=False, delta=1e-12):
    """Factorized conjugate gradient squared: Arnoldi bases, two core products per iteration
    (V = F(P), then F(U + Q)). After k+1 iterations Xc is (2k+2)s square, like Algorithm 4.2."""
    s = C1.shape[1]
    V, W = _bases(A, B, C1, C2, "arnoldi", lyapunov, delta)
    sd = _Side(V, W, lyapunov)
    R = V.R @ W.R.T
    Rt = R.copy()
    U, P = R.copy(), R.copy()
    rho = inner(Rt, R)
    nr0 = np.linalg.norm(R)
    X = np.zeros((0, 0))
    info = {"alpha": [], "beta": [], "rho": [rho], "relres": [], "status": NOT_CONVERGED,
            "iters": 0, "normR0": nr0}
    for k in range(max_iter):
        p = (2 * k + 1) * s
        Vk = sd.op(P)
        den = inner(Rt, Vk[:s, :s])
        if den == 0.0 or rho == 0.0 or not np.isfinite(den):
            info["status"] = BREAKDOWN
            break
        alpha = rho / den
        Q = pad(U, p + s) - alpha * Vk
        Wk = pad(U, p + s) + Q
        X = pad(X, p + s) + alpha * Wk
        R = pad(R, p + 2 * s) - alpha * sd.op(Wk)
        rel = np.linalg.norm(R) / nr0
        info["alpha"].append(alpha)
        info["relres"].append(rel)
        info["iters"] = k + 1
        if rel <= tol:
            info["status"] = CONVERGED
            break
        rho_new = inner(Rt, R[:s, :s])
        beta = rho_new / rho
        info["beta"].append(beta)
        info["rho"].append(rho_new)
        U = R + beta * pad(Q, p + 2 * s)
        P = U + beta * (pad(Q, p + 2 * s) + beta * pad(P, p + 2 * s))
        rho = rho_new
    return (*_out(V, W, X, s, A, B), info)


def factored_gpbicg(A, B, C1, C2, tol=1e-8, max_iter=200, lyapunov=False, delta=1e-12,
                    eta_zero=False):
    """Factorized GPBiCG: Arnoldi bases, two core products per iteration (F(p_n), F(t_n)); the
    cores of p, u, t, y, z, w, r, x grow by 2s per iteration. eta_zero gives BiCGSTAB."""
    s = C1.shape[1]
    V, W = _bases(A, B, C1, C2, "arnoldi", lyapunov, delta)
    sd = _Side(V, W, lyapunov)
    R = V.R @ W.R.T
    Rt = R.copy()
    nr0 = np.linalg.norm(R)
    rho = inner(Rt, R)
    zero = np.zeros((s, s))
    Z, Pm, Um, Tm, Wm = zero, zero, zero, zero, zero
    beta = 0.0
    X = np.zeros((0, 0))
    info = {"alpha": [], "zeta": [], "eta": [], "beta": [], "relres": [],
            "status": NOT_CONVERGED, "iters": 0, "normR0": nr0}
    for k in range(max_iter):
        p = (2 * k + 1) * s
        P = R + beta * (pad(Pm, p) - pad(Um, p))
        AP = sd.op(P)
        den = inner(Rt, AP[:s, :s])
        if den == 0.0 or rho == 0.0 or not np.isfinite(den):
            info["status"] = BREAKDOWN
            break
        alpha = rho / den
        q = p + s
        Y = pad(Tm, q) - pad(R, q) - alpha * pad(Wm, q) + alpha * AP
        T = pad(R, q) - alpha * AP
        AT = sd.op(T)
        Tq = pad(T, q + s)
        tt, ts = inner(AT, AT), inner(AT, Tq)
        if k == 0 or eta_zero:
            if tt == 0.0:
                info["status"] = BREAKDOWN
                break
            zeta, eta = ts / tt, 0.0
        else:
            Yq = pad(Y, q + s)
            zeta, eta = gpbicg_zeta_eta(tt, inner(Y, Y), inner(AT, Yq), inner(Y, T), ts)
        if zeta == 0.0 or not np.isfinite(zeta) or not np.isfinite(eta):
            info["status"] = BREAKDOWN
            break
        U = zeta * AP + eta * (pad(Tm, q) - pad(R, q) + beta * pad(Um, q))
        Z = zeta * pad(R, q) + eta * pad(Z, q) - alpha * U
        X = pad(X, q) + alpha * pad(P, q) + Z
        Rn = pad(T, q + s) - eta * pad(Y, q + s) - zeta * AT
        rel = np.linalg.norm(Rn) / nr0
        info["alpha"].append(alpha)
        info["zeta"].append(zeta)
        info["eta"].append(eta)
        info["relres"].append(rel)
        info["iters"] = k + 1
        if rel <= tol:
            info["status"] = CONVERGED
            break
        rho_new = inner(Rt, Rn[:s, :s])
        beta = (alpha / zeta) * (rho_new / rho)
        info["beta"].append(beta)
        Wm = AT + beta * pad(AP, q + s)
        Pm, Um, Tm, R, rho = P, U, T, Rn, rho_new
    return (*_out(V, W, X, s, A, B), info)


METHODS = {"cr": factored_cr, "cgs": factored_cgs, "gpbicg": factored_gpbicg}
