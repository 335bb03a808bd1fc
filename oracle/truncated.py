"""Truncated CG (Algorithm A.1) and truncated BiCGSTAB (Algorithm A.2): the matrix-oriented
methods with every iterate in low-rank form ``Z = L D N^T`` and low-rank truncation after the
operations the algorithms mark, the paper's comparison methods (Section 5.2, Appendix A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Low-rank arithmetic (Appendix A and the cost comparison of Appendix B): a sum stacks the factors
(``[L1 L2] blkdiag(a D1, b D2) [N1 N2]^T``), the operator is ``A Z + Z B = [A L, L]
blkdiag(D, D) [N, B^T N]^T`` (the rank doubles), an inner product is
``tr(D1^T (L1^T L2) D2 (N2^T N1))``.

Reading of the truncation operator T (defined in a cited work that is not available here): thin
QR factorizations ``L = Q_L R_L``, ``N = Q_N R_N`` (Householder, NumPy), an SVD of the small core
``R_L D R_N^T = U diag(sigma) Y^T``, and the singular values ``sigma_i > eps_T sigma_1`` kept:
``T(Z) = (Q_L U_k) diag(sigma_k) (Q_N Y_k)^T``. Norms are taken after the QR step as the
Frobenius norm of the small core, so no squared-norm cancellation enters the stopping test.
Options follow Examples 5.3 and 5.4: truncated CG truncates R (Q not), truncated BiCGSTAB uses
variant 1 (the recursive residual) and truncates Q and S (T not).
"""
from __future__ import annotations

import numpy as np

CONVERGED, NOT_CONVERGED, BREAKDOWN = 0, 1, 2


class LowRank:
    """Z = L @ D @ N.T with L (n x r), D (r x r), N (m x r)."""

    def __init__(self, L, D, N):
        self.L, self.D, self.N = L, D, N

    @property
    def rank(self) -> int:
        return self.D.shape[0]

    def dense(self):
        return self.L @ self.D @ self.N.T


def lr_rhs(C1, C2):
    return LowRank(C1.copy(), np.eye(C1.shape[1]), C2.copy())


def lr_zero(n, m):
    return LowRank(np.zeros((n, 0)), np.zeros((0, 0)), np.zeros((m, 0)))


def lr_comb(*terms):
    """sum of c_i Z_i, by stacking the factors."""
    Ls, Ns, Ds = [], [], []
    for c, Z in terms:
        Ls.append(Z.L)
        Ns.append(Z.N)
        Ds.append(c * Z.D)
    r = sum(D.shape[0] for D in Ds)
    D = np.zeros((r, r))
    o = 0
    for Db in Ds:
        k = Db.shape[0]
        D[o:o + k, o:o + k] = Db
        o += k
    return LowRank(np.hstack(Ls), D, np.hstack(Ns))


def lr_op(A, B, Z):
    """A Z + Z B = (A L) D N^T + L D (B^T N)^T."""
    r = Z.rank
    D = np.zeros((2 * r, 2 * r))
    D[:r, :r] = Z.D
    D[r:, r:] = Z.D
    return LowRank(np.hstack([A @ Z.L, Z.L]), D, np.hstack([Z.N, B.T @ Z.N]))


def lr_inner(Z1, Z2) -> float:
    """<Z1, Z2> = tr(D1^T (L1^T L2) D2 (N2^T N1))."""
    return float(np.sum((Z1.D.T @ (Z1.L.T @ Z2.L) @ Z2.D) * (Z1.N.T @ Z2.N)))


def _core(Z):
    QL, RL = np.linalg.qr(Z.L, mode="reduced")
    QN, RN = np.linalg.qr(Z.N, mode="reduced")
    return QL, RL @ Z.D @ RN.T, QN


def lr_norm(Z) -> float:
    if Z.rank == 0:
        return 0.0
    return float(np.linalg.norm(_core(Z)[1]))


def lr_truncate(Z, eps):
    """T(Z): singular values above eps times the largest kept."""
    if Z.rank == 0:
        return Z
    QL, M, QN = _core(Z)
    U, sig, Yt = np.linalg.svd(M)
    if sig.size == 0 or sig[0] == 0.0:
        return lr_zero(Z.L.shape[0], Z.N.shape[0])
    k = int(np.sum(sig > eps * sig[0]))
    return LowRank(QL @ U[:, :k], np.diag(sig[:k]), QN @ Yt[:k].T)


def truncated_cg(A, B, C1, C2, tol, max_iter, eps_t, trunc_q=False, trunc_r=True):
    """Algorithm A.1 (written for A X + X A^T = C1 C1^T; the same steps for symmetric A, B and
    C1 C2^T): alpha = <R, P> / <P, Q>, X = T(X + alpha P), R recomputed as C - A X - X B
    (optionally truncated), beta = -<R, Q> / <P, Q>, P = T(R + beta P)."""
    C = lr_rhs(C1, C2)
    n, m = C1.shape[0], C2.shape[0]
    X = lr_zero(n, m)
    R = C
    P = R
    nr0 = lr_norm(C)
    info = {"alpha": [], "beta": [], "relres": [], "rank_x": [], "status": NOT_CONVERGED,
            "iters": 0}
    for k in range(max_iter):
        Q = lr_op(A, B, P)
        if trunc_q:
            Q = lr_truncate(Q, eps_t)
        xi = lr_inner(P, Q)
        if not (xi > 0.0):
            info["status"] = BREAKDOWN
            break
        alpha = lr_inner(R, P) / xi
        X = lr_truncate(lr_comb((1.0, X), (alpha, P)), eps_t)
        R = lr_comb((1.0, C), (-1.0, lr_op(A, B, X)))
        if trunc_r:
            R = lr_truncate(R, eps_t)
        rel = lr_norm(R) / nr0
        info["alpha"].append(alpha)
        info["relres"].append(rel)
        info["rank_x"].append(X.rank)
        info["iters"] = k + 1
        if rel <= tol:
            info["status"] = CONVERGED
            break
        beta = -lr_inner(R, Q) / xi
        info["beta"].append(beta)
        P = lr_truncate(lr_comb((1.0, R), (beta, P)), eps_t)
    return X, info


def truncated_bicgstab(A, B, C1, C2, tol, max_iter, eps_t, variant=1, trunc_q=True,
                       trunc_s=True, trunc_t=False, trunc_r2=False):
    """Algorithm A.2 with R~0 = R0; variant 1 updates R = T(S - omega T), variant 2 recomputes
    R = C - A X - X B (optionally truncated)."""
    C = lr_rhs(C1, C2)
    n, m = C1.shape[0], C2.shape[0]
    X = lr_zero(n, m)
    R = C
    Rt = C
    P = R
    rho = lr_inner(R, Rt)
    nr0 = lr_norm(C)
    info = {"alpha": [], "omega": [], "beta": [], "relres": [], "rank_x": [],
            "status": NOT_CONVERGED, "iters": 0}
    for k in range(max_iter):
        Q = lr_op(A, B, P)
        if trunc_q:
            Q = lr_truncate(Q, eps_t)
        den = lr_inner(Rt, Q)
        if den == 0.0:
            info["status"] = BREAKDOWN
            break
        alpha = rho / den
        S = lr_comb((1.0, R), (-alpha, Q))
        if trunc_s:
            S = lr_truncate(S, eps_t)
        Tm = lr_op(A, B, S)
        if trunc_t:
            Tm = lr_truncate(Tm, eps_t)
        tt = lr_inner(Tm, Tm)
        if tt == 0.0:
            info["status"] = BREAKDOWN
            break
        omega = lr_inner(Tm, S) / tt
        X = lr_truncate(lr_comb((1.0, X), (alpha, P), (omega, S)), eps_t)
        if variant == 1:
            R = lr_truncate(lr_comb((1.0, S), (-omega, Tm)), eps_t)
        else:
            R = lr_comb((1.0, C), (-1.0, lr_op(A, B, X)))
            if trunc_r2:
                R = lr_truncate(R, eps_t)
        rel = lr_norm(R) / nr0
        info["alpha"].append(alpha)
        info["omega"].append(omega)
        info["relres"].append(rel)
        info["rank_x"].append(X.rank)
        info["iters"] = k + 1
        if rel <= tol:
            info["status"] = CONVERGED
            break
        rho_new = lr_inner(Rt, R)
        if rho_new == 0.0:
            info["status"] = BREAKDOWN
            break
        beta = (alpha / omega) * (rho_new / rho)
        info["beta"].append(beta)
        P = lr_truncate(lr_comb((1.0, R), (beta, P), (-beta * omega, Q)), eps_t)
        rho = rho_new
    return X, info
