"""Factorized CG (Algorithm 4.1), factorized BiCGSTAB (Algorithm 4.2) and the Lyapunov case
(Section 4.3) in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Iterates are kept as ``Z = V Zc W^T`` with small cores ``Zc`` (Corollary 3.3). The bases come from
a block Lanczos process (Algorithm 4.1; A and B symmetric) or a block Arnoldi process
(Algorithm 4.2), both satisfying eq. (3.8): ``A V_k = V_{k+1} H_{k+1,k}``,
``B^T W_k = W_{k+1} G_{k+1,k}``. Core algebra follows eqs. (3.9)-(3.11).

Readings where the paper leaves a choice open (all listed in the design notes):

* Block QR (Alg. 4.1 step 1, Alg. 4.2 step 2 and every new block): Householder QR with the sign
  convention ``diag(R) >= 0``.
* Block Lanczos: three-term recurrence ``U = A V_j - V_{j-1} H_{j,j-1}^T``, ``H_jj = V_j^T U``,
  ``U -= V_j H_jj``, then QR of U; no reorthogonalization against older blocks (the per-step cost
  stated after eq. (3.11) excludes it).
* Block Arnoldi: block modified Gram-Schmidt over all previous blocks, applied twice.
* Krylov closure: if after orthogonalization ``||U||_F <= delta * ||M V_j||_F``, a zero block is
  appended with a zero subdiagonal block. If only some directions vanish, U is orthonormalised
  through its SVD and the vanishing directions become zero columns.
* Breakdown: CG stops with status 2 when ``<P, Q> <= 0``; BiCGSTAB when ``<R~0, Q(1:s,1:s)> = 0``,
  ``<T, T> = 0``, ``omega = 0`` or ``rho = 0``. The last completed iterate is returned.
* On reaching ``max_iter`` the last iterate is returned with status 1.
"""
from __future__ import annotations

import numpy as np

CONVERGED, NOT_CONVERGED, BREAKDOWN = 0, 1, 2


class RhsRankError(ValueError):
    """C1 or C2 does not have full column rank."""


def qr_pos(U):
    """Thin Householder QR with ``diag(R) >= 0``."""
    Q, R = np.linalg.qr(U, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d, d[:, None] * R


def orthonormalize(U, ref, delta):
    """Return (V, Hsub) with ``U ~= V Hsub``, V having orthonormal or zero columns (closure rule)."""
    s = U.shape[1]
    if not np.linalg.norm(U) > delta * ref:
        return np.zeros_like(U), np.zeros((s, s))
    Q, R = qr_pos(U)
    if np.min(np.abs(np.diag(R))) > delta * ref:
        return Q, R
    Y, sig, Zt = np.linalg.svd(U, full_matrices=False)
    keep = sig > delta * ref
    V = np.zeros_like(U)
    Hs = np.zeros((s, s))
    V[:, keep] = Y[:, keep]
    Hs[keep, :] = sig[keep, None] * Zt[keep, :]
    return V, Hs


class BlockKrylov:
    """Orthonormal basis of the block Krylov space K_j(M, C), one block of s columns per step,
    with the block Hessenberg matrix of eq. (3.8)."""

    def __init__(self, M, C, method: str, delta: float = 1e-12):
        assert method in ("lanczos", "arnoldi")
        self.M, self.method, self.delta = M, method, delta
        self.s = C.shape[1]
        V1, R = qr_pos(C)
        if np.min(np.abs(np.diag(R))) <= 1e-14 * max(np.linalg.norm(C), 1e-300):
            raise RhsRankError("right-hand-side factor is rank deficient")
        self.R = R
        self.blocks = [V1]
        cap = 16 * self.s
        self._H = np.zeros((cap + self.s, cap))

    @property
    def nblocks(self) -> int:
        return len(self.blocks)

    def H(self, rows: int, cols: int):
        return self._H[:rows, :cols]

    def basis(self, nblocks: int | None = None):
        nb = self.nblocks if nblocks is None else nblocks
        return np.hstack(self.blocks[:nb])

    def _grow(self, need_cols: int):
        if need_cols <= self._H.shape[1]:
            return
        cap = max(need_cols, 2 * self._H.shape[1])
        H = np.zeros((cap + self.s, cap))
        H[: self._H.shape[0], : self._H.shape[1]] = self._H
        self._H = H

    def step(self):
        """Apply M to the newest block V_j, orthogonalize, append V_{j+1} and column block j of H."""
        s = self.s
        j = self.nblocks - 1
        self._grow((j + 1) * s)
        U = self.M @ self.blocks[j]
        ref = np.linalg.norm(U)
        col = np.zeros(((j + 2) * s, s))
        if self.method == "lanczos":
            if j > 0:
                h_up = self._H[j * s:(j + 1) * s, (j - 1) * s:j * s].T.copy()
                U = U - self.blocks[j - 1] @ h_up
                col[(j - 1) * s:j * s] = h_up
            h_jj = self.blocks[j].T @ U
            U = U - self.blocks[j] @ h_jj
            col[j * s:(j + 1) * s] = h_jj
        else:
            for _sweep in range(2):
                for i in range(j + 1):
                    c = self.blocks[i].T @ U
                    U = U - self.blocks[i] @ c
                    col[i * s:(i + 1) * s] += c
        Vn, Hn = orthonormalize(U, ref, self.delta)
        col[(j + 1) * s:] = Hn
        self._H[: (j + 2) * s, j * s:(j + 1) * s] = col
        self.blocks.append(Vn)


def pad(Z, size):
    """Embed Z in the upper-left corner of a size x size zero matrix (the block padding of
    Algorithms 4.1 and 4.2)."""
    out = np.zeros((size, size))
    out[: Z.shape[0], : Z.shape[1]] = Z
    return out


def inner(X, Y) -> float:
    """Core inner product, eq. (3.10)."""
    return float(np.sum(X * Y))


def sylvester_core(P, H, G):
    """Eq. (3.11): ``[H P, 0] + [P G^T; 0]`` for P (p x p) and H, G ((p+s) x p)."""
    p = P.shape[0]
    q = H.shape[0]
    Q = np.zeros((q, q))
    Q[:, :p] += H @ P
    Q[:p, :] += P @ G.T
    return Q


def _bases(A, B, C1, C2, method, lyapunov, delta):
    V = BlockKrylov(A, C1, method, delta)
    if lyapunov:
        return V, V
    return V, BlockKrylov(B.T.tocsr(), C2, method, delta)


def factored_cg(A, B, C1, C2, tol=1e-8, max_iter=200, lyapunov=False, delta=1e-12):
    """Algorithm 4.1 (Lyapunov form of Section 4.3 when ``lyapunov``: W = V, G = H).

    Returns ``(Vk, Xc, Wk, info)`` with ``Vk Xc Wk^T`` the approximate solution."""
    s = C1.shape[1]
    V, W = _bases(A, B, C1, C2, "lanczos", lyapunov, delta)
    R = V.R @ W.R.T
    P = R.copy()
    rho = inner(R, R)
    nr0 = np.sqrt(rho)
    X = np.zeros((0, 0))
    info = {"alpha": [], "beta": [], "rho": [rho], "relres": [], "status": NOT_CONVERGED,
            "iters": 0, "normR0": nr0}
    for k in range(max_iter):
        V.step()
        if not lyapunov:
            W.step()
        p = (k + 1) * s
        Q = sylvester_core(P, V.H(p + s, p), W.H(p + s, p))
        pq = inner(P, Q[:p, :p])
        if not (pq > 0.0 and np.isfinite(pq)):
            info["status"] = BREAKDOWN
            break
        alpha = rho / pq
        X = pad(X, p) + alpha * P
        R = pad(R, p + s) - alpha * Q
        rel = np.linalg.norm(R) / nr0
        info["alpha"].append(alpha)
        info["relres"].append(rel)
        info["iters"] = k + 1
        if rel <= tol:
            info["status"] = CONVERGED
            break
        rho_new = inner(R, R)
        beta = rho_new / rho
        info["beta"].append(beta)
        info["rho"].append(rho_new)
        P = R + beta * pad(P, p + s)
        rho = rho_new
    r = X.shape[0]
    nb = r // s
    return V.basis(nb) if nb else np.zeros((A.shape[0], 0)), X, \
        (W.basis(nb) if nb else np.zeros((B.shape[0], 0))), info


def factored_bicgstab(A, B, C1, C2, tol=1e-8, max_iter=200, lyapunov=False, delta=1e-12):
    """Algorithm 4.2 with R~0 = R0 (Lyapunov form when ``lyapunov``).

    Returns ``(V, Xc, W, info)``; after k+1 iterations Xc is (2k+2)s square."""
    s = C1.shape[1]
    V, W = _bases(A, B, C1, C2, "arnoldi", lyapunov, delta)
    R = V.R @ W.R.T
    Rt = R.copy()
    P = R.copy()
    rho = inner(Rt, R)
    nr0 = np.linalg.norm(R)
    X = np.zeros((0, 0))
    info = {"alpha": [], "omega": [], "beta": [], "rho": [rho], "relres": [],
            "status": NOT_CONVERGED, "iters": 0, "normR0": nr0}

    def step_both():
        V.step()
        if not lyapunov:
            W.step()

    for k in range(max_iter):
        p = (2 * k + 1) * s
        step_both()
        Q = sylvester_core(P, V.H(p + s, p), W.H(p + s, p))
        den = inner(Rt, Q[:s, :s])
        if den == 0.0 or not np.isfinite(den):
            info["status"] = BREAKDOWN
            break
        alpha = rho / den
        S = pad(R, p + s) - alpha * Q
        step_both()
        T = sylvester_core(S, V.H(p + 2 * s, p + s), W.H(p + 2 * s, p + s))
        tt = inner(T, T)
        if tt == 0.0 or not np.isfinite(tt):
            info["status"] = BREAKDOWN
            break
        omega = inner(T[: p + s, : p + s], S) / tt
        if omega == 0.0:
            info["status"] = BREAKDOWN
            break
        X = pad(X, p + s) + pad(alpha * P, p + s) + omega * S
        R = pad(S, p + 2 * s) - omega * T
        rel = np.linalg.norm(R) / nr0
        info["alpha"].append(alpha)
        info["omega"].append(omega)
        info["relres"].append(rel)
        info["iters"] = k + 1
        if rel <= tol:
            info["status"] = CONVERGED
            break
        rho_new = inner(Rt, R[:s, :s])
        if rho_new == 0.0:
            info["status"] = BREAKDOWN
            break
        beta = (alpha / omega) * (rho_new / rho)
        info["beta"].append(beta)
        info["rho"].append(rho_new)
        P = R + beta * (pad(P, p + 2 * s) - omega * pad(Q, p + 2 * s))
        rho = rho_new
    r = X.shape[0]
    nb = r // s
    return V.basis(nb) if nb else np.zeros((A.shape[0], 0)), X, \
        (W.basis(nb) if nb else np.zeros((B.shape[0], 0))), info


def solve(problem, method=None, tol=None, max_iter=None):
    """Run the factored method a :class:`workloads.Problem` names."""
    method = method or problem.method
    fn = factored_cg if method == "cg" else factored_bicgstab
    return fn(problem.A, problem.B, problem.C1, problem.C2,
              tol=problem.tol if tol is None else tol,
              max_iter=problem.max_iter if max_iter is None else max_iter,
              lyapunov=problem.lyapunov)
