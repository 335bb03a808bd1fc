"""Pins for the CPU oracle: closed forms, exact solves, the paper's identities and invariants.

Each test ties the oracle to something other than itself: a closed-form solution, a dense direct
solve from a different library routine, the mathematical equivalence of the factored and
matrix-oriented methods (Section 5.1), the identities eqs. (3.8)-(3.11) and Corollary 3.2, and the
paper's own iteration counts (table tab:ex3) as a sanity band.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import direct, factored, matrix_oriented, residual
from workloads import configs, stencils

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------------------------------------
# P1: closed form. A = a I, B = b I: X = C1 C2^T / (a + b); both bases close after one block.
@pytest.mark.parametrize("method", ["cg", "bicgstab"])
@pytest.mark.parametrize("s", [1, 2, 3])
def test_closed_form_scaled_identity(method, s):
    n, m, a, b = 9, 7, 3.0, 1.5
    A = sp.csr_matrix(a * np.eye(n))
    B = sp.csr_matrix(b * np.eye(m))
    C1, C2 = stencils.gaussian_rhs(n, m, s, 5)
    fn = factored.factored_cg if method == "cg" else factored.factored_bicgstab
    V, X, W, info = fn(A, B, C1, C2, tol=1e-12, max_iter=5)
    assert info["status"] == factored.CONVERGED and info["iters"] == 1
    assert _rel(V @ X @ W.T, C1 @ C2.T / (a + b)) < 1e-14


# P2: finite termination. Diagonal A, B with p and q distinct eigenvalues: F has at most p*q
# distinct eigenvalues, so CG reaches the solution within p*q iterations.
def test_finite_termination_diagonal():
    p_vals = np.array([1.0, 2.0, 5.0])
    q_vals = np.array([0.5, 3.0])
    A = sp.csr_matrix(np.diag(np.repeat(p_vals, 4)))
    B = sp.csr_matrix(np.diag(np.repeat(q_vals, 5)))
    C1, C2 = stencils.gaussian_rhs(12, 10, 1, 3)
    V, X, W, info = factored.factored_cg(A, B, C1, C2, tol=1e-11, max_iter=50)
    assert info["status"] == factored.CONVERGED
    assert info["iters"] <= len(p_vals) * len(q_vals)
    Xd = direct.kron_solve(A, B, C1, C2)
    assert _rel(V @ X @ W.T, Xd) < 1e-9


# P3: the two direct solvers (different algorithms and library routines) agree; the factored
# methods converge to the same X within the conditioning of F times the tolerance.
def test_direct_solvers_agree():
    p = configs.tiny_sylvester(10, 8, 2, seed=3, pe=20.0)
    Xk = direct.kron_solve(p.A, p.B, p.C1, p.C2)
    Xb = direct.bartels_stewart(p.A, p.B, p.C1, p.C2)
    assert _rel(Xk, Xb) < 1e-12
    # the Kronecker matrix applies the Sylvester operator with column-stacking vec (eq. (1.2))
    X = np.random.default_rng(0).standard_normal((10, 8))
    F = direct.kron_matrix(p.A, p.B)
    lhs = (F @ X.reshape(-1, order="F")).reshape((10, 8), order="F")
    assert _rel(lhs, p.A.toarray() @ X + X @ p.B.toarray()) < 1e-14


@pytest.mark.parametrize("method,pe", [("cg", 0.0), ("bicgstab", 0.0), ("bicgstab", 25.0)])
def test_factored_matches_direct(method, pe):
    p = configs.tiny_sylvester(12, 9, 2, seed=11, pe=pe, method=method)
    V, X, W, info = factored.solve(p, tol=1e-12, max_iter=300)
    assert info["status"] == factored.CONVERGED
    Xd = direct.kron_solve(p.A, p.B, p.C1, p.C2)
    F = direct.kron_matrix(p.A, p.B)
    kappa = np.linalg.cond(F)
    assert _rel(V @ X @ W.T, Xd) <= 10 * kappa * 1e-12


# P4: the residual identity, densely and from the factors.
@pytest.mark.parametrize("method", ["cg", "bicgstab"])
def test_residual_identity(method):
    A = stencils.cd2d(8, 6, 0.0 if method == "cg" else 8.0)
    B = stencils.cd1d(40, 0.0 if method == "cg" else 8.0)
    p = stencils.make_problem("r", A, B, 2, 21, method=method)
    V, X, W, info = factored.solve(p, tol=1e-8, max_iter=300)
    assert info["status"] == factored.CONVERGED
    ad, rd = residual.dense_residual(p.A, p.B, p.C1, p.C2, V, X, W)
    af, rf = residual.factored_residual(p.A, p.B, p.C1, p.C2, V, X, W)
    assert abs(rd - rf) <= 1e-12 + 1e-6 * rd
    assert rd <= 1.5e-8
    # the recursive residual of the last iteration is the one the algorithm stops on
    assert info["relres"][-1] <= 1e-8


# ---------------------------------------------------------------------------------------------
# P5: factored and matrix-oriented methods are mathematically equivalent (Section 5.1).
def _equiv_problem(method):
    pe = 0.0 if method == "cg" else 12.0
    A = stencils.cd2d(12, 10, pe)
    B = stencils.cd1d(50, pe)
    return stencils.make_problem("eq", A, B, 2, 31, method=method)


@pytest.mark.parametrize("method", ["cg", "bicgstab"])
def test_factored_equals_matrix_oriented(method):
    p = _equiv_problem(method)
    if method == "cg":
        _, _, _, fi = factored.factored_cg(p.A, p.B, p.C1, p.C2, tol=1e-8, max_iter=400)
        _, mi = matrix_oriented.matrix_cg(p.A, p.B, p.C1, p.C2, 1e-8, 400)
        keys = ["alpha", "beta"]
    else:
        _, _, _, fi = factored.factored_bicgstab(p.A, p.B, p.C1, p.C2, tol=1e-8, max_iter=400)
        _, mi = matrix_oriented.matrix_bicgstab(p.A, p.B, p.C1, p.C2, 1e-8, 400)
        keys = ["alpha", "omega", "beta"]
    # BiCGSTAB amplifies the different rounding of the two forms (Example 5.2 observes the
    # histories separating late), so the tight bound covers the first 12 iterations.
    for key in keys + ["relres"]:
        a = np.array(fi[key][:20])
        b = np.array(mi[key][:20])
        err = np.abs(a - b) / np.abs(b)
        assert np.max(err[:12]) < 1e-10, key
        assert np.max(err) < 1e-8, key
    assert fi["status"] == mi["status"] == factored.CONVERGED
    assert abs(fi["iters"] - mi["iters"]) <= max(1, math.ceil(0.03 * mi["iters"]))


# ---------------------------------------------------------------------------------------------
# P6: invariants of the bases and of the core algebra.
def _arnoldi(M, C, steps, method="arnoldi"):
    K = factored.BlockKrylov(M, C, method)
    for _ in range(steps):
        K.step()
    return K


@pytest.mark.parametrize("method", ["arnoldi", "lanczos"])
def test_krylov_relation_eq38(method):
    pe = 10.0 if method == "arnoldi" else 0.0
    A = stencils.cd2d(9, 8, pe)
    C1, _ = stencils.gaussian_rhs(72, 1, 3, 4)
    K = _arnoldi(A, C1, 8, method)
    s, k = 3, 8
    Vk1 = K.basis(k + 1)
    Vk = K.basis(k)
    H = K.H((k + 1) * s, k * s)
    normA = sp.linalg.norm(A)
    assert np.linalg.norm(A @ Vk - Vk1 @ H) <= 1e-13 * normA
    orth = np.linalg.norm(Vk1.T @ Vk1 - np.eye((k + 1) * s))
    assert orth <= (1e-12 if method == "arnoldi" else 1e-9)
    # the first block spans C1: C1 = V1 R with R upper triangular and positive diagonal
    assert np.allclose(K.blocks[0] @ K.R, C1, atol=1e-13 * np.linalg.norm(C1))
    assert np.all(np.diag(K.R) > 0) and np.allclose(np.tril(K.R, -1), 0)
    # Lanczos: H is block tridiagonal with H_{j-1,j} = H_{j,j-1}^T
    if method == "lanczos":
        for j in range(2, k):
            assert np.allclose(H[(j - 1) * s:j * s, j * s:(j + 1) * s],
                               H[j * s:(j + 1) * s, (j - 1) * s:j * s].T)
            assert np.all(H[: (j - 1) * s, j * s:(j + 1) * s] == 0)


def _eq311_error(core_fn):
    """max relative error of eq. (3.11) on random cores: A Z + Z B = V_{k+1} L(Zc) W_{k+1}^T."""
    A = stencils.cd2d(7, 6, 9.0)
    B = stencils.cd1d(30, 5.0)
    C1, C2 = stencils.gaussian_rhs(42, 30, 2, 8)
    V = _arnoldi(A, C1, 5)
    W = _arnoldi(B.T.tocsr(), C2, 5)
    s, k = 2, 5
    Zc = np.random.default_rng(1).standard_normal((k * s, k * s))
    Z = V.basis(k) @ Zc @ W.basis(k).T
    lhs = A @ Z + (B.T @ Z.T).T
    Q = core_fn(Zc, V.H((k + 1) * s, k * s), W.H((k + 1) * s, k * s))
    rhs = V.basis(k + 1) @ Q @ W.basis(k + 1).T
    return _rel(rhs, lhs)


def test_sylvester_operator_eq311():
    assert _eq311_error(factored.sylvester_core) < 1e-13


def test_inner_product_eq310_and_rank_bound():
    p = _equiv_problem("bicgstab")
    V, X, W, info = factored.factored_bicgstab(p.A, p.B, p.C1, p.C2, tol=1e-30, max_iter=6)
    k = info["iters"]
    s = p.s
    assert X.shape == ((2 * k) * s, (2 * k) * s)
    Xf = V @ X @ W.T
    Y = np.random.default_rng(2).standard_normal(X.shape)
    Yf = V @ Y @ W.T
    assert abs(np.sum(Xf * Yf) - np.sum(X * Y)) <= 1e-12 * np.linalg.norm(X) * np.linalg.norm(Y)
    # rank X_k <= 2ks for BiCGSTAB
    assert np.linalg.matrix_rank(Xf) <= 2 * k * s
    p = _equiv_problem("cg")
    V, X, W, info = factored.factored_cg(p.A, p.B, p.C1, p.C2, tol=1e-30, max_iter=7)
    assert np.linalg.matrix_rank(V @ X @ W.T) <= info["iters"] * p.s


# P7: Corollary 3.2. For z = sum_i rho_i F^i c, Z = [C1, A C1, ...] Zhat [C2, B^T C2, ...]^T with
# Zhat_ij = binom(i+j-2, i-1) rho_{i+j-2} I_s (1-based, zero when i + j > k + 1).
def test_binomial_structure_cor32():
    n, m, s, k = 6, 5, 2, 4
    A = stencils.cd1d(n, 7.0)
    B = stencils.cd1d(m, 3.0)
    C1, C2 = stencils.gaussian_rhs(n, m, s, 9)
    rho = np.random.default_rng(4).standard_normal(k)
    F = direct.kron_matrix(A, B)
    c = (C1 @ C2.T).reshape(-1, order="F")
    z = sum(rho[i] * np.linalg.matrix_power(F, i) @ c for i in range(k))
    Z = z.reshape((n, m), order="F")
    Ad, Bd = A.toarray(), B.toarray()
    KA = np.hstack([np.linalg.matrix_power(Ad, i) @ C1 for i in range(k)])
    KB = np.hstack([np.linalg.matrix_power(Bd.T, i) @ C2 for i in range(k)])
    Zhat = np.zeros((k * s, k * s))
    for i in range(1, k + 1):
        for j in range(1, k + 1):
            if i + j <= k + 1:
                Zhat[(i - 1) * s:i * s, (j - 1) * s:j * s] = \
                    math.comb(i + j - 2, i - 1) * rho[i + j - 2] * np.eye(s)
    assert _rel(KA @ Zhat @ KB.T, Z) < 1e-12


def test_repeated_core_operator_reproduces_powers():
    """Applying eq. (3.11) i times to R0 reproduces F^i c (Proposition 3.1)."""
    n, m, s = 8, 7, 2
    A = stencils.cd1d(n, 6.0)
    B = stencils.cd1d(m, 2.0)
    C1, C2 = stencils.gaussian_rhs(n, m, s, 12)
    V = _arnoldi(A, C1, 3)
    W = _arnoldi(B.T.tocsr(), C2, 3)
    F = direct.kron_matrix(A, B)
    c = (C1 @ C2.T).reshape(-1, order="F")
    Z = V.R @ W.R.T
    for i in range(1, 4):
        Z = factored.sylvester_core(Z, V.H((i + 1) * s, i * s), W.H((i + 1) * s, i * s))
        full = V.basis(i + 1) @ Z @ W.basis(i + 1).T
        ref = (np.linalg.matrix_power(F, i) @ c).reshape((n, m), order="F")
        assert _rel(full, ref) < 1e-12


# ---------------------------------------------------------------------------------------------
# P8: the paper's own iteration counts (table tab:ex3) as a sanity band.
@pytest.mark.parametrize("s", [1, 3])
def test_paper_anchor_tab_ex3(s):
    with open(os.path.join(GOLDEN, "tab_ex3_iterations.json")) as f:
        gold = json.load(f)
    A = stencils.cd2d(*gold["grid"])
    p = stencils.make_problem("anchor", A, None, s, 11 + s, lyapunov=True)
    _, _, _, info = factored.factored_cg(p.A, p.B, p.C1, p.C2, tol=gold["tolerance"],
                                          max_iter=600, lyapunov=True)
    ref = gold["iterations"][str(s)]
    assert info["status"] == factored.CONVERGED
    assert abs(info["iters"] - ref) <= 0.25 * ref


# P9: the Lyapunov form (Section 4.3) equals the general method with B = A^T, C2 = C1.
@pytest.mark.parametrize("method", ["cg", "bicgstab"])
def test_lyapunov_equals_sylvester(method):
    A = stencils.cd2d(9, 7, 0.0 if method == "cg" else 9.0)
    p = stencils.make_problem("ly", A, None, 2, 17, lyapunov=True)
    fn = factored.factored_cg if method == "cg" else factored.factored_bicgstab
    V1, X1, W1, i1 = fn(p.A, p.B, p.C1, p.C2, tol=1e-8, max_iter=200, lyapunov=True)
    V2, X2, W2, i2 = fn(p.A, p.B, p.C1, p.C2, tol=1e-8, max_iter=200, lyapunov=False)
    assert i1["iters"] == i2["iters"]
    S1 = V1 @ X1 @ W1.T
    assert _rel(S1, V2 @ X2 @ W2.T) < 1e-10
    assert _rel(S1, S1.T) < 1e-10


# ---------------------------------------------------------------------------------------------
# Status outcomes.
def test_breakdown_cg_indefinite():
    A = sp.csr_matrix(np.diag([1.0, -2.0, 0.5]))
    B = sp.csr_matrix(np.diag([0.1, 0.2]))
    C1 = np.array([[1.0], [1.0], [0.0]])
    C2 = np.array([[1.0], [0.0]])
    _, _, _, info = factored.factored_cg(A, B, C1, C2, tol=1e-12, max_iter=10)
    assert info["status"] == factored.BREAKDOWN


def test_breakdown_bicgstab_skew():
    A = sp.csr_matrix(np.array([[0.0, 1.0], [-1.0, 0.0]]))
    B = sp.csr_matrix(np.zeros((1, 1)))
    C1 = np.array([[1.0], [0.0]])  # <R~0, F R0> = <e1, A e1> = 0 exactly: alpha is undefined
    C2 = np.array([[1.0]])
    _, _, _, info = factored.factored_bicgstab(A, B, C1, C2, tol=1e-12, max_iter=10)
    assert info["status"] == factored.BREAKDOWN


def test_max_iter_returns_valid_factors():
    p = configs.c1_cg_1d()
    V, X, W, info = factored.factored_cg(p.A, p.B, p.C1, p.C2, tol=1e-8, max_iter=30)
    assert info["status"] == factored.NOT_CONVERGED and info["iters"] == 30
    assert V.shape == (256, 30) and X.shape == (30, 30) and W.shape == (192, 30)
    _, rel = residual.dense_residual(p.A, p.B, p.C1, p.C2, V, X, W)
    assert abs(rel - info["relres"][-1]) < 1e-6


def test_rank_deficient_rhs_rejected():
    A = stencils.cd1d(10)
    C1 = np.ones((10, 2))
    C2 = np.random.default_rng(0).standard_normal((10, 2))
    with pytest.raises(factored.RhsRankError):
        factored.factored_cg(A, A, C1, C2)


def test_closure_partial_deflation():
    """A with 2 distinct eigenvalues and s = 3: the block Krylov space of A has dimension 6, so
    the second block is partly deflated; the solution is still exact."""
    d = np.repeat([1.0, 4.0], 5)
    A = sp.csr_matrix(np.diag(d))
    B = stencils.cd1d(6)
    C1, C2 = stencils.gaussian_rhs(10, 6, 3, 2)
    V, X, W, info = factored.factored_cg(A, B, C1, C2, tol=1e-12, max_iter=60)
    assert info["status"] == factored.CONVERGED
    assert _rel(V @ X @ W.T, direct.kron_solve(A, B, C1, C2)) < 1e-9
