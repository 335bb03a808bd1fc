"""Seeded synthetic inputs: finite-difference stencil matrices in CSR and Gaussian RHS factors.

This module only builds inputs. It holds none of the solver's arithmetic, so both the CPU
oracle and the GPU path may take their matrices and right-hand sides from here.

Operators (Dirichlet boundary, lexicographic ordering with x fastest):

* 1D convection-diffusion ``-u'' + v u'`` discretised by central differences on N interior
  points, h = 1/(N+1). In unit-coefficient form (every entry multiplied by h^2) the row
  stencil is ``(-1-g, 2, -1+g)`` with cell Peclet number ``g = v*h/2``; ``v = 0`` gives the
  Laplacian ``tridiag(-1, 2, -1)``.
* 2D / 3D operators are Kronecker sums of 1D operators, one per direction, each with its
  own ``g_d = Pe*h_d/2``: ``A2 = I_y (x) T_x + T_y (x) I_x`` and likewise in 3D.

``scale="unit"`` keeps the unit-coefficient form; ``scale="physical"`` multiplies each 1D
factor by ``(N_d+1)^2`` (the 1/h^2 of the continuous operator). Every CSR array is canonical:
int32 ``indptr``/``indices`` with sorted, duplicate-free column indices and float64 values.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


def _canonical(M: sp.spmatrix) -> sp.csr_matrix:
    M = sp.csr_matrix(M, dtype=np.float64)
    M.sum_duplicates()
    M.eliminate_zeros()
    M.sort_indices()
    M.indptr = M.indptr.astype(np.int32)
    M.indices = M.indices.astype(np.int32)
    return M


def cd1d(N: int, pe: float = 0.0, scale: str = "unit") -> sp.csr_matrix:
    """1D convection-diffusion (Laplacian when pe == 0) on N interior points."""
    if N < 1:
        raise ValueError("N must be positive")
    h = 1.0 / (N + 1)
    g = pe * h / 2.0
    lo = np.full(N - 1, -1.0 - g)
    up = np.full(N - 1, -1.0 + g)
    T = sp.diags([lo, np.full(N, 2.0), up], [-1, 0, 1], shape=(N, N), format="csr")
    if scale == "physical":
        T = T * float((N + 1) ** 2)
    elif scale != "unit":
        raise ValueError(f"unknown scale {scale!r}")
    return _canonical(T)


def cd2d(Nx: int, Ny: int, pe: float = 0.0, scale: str = "unit") -> sp.csr_matrix:
    Tx, Ty = cd1d(Nx, pe, scale), cd1d(Ny, pe, scale)
    A = sp.kron(sp.identity(Ny), Tx) + sp.kron(Ty, sp.identity(Nx))
    return _canonical(A)


def cd3d(Nx: int, Ny: int, Nz: int, pe: float = 0.0, scale: str = "unit") -> sp.csr_matrix:
    Tx, Ty, Tz = cd1d(Nx, pe, scale), cd1d(Ny, pe, scale), cd1d(Nz, pe, scale)
    Ix, Iy, Iz = sp.identity(Nx), sp.identity(Ny), sp.identity(Nz)
    A = sp.kron(sp.kron(Iz, Iy), Tx) + sp.kron(sp.kron(Iz, Ty), Ix) + sp.kron(sp.kron(Tz, Iy), Ix)
    return _canonical(A)


def gaussian_rhs(n: int, m: int, s: int, seed: int, lyapunov: bool = False):
    """C1 ~ N(0,1)^{n x s}, then C2 ~ N(0,1)^{m x s} from the same PCG64 stream (C2 = C1 for
    a Lyapunov problem). Returned C-contiguous float64."""
    rng = np.random.default_rng(seed)
    C1 = np.ascontiguousarray(rng.standard_normal((n, s)))
    if lyapunov:
        return C1, C1.copy()
    C2 = np.ascontiguousarray(rng.standard_normal((m, s)))
    return C1, C2


@dataclass
class Problem:
    """One Sylvester problem ``A X + X B = C1 C2^T`` (Lyapunov when ``lyapunov``: B = A^T, C2 = C1)."""

    name: str
    A: sp.csr_matrix
    B: sp.csr_matrix
    C1: np.ndarray
    C2: np.ndarray
    lyapunov: bool = False
    method: str = "cg"  # "cg" | "bicgstab"
    tol: float = 1e-8
    max_iter: int = 200
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def m(self) -> int:
        return self.B.shape[0]

    @property
    def s(self) -> int:
        return self.C1.shape[1]


def make_problem(name, A, B, s, seed, lyapunov=False, **kw) -> Problem:
    if lyapunov:
        B = _canonical(A.T)
    C1, C2 = gaussian_rhs(A.shape[0], B.shape[0], s, seed, lyapunov)
    return Problem(name, A, B, C1, C2, lyapunov=lyapunov, **kw)
