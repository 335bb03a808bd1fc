"""Dense direct solves of ``A X + X B = C1 C2^T`` for tiny sizes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* :func:`kron_solve` - the Kronecker form eq. (1.2), ``(I_m (x) A + B^T (x) I_n) vec X = vec C`` with
  vec stacking columns, solved by dense LU.
* :func:`bartels_stewart` - the Schur-based method cited in Section 1 (SciPy's implementation).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _dense(M):
    return M.toarray() if hasattr(M, "toarray") else np.asarray(M, dtype=np.float64)


def kron_matrix(A, B):
    """``F = I_m (x) A + B^T (x) I_n`` (eq. (1.2))."""
    A, B = _dense(A), _dense(B)
    n, m = A.shape[0], B.shape[0]
    return np.kron(np.eye(m), A) + np.kron(B.T, np.eye(n))


def kron_solve(A, B, C1, C2):
    A, B = _dense(A), _dense(B)
    n, m = A.shape[0], B.shape[0]
    if n * m > 4096:
        raise ValueError("kron_solve is for n*m <= 4096")
    c = (C1 @ C2.T).reshape(-1, order="F")
    x = np.linalg.solve(kron_matrix(A, B), c)
    return x.reshape((n, m), order="F")


def bartels_stewart(A, B, C1, C2):
    return sla.solve_sylvester(_dense(A), _dense(B), C1 @ C2.T)
