"""Low-rank compression of a factored solution ``X = V Xc W^T`` (the form of Corollary 3.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

With V and W of orthonormal columns the singular values of X are those of the core Xc, and
``Xc = U diag(sigma) Y^T`` gives ``X = (V U) diag(sigma) (W Y)^T``. Truncating to the k largest
singular values leaves the Frobenius error ``sqrt(sum_{i > k} sigma_i^2)`` (Eckart-Young); k is
the smallest rank whose error is at most ``rel_tol ||X||_F``. The core's SVD is a library
primitive (LAPACK through NumPy).
"""
from __future__ import annotations

import numpy as np


def truncation_rank(sigma, rel_tol, max_rank=None):
    """Smallest k with sqrt(sum_{i >= k} sigma_i^2) <= rel_tol * ||sigma||_2 (sigma descending)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    total = np.sqrt(np.sum(sigma ** 2))
    tail = np.sqrt(np.cumsum((sigma ** 2)[::-1])[::-1])  # tail[k] = ||sigma[k:]||
    tail = np.append(tail, 0.0)
    k = int(np.argmax(tail <= rel_tol * total))
    if max_rank is not None:
        k = min(k, int(max_rank))
    return k


def compress(V, Xc, W, rel_tol, max_rank=None):
    """Returns (Z1, sigma, Z2) with X ~= Z1 diag(sigma) Z2^T and the rank-k truncation error."""
    U, sig, Yt = np.linalg.svd(Xc, full_matrices=False)
    k = truncation_rank(sig, rel_tol, max_rank)
    return V @ U[:, :k], sig[:k], W @ Yt[:k].T, float(np.sqrt(np.sum(sig[k:] ** 2)))
