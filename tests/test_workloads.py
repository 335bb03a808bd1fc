"""Pins for the seeded input generators: CSR canonical form, nnz formulas, symmetry and the
closed-form eigenvalues of the Dirichlet stencils."""
import numpy as np
import pytest
import scipy.sparse as sp

from workloads import configs, stencils


def _canonical(M):
    assert M.indptr.dtype == np.int32 and M.indices.dtype == np.int32
    assert M.data.dtype == np.float64
    for i in range(M.shape[0]):
        cols = M.indices[M.indptr[i]:M.indptr[i + 1]]
        assert np.all(np.diff(cols) > 0)


@pytest.mark.parametrize("N,pe", [(7, 0.0), (31, 10.0)])
def test_cd1d_stencil_and_spectrum(N, pe):
    T = stencils.cd1d(N, pe)
    _canonical(T)
    assert T.nnz == 3 * N - 2
    g = pe / (2 * (N + 1))
    d = T.toarray()
    assert np.all(np.diag(d) == 2.0)
    assert np.allclose(np.diag(d, -1), -1 - g) and np.allclose(np.diag(d, 1), -1 + g)
    # eigenvalues of tridiag(a, 2, c): 2 + 2 sqrt(a c) cos(k pi / (N+1))
    k = np.arange(1, N + 1)
    ev = np.sort(2 - 2 * np.sqrt((1 + g) * (1 - g)) * np.cos(k * np.pi / (N + 1)))
    assert np.allclose(np.sort(np.linalg.eigvals(d).real), ev, atol=1e-12)


def test_physical_scaling():
    T = stencils.cd1d(9, 0.0, "physical")
    assert np.allclose(T.toarray(), 100.0 * stencils.cd1d(9).toarray())


def test_cd2d_cd3d_structure():
    A = stencils.cd2d(6, 5, 4.0)
    _canonical(A)
    assert A.shape == (30, 30)
    assert A.nnz == 5 * 30 - 2 * 6 - 2 * 5
    A0 = stencils.cd2d(6, 5)
    assert (A0 - A0.T).nnz == 0
    ex = np.add.outer(2 - 2 * np.cos(np.arange(1, 6) * np.pi / 6),
                      2 - 2 * np.cos(np.arange(1, 7) * np.pi / 7)).ravel()
    assert np.allclose(np.sort(np.linalg.eigvalsh(A0.toarray())), np.sort(ex))
    # x is the fastest index: row 0 couples to 1 (x neighbour) and 6 (y neighbour)
    assert list(A0.indices[A0.indptr[0]:A0.indptr[1]]) == [0, 1, 6]
    A3 = stencils.cd3d(4, 3, 5, 2.0)
    _canonical(A3)
    n = 60
    assert A3.nnz == 7 * n - 2 * (3 * 5) - 2 * (4 * 5) - 2 * (4 * 3)


def test_config_shapes():
    p = configs.c1_cg_1d()
    assert (p.n, p.m, p.s) == (256, 192, 1)
    assert p.A.nnz == 766 and p.B.nnz == 574
    assert np.allclose(p.A.diagonal(), 2 * 257 ** 2)
    p = configs.c2_bicgstab()
    assert (p.n, p.m, p.s) == (16384, 8192, 2)
    assert p.A.nnz == 81408 and p.B.nnz == 24574
    C1, C2 = stencils.gaussian_rhs(p.n, p.m, 2, 1002)
    assert np.array_equal(C1, p.C1) and np.array_equal(C2, p.C2)


def test_batch_recipe():
    probs = configs.batch64(count=8)
    for i, p in enumerate(probs):
        assert 1024 <= p.n <= 32768 and 512 <= p.m <= 16384 and p.s in (1, 2, 4)
        assert p.method == ("cg" if i % 2 == 0 else "bicgstab")
        if p.method == "cg":
            assert (p.A - p.A.T).nnz == 0 and (p.B - p.B.T).nnz == 0
