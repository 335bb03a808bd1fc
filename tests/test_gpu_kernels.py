"""GPU parity of the building blocks behind the C ABI: FP64 MFMA GEMM, CSR SpMM and the exact CSR
transpose. Expected values are plain NumPy/SciPy products of the same seeded inputs."""
import numpy as np
import pytest
import scipy.sparse as sp

from workloads import configs, stencils

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sylv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_28274_amd import sylv as _s
    return _s


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (16, 16, 4), (70, 53, 37), (130, 64, 200),
                                   (64, 129, 1000)])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_dgemm_mfma(sylv, M, N, K, ta, tb):
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    ref = 1.5 * ((A.T if ta else A) @ (B.T if tb else B)) - 0.5 * C0
    dA, dB, dC = _dev(A), _dev(B), _dev(C0)
    a_rs, a_cs = (1, M) if ta else (K, 1)
    b_rs, b_cs = (1, K) if tb else (N, 1)
    sylv.sylv_dgemm(M, N, K, 1.5, dA, a_rs, a_cs, dB, b_rs, b_cs, -0.5, dC, N)
    got = dC.cpu().numpy()
    scale = np.abs(A).max() * np.abs(B).max() * K + 1
    assert np.max(np.abs(got - ref)) <= 1e-14 * scale


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 8])
def test_spmm_small(sylv, s):
    A = stencils.cd2d(37, 29, 5.0)
    X = np.random.default_rng(s).standard_normal((A.shape[0], s))
    rp, ci, va = sylv.csr_tensors(A)
    csr = sylv.make_csr(A.shape[0], rp, ci, va)
    dX = _dev(X)
    dY = torch.empty_like(dX)
    sylv.sylv_spmm(csr, s, dX, dY)
    ref = A @ X
    assert np.max(np.abs(dY.cpu().numpy() - ref)) <= 1e-14 * np.abs(ref).max()


def test_spmm_c2_sizes(sylv):
    p = configs.c2_bicgstab()
    for M, s in ((p.A, 2), (p.B.T.tocsr(), 2)):
        M = stencils._canonical(M)
        X = np.random.default_rng(3).standard_normal((M.shape[0], s))
        rp, ci, va = sylv.csr_tensors(M)
        csr = sylv.make_csr(M.shape[0], rp, ci, va)
        dX = _dev(X)
        dY = torch.empty_like(dX)
        sylv.sylv_spmm(csr, s, dX, dY)
        ref = M @ X
        assert np.max(np.abs(dY.cpu().numpy() - ref)) <= 1e-14 * np.abs(ref).max()


def _transpose_case(sylv, M):
    rows = M.shape[0]
    rp, ci, va = sylv.csr_tensors(M)
    csr = sylv.make_csr(rows, rp, ci, va)
    orp = torch.empty(rows + 1, dtype=torch.int32, device="cuda")
    oci = torch.empty(max(M.nnz, 1), dtype=torch.int32, device="cuda")
    ova = torch.empty(max(M.nnz, 1), dtype=torch.float64, device="cuda")
    scr = torch.empty(sylv.sylv_csr_transpose_scratch_bytes(rows), dtype=torch.uint8, device="cuda")
    sylv.sylv_csr_transpose(csr, orp, oci, ova, scr)
    T = stencils._canonical(M.T)
    assert np.array_equal(orp.cpu().numpy(), T.indptr)
    assert np.array_equal(oci.cpu().numpy()[:M.nnz], T.indices)
    assert np.array_equal(ova.cpu().numpy()[:M.nnz], T.data)  # exact copies of the values


def test_csr_transpose_bit_exact(sylv):
    _transpose_case(sylv, configs.c2_bicgstab().B)
    _transpose_case(sylv, stencils.cd2d(256, 256, 10.0))
    rng = np.random.default_rng(5)
    R = sp.random(3000, 3000, density=0.002, format="csr", random_state=rng)
    R = R + sp.diags(rng.standard_normal(3000))
    _transpose_case(sylv, stencils._canonical(R))
