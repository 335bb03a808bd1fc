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


def _sell_case(sylv, M, s, expect_ok=True):
    rp, ci, va = sylv.csr_tensors(M)
    csr = sylv.make_csr(M.shape[0], rp, ci, va)
    buf = torch.empty(sylv.sylv_sell_bytes(csr), dtype=torch.uint8, device="cuda")
    if not expect_ok:
        with pytest.raises(sylv.SylvError) as ei:
            sylv.sylv_sell_build(csr, buf)
        assert ei.value.code == sylv.SYLV_ERR_WORKSPACE
        return
    sylv.sylv_sell_build(csr, buf)
    X = np.random.default_rng(s).standard_normal((M.shape[0], s))
    dX = _dev(X)
    dY = torch.empty_like(dX)
    sylv.sylv_sell_spmm(csr, buf, s, dX, dY)
    ref = M @ X
    assert np.max(np.abs(dY.cpu().numpy() - ref)) <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("s", [1, 2, 3, 4, 7, 8])
def test_sell_spmm_stencils(sylv, s):
    _sell_case(sylv, stencils.cd2d(37, 29, 5.0), s)           # rows not a multiple of 64
    _sell_case(sylv, stencils.cd3d(16, 8, 9, 10.0), s)


@pytest.mark.parametrize("grid,s", [("2d1024", 1), ("2d1023", 1), ("3d64", 4)])
def test_sell_spmm_chained_full_size(sylv, grid, s):
    # the operators the bandwidth figure is measured on, at full size; three products issued
    # back to back on one stream without waiting in between (the call only enqueues). Over
    # 2048 x 256 rows with one column each thread takes two rows; 1023^2 rows leave a ragged
    # last workgroup (its second block of 256 rows partly past the end)
    M = {"2d1024": lambda: stencils.cd2d(1024, 1024, 0.0),
         "2d1023": lambda: stencils.cd2d(1023, 1023, 3.0),
         "3d64": lambda: stencils.cd3d(64, 64, 64, 10.0)}[grid]()
    rp, ci, va = sylv.csr_tensors(M)
    csr = sylv.make_csr(M.shape[0], rp, ci, va)
    buf = torch.empty(sylv.sylv_sell_bytes(csr), dtype=torch.uint8, device="cuda")
    sylv.sylv_sell_build(csr, buf)
    X = np.random.default_rng(5).standard_normal((M.shape[0], s))
    d = [_dev(X)] + [torch.empty_like(_dev(X)) for _ in range(3)]
    for k in range(3):
        sylv.sylv_sell_spmm(csr, buf, s, d[k], d[k + 1])
    ref = M @ (M @ (M @ X))
    assert np.max(np.abs(d[3].cpu().numpy() - ref)) <= 1e-13 * np.abs(ref).max()


def _sell_fits(M):
    # documented rule: padded size (64 x slice max row length, summed) <= nnz + nnz/4 + 64 slices
    n = M.shape[0]
    lens = np.diff(M.indptr)
    padded = sum(64 * int(lens[k:k + 64].max()) for k in range(0, n, 64))
    return padded <= M.nnz + M.nnz // 4 + 64 * ((n + 63) // 64) + 64


def test_sell_spmm_uneven_rows(sylv):
    rng = np.random.default_rng(9)
    n = 1000
    # one long row: padding beyond the reserved capacity is refused (the solver keeps CSR)
    R = sp.random(n, n, density=0.001, format="csr", random_state=rng) + sp.identity(n)
    R = R.tolil()
    R[5, :400] = 1.0
    R = stencils._canonical(R.tocsr())
    assert not _sell_fits(R)
    _sell_case(sylv, R, 2, expect_ok=False)
    # rows of 3..6 entries fit and give exact products
    T = stencils.cd1d(n, 3.0).tolil()
    for i in range(0, n, 7):
        T[i, (i + 11) % n] = 0.5
        T[i, (i + 29) % n] = -0.25
    T = stencils._canonical(T.tocsr())
    assert _sell_fits(T)
    _sell_case(sylv, T, 3)
