"""sylv_csr_transpose_noalloc: the CSR transpose with its scratch in the library's static device
array, for callers that cannot allocate. Its output must equal the allocating entry point's
(sylv_csr_transpose, caller scratch) bit for bit, on two calls in a row with the second input
smaller (the shared scratch keeps the first call's contents and must be cleared), and the exact
transpose (SciPy's, with sorted indices)."""
import numpy as np
import pytest
import scipy.sparse as sp

from workloads import stencils

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sylv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_28274_amd import sylv as _s
    return _s


def _random_csr(rows, density, seed):
    rng = np.random.default_rng(seed)
    M = sp.random(rows, rows, density=density, random_state=rng, format="csr")
    M = M + sp.identity(rows, format="csr")
    return stencils._canonical(M)


def _transpose_both(sylv, M):
    rows, nnz = M.shape[0], M.nnz
    rp, ci, va = sylv.csr_tensors(M)
    csr = sylv.make_csr(rows, rp, ci, va)
    outs = []
    for noalloc in (False, True):
        orp = torch.full((rows + 1,), -7, dtype=torch.int32, device="cuda")
        oci = torch.full((max(nnz, 1),), -7, dtype=torch.int32, device="cuda")
        ova = torch.full((max(nnz, 1),), np.nan, dtype=torch.float64, device="cuda")
        if noalloc:
            sylv.sylv_csr_transpose_noalloc(csr, orp, oci, ova)
            torch.cuda.synchronize()
        else:
            scr = torch.empty(sylv.sylv_csr_transpose_scratch_bytes(rows), dtype=torch.uint8,
                              device="cuda")
            sylv.sylv_csr_transpose(csr, orp, oci, ova, scr)
        outs.append((orp.cpu().numpy(), oci.cpu().numpy()[:nnz], ova.cpu().numpy()[:nnz]))
    return outs


@pytest.mark.parametrize("first,second", [((20000, 3e-4, 1), (3000, 2e-3, 2)),
                                          ((256 * 256, 0, 3), (1000, 0, 4))])
def test_noalloc_transpose_matches_allocating_entry_point(sylv, first, second):
    for rows, dens, seed in (first, second):
        M = _random_csr(rows, dens, seed) if dens else stencils.cd2d(int(np.sqrt(rows)),
                                                                       rows // int(np.sqrt(rows)),
                                                                       7.0)
        (a_rp, a_ci, a_va), (b_rp, b_ci, b_va) = _transpose_both(sylv, M)
        assert np.array_equal(a_rp, b_rp) and np.array_equal(a_ci, b_ci)
        assert np.array_equal(a_va.view(np.int64), b_va.view(np.int64))
        T = stencils._canonical(M.T)
        assert np.array_equal(b_rp, T.indptr) and np.array_equal(b_ci, T.indices)
        assert np.array_equal(b_va, T.data)


def test_noalloc_transpose_rejects_rows_over_the_limit(sylv):
    rows = sylv.SYLV_NOALLOC_TRANSPOSE_MAX_ROWS + 1
    rp = torch.zeros(rows + 1, dtype=torch.int32, device="cuda")
    csr = sylv.sylv_csr(rows, 0, int(rp.data_ptr()), 0, 0)
    orp = torch.empty(rows + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(sylv.SylvError) as ei:
        sylv.sylv_csr_transpose_noalloc(csr, orp, None, None)
    assert ei.value.code == sylv.SYLV_ERR_WORKSPACE
