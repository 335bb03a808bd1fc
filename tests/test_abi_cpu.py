"""CPU checks of the C ABI: the library loads without a GPU, exports every function the header
declares, and its host-only calls (options, workspace sizing, status strings) behave as stated.
No device compute runs here."""
import ctypes

import numpy as np
import pytest

from workloads import configs

sylv = pytest.importorskip("paper_2605_28274_amd.sylv")


def test_exports_every_declared_symbol():
    names = sylv.declared_functions()
    assert len(names) >= 14
    lib = ctypes.CDLL(sylv.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings_and_defaults():
    assert sylv.status_string(0) == "converged"
    assert "rank" in sylv.status_string(sylv.SYLV_ERR_RHS_RANK)
    assert sylv.status_string(12345) == "unknown status"
    o = sylv.default_options()
    assert o.max_iter > 0 and o.check_every > 0 and o.closure_tol == 0.0
    assert o.precision == sylv.SYLV_FP64
    assert o.streams == 0  # automatic: second stream for large bases
    assert o.reorth == 0   # automatic: lagged second pass where available


def _problem(n=256, m=192, s=1, lyap=0, nnzA=766, nnzB=574):
    # pointers are never dereferenced by the sizing call; any non-null value works
    fake = 0x1000
    A = sylv.sylv_csr(n, nnzA, fake, fake, fake)
    B = sylv.sylv_csr(m, nnzB, fake, fake, fake)
    return sylv.sylv_problem(n, m, s, A, B, lyap, fake, s, fake, s)


def test_workspace_bytes_grows_with_max_iter_and_method():
    p = _problem()
    cg = sylv.sylv_workspace_bytes(p, sylv.default_options(sylv.SYLV_METHOD_CG, 100))
    cg2 = sylv.sylv_workspace_bytes(p, sylv.default_options(sylv.SYLV_METHOD_CG, 200))
    bi = sylv.sylv_workspace_bytes(p, sylv.default_options(sylv.SYLV_METHOD_BICGSTAB, 100))
    assert 0 < cg < cg2 and cg < bi


@pytest.mark.parametrize("bad", [
    dict(n=0), dict(s=0), dict(s=9), dict(s=300), dict(lyap=1),
])
def test_workspace_bytes_rejects_invalid(bad):
    kw = dict(n=256, m=192, s=1, lyap=0)
    kw.update(bad)
    p = _problem(**kw)
    assert sylv.sylv_workspace_bytes(p, sylv.default_options(sylv.SYLV_METHOD_CG, 10)) == 0


def test_workspace_bytes_rejects_bad_options():
    p = _problem()
    o = sylv.default_options(sylv.SYLV_METHOD_CG, 0)
    assert sylv.sylv_workspace_bytes(p, o) == 0
    o = sylv.default_options(7, 10)
    assert sylv.sylv_workspace_bytes(p, o) == 0


def test_create_rejects_missing_workspace_without_device_work():
    p = _problem()
    o = sylv.default_options(sylv.SYLV_METHOD_CG, 10)
    h = ctypes.c_void_p()
    rc = sylv._lib.sylv_create(ctypes.byref(h), ctypes.byref(p), ctypes.byref(o), None, 0, None)
    assert rc == sylv.SYLV_ERR_WORKSPACE
    rc = sylv._lib.sylv_create(None, ctypes.byref(p), ctypes.byref(o), None, 0, None)
    assert rc == sylv.SYLV_ERR_INVALID


def test_c2_workspace_is_modest():
    p = configs.c2_bicgstab()
    prob = _problem(p.n, p.m, p.s, 0, p.A.nnz, p.B.nnz)
    nb = sylv.sylv_workspace_bytes(prob, sylv.default_options(sylv.SYLV_METHOD_BICGSTAB, 800))
    assert 0 < nb < 4 * 2**30


def test_precision_and_refine_options_validated():
    p = _problem()
    base = sylv.default_options(sylv.SYLV_METHOD_BICGSTAB, 50, precision=sylv.SYLV_MIXED_FP32)
    fp64 = sylv.default_options(sylv.SYLV_METHOD_BICGSTAB, 50)
    ref = sylv.default_options(sylv.SYLV_METHOD_BICGSTAB, 50, precision=sylv.SYLV_MIXED_FP32,
                               refine_max=2)
    # FP32 bases need less workspace; refinement adds correction contexts and buffers
    assert 0 < sylv.sylv_workspace_bytes(p, base) < sylv.sylv_workspace_bytes(p, fp64)
    assert sylv.sylv_workspace_bytes(p, ref) > sylv.sylv_workspace_bytes(p, base)
    for bad in (dict(refine_max=5), dict(refine_max=1, refine_rank=0),
                dict(refine_max=1, refine_rank=9), dict(refine_max=1, refine_max_iter=0),
                dict(precision=3), dict(streams=3), dict(streams=-1), dict(reorth=3),
                dict(reorth=2)):  # the lagged pass needs FP64 bases (base is FP32)
        kw = dict(precision=sylv.SYLV_MIXED_FP32) if bad == dict(reorth=2) else {}
        kw.update(bad)
        o = sylv.default_options(sylv.SYLV_METHOD_BICGSTAB, 50, **kw)
        assert sylv.sylv_workspace_bytes(p, o) == 0, bad
    # lagged pass: FP64 bases with s <= 4 only
    assert sylv.sylv_workspace_bytes(p, sylv.default_options(sylv.SYLV_METHOD_BICGSTAB, 50,
                                                             reorth=2)) > 0
    p5 = _problem(s=5)
    assert sylv.sylv_workspace_bytes(p5, sylv.default_options(sylv.SYLV_METHOD_BICGSTAB, 50,
                                                              reorth=2)) == 0
    assert sylv.sylv_workspace_bytes(p5, sylv.default_options(sylv.SYLV_METHOD_BICGSTAB, 50)) > 0


def test_bf16split_precision_is_fp64_bases_with_split_grams():
    p = _problem(n=4096, m=2048, s=2, nnzA=20000, nnzB=6000)
    size = lambda **kw: sylv.sylv_workspace_bytes(
        p, sylv.default_options(sylv.SYLV_METHOD_BICGSTAB, 50, **kw))
    # the same workspace as FP64 bases with split-BF16 residual Grams (form 1, or 2 when asked)
    assert size(precision=sylv.SYLV_MIXED_BF16SPLIT) == size(gram_precision=1) > size()
    assert size(precision=sylv.SYLV_MIXED_BF16SPLIT, gram_precision=2) == size(gram_precision=2)
