"""Thin ctypes binding of libsylv (C ABI in ``include/sylv.h``).

Argument marshalling only: every step of the solve runs in the HIP kernels of ``libsylv.so``.
PyTorch provides the device memory (CSR arrays, right-hand sides, workspace, outputs) and the
stream. Importing this module raises if the library has not been built; there is no fallback.

Functions keep the C names (``sylv_create``, ``sylv_factored_cg``, ...). :class:`Solver` bundles
one context with the device tensors it borrows, so they stay alive as long as the context.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, byref, c_double, c_int, c_int64, c_size_t, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsylv.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "sylv.h")

SYLV_OK, SYLV_NOT_CONVERGED, SYLV_BREAKDOWN = 0, 1, 2
SYLV_ERR_INVALID, SYLV_ERR_HIP, SYLV_ERR_WORKSPACE = -1, -2, -3
SYLV_ERR_RHS_RANK, SYLV_ERR_STATE = -4, -5
SYLV_METHOD_CG, SYLV_METHOD_BICGSTAB = 0, 1
SYLV_METHOD_CR, SYLV_METHOD_CGS, SYLV_METHOD_GPBICG = 2, 3, 4
SYLV_FP64, SYLV_MIXED_FP32, SYLV_MIXED_BF16SPLIT = 0, 1, 2
SYLV_BATCH_STREAMS, SYLV_BATCH_GROUPED, SYLV_BATCH_GRAPH = 0, 1, 2


class SylvError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = f"{what}: {status_string(code)} ({code})"
        if code == SYLV_ERR_HIP:
            msg += f" [{_lib.sylv_last_error().decode()}]"
        super().__init__(msg)
        self.code = code


def _load():
    # torch ships its own HIP runtime; loading it first makes libsylv bind to that same runtime
    # (one HIP runtime per process, shared device memory and streams)
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first (__graft_entry__.build())")
    return ctypes.CDLL(LIB_PATH)


_lib = _load()


class sylv_csr(ctypes.Structure):
    _fields_ = [("rows", c_int64), ("nnz", c_int64), ("row_ptr", c_void_p),
                ("col_idx", c_void_p), ("values", c_void_p)]


class sylv_problem(ctypes.Structure):
    _fields_ = [("n", c_int64), ("m", c_int64), ("s", c_int64), ("A", sylv_csr), ("B", sylv_csr),
                ("lyapunov", c_int), ("C1", c_void_p), ("ldc1", c_int64), ("C2", c_void_p),
                ("ldc2", c_int64)]


class sylv_options(ctypes.Structure):
    _fields_ = [("method", c_int), ("max_iter", c_int), ("check_every", c_int),
                ("record_history", c_int), ("closure_tol", c_double), ("precision", c_int),
                ("refine_max", c_int), ("refine_max_iter", c_int), ("refine_rank", c_int),
                ("refine_inner_tol", c_double), ("streams", c_int), ("reorth", c_int),
                ("gram_precision", c_int), ("verify", c_int)]


class sylv_result(ctypes.Structure):
    _fields_ = [("status", c_int), ("iters", c_int), ("rank_v", c_int64), ("rank_w", c_int64),
                ("rel_res_recursive", c_double), ("seconds", c_double), ("outer_steps", c_int),
                ("rel_res_true", c_double)]


_lib.sylv_default_options.argtypes = [POINTER(sylv_options)]
_lib.sylv_default_options.restype = None
_lib.sylv_workspace_bytes.argtypes = [POINTER(sylv_problem), POINTER(sylv_options)]
_lib.sylv_workspace_bytes.restype = c_size_t
_lib.sylv_create.argtypes = [POINTER(c_void_p), POINTER(sylv_problem), POINTER(sylv_options),
                             c_void_p, c_size_t, c_void_p]
_lib.sylv_create.restype = c_int
for _f in ("sylv_factored_cg", "sylv_factored_bicgstab", "sylv_factored_cr", "sylv_factored_cgs",
           "sylv_factored_gpbicg"):
    getattr(_lib, _f).argtypes = [c_void_p, c_double, c_int, POINTER(sylv_result)]
    getattr(_lib, _f).restype = c_int
_lib.sylv_compress.argtypes = [c_void_p, c_double, c_int64, POINTER(c_int64), POINTER(c_double)]
_lib.sylv_compress.restype = c_int
_lib.sylv_get_compressed.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_int64,
                                     POINTER(c_int64)]
_lib.sylv_get_compressed.restype = c_int
_lib.sylv_residual_norm.argtypes = [c_void_p, POINTER(c_double), POINTER(c_double)]
_lib.sylv_residual_norm.restype = c_int
_lib.sylv_get_factors.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                                  c_int64, POINTER(c_int64), POINTER(c_int64)]
_lib.sylv_get_factors.restype = c_int
_lib.sylv_get_history.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                  POINTER(c_int)]
_lib.sylv_get_history.restype = c_int
_lib.sylv_destroy.argtypes = [c_void_p]
_lib.sylv_destroy.restype = None
_lib.sylv_status_string.argtypes = [c_int]
_lib.sylv_status_string.restype = ctypes.c_char_p
_lib.sylv_last_error.argtypes = []
_lib.sylv_last_error.restype = ctypes.c_char_p
_lib.sylv_spmm.argtypes = [POINTER(sylv_csr), c_int64, c_void_p, c_int64, c_void_p, c_int64,
                           c_void_p]
_lib.sylv_spmm.restype = c_int
_lib.sylv_csr_transpose_scratch_bytes.argtypes = [c_int64]
_lib.sylv_csr_transpose_scratch_bytes.restype = c_size_t
_lib.sylv_csr_transpose.argtypes = [POINTER(sylv_csr), c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_void_p]
_lib.sylv_csr_transpose.restype = c_int
_lib.sylv_csr_transpose_noalloc.argtypes = [POINTER(sylv_csr), c_void_p, c_void_p, c_void_p,
                                            c_void_p]
_lib.sylv_csr_transpose_noalloc.restype = c_int
SYLV_NOALLOC_TRANSPOSE_MAX_ROWS = 1 << 21
class sylv_kernel_stat(ctypes.Structure):
    _fields_ = [("family", c_int), ("launches", c_int64), ("ms", c_double), ("bytes", c_double),
                ("flops", c_double)]


_lib.sylv_set_profiling.argtypes = [c_void_p, c_int]
_lib.sylv_set_profiling.restype = c_int
_lib.sylv_get_kernel_stats.argtypes = [c_void_p, POINTER(sylv_kernel_stat), c_int, POINTER(c_int)]
_lib.sylv_get_kernel_stats.restype = c_int
_lib.sylv_kernel_family_name.argtypes = [c_int]
_lib.sylv_kernel_family_name.restype = ctypes.c_char_p
_lib.sylv_sell_bytes.argtypes = [POINTER(sylv_csr)]
_lib.sylv_sell_bytes.restype = c_size_t
_lib.sylv_sell_build.argtypes = [POINTER(sylv_csr), c_void_p, c_size_t, c_void_p]
_lib.sylv_sell_build.restype = c_int
_lib.sylv_sell_spmm.argtypes = [POINTER(sylv_csr), c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                                c_int64, c_void_p]
_lib.sylv_sell_spmm.restype = c_int
_lib.sylv_dgemm.argtypes = [c_int64, c_int64, c_int64, c_double, c_void_p, c_int64, c_int64,
                            c_void_p, c_int64, c_int64, c_double, c_void_p, c_int64, c_void_p]
_lib.sylv_dgemm.restype = c_int
_lib.sylv_gram_work_bytes.argtypes = [c_int64, c_int64, c_int64]
_lib.sylv_gram_work_bytes.restype = c_size_t
_lib.sylv_gram.argtypes = [c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64, c_int,
                           c_int, c_void_p, c_int64, c_void_p, c_size_t, c_void_p]
_lib.sylv_gram.restype = c_int
_lib.sylv_batch_workspace_bytes.argtypes = [c_int, c_void_p, c_void_p]
_lib.sylv_batch_workspace_bytes.restype = c_size_t
_lib.sylv_batch_create.argtypes = [POINTER(c_void_p), c_int, c_void_p, c_void_p, c_void_p,
                                   c_size_t, c_int]
_lib.sylv_batch_create.restype = c_int
_lib.sylv_batch_create_ex.argtypes = [POINTER(c_void_p), c_int, c_void_p, c_void_p, c_void_p,
                                      c_size_t, c_int, c_int]
_lib.sylv_batch_create_ex.restype = c_int
_lib.sylv_batch_groups.argtypes = [c_void_p]
_lib.sylv_batch_groups.restype = c_int
_lib.sylv_batch_solve.argtypes = [c_void_p, c_double, c_void_p]
_lib.sylv_batch_solve.restype = c_int
_lib.sylv_batch_context.argtypes = [c_void_p, c_int]
_lib.sylv_batch_context.restype = c_void_p
_lib.sylv_batch_destroy.argtypes = [c_void_p]
_lib.sylv_batch_destroy.restype = None


def declared_functions(header: str = HEADER_PATH) -> list[str]:
    """Names of the functions ``include/sylv.h`` declares."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sylv_[a-z_]+)\s*\(", text)))


def status_string(code: int) -> str:
    return _lib.sylv_status_string(int(code)).decode()


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return c_void_p(torch.cuda.current_stream().cuda_stream)
    return c_void_p(int(stream))


# ---- CSR helpers (device tensors) ----------------------------------------------------------

def csr_tensors(M, device="cuda"):
    """(row_ptr int32, col_idx int32, values float64) device tensors of a SciPy CSR matrix."""
    import torch
    rp = torch.as_tensor(np.ascontiguousarray(M.indptr, dtype=np.int32), device=device)
    ci = torch.as_tensor(np.ascontiguousarray(M.indices, dtype=np.int32), device=device)
    va = torch.as_tensor(np.ascontiguousarray(M.data, dtype=np.float64), device=device)
    return rp, ci, va


def make_csr(rows: int, rp, ci, va) -> sylv_csr:
    return sylv_csr(rows, int(ci.numel()), _ptr(rp), _ptr(ci), _ptr(va))


def default_options(method: int = SYLV_METHOD_BICGSTAB, max_iter: int = 200, **kw) -> sylv_options:
    o = sylv_options()
    _lib.sylv_default_options(byref(o))
    o.method = method
    o.max_iter = max_iter
    for k, v in kw.items():
        setattr(o, k, v)
    return o


# ---- C-named wrappers ----------------------------------------------------------------------

def sylv_workspace_bytes(problem: sylv_problem, options: sylv_options) -> int:
    return int(_lib.sylv_workspace_bytes(byref(problem), byref(options)))


def sylv_create(problem: sylv_problem, options: sylv_options, workspace, stream=None):
    h = c_void_p()
    rc = _lib.sylv_create(byref(h), byref(problem), byref(options), c_void_p(_ptr(workspace)),
                          c_size_t(workspace.numel() * workspace.element_size()), _stream(stream))
    if rc != 0:
        raise SylvError(rc, "sylv_create")
    return h


def _solve(fn, ctx, tol, max_iter):
    res = sylv_result()
    rc = fn(ctx, c_double(tol), c_int(max_iter), byref(res))
    if rc < 0:
        raise SylvError(rc, fn.__name__)
    return res


def sylv_factored_cg(ctx, tol: float, max_iter: int) -> sylv_result:
    return _solve(_lib.sylv_factored_cg, ctx, tol, max_iter)


def sylv_factored_bicgstab(ctx, tol: float, max_iter: int) -> sylv_result:
    return _solve(_lib.sylv_factored_bicgstab, ctx, tol, max_iter)


def sylv_factored_cr(ctx, tol: float, max_iter: int) -> sylv_result:
    return _solve(_lib.sylv_factored_cr, ctx, tol, max_iter)


def sylv_factored_cgs(ctx, tol: float, max_iter: int) -> sylv_result:
    return _solve(_lib.sylv_factored_cgs, ctx, tol, max_iter)


def sylv_factored_gpbicg(ctx, tol: float, max_iter: int) -> sylv_result:
    return _solve(_lib.sylv_factored_gpbicg, ctx, tol, max_iter)


METHOD_CODES = {"cg": SYLV_METHOD_CG, "bicgstab": SYLV_METHOD_BICGSTAB, "cr": SYLV_METHOD_CR,
                "cgs": SYLV_METHOD_CGS, "gpbicg": SYLV_METHOD_GPBICG}
SOLVERS = {SYLV_METHOD_CG: "sylv_factored_cg", SYLV_METHOD_BICGSTAB: "sylv_factored_bicgstab",
           SYLV_METHOD_CR: "sylv_factored_cr", SYLV_METHOD_CGS: "sylv_factored_cgs",
           SYLV_METHOD_GPBICG: "sylv_factored_gpbicg"}


def sylv_compress(ctx, rel_tol: float, max_rank: int = -1):
    """Returns (status, rank, achieved relative error)."""
    k, err = c_int64(), c_double()
    rc = _lib.sylv_compress(ctx, c_double(rel_tol), c_int64(max_rank), byref(k), byref(err))
    if rc < 0:
        raise SylvError(rc, "sylv_compress")
    return rc, k.value, err.value


def sylv_get_compressed(ctx, Z1=None, sigma=None, Z2=None):
    k = c_int64()
    ld = lambda t: int(t.stride(0)) if t is not None and t.dim() == 2 else 0  # noqa: E731
    rc = _lib.sylv_get_compressed(ctx, c_void_p(_ptr(Z1)), ld(Z1), c_void_p(_ptr(sigma)),
                                  c_void_p(_ptr(Z2)), ld(Z2), byref(k))
    if rc != 0:
        raise SylvError(rc, "sylv_get_compressed")
    return k.value


def sylv_residual_norm(ctx):
    a, r = c_double(), c_double()
    rc = _lib.sylv_residual_norm(ctx, byref(a), byref(r))
    if rc != 0:
        raise SylvError(rc, "sylv_residual_norm")
    return a.value, r.value


def sylv_get_factors(ctx, V=None, Xc=None, W=None):
    """Copies the factors into the given device tensors (any may be None); returns the ranks."""
    rv, rw = c_int64(), c_int64()
    ld = lambda t: int(t.stride(0)) if t is not None else 0  # noqa: E731
    rc = _lib.sylv_get_factors(ctx, c_void_p(_ptr(V)), ld(V), c_void_p(_ptr(Xc)), ld(Xc),
                               c_void_p(_ptr(W)), ld(W), byref(rv), byref(rw))
    if rc != 0:
        raise SylvError(rc, "sylv_get_factors")
    return rv.value, rw.value


def sylv_get_history(ctx, cap: int):
    rel, al, be, om = (np.zeros(cap) for _ in range(4))
    cnt = c_int()
    p = lambda a: a.ctypes.data_as(c_void_p)  # noqa: E731
    rc = _lib.sylv_get_history(ctx, p(rel), p(al), p(be), p(om), c_int(cap), byref(cnt))
    if rc != 0:
        raise SylvError(rc, "sylv_get_history")
    n = min(cnt.value, cap)
    return {"relres": rel[:n], "alpha": al[:n], "beta": be[:n], "omega": om[:n],
            "iters": cnt.value}


def sylv_destroy(ctx) -> None:
    _lib.sylv_destroy(ctx)


def sylv_set_profiling(ctx, on: bool) -> None:
    rc = _lib.sylv_set_profiling(ctx, 1 if on else 0)
    if rc != 0:
        raise SylvError(rc, "sylv_set_profiling")


def sylv_kernel_family_name(family: int) -> str:
    return _lib.sylv_kernel_family_name(int(family)).decode()


def sylv_get_kernel_stats(ctx) -> list[dict]:
    buf = (sylv_kernel_stat * 32)()
    cnt = c_int()
    rc = _lib.sylv_get_kernel_stats(ctx, buf, 32, byref(cnt))
    if rc != 0:
        raise SylvError(rc, "sylv_get_kernel_stats")
    return [{"family": sylv_kernel_family_name(b.family), "launches": b.launches, "ms": b.ms,
             "bytes": b.bytes, "flops": b.flops} for b in buf[:cnt.value]]


def sylv_spmm(csr: sylv_csr, s: int, X, Y, stream=None) -> None:
    rc = _lib.sylv_spmm(byref(csr), s, c_void_p(_ptr(X)), int(X.stride(0)), c_void_p(_ptr(Y)),
                        int(Y.stride(0)), _stream(stream))
    if rc != 0:
        raise SylvError(rc, "sylv_spmm")


def sylv_sell_bytes(csr: sylv_csr) -> int:
    return int(_lib.sylv_sell_bytes(byref(csr)))


def sylv_sell_build(csr: sylv_csr, buf, stream=None) -> None:
    rc = _lib.sylv_sell_build(byref(csr), c_void_p(_ptr(buf)),
                              c_size_t(buf.numel() * buf.element_size()), _stream(stream))
    if rc != 0:
        raise SylvError(rc, "sylv_sell_build")


def sylv_sell_spmm(csr: sylv_csr, buf, s: int, X, Y, stream=None) -> None:
    rc = _lib.sylv_sell_spmm(byref(csr), c_void_p(_ptr(buf)), s, c_void_p(_ptr(X)),
                             int(X.stride(0)), c_void_p(_ptr(Y)), int(Y.stride(0)),
                             _stream(stream))
    if rc != 0:
        raise SylvError(rc, "sylv_sell_spmm")


def sylv_csr_transpose(csr: sylv_csr, out_rp, out_ci, out_va, scratch, stream=None) -> None:
    rc = _lib.sylv_csr_transpose(byref(csr), c_void_p(_ptr(out_rp)), c_void_p(_ptr(out_ci)),
                                 c_void_p(_ptr(out_va)), c_void_p(_ptr(scratch)), _stream(stream))
    if rc != 0:
        raise SylvError(rc, "sylv_csr_transpose")


def sylv_csr_transpose_noalloc(csr: sylv_csr, out_rp, out_ci, out_va, stream=None) -> None:
    """Enqueues the transpose on the stream and returns (no synchronization)."""
    rc = _lib.sylv_csr_transpose_noalloc(byref(csr), c_void_p(_ptr(out_rp)),
                                         c_void_p(_ptr(out_ci)), c_void_p(_ptr(out_va)),
                                         _stream(stream))
    if rc != 0:
        raise SylvError(rc, "sylv_csr_transpose_noalloc")


def sylv_dgemm(M, N, K, alpha, A, a_rs, a_cs, B, b_rs, b_cs, beta, C, ldc, stream=None) -> None:
    rc = _lib.sylv_dgemm(M, N, K, alpha, c_void_p(_ptr(A)), a_rs, a_cs, c_void_p(_ptr(B)), b_rs,
                         b_cs, beta, c_void_p(_ptr(C)), ldc, _stream(stream))
    if rc != 0:
        raise SylvError(rc, "sylv_dgemm")


def sylv_gram_work_bytes(M: int, N: int, K: int) -> int:
    return int(_lib.sylv_gram_work_bytes(M, N, K))


def sylv_gram(M, N, K, A, lda, B, ldb, C, ldc, symmetric=False, accumulate=False, work=None,
              work_bytes=0, stream=None) -> None:
    """C = A^T B (C += with accumulate) for row-major K x M and K x N device operands."""
    rc = _lib.sylv_gram(M, N, K, c_void_p(_ptr(A)), lda, c_void_p(_ptr(B)), ldb,
                        1 if symmetric else 0, 1 if accumulate else 0, c_void_p(_ptr(C)), ldc,
                        c_void_p(_ptr(work)), work_bytes, _stream(stream))
    if rc != 0:
        raise SylvError(rc, "sylv_gram")


def sylv_csr_transpose_scratch_bytes(rows: int) -> int:
    return int(_lib.sylv_csr_transpose_scratch_bytes(rows))


# ---- one context with the device memory it borrows -----------------------------------------

class Solver:
    """Holds the device copies of (A, B, C1, C2), the workspace and the context of one problem.

    ``A``, ``B``: SciPy CSR matrices (int32 indices, float64 values); ``C1``, ``C2``: float64
    arrays (n x s, m x s). ``method`` and ``max_iter`` size the workspace."""

    def __init__(self, A, B, C1, C2, lyapunov=False, method=SYLV_METHOD_BICGSTAB, max_iter=200,
                 check_every=16, closure_tol=0.0, precision=0, refine_max=0, refine_max_iter=100,
                 refine_rank=8, refine_inner_tol=0.0, streams=0, reorth=0, gram_precision=0,
                 verify=1, device="cuda", stream=None):
        import torch
        self.device = device
        self.n, self.s = C1.shape
        self.m = self.n if lyapunov else B.shape[0]
        self._A = csr_tensors(A, device)
        self._B = self._A if lyapunov else csr_tensors(B, device)
        self._C1 = torch.as_tensor(np.ascontiguousarray(C1, dtype=np.float64), device=device)
        self._C2 = self._C1 if lyapunov else torch.as_tensor(
            np.ascontiguousarray(C2, dtype=np.float64), device=device)
        self.problem = sylv_problem(
            self.n, self.m, self.s, make_csr(self.n, *self._A), make_csr(self.m, *self._B),
            1 if lyapunov else 0, _ptr(self._C1), self.s, _ptr(self._C2), self.s)
        self.options = default_options(method, max_iter, check_every=check_every,
                                       closure_tol=closure_tol, precision=precision,
                                       refine_max=refine_max, refine_max_iter=refine_max_iter,
                                       refine_rank=refine_rank, refine_inner_tol=refine_inner_tol,
                                       streams=streams, reorth=reorth,
                                       gram_precision=gram_precision, verify=verify)
        nbytes = sylv_workspace_bytes(self.problem, self.options)
        if nbytes == 0:
            raise SylvError(SYLV_ERR_INVALID, "sylv_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream
        self.ctx = sylv_create(self.problem, self.options, self.workspace, stream)
        self.max_iter = max_iter

    def factored_cg(self, tol, max_iter=None):
        return sylv_factored_cg(self.ctx, tol, max_iter or self.max_iter)

    def factored_bicgstab(self, tol, max_iter=None):
        return sylv_factored_bicgstab(self.ctx, tol, max_iter or self.max_iter)

    def solve(self, tol, max_iter=None):
        """The method the context was created for."""
        fn = globals()[SOLVERS[self.options.method]]
        return fn(self.ctx, tol, max_iter or self.max_iter)

    def residual_norm(self):
        return sylv_residual_norm(self.ctx)

    def get_factors(self):
        """(V, Xc, W) as float64 device tensors."""
        import torch
        rv, rw = sylv_get_factors(self.ctx)
        V = torch.empty((self.n, max(rv, 1)), dtype=torch.float64, device=self.device)
        X = torch.empty((max(rv, 1), max(rw, 1)), dtype=torch.float64, device=self.device)
        W = torch.empty((self.m, max(rw, 1)), dtype=torch.float64, device=self.device)
        if rv:
            sylv_get_factors(self.ctx, V, X, W)
        return V[:, :rv], X[:rv, :rw], W[:, :rw]

    def compress(self, rel_tol, max_rank=-1):
        """Truncated SVD of the solution: (status, Z1, sigma, Z2, achieved relative error) with
        X ~= Z1 diag(sigma) Z2^T, device tensors."""
        import torch
        st, k, err = sylv_compress(self.ctx, rel_tol, max_rank)
        Z1 = torch.empty((self.n, max(k, 1)), dtype=torch.float64, device=self.device)
        Z2 = torch.empty((self.m, max(k, 1)), dtype=torch.float64, device=self.device)
        sig = torch.empty(max(k, 1), dtype=torch.float64, device=self.device)
        if k:
            sylv_get_compressed(self.ctx, Z1, sig, Z2)
        return st, Z1[:, :k], sig[:k], Z2[:, :k], err

    def get_history(self, cap=None):
        return sylv_get_history(self.ctx, cap or self.max_iter)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            sylv_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- batches ----------------------------------------------------------------------------------

def sylv_batch_workspace_bytes(problems, options) -> int:
    P = (sylv_problem * len(problems))(*problems)
    O = (sylv_options * len(options))(*options)
    return int(_lib.sylv_batch_workspace_bytes(len(problems), P, O))


def sylv_batch_create(problems, options, workspace, nstreams: int):
    P = (sylv_problem * len(problems))(*problems)
    O = (sylv_options * len(options))(*options)
    h = c_void_p()
    rc = _lib.sylv_batch_create(byref(h), len(problems), P, O, c_void_p(_ptr(workspace)),
                                c_size_t(workspace.numel() * workspace.element_size()),
                                int(nstreams))
    if rc != 0:
        raise SylvError(rc, "sylv_batch_create")
    return h


def sylv_batch_create_ex(problems, options, workspace, nstreams: int, form: int):
    P = (sylv_problem * len(problems))(*problems)
    O = (sylv_options * len(options))(*options)
    h = c_void_p()
    rc = _lib.sylv_batch_create_ex(byref(h), len(problems), P, O, c_void_p(_ptr(workspace)),
                                   c_size_t(workspace.numel() * workspace.element_size()),
                                   int(nstreams), int(form))
    if rc != 0:
        raise SylvError(rc, "sylv_batch_create_ex")
    return h


def sylv_batch_groups(batch) -> int:
    return int(_lib.sylv_batch_groups(batch))


def sylv_batch_solve(batch, tol: float, count: int):
    R = (sylv_result * count)()
    rc = _lib.sylv_batch_solve(batch, c_double(tol), R)
    if rc < 0:
        raise SylvError(rc, "sylv_batch_solve")
    return list(R)


def sylv_batch_context(batch, i: int):
    return c_void_p(_lib.sylv_batch_context(batch, int(i)))


def sylv_batch_destroy(batch) -> None:
    _lib.sylv_batch_destroy(batch)


class Batch:
    """Device copies and contexts of a batch of problems (workloads.Problem-like objects with
    A, B, C1, C2, lyapunov, method, max_iter), solved together by sylv_batch_solve."""

    def __init__(self, problems, nstreams=8, precision=0, device="cuda", form=None, verify=1):
        import torch
        self._keep = []
        probs, opts = [], []
        for p in problems:
            A = csr_tensors(p.A, device)
            Bm = A if p.lyapunov else csr_tensors(p.B, device)
            C1 = torch.as_tensor(np.ascontiguousarray(p.C1, dtype=np.float64), device=device)
            C2 = C1 if p.lyapunov else torch.as_tensor(
                np.ascontiguousarray(p.C2, dtype=np.float64), device=device)
            self._keep += [A, Bm, C1, C2]
            n, s = p.C1.shape
            m = n if p.lyapunov else p.B.shape[0]
            probs.append(sylv_problem(n, m, s, make_csr(n, *A), make_csr(m, *Bm),
                                      1 if p.lyapunov else 0, _ptr(C1), s, _ptr(C2), s))
            method = METHOD_CODES[p.method]
            opts.append(default_options(method, p.max_iter, precision=precision, verify=verify))
        self.problems, self.options = probs, opts
        nbytes = sylv_batch_workspace_bytes(probs, opts)
        if nbytes == 0:
            raise SylvError(SYLV_ERR_INVALID, "sylv_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.form = SYLV_BATCH_STREAMS if form is None else form
        self.handle = sylv_batch_create_ex(probs, opts, self.workspace, nstreams, self.form)
        self.count = len(probs)

    def solve(self, tol):
        return sylv_batch_solve(self.handle, tol, self.count)

    def context(self, i):
        return sylv_batch_context(self.handle, i)

    def groups(self):
        return sylv_batch_groups(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None:
            sylv_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
