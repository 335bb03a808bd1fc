"""The C ABI under AddressSanitizer and UndefinedBehaviorSanitizer on the host code.

The build script builds hostsan/libsylv_hostsan.so (host code instrumented, kernels as in
libsylv.so) and the C driver hostsan/abi_hostcheck (tests/abi_hostcheck.c) next to libsylv.so.

* CPU: every entry point with missing pointers, sizes out of range (up to the int64 limit),
  malformed CSR headers and unknown options returns its documented error without device work,
  and the workspace sizing runs over many valid problems, with no sanitizer report.
* GPU: single solves of every method (FP64, FP32 bases with refinement, Lyapunov), residual,
  factors, history, compression, kernel statistics, batches in the three forms (worker and
  finisher threads) and the building-block calls, with no sanitizer report and every check met.
"""
import os
import subprocess

import pytest

from paper_2605_28274_amd.csrc import build as _build

# the HIP runtime keeps allocations until the process ends: leak reports would name it, not us
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:protect_shadow_gap=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _driver(build_if_missing: bool) -> str:
    if not os.path.exists(_build.SAN_DRIVER):
        if not build_if_missing:
            pytest.fail("hostsan/abi_hostcheck is not built (run the build script first)")
        _build.build()
    return _build.SAN_DRIVER


def _run(mode: str, timeout: int, build_if_missing: bool) -> subprocess.CompletedProcess:
    drv = _driver(build_if_missing)
    print(f"running {drv} {mode}", flush=True)
    r = subprocess.run([drv, mode], env=ENV, capture_output=True, text=True, timeout=timeout)
    print(r.stdout[-4000:], r.stderr[-4000:], flush=True)
    return r


def test_argument_handling_under_sanitizers():
    r = _run("args", 120, build_if_missing=True)
    assert "Sanitizer" not in r.stderr, r.stderr
    assert r.returncode == 0 and "0 failed" in r.stdout, r.stdout


@pytest.mark.gpu
def test_solves_and_batches_under_host_sanitizers():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = _run("solve", 300, build_if_missing=False)
    assert "Sanitizer" not in r.stderr, r.stderr
    assert r.returncode == 0 and "0 failed" in r.stdout, r.stdout
    for name in ("cg", "bicgstab", "cr", "cgs", "gpbicg", "lyapunov_cg", "batch form 2"):
        assert name in r.stdout
