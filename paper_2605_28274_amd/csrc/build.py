"""Builds libsylv.so (HIP, gfx950) in-tree: one hipcc compile per translation unit, then a link.

Usage: python -m paper_2605_28274_amd.csrc.build   (or build() from __graft_entry__)

The same call builds a second copy, hostsan/libsylv_hostsan.so, with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code only (the kernels are compiled exactly as in
libsylv.so and are not instrumented), and the C driver hostsan/abi_hostcheck that calls the ABI
through it (tests/abi_hostcheck.c): argument handling without a GPU, real solves and batches on
one.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libsylv.so")
SAN_DIR = os.path.join(PKG, "hostsan")
SAN_LIB = os.path.join(SAN_DIR, "libsylv_hostsan.so")
SAN_DRIVER = os.path.join(SAN_DIR, "abi_hostcheck")
DRIVER_SRC = os.path.join(ROOT, "tests", "abi_hostcheck.c")

SOURCES = ["api.hip", "sparse.hip", "krylov.hip", "arnoldi.hip", "core.hip", "dense.hip",
           "residual.hip", "refine.hip", "batch.hip", "gram_bf16.hip", "core_more.hip", "compress.hip"] + [f"arnoldi_s{s}.hip" for s in range(1, 9)]
ARCH = os.environ.get("SYLV_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = os.environ.get("SYLV_CLANGXX", "/opt/rocm/llvm/bin/clang++")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    # packed FP32 instructions stay off (they are never needed in this FP64 code either)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{HERE}",
]
# host-code sanitizers: every option goes to the host pass only, so the device code is the same
# as libsylv.so's
SAN_FLAGS = ["-Xarch_host", "-g", "-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all",
             "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd: list[str], what: str) -> None:
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"{what} failed")


def _compile(src: str, out_dir: str, flags: list[str]) -> str:
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    _run([HIPCC, *flags, "-c", os.path.join(HERE, src), "-o", obj], f"hipcc on {src}")
    return obj


def _link(objs: list[str], out: str) -> None:
    tmp = out + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", *objs, "-o", tmp],
         f"link of {os.path.basename(out)}")
    os.replace(tmp, out)


def _driver() -> None:
    # clang++ links the C driver so that the sanitizers' C++ runtime parts come along; the
    # library is found next to the driver wherever the tree is copied
    tmp = SAN_DRIVER + ".tmp"
    _run([CLANGXX, "-x", "c", "-std=c11", "-O1", "-g", "-Wall", "-D__HIP_PLATFORM_AMD__",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
          f"-I{INCLUDE}", f"-I{ROCM}/include", DRIVER_SRC, "-x", "none", SAN_LIB,
          f"-L{ROCM}/lib", "-lamdhip64", "-Wl,-rpath,$ORIGIN", f"-Wl,-rpath,{ROCM}/lib", "-o",
          tmp], "build of abi_hostcheck")
    os.replace(tmp, SAN_DRIVER)


def build(verbose: bool = False, sanitized: bool = True) -> str:
    """Compiles every translation unit (and, with sanitized, its host-sanitized twin) in one
    pool, links libsylv.so (and hostsan/libsylv_hostsan.so plus its driver); returns LIB."""
    san_obj = os.path.join(BUILD_DIR, "hostsan")
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = [(src, BUILD_DIR, FLAGS) for src in SOURCES]
    if sanitized:
        os.makedirs(san_obj, exist_ok=True)
        os.makedirs(SAN_DIR, exist_ok=True)
        jobs += [(src, san_obj, FLAGS + SAN_FLAGS) for src in SOURCES]
    # the sanitized twins go first: together the two sets keep every core busy to the end
    jobs = jobs[len(SOURCES):] + jobs[:len(SOURCES)] if sanitized else jobs
    with ThreadPoolExecutor(max_workers=os.cpu_count() or 4) as ex:
        objs = list(ex.map(lambda j: _compile(*j), jobs))
    plain = [o for o in objs if os.path.dirname(o) == BUILD_DIR]
    _link(plain, LIB)
    if verbose:
        print("built", LIB)
    if sanitized:
        _link([o for o in objs if os.path.dirname(o) == san_obj], SAN_LIB)
        _driver()
        if verbose:
            print("built", SAN_LIB, "and", SAN_DRIVER)
    return LIB


if __name__ == "__main__":
    build(verbose=True, sanitized="--no-hostsan" not in sys.argv)
