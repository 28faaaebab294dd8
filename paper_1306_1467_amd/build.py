"""Builds libvjboost.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with packed FP32 vector
instructions disabled and no floating-point contraction or fast-math (the
compensated sums rely on exact IEEE rounding of each addition).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libvjboost.so")

SOURCES = ["api.cpp", "features.cpp", "batch.cpp", "tune.cpp", "k_prep.hip", "k_sort.hip", "k_scan.hip", "k_update.hip", "k_batch.hip",
           "k_probe.hip", "k_classify.hip"]
ARCH = os.environ.get("VJBOOST_ARCH", "gfx950")


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def common_flags():
    return ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-ffp-contract=off", "-fno-fast-math",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")]


# Per-file extra flags (none at present: every unit honours NaNs; the scan's
# quiet-NaN candidate masks rely on IEEE semantics, see scan_core.h).
EXTRA: dict = {}


# Sanitizer build of the host code (device code is built as usual): the
# host-side C++ of every unit with AddressSanitizer and UndefinedBehavior-
# Sanitizer, into _build/san/libvjboost.so.  Load it with VJBOOST_LIB and the
# clang ASan runtime preloaded (see SAN_RUNTIME).
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined", "-g"]
SAN_BUILD = os.path.join(BUILD, "san")
SAN_LIB = os.path.join(SAN_BUILD, "libvjboost.so")


def san_runtime() -> str:
    """Path of the clang ASan runtime the sanitized library needs preloaded."""
    r = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


def _compile(src: str, sanitize: bool = False) -> str:
    out_dir = SAN_BUILD if sanitize else BUILD
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    extra = SAN_FLAGS if sanitize else []
    cmd = [hipcc()] + common_flags() + EXTRA.get(src, []) + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    os.makedirs(SAN_BUILD if sanitize else BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), srcs))
    lib = SAN_LIB if sanitize else LIB
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if sanitize:
        cmd += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--sanitize":
        build(verbose=True, sanitize=True)
        print("preload:", san_runtime())
    else:
        build(verbose=True)
    sys.exit(0)
