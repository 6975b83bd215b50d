"""Builds libsetd.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2310_07551_amd.build [-v] [--sanitize]
Each .hip source is compiled to an object in parallel, then linked into a
shared library next to this file.

--sanitize builds libsetd_san.so instead: the host code (argument checking,
tables, orchestration) instrumented with AddressSanitizer and
UndefinedBehaviorSanitizer (host pass only; the GPU code is built as usual).
Load it with the sanitizer runtime preloaded (sanitizer_runtime() names it).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsetd.so")
OBJDIR = os.path.join(HERE, "_build")
SAN_LIB = os.path.join(HERE, "libsetd_san.so")
SAN_OBJDIR = os.path.join(HERE, "_build_san")
# host-side sanitizers: each -fsanitize= applies to the host compilation only
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-g", "-shared-libsan"]

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _compile(src: str, verbose: bool, objdir: str = OBJDIR, extra=()) -> str:
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, *extra, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, res.stdout, res.stderr))
    if verbose and res.stderr.strip():
        print(res.stderr, flush=True)
    return obj


def sanitizer_runtime() -> str:
    """Path of the AddressSanitizer runtime of the compiler that built libsetd_san.so."""
    res = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return res.stdout.strip()


def build(verbose: bool = False, sanitize: bool = False, lib_path: str = None, obj_dir: str = None) -> str:
    objdir = obj_dir or (SAN_OBJDIR if sanitize else OBJDIR)
    lib = lib_path or (SAN_LIB if sanitize else LIB)
    extra = SAN_FLAGS if sanitize else []
    os.makedirs(objdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, objdir, extra), srcs))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *extra, "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (res.stdout, res.stderr))
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
