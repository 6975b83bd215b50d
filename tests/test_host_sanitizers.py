"""The host side of the C ABI (argument checking, size arithmetic, error
reporting) under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is rebuilt with both sanitizers on its host code (the GPU code is
unchanged) into a temporary directory, and the argument-validation checks of
tests/test_abi.py run against it in a child process with the sanitizer
runtime preloaded; any report aborts the child.  No GPU is needed: every
call returns before it would touch a device.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, %(root)r)
from paper_2310_07551_amd import _lib
_lib.load(%(lib)r)
import tests.test_abi as t
t.test_header_declares_the_boundary()
t.test_library_exports_every_declared_symbol()
t.test_version_and_empty_error()
t.test_workspace_size_is_host_only()
t.test_validation_errors_before_any_launch()
t.test_python_binding_raises_on_error()
print("sanitized checks done")
"""


def test_abi_validation_under_host_sanitizers(tmp_path):
    from paper_2310_07551_amd import build
    lib = build.build(sanitize=True, lib_path=str(tmp_path / "libsetd_san.so"), obj_dir=str(tmp_path / "obj"))
    rt = build.sanitizer_runtime()
    if not os.path.exists(rt):
        pytest.skip("no AddressSanitizer runtime next to hipcc's clang")
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([sys.executable, "-c", CHILD % {"root": ROOT, "lib": lib}], env=env, cwd=ROOT,
                         capture_output=True, text=True, timeout=300)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "sanitized checks done" in out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
