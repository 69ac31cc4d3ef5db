"""The library's host code (argument checks, workspace layouts and sizes,
status strings, the solver-choice inputs) under AddressSanitizer and UBSan:
api.hip is compiled with host-side sanitizers (device code is not
instrumented) and driven by tests/host_check/host_check.cpp over 1600 shapes
and the error paths; every call returns before any launch, so no GPU is
needed."""
import os
import shutil
import subprocess

import pytest

from paper_2606_19224_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))


def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    if not shutil.which("g++") or not os.path.exists(B.HIPCC):
        pytest.skip("no host compiler")
    if not all(os.path.exists(os.path.join(B.BUILD, os.path.basename(s) + ".o"))
               for s in B.sources()):
        pytest.skip("library objects not built")
    exe = B.build_host_checked(os.path.join(HERE, "host_check", "host_check.cpp"), str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "0 failures" in res.stdout
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr
