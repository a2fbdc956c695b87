"""The library's host code (the C ABI's argument checks, point validation,
item checks, workspace and checkpoint handling) built with AddressSanitizer
and UndefinedBehaviorSanitizer on the host side and driven by
tests/sanitize/host_driver.cpp: on the CPU the checks that run before any
device call, on a GPU also evaluation, the adjoint, an adaptive run and
checkpoint save / load with truncated and corrupted blobs.  Every call must
return its documented status and no sanitizer may report."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "bin", "rift_host_asan")


def _exe():
    if not os.path.exists(EXE):
        sys.path.insert(0, os.path.join(HERE, "sanitize"))
        import build_host_asan
        build_host_asan.build()
    return EXE


def _run(mode, leaks):
    env = dict(os.environ, ASAN_OPTIONS=f"detect_leaks={1 if leaks else 0}:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([_exe(), mode], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "runtime error" not in out and "AddressSanitizer" not in out and "LeakSanitizer" not in out, out
    assert r.stdout.splitlines()[-1].startswith("ok "), out
    return r.stdout


def test_host_code_under_sanitizers():
    print(_run("host", leaks=True).strip().splitlines()[-1])


@pytest.mark.gpu
def test_host_code_under_sanitizers_on_device():
    # the HIP runtime keeps its own allocations until exit: no leak check here
    print(_run("device", leaks=False), flush=True)
