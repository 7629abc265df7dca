"""The CPU checks of the C ABI (tests/test_abi.py) against a libgg whose host
code is built with AddressSanitizer and UndefinedBehaviorSanitizer: argument
validation, error strings and plan-creation failure paths run without memory
or undefined-behaviour errors.  Host code only; no GPU is used."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/lib/llvm/bin/clang"


def _asan_runtime():
    if not os.path.exists(CLANG):
        return None
    rdir = subprocess.run([CLANG, "--print-runtime-dir"], capture_output=True, text=True).stdout.strip()
    # the runtime sits in the per-target directory or in the older lib/linux one
    for path in (os.path.join(rdir, "libclang_rt.asan.so"), os.path.join(rdir, "libclang_rt.asan-x86_64.so"),
                 os.path.join(os.path.dirname(rdir), "linux", "libclang_rt.asan-x86_64.so")):
        if os.path.exists(path):
            return path
    return None


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_abi_checks_under_host_sanitizers():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("clang ASan runtime not found")
    from paper_2511_10353_amd import build
    lib = build.build_host_sanitized()
    env = dict(os.environ, LD_PRELOAD=rt, GG_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_abi.py"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = res.stdout[-4000:] + res.stderr[-4000:]
    assert res.returncode == 0, out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
    assert " passed" in res.stdout
