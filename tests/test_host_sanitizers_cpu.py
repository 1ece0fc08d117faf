"""The host runtime (plan, layout, validation, every entry point's host path, the
autotuner's host logic) under AddressSanitizer and UndefinedBehaviorSanitizer: the
library's host code built with both (build_lib --sanitize; the device code as usual),
the host-side test files run against it with the sanitizer runtime preloaded.  The
address-space-capped catch-all test is left out: the sanitizer's shadow memory does not
fit under that cap."""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sanitized_library():
    from paper_0902_0827_amd import build_lib
    lib = build_lib.SAN_LIB
    sources = glob.glob(os.path.join(build_lib.CSRC, "*")) + glob.glob(os.path.join(build_lib.INCLUDE, "*"))
    if not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(f) for f in sources):
        lib = build_lib.build(sanitize=True)
    return lib


def test_host_runtime_is_clean_under_asan_and_ubsan():
    if not os.path.exists(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc is not available")
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("the clang AddressSanitizer runtime is not installed")
    lib = _sanitized_library()
    env = dict(os.environ, LD_PRELOAD=rt[-1], NBHIP_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", "tests/test_abi_cpu.py", "tests/test_autotune_cpu.py", "-q",
           "-p", "no:cacheprovider", "-m", "not gpu",
           "--deselect", "tests/test_abi_cpu.py::test_no_exception_crosses_the_abi"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, out
    assert " passed" in r.stdout
