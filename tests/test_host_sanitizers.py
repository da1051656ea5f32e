"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer: libsr's
sr_api.cpp (argument checks, workspace carving and size arithmetic) is rebuilt with both
sanitizers and the CPU ABI tests run against it in a child process that preloads the ASan
runtime.  Any sanitizer report fails the child (UBSan halts on the first error)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc_present():
    from paper_1108_0900_amd import build
    return os.path.exists(build.HIPCC) and os.path.exists(build.CLANGXX)


@pytest.mark.skipif(not _hipcc_present(), reason="hipcc / clang++ not installed")
def test_abi_tests_pass_under_host_sanitizers():
    from paper_1108_0900_amd import build
    lib = build.build_host_sanitized()
    runtime = build.sanitizer_runtime()
    assert os.path.exists(runtime), runtime
    # the library really carries the instrumentation (it calls into both runtimes)
    syms = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True).stdout
    assert "__asan_report_load8" in syms and "__ubsan_handle_" in syms
    env = dict(os.environ)
    env.update({"SR_LIBRARY": lib, "LD_PRELOAD": runtime,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                          os.path.join(ROOT, "tests", "test_abi.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out
