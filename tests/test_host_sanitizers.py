"""The host logic of the library (argument checks, the serving engine's
scheduler, queues, cancellation and threads) under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

The library is rebuilt with host-side instrumentation (the device code is
the ordinary one) into _build/libknn_asan.so, and the CPU test files of the
C ABI and of the dry-run server are run in a child process that preloads the
toolchain's ASan runtime and loads that build (KNN_LIB_PATH).  Any report of
either sanitizer fails the test.
"""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def asan_lib():
    import paper_0804_1448_amd.build as B

    srcs = [os.path.join(B.CSRC, s) for s in B.SOURCES] + [os.path.join(ROOT, "include", "knn.h")]
    srcs += [os.path.join(B.CSRC, f) for f in os.listdir(B.CSRC) if f.endswith(".h")]
    if not os.path.exists(B.ASAN_LIB) or os.path.getmtime(B.ASAN_LIB) < max(os.path.getmtime(s) for s in srcs):
        B.build_host_sanitized()
    return B.ASAN_LIB, B.asan_runtime()


def test_build_is_instrumented(asan_lib):
    lib, _ = asan_lib
    out = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True, check=True).stdout
    assert "__asan_report_load8" in out, "no AddressSanitizer checks in the host code"
    assert "__ubsan_handle_" in out, "no UndefinedBehaviorSanitizer checks in the host code"


def test_host_logic_is_clean_under_sanitizers(asan_lib):
    lib, runtime = asan_lib
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": runtime,
        "KNN_LIB_PATH": lib,
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    probe = ("import paper_0804_1448_amd._lib as L; L.load(); "
             "maps = open('/proc/self/maps').read(); "
             "assert 'libknn_asan.so' in maps and 'libclang_rt.asan' in maps, 'sanitized build not loaded'")
    res = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_server_sched.py",
                          "tests/test_abi.py"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    text = res.stdout + res.stderr
    assert res.returncode == 0, text[-4000:]
    assert "AddressSanitizer" not in text and "runtime error:" not in text, text[-4000:]
