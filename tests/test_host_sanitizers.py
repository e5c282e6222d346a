"""The CPU test suite once more, against AddressSanitizer + UndefinedBehavior-
Sanitizer builds of the library's host code (plan creation, argument
validation, the C ABI, table generation) and of the C oracle, in a child
process with the sanitizer runtime preloaded.  Any report fails the test."""
import glob
import os
import subprocess
import sys

import pytest

from paper_2504_07264_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _clang():
    for cand in ("/opt/rocm/lib/llvm/bin/clang", "/opt/rocm/llvm/bin/clang"):
        if os.path.exists(cand):
            return cand
    return None


@pytest.mark.skipif(_clang() is None, reason="ROCm's clang (sanitizer runtime) is not installed")
def test_cpu_suite_under_host_sanitizers(tmp_path):
    import oracle

    out = str(tmp_path)
    lib = build.build_sanitized(out)
    olib = oracle.build_sanitized(os.path.join(out, "liboracle.so"), _clang())
    runtime = build.asan_runtime()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": runtime,
        "LD_LIBRARY_PATH": os.path.join(os.path.dirname(os.path.dirname(_clang())), "lib")
        + (":" + env["LD_LIBRARY_PATH"] if env.get("LD_LIBRARY_PATH") else ""),
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:log_path=%s/asan" % out,
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:log_path=%s/ubsan" % out,
        "SPLIT_DFT_LIB": lib,
        "ORACLE_LIB": olib,
    })
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-x", "-q",
           "-p", "no:cacheprovider", "--ignore", os.path.abspath(__file__)]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    reports = sorted(glob.glob(os.path.join(out, "asan*")) + glob.glob(os.path.join(out, "ubsan*")))
    text = "".join(open(r).read()[:4000] for r in reports)
    assert res.returncode == 0 and not reports, (res.stdout[-3000:] + res.stderr[-3000:] + text)
    assert " passed" in res.stdout
