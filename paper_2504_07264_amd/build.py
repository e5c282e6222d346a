"""Build the HIP library ``libsplitdft.so`` in-tree with hipcc for gfx950.

Run as ``python -m paper_2504_07264_amd.build``.  All sources are compiled
in one hipcc invocation per file and linked into one shared library next to
this file, where the Python binding loads it.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD_DIR = os.path.join(PKG, "_build")
LIB_PATH = os.path.join(PKG, "libsplitdft.so")
# Benchmark-only kernels, not part of the transform library: HBM streaming
# for the copy ceiling, and the L2 hand-over model of a two-pass transform
BENCH_LIB_PATH = os.path.join(PKG, "libsplitdft_bench.so")
BENCH_SOURCES = ["bench_copy.hip", "bench_l2.hip"]

SOURCES = ["fft_lds.hip", "fft_tile.hip", "fft_many.hip", "fft_mfma.hip", "twiddle.cpp", "mfma_tables.cpp",
           "api.cpp", "api_many.cpp", "noalloc.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # The operation forms of the transform are written out explicitly (fmaf
    # where a fused multiply-add is meant); nothing else may be contracted.
    "-ffp-contract=off",
    # No packed FP32 instructions in device code.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the split-format DFT library needs ROCm's hipcc")


def _compile(cc, src, verbose):
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [cc, *HIPCC_FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s%s" % (src, res.stdout, res.stderr))
    return obj


def _link(cc, objs, path, verbose):
    tmp = path + ".tmp%d" % os.getpid()
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (res.stdout, res.stderr))
    os.replace(tmp, path)


def build(verbose: bool = False) -> str:
    """Compile every source and link libsplitdft.so (and the benchmark's
    libsplitdft_bench.so); returns the transform library's path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    srcs = SOURCES + BENCH_SOURCES
    with ThreadPoolExecutor(max_workers=min(4, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(cc, s, verbose), srcs))
    _link(cc, objs[:len(SOURCES)], LIB_PATH, verbose)
    _link(cc, objs[len(SOURCES):], BENCH_LIB_PATH, verbose)
    return LIB_PATH


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build, for CPU
# tests: the host C++ sources (plan creation, argument validation, the C ABI,
# table generation) are instrumented; the HIP sources (kernels and their
# launchers) are linked from the regular build.
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-fno-omit-frame-pointer", "-shared-libsan", "-g", "-O1"]


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime the sanitized builds link against
    (to preload into an uninstrumented Python)."""
    cc = hipcc()
    res = subprocess.run([cc, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = res.stdout.strip()
    if res.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        import glob

        found = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        if not found:
            raise RuntimeError("clang AddressSanitizer runtime not found")
        path = found[0]
    return path


def build_sanitized(out_dir: str, verbose: bool = False) -> str:
    """Link out_dir/libsplitdft.so from ASan + UBSan builds of the host C++
    sources and the regular objects of the HIP sources; returns its path."""
    os.makedirs(out_dir, exist_ok=True)
    cc = hipcc()
    flags = [f for f in HIPCC_FLAGS if f != "-O3"] + SANITIZE_FLAGS

    def one(src):
        if src.endswith(".hip"):
            obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
            return obj if os.path.exists(obj) else _compile(cc, src, verbose)
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        cmd = [cc, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("sanitized compile failed for %s:\n%s%s" % (src, res.stdout, res.stderr))
        return obj

    os.makedirs(BUILD_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(one, SOURCES))
    path = os.path.join(out_dir, "libsplitdft.so")
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
           "-fsanitize=undefined", "-shared-libsan", *objs, "-o", path]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("sanitized link failed:\n%s%s" % (res.stdout, res.stderr))
    return path


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(sys.argv[sys.argv.index("--sanitize") + 1], verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
