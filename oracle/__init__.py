"""CPU oracle for the split-format DFT (Cariow, arXiv 2504.07264).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_2504_07264_amd``) never imports it, and it never imports the
product: the two share no code, tables or constant generators.

The arithmetic lives in ``split_oracle.c`` (plain C, FP64, compiled with gcc
and floating-point contraction off); this module marshals numpy arrays to it.
``factors.py`` builds the factors of eq. (6) and eq. (9) as dense matrices
straight from their Kronecker definitions in Section III.

Functions (all take and return numpy arrays of shape ``[batch, n]``):

* ``dft_direct``      O1, eq. (5) evaluated directly in FP64, O(N^2)
* ``dft_direct_bins`` O1 at selected output bins of one row
* ``adjoint_direct``  O1 adjoint, E_2N^T of eq. (5), evaluated directly
* ``split_fft``       O2, eq. (6) factor by factor in FP64
* ``split_fft_f32``   O2f, the same factors in FP32 with one fixed op form
* ``split_adjoint_f32`` O2f applied to the adjoint through the plane swap
* ``split_fft_dif`` / ``split_fft_dif_f32``  O3, eq. (9)
* ``omega``, ``twiddle_table_f32``  the twiddle blocks of Section III
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "split_oracle.c")
# ORACLE_LIB: another build of the same source (the host-sanitizer build of
# the CPU tests); by default the in-tree one
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

_CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile split_oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_sanitized(path: str, cc: str = "clang") -> str:
    """Compile split_oracle.c with AddressSanitizer + UndefinedBehaviorSanitizer
    (clang, shared sanitizer runtime) into ``path``."""
    flags = [f for f in _CFLAGS if f not in ("-O2", "-fopenmp")]
    subprocess.check_call([cc, *flags, "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
                           "-fno-omit-frame-pointer", "-shared-libsan", _SRC, "-o", path, "-lm"])
    return path


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if (not os.path.exists(_LIB_PATH)
                or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        i64, i32 = ctypes.c_int64, ctypes.c_int
        p = ctypes.c_void_p
        lib.oracle_omega_f64.argtypes = [i64, i32, p, p]
        lib.oracle_omega_f64.restype = None
        lib.oracle_twiddle_table_f32.argtypes = [i32, p, p]
        lib.oracle_twiddle_table_f32.restype = None
        lib.oracle_twiddle_table_f64.argtypes = [i32, p, p]
        lib.oracle_twiddle_table_f64.restype = None
        lib.oracle_bit_reverse.argtypes = [i64, i32]
        lib.oracle_bit_reverse.restype = i64
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = i32
        for name in ("oracle_dft_direct_f64", "oracle_adjoint_direct_f64",
                     "oracle_split_fft_f64", "oracle_split_fft_f32",
                     "oracle_split_fft_dif_f64", "oracle_split_fft_dif_f32"):
            fn = getattr(lib, name)
            fn.argtypes = [i64, i64, p, p, p, p, i32]
            fn.restype = i32
        lib.oracle_dft_direct_bins_f64.argtypes = [i64, p, p, i64, p, p, p]
        lib.oracle_dft_direct_bins_f64.restype = i32
        _lib = lib
        return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _as2d(a, dtype) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    if a.ndim == 1:
        a = a[None, :]
    if a.ndim != 2:
        raise ValueError("expected [batch, n] or [n]")
    return a


def _pair(xr, xi, dtype):
    xr = _as2d(xr, dtype)
    xi = _as2d(xi, dtype)
    if xr.shape != xi.shape:
        raise ValueError("real and imaginary planes differ in shape")
    return xr, xi


def _run(name, xr, xi, dtype, nthreads):
    xr, xi = _pair(xr, xi, dtype)
    batch, n = xr.shape
    yr = np.empty_like(xr)
    yi = np.empty_like(xi)
    rc = getattr(_load(), name)(n, batch, _ptr(xr), _ptr(xi), _ptr(yr), _ptr(yi), nthreads)
    if rc != 0:
        raise ValueError("%s rejected n=%d batch=%d" % (name, n, batch))
    return yr, yi


def max_threads() -> int:
    """Threads the oracle's OpenMP loops use by default."""
    return int(_load().oracle_max_threads())


def bit_reverse(k: int, m: int) -> int:
    return int(_load().oracle_bit_reverse(k, m))


def omega(q: int, i: int):
    """(cos, sin) of omega^(i,q) in FP64 (Section III, under eq. 6)."""
    c = ctypes.c_double()
    s = ctypes.c_double()
    _load().oracle_omega_f64(q, i, ctypes.byref(c), ctypes.byref(s))
    return c.value, s.value


def twiddle_table_f64(m: int):
    n = 1 << m
    c = np.empty(n, np.float64)
    s = np.empty(n, np.float64)
    _load().oracle_twiddle_table_f64(m, _ptr(c), _ptr(s))
    return c, s


def twiddle_table_f32(m: int):
    """Entry 2^(i-1)+q = FP32 rounding of omega^(i,q); entry 0 = angle 0."""
    n = 1 << m
    c = np.empty(n, np.float32)
    s = np.empty(n, np.float32)
    _load().oracle_twiddle_table_f32(m, _ptr(c), _ptr(s))
    return c, s


def dft_direct(xr, xi, nthreads: int = 0):
    """O1: eq. (5) evaluated directly in FP64."""
    return _run("oracle_dft_direct_f64", xr, xi, np.float64, nthreads)


def dft_direct_bins(xr, xi, ks):
    """O1 at output bins ``ks`` of one row (1-D inputs of length n)."""
    xr = np.ascontiguousarray(np.asarray(xr, np.float64).ravel())
    xi = np.ascontiguousarray(np.asarray(xi, np.float64).ravel())
    ks = np.ascontiguousarray(np.asarray(ks, np.int64).ravel())
    yr = np.empty(ks.size, np.float64)
    yi = np.empty(ks.size, np.float64)
    rc = _load().oracle_dft_direct_bins_f64(xr.size, _ptr(xr), _ptr(xi), ks.size, _ptr(ks),
                                            _ptr(yr), _ptr(yi))
    if rc != 0:
        raise ValueError("bad arguments")
    return yr, yi


def adjoint_direct(gr, gi, nthreads: int = 0):
    """O1 adjoint: [[C, -S], [S, C]] applied directly in FP64."""
    return _run("oracle_adjoint_direct_f64", gr, gi, np.float64, nthreads)


def split_fft(xr, xi, nthreads: int = 0):
    """O2: eq. (6) applied factor by factor in FP64."""
    return _run("oracle_split_fft_f64", xr, xi, np.float64, nthreads)


def split_fft_f32(xr, xi, nthreads: int = 0):
    """O2f: eq. (6) in FP32 with the fixed operation forms (structural mirror)."""
    return _run("oracle_split_fft_f32", xr, xi, np.float32, nthreads)


def split_adjoint_f32(gr, gi, nthreads: int = 0):
    """O2f applied to the adjoint: C gr - S gi and S gr + C gi equal the
    forward transform of (gi, gr) with its two output planes swapped."""
    yr, yi = split_fft_f32(gi, gr, nthreads)
    return yi, yr


def split_fft_dif(xr, xi, nthreads: int = 0):
    """O3: eq. (9) factor by factor in FP64."""
    return _run("oracle_split_fft_dif_f64", xr, xi, np.float64, nthreads)


def split_fft_dif_f32(xr, xi, nthreads: int = 0):
    """O3 in FP32 with the fixed operation forms."""
    return _run("oracle_split_fft_dif_f32", xr, xi, np.float32, nthreads)


def rel_l2_per_row(yr, yi, rr, ri) -> np.ndarray:
    """Relative L2 error of each transform, both planes together."""
    yr = np.asarray(yr, np.float64)
    yi = np.asarray(yi, np.float64)
    rr = np.asarray(rr, np.float64)
    ri = np.asarray(ri, np.float64)
    num = np.sqrt(((yr - rr) ** 2 + (yi - ri) ** 2).sum(axis=-1))
    den = np.sqrt((rr ** 2 + ri ** 2).sum(axis=-1))
    out = np.where(den > 0, num / np.where(den > 0, den, 1.0), num)
    return out


def tolerance(n: int) -> float:
    """Per-transform relative L2 bound for FP32 results: 2e-7*log2(N) + 1e-7."""
    m = int(n).bit_length() - 1
    return 2e-7 * m + 1e-7
