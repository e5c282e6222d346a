"""ctypes binding of ``libsplitdft.so`` (the C ABI declared in include/split_dft.h).

Argument marshalling only: tensors are checked for shape, dtype and device,
their device pointers and the current HIP stream are handed to the library,
and a non-OK status is raised as ``SplitDFTError``.  Every step of the
transform runs in the library's kernels; there is no fallback path.  PyTorch
provides device memory and streams.

``torch`` is imported before the library is loaded so that the library binds
to the HIP runtime torch already holds (same soname), and torch's pointers
and streams are valid in it.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsplitdft.so")

OK = 0
STATUS_NAMES = {
    0: "OK", 1: "INVALID_LENGTH", 2: "INVALID_BATCH", 3: "NULL_POINTER", 4: "MISALIGNED",
    5: "ALIASING", 6: "UNSUPPORTED", 7: "OUT_OF_MEMORY", 8: "HIP", 9: "INVALID_PLAN",
}
FP32 = 0
BF16X2 = 1
FP16X2 = 2
BF16X3 = 3
PRECISIONS = {"fp32": FP32, "bf16x2": BF16X2, "fp16x2": FP16X2, "bf16x3": BF16X3}
MAX_LOG2N = 16

EXPORTED = (
    "split_dft_plan", "split_dft_exec", "split_dft_adjoint", "split_dft_exec_ws", "split_dft_adjoint_ws",
    "split_dft_destroy",
    "split_dft_workspace_bytes", "split_dft_plan_info", "split_dft_plan_describe", "split_dft_twiddle_table",
    "split_dft_status_string", "split_dft_last_error",
)

_lib = None
_lock = threading.Lock()


class SplitDFTError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.status_name = STATUS_NAMES.get(status, str(status))
        super().__init__("split_dft %s: %s" % (self.status_name, message))


def lib() -> ctypes.CDLL:
    """Load libsplitdft.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsplitdft.so is missing at %s; build it with "
                               "`python -m paper_2504_07264_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, u32, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int
        L.split_dft_plan.argtypes = [ctypes.POINTER(vp), i64, i64, u32]
        L.split_dft_plan.restype = ci
        for name in ("split_dft_exec", "split_dft_adjoint"):
            fn = getattr(L, name)
            fn.argtypes = [vp, vp, vp, vp, vp, vp]
            fn.restype = ci
        for name in ("split_dft_exec_ws", "split_dft_adjoint_ws"):
            fn = getattr(L, name)
            fn.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
            fn.restype = ci
        L.split_dft_destroy.argtypes = [vp]
        L.split_dft_destroy.restype = ci
        L.split_dft_workspace_bytes.argtypes = [vp]
        L.split_dft_workspace_bytes.restype = ctypes.c_size_t
        pi = ctypes.POINTER(ci)
        pi64 = ctypes.POINTER(i64)
        L.split_dft_plan_info.argtypes = [vp, pi64, pi64, pi, pi, pi]
        L.split_dft_plan_info.restype = ci
        L.split_dft_plan_describe.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
        L.split_dft_plan_describe.restype = ci
        L.split_dft_twiddle_table.argtypes = [ci, vp, vp]
        L.split_dft_twiddle_table.restype = ci
        L.split_dft_status_string.argtypes = [ci]
        L.split_dft_status_string.restype = ctypes.c_char_p
        L.split_dft_last_error.argtypes = []
        L.split_dft_last_error.restype = ctypes.c_char_p
        _lib = L
        return L


def check(status: int) -> None:
    if status != OK:
        msg = lib().split_dft_last_error()
        raise SplitDFTError(status, msg.decode() if msg else "")


def variant_flag(index: int) -> int:
    """Plan flag bits that select compiled schedule ``index`` (0-based)."""
    return (int(index) + 1) << 8


def twiddle_table(m: int):
    """The library's FP32 twiddle table for length 2^m (host computation)."""
    import numpy as np

    n = 1 << m
    c = np.empty(n, np.float32)
    s = np.empty(n, np.float32)
    check(lib().split_dft_twiddle_table(m, c.ctypes.data, s.ctypes.data))
    return c, s


def _stream_handle(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Plan:
    """A plan for ``batch`` split-format DFTs of length ``n`` on the current device."""

    def __init__(self, n: int, batch: int, flags: int = FP32, device=None):
        L = lib()
        self.n = int(n)
        self.batch = int(batch)
        self.flags = int(flags)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L.split_dft_plan(ctypes.byref(h), self.n, self.batch, self.flags))
        self._h = h

    @property
    def handle(self):
        return self._h

    def info(self):
        n, b = ctypes.c_int64(), ctypes.c_int64()
        m, ept, tpw = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().split_dft_plan_info(self._h, ctypes.byref(n), ctypes.byref(b), ctypes.byref(m),
                                        ctypes.byref(ept), ctypes.byref(tpw)))
        return {"n": n.value, "batch": b.value, "log2n": m.value, "ept": ept.value, "tpw": tpw.value}

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(256)
        check(lib().split_dft_plan_describe(self._h, buf, len(buf)))
        return buf.value.decode()

    def workspace_bytes(self) -> int:
        return int(lib().split_dft_workspace_bytes(self._h))

    def _check_plane(self, t: torch.Tensor, name: str) -> None:
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch.Tensor" % name)
        if t.dtype != torch.float32:
            raise TypeError("%s must be float32, got %s" % (name, t.dtype))
        if t.device != self.device:
            raise ValueError("%s is on %s, the plan on %s" % (name, t.device, self.device))
        if t.numel() != self.n * self.batch or (t.dim() >= 1 and t.shape[-1] != self.n):
            raise ValueError("%s must hold [batch=%d, n=%d] floats, got shape %s"
                             % (name, self.batch, self.n, tuple(t.shape)))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)

    def _call(self, fn, ar, ai, out_r, out_i):
        for t, nm in ((ar, "input real"), (ai, "input imag")):
            self._check_plane(t, nm)
        if out_r is None:
            out_r = torch.empty_like(ar)
        if out_i is None:
            out_i = torch.empty_like(ai)
        self._check_plane(out_r, "output real")
        self._check_plane(out_i, "output imag")
        with torch.cuda.device(self.device):
            check(fn(self._h, ar.data_ptr(), ai.data_ptr(), out_r.data_ptr(), out_i.data_ptr(),
                     _stream_handle(self.device)))
        return out_r, out_i

    def exec(self, xr, xi, yr=None, yi=None):
        """Forward transform: (C xr + S xi, C xi - S xr) per row."""
        return self._call(lib().split_dft_exec, xr, xi, yr, yi)

    def adjoint(self, gr, gi, gxr=None, gxi=None):
        """Adjoint transform: (C gr - S gi, S gr + C gi) per row."""
        return self._call(lib().split_dft_adjoint, gr, gi, gxr, gxi)

    def close(self) -> None:
        h, self._h = getattr(self, "_h", None), None
        if h is not None and h.value and _lib is not None:
            with torch.cuda.device(self.device):
                check(_lib.split_dft_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


_plan_cache = {}
_plan_cache_lock = threading.Lock()


def cached_plan(n: int, batch: int, device: torch.device, flags: int = FP32) -> Plan:
    key = (int(n), int(batch), str(device), int(flags))
    with _plan_cache_lock:
        p = _plan_cache.get(key)
        if p is None:
            p = Plan(n, batch, flags, device)
            _plan_cache[key] = p
        return p


def split_dft(xr: torch.Tensor, xi: torch.Tensor, out=None):
    """Forward split-format DFT of the rows of xr, xi ([..., n], float32, on a GPU)."""
    n = xr.shape[-1]
    p = cached_plan(n, xr.numel() // max(n, 1), xr.device)
    yr, yi = (None, None) if out is None else out
    return p.exec(xr, xi, yr, yi)


def split_dft_adjoint(gr: torch.Tensor, gi: torch.Tensor, out=None):
    """Adjoint split-format DFT (N times the inverse DFT) of the rows of gr, gi."""
    n = gr.shape[-1]
    p = cached_plan(n, gr.numel() // max(n, 1), gr.device)
    r, i = (None, None) if out is None else out
    return p.adjoint(gr, gi, r, i)
