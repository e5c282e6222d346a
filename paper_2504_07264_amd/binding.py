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
# SPLIT_DFT_LIB: another build of the same library (the host-sanitizer build
# of the CPU tests); by default the in-tree one
LIB_PATH = os.environ.get("SPLIT_DFT_LIB") or os.path.join(_PKG, "libsplitdft.so")

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
DIF = 1 << 24  # decimation-in-frequency factorisation (eq. 9)
CALLER_WORKSPACE = 1 << 30  # the plan allocates no workspace; each call brings one
MAX_LOG2N = 16

EXPORTED = (
    "split_dft_plan", "split_dft_exec", "split_dft_adjoint", "split_dft_exec_ws", "split_dft_adjoint_ws",
    "split_dft_exec_adjoint", "split_dft_exec_adjoint_ws", "split_dft_exec_noalloc",
    "split_dft_destroy",
    "split_dft_workspace_bytes", "split_dft_plan_info", "split_dft_plan_describe", "split_dft_twiddle_table",
    "split_dft_status_string", "split_dft_last_error",
    "split_dft_many_plan", "split_dft_many_offsets", "split_dft_many_info", "split_dft_many_workspace_bytes",
    "split_dft_many_exec", "split_dft_many_exec_ws", "split_dft_many_adjoint", "split_dft_many_adjoint_ws",
    "split_dft_many_exec_adjoint", "split_dft_many_exec_adjoint_ws", "split_dft_many_graph",
    "split_dft_many_graph_ws", "split_dft_graph_launch", "split_dft_graph_destroy", "split_dft_many_destroy",
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
        for name in ("split_dft_exec", "split_dft_adjoint", "split_dft_exec_noalloc"):
            fn = getattr(L, name)
            fn.argtypes = [vp, vp, vp, vp, vp, vp]
            fn.restype = ci
        for name in ("split_dft_exec_ws", "split_dft_adjoint_ws"):
            fn = getattr(L, name)
            fn.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
            fn.restype = ci
        L.split_dft_exec_adjoint.argtypes = [vp] + [vp] * 8 + [vp]
        L.split_dft_exec_adjoint.restype = ci
        L.split_dft_exec_adjoint_ws.argtypes = [vp] + [vp] * 8 + [vp, ctypes.c_size_t, vp]
        L.split_dft_exec_adjoint_ws.restype = ci
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
        L.split_dft_many_plan.argtypes = [ctypes.POINTER(vp), vp, i64, u32]
        L.split_dft_many_plan.restype = ci
        L.split_dft_many_offsets.argtypes = [vp, vp]
        L.split_dft_many_offsets.restype = ci
        L.split_dft_many_info.argtypes = [vp, pi64, pi64, pi, pi, ctypes.POINTER(ctypes.c_size_t)]
        L.split_dft_many_info.restype = ci
        L.split_dft_many_workspace_bytes.argtypes = [vp]
        L.split_dft_many_workspace_bytes.restype = ctypes.c_size_t
        for name in ("split_dft_many_exec", "split_dft_many_adjoint"):
            fn = getattr(L, name)
            fn.argtypes = [vp, vp, vp, vp, vp, vp]
            fn.restype = ci
        for name in ("split_dft_many_exec_ws", "split_dft_many_adjoint_ws"):
            fn = getattr(L, name)
            fn.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
            fn.restype = ci
        L.split_dft_many_exec_adjoint.argtypes = [vp] + [vp] * 8 + [vp]
        L.split_dft_many_exec_adjoint.restype = ci
        L.split_dft_many_exec_adjoint_ws.argtypes = [vp] + [vp] * 8 + [vp, ctypes.c_size_t, vp]
        L.split_dft_many_exec_adjoint_ws.restype = ci
        L.split_dft_many_graph.argtypes = [vp] + [vp] * 8 + [ctypes.POINTER(vp)]
        L.split_dft_many_graph.restype = ci
        L.split_dft_many_graph_ws.argtypes = [vp] + [vp] * 8 + [vp, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.split_dft_many_graph_ws.restype = ci
        L.split_dft_graph_launch.argtypes = [vp, vp]
        L.split_dft_graph_launch.restype = ci
        L.split_dft_graph_destroy.argtypes = [vp]
        L.split_dft_graph_destroy.restype = ci
        L.split_dft_many_destroy.argtypes = [vp]
        L.split_dft_many_destroy.restype = ci
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


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream_handle(device) -> int:
    """The current stream of ``device`` (a torch.device or an index) as a raw
    hipStream_t value."""
    index = device if isinstance(device, int) else device.index
    if _raw_stream is not None:
        return _raw_stream(index)
    return torch.cuda.current_stream(index).cuda_stream


def _device_of(device) -> torch.device:
    """A CUDA device with its index filled in (the current device when none is given)."""
    if device is None:
        return torch.device("cuda", torch.cuda.current_device())
    d = torch.device(device)
    if d.type != "cuda":
        raise ValueError("split_dft runs on a GPU device, got %s" % d)
    return d if d.index is not None else torch.device("cuda", torch.cuda.current_device())


def _workspace_arg(workspace, nbytes: int, index: int, like: torch.Tensor):
    """(pointer, bytes, tensor) of the workspace of one call: the caller's
    tensor, or one allocated here through torch's caching allocator on the
    current stream (freed back to the allocator when the call returns; the
    allocator hands it out again only on the same stream)."""
    if workspace is None:
        if nbytes == 0:
            return None, 0, None
        workspace = torch.empty((nbytes + 3) // 4, dtype=torch.float32, device=like.device)
    elif (not isinstance(workspace, torch.Tensor) or not workspace.is_cuda
          or workspace.get_device() != index or not workspace.is_contiguous()):
        raise ValueError("workspace must be a contiguous tensor on cuda:%d" % index)
    return workspace.data_ptr(), workspace.numel() * workspace.element_size(), workspace


class Plan:
    """A plan for ``batch`` split-format DFTs of length ``n`` on the current device.

    Two-pass lengths (n >= 2^15) need a workspace.  By default the plan owns
    none: every call takes the ``workspace=`` tensor given, or allocates one
    through torch's caching allocator on the current stream, so calls on
    different streams never share it.  ``own_workspace=True`` makes the
    library allocate one per plan instead (calls then must not overlap on
    different streams unless they pass their own)."""

    def __init__(self, n: int, batch: int, flags: int = FP32, device=None, own_workspace: bool = False):
        L = lib()
        self.n = int(n)
        self.batch = int(batch)
        self.flags = int(flags) | (0 if own_workspace else CALLER_WORKSPACE)
        self.device = _device_of(device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L.split_dft_plan(ctypes.byref(h), self.n, self.batch, self.flags))
        self._h = h
        self._index = self.device.index
        self._numel = self.n * self.batch
        self._ws_bytes = int(L.split_dft_workspace_bytes(h))
        self._own_ws = bool(own_workspace)

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
        # cheap attribute checks only: this runs four times per launch
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch.Tensor" % name)
        if t.dtype is not torch.float32:
            raise TypeError("%s must be float32, got %s" % (name, t.dtype))
        if not t.is_cuda or t.get_device() != self._index:
            raise ValueError("%s is on %s, the plan on %s" % (name, t.device, self.device))
        if t.numel() != self._numel or (t.dim() >= 1 and t.shape[-1] != self.n):
            raise ValueError("%s must hold [batch=%d, n=%d] floats, got shape %s"
                             % (name, self.batch, self.n, tuple(t.shape)))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)

    def _planes(self, ar, ai, out_r, out_i, names):
        self._check_plane(ar, names[0])
        self._check_plane(ai, names[1])
        if out_r is None:
            out_r = torch.empty_like(ar)
        if out_i is None:
            out_i = torch.empty_like(ai)
        self._check_plane(out_r, names[2])
        self._check_plane(out_i, names[3])
        return out_r, out_i

    def _run(self, fn, fn_ws, ptrs, workspace, like):
        # a workspace goes to the _ws entry point: the caller's, or (plans
        # without their own) one allocated here for this call
        need = 0 if self._own_ws else self._ws_bytes
        wptr, wbytes, keep = _workspace_arg(workspace, need, self._index, like)
        if wptr is None:
            args = (self._h,) + ptrs + (_stream_handle(self._index),)
        else:
            fn = fn_ws
            args = (self._h,) + ptrs + (wptr, wbytes, _stream_handle(self._index))
        if torch.cuda.current_device() == self._index:
            check(fn(*args))
        else:
            with torch.cuda.device(self._index):
                check(fn(*args))
        del keep  # the caching allocator reuses it in stream order

    def exec(self, xr, xi, yr=None, yi=None, workspace=None):
        """Forward transform: (C xr + S xi, C xi - S xr) per row.  ``workspace``
        (optional, two-pass lengths): a contiguous device tensor of at least
        ``workspace_bytes()`` bytes, else one is allocated for the call."""
        yr, yi = self._planes(xr, xi, yr, yi, ("input real", "input imag", "output real", "output imag"))
        L = lib()
        self._run(L.split_dft_exec, L.split_dft_exec_ws,
                  (xr.data_ptr(), xi.data_ptr(), yr.data_ptr(), yi.data_ptr()), workspace, xr)
        return yr, yi

    def adjoint(self, gr, gi, gxr=None, gxi=None, workspace=None):
        """Adjoint transform: (C gr - S gi, S gr + C gi) per row (``workspace``
        as for exec)."""
        gxr, gxi = self._planes(gr, gi, gxr, gxi, ("input real", "input imag", "output real", "output imag"))
        L = lib()
        self._run(L.split_dft_adjoint, L.split_dft_adjoint_ws,
                  (gr.data_ptr(), gi.data_ptr(), gxr.data_ptr(), gxi.data_ptr()), workspace, gr)
        return gxr, gxi

    def exec_adjoint(self, xr, xi, gr, gi, out=None, workspace=None):
        """Forward transform of (xr, xi) and adjoint transform of (gr, gi) in
        one call (one kernel launch for single-pass FP32 schedules); returns
        (yr, yi, gxr, gxi)."""
        yr, yi, gxr, gxi = (None,) * 4 if out is None else out
        yr, yi = self._planes(xr, xi, yr, yi, ("xr", "xi", "yr", "yi"))
        gxr, gxi = self._planes(gr, gi, gxr, gxi, ("gr", "gi", "gxr", "gxi"))
        L = lib()
        self._run(L.split_dft_exec_adjoint, L.split_dft_exec_adjoint_ws,
                  (xr.data_ptr(), xi.data_ptr(), yr.data_ptr(), yi.data_ptr(), gr.data_ptr(), gi.data_ptr(),
                   gxr.data_ptr(), gxi.data_ptr()), workspace, xr)
        return yr, yi, gxr, gxi

    def exec_noalloc(self, xr, xi, yr, yi):
        """Forward transform into the given outputs through the library's
        static scratch array: the call allocates nothing (for code under
        graph capture).  Calls that overlap in time on one GPU race on that
        array."""
        yr, yi = self._planes(xr, xi, yr, yi, ("input real", "input imag", "output real", "output imag"))
        args = (self._h, xr.data_ptr(), xi.data_ptr(), yr.data_ptr(), yi.data_ptr(), _stream_handle(self._index))
        if torch.cuda.current_device() == self._index:
            check(lib().split_dft_exec_noalloc(*args))
        else:
            with torch.cuda.device(self._index):
                check(lib().split_dft_exec_noalloc(*args))
        return yr, yi

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


PLAN_CACHE_SIZE = 8  # most recently used plans kept (each holds its device tables)


def cached_plan(n: int, batch: int, device: torch.device, flags: int = FP32) -> Plan:
    """A plan for (n, batch, device, flags) from a small most-recently-used
    cache; an evicted plan is destroyed once nothing references it."""
    key = (int(n), int(batch), str(device), int(flags))
    with _plan_cache_lock:
        p = _plan_cache.pop(key, None)
        if p is None:
            p = Plan(n, batch, flags, device)
        _plan_cache[key] = p  # most recent last
        while len(_plan_cache) > PLAN_CACHE_SIZE:
            _plan_cache.pop(next(iter(_plan_cache)))
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


MANY_ONE_KERNEL = 1 << 24


def many_flags(build: int = -1, workgroups_per_cu: int = 0, one_kernel: bool = False,
               per_length_from: int = 0) -> int:
    """Grouped-plan flag bits: kernel build (-1 = default), workgroups per CU
    (0 = max), whether every length runs in the persistent kernel, and log2 of
    the shortest length run by per-length launches (0 = default)."""
    return (((int(build) + 1) << 8) + (int(workgroups_per_cu) << 16) + (MANY_ONE_KERNEL if one_kernel else 0)
            + (int(per_length_from) << 25))


class ManyPlan:
    """Grouped plan for a ragged batch: transform k has length lengths[k] and
    occupies [offsets[k], offsets[k+1]) of each flat FP32 plane.  Workspace
    as for ``Plan``: by default each call takes ``workspace=`` or allocates
    one through torch (``own_workspace=True``: the library's)."""

    def __init__(self, lengths, flags: int = FP32, device=None, own_workspace: bool = False):
        import numpy as np

        L = lib()
        self.lengths = np.ascontiguousarray(np.asarray(lengths, dtype=np.int64).ravel())
        self.device = _device_of(device)
        self._index = self.device.index
        self.flags = int(flags) | (0 if own_workspace else CALLER_WORKSPACE)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L.split_dft_many_plan(ctypes.byref(h), self.lengths.ctypes.data, self.lengths.size, self.flags))
        self._h = h
        offs = np.empty(self.lengths.size + 1, np.int64)
        check(L.split_dft_many_offsets(h, offs.ctypes.data))
        self.offsets = offs
        self.points = int(offs[-1])
        self._ws_bytes = int(L.split_dft_many_workspace_bytes(h))
        self._own_ws = bool(own_workspace)

    def info(self):
        c, p = ctypes.c_int64(), ctypes.c_int64()
        wg, it = ctypes.c_int(), ctypes.c_int()
        ws = ctypes.c_size_t()
        check(lib().split_dft_many_info(self._h, ctypes.byref(c), ctypes.byref(p), ctypes.byref(wg),
                                        ctypes.byref(it), ctypes.byref(ws)))
        return {"count": c.value, "points": p.value, "workgroups": wg.value, "items": it.value,
                "workspace_bytes": ws.value}

    def workspace_bytes(self) -> int:
        return int(lib().split_dft_many_workspace_bytes(self._h))

    def _plane(self, t, name):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32:
            raise TypeError("%s must be a float32 tensor" % name)
        if t.device != self.device or not t.is_contiguous() or t.numel() != self.points:
            raise ValueError("%s must be a contiguous tensor of %d floats on %s" % (name, self.points, self.device))
        return t.data_ptr()

    def _new(self, like):
        return torch.empty_like(like)

    def _ws(self, workspace, like):
        return _workspace_arg(workspace, 0 if self._own_ws else self._ws_bytes, self._index, like)

    def _call(self, name, ptrs, workspace, like):
        wptr, wbytes, keep = self._ws(workspace, like)
        L = lib()
        with torch.cuda.device(self.device):
            if wptr is None:
                check(getattr(L, name)(self._h, *ptrs, _stream_handle(self.device)))
            else:
                check(getattr(L, name + "_ws")(self._h, *ptrs, wptr, wbytes, _stream_handle(self.device)))
        del keep

    def exec(self, xr, xi, yr=None, yi=None, workspace=None):
        yr = self._new(xr) if yr is None else yr
        yi = self._new(xi) if yi is None else yi
        args = [self._plane(t, n) for t, n in ((xr, "xr"), (xi, "xi"), (yr, "yr"), (yi, "yi"))]
        self._call("split_dft_many_exec", args, workspace, xr)
        return yr, yi

    def adjoint(self, gr, gi, gxr=None, gxi=None, workspace=None):
        gxr = self._new(gr) if gxr is None else gxr
        gxi = self._new(gi) if gxi is None else gxi
        args = [self._plane(t, n) for t, n in ((gr, "gr"), (gi, "gi"), (gxr, "gxr"), (gxi, "gxi"))]
        self._call("split_dft_many_adjoint", args, workspace, gr)
        return gxr, gxi

    def exec_adjoint(self, xr, xi, gr, gi, out=None, workspace=None):
        yr, yi, gxr, gxi = out if out is not None else (self._new(xr), self._new(xi), self._new(gr), self._new(gi))
        names = ("xr", "xi", "yr", "yi", "gr", "gi", "gxr", "gxi")
        args = [self._plane(t, n) for t, n in zip((xr, xi, yr, yi, gr, gi, gxr, gxi), names)]
        self._call("split_dft_many_exec_adjoint", args, workspace, xr)
        return yr, yi, gxr, gxi

    def graph(self, xr, xi, yr, yi, gr=None, gi=None, gxr=None, gxi=None, workspace=None):
        """Capture exec (and the adjoint when g planes are given) on these
        buffers.  The returned graph holds references to the tensors and to
        its workspace (allocated here through torch unless given), so they
        stay allocated while it exists."""
        tensors = [xr, xi, yr, yi]
        ptrs = [self._plane(t, n) for t, n in zip(tensors, ("xr", "xi", "yr", "yi"))]
        if gr is None:
            ptrs += [None] * 4
        else:
            more = [gr, gi, gxr, gxi]
            ptrs += [self._plane(t, n) for t, n in zip(more, ("gr", "gi", "gxr", "gxi"))]
            tensors += more
        wptr, wbytes, ws = self._ws(workspace, xr)
        g = ctypes.c_void_p()
        L = lib()
        with torch.cuda.device(self.device):
            if wptr is None:
                check(L.split_dft_many_graph(self._h, *ptrs, ctypes.byref(g)))
            else:
                check(L.split_dft_many_graph_ws(self._h, *ptrs, wptr, wbytes, ctypes.byref(g)))
        return ManyGraph(g, self, tensors + ([ws] if ws is not None else []))

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h is not None and h.value and _lib is not None:
            check(_lib.split_dft_many_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class ManyGraph:
    """An instantiated HIP graph of one grouped launch on fixed buffers.  The
    library keeps the plan's device data until both the plan and the graph
    are destroyed; the graph object holds the captured tensors (and its
    workspace) so that their memory is not reused while it can replay."""

    def __init__(self, handle, plan, tensors=()):
        self._h = handle
        self._device = plan.device
        self._tensors = list(tensors)

    def launch(self, stream=None):
        s = _stream_handle(self._device) if stream is None else stream
        check(lib().split_dft_graph_launch(self._h, s))

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h is not None and h.value and _lib is not None:
            check(_lib.split_dft_graph_destroy(h))
        self._tensors = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
