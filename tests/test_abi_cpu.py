"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments before any HIP call, and builds the same
twiddle table as the oracle's independent generator."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2504_07264_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "split_dft.h")


@pytest.fixture(scope="module")
def L():
    return binding.lib()


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(split_dft_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_symbols():
    assert set(header_functions()) == set(binding.EXPORTED)


def test_library_exports_every_declared_symbol(L):
    for name in header_functions():
        assert hasattr(L, name), name


def _plan(L, n, batch, flags=0):
    h = ctypes.c_void_p()
    st = L.split_dft_plan(ctypes.byref(h), n, batch, flags)
    return st, h


@pytest.mark.parametrize("n", [0, -4, 3, 12, 1000, 1 << 17, 1 << 20])
def test_plan_rejects_bad_length(L, n):
    st, h = _plan(L, n, 4)
    assert st == 1 and h.value is None
    assert b"n must be" in L.split_dft_last_error()


@pytest.mark.parametrize("batch", [0, -1, (1 << 62)])
def test_plan_rejects_bad_batch(L, batch):
    st, _ = _plan(L, 1024, batch)
    assert st == 2


def test_plan_rejects_unknown_flags(L):
    assert _plan(L, 16, 4, 0x7)[0] == 6
    assert _plan(L, 16, 4, 1 << 20)[0] == 6
    assert _plan(L, 16, 4, 1 << 31)[0] == 6
    assert _plan(L, 16, 4, binding.CALLER_WORKSPACE | (1 << 29))[0] == 6
    # a schedule selector beyond the compiled ones
    assert _plan(L, 16, 4, binding.variant_flag(200))[0] == 6


@pytest.mark.parametrize("n", [16, 128, 512, 1 << 16])
@pytest.mark.parametrize("mode", [binding.BF16X2, binding.FP16X2, binding.BF16X3])
def test_matrix_core_modes_need_n256(L, n, mode):
    st, h = _plan(L, n, 4, mode)
    assert st == 6 and h.value is None


def test_dif_flag_domain(L):
    # every length has a DIF schedule (two passes from 2^15); selectors beyond
    # the compiled ones, matrix-core modes and unknown bits are rejected
    assert _plan(L, 1 << 15, 4, binding.DIF | binding.variant_flag(200))[0] == 6
    assert _plan(L, 1 << 16, 4, binding.DIF | binding.variant_flag(200))[0] == 6
    assert _plan(L, 256, 4, binding.DIF | binding.BF16X2)[0] == 6
    assert _plan(L, 256, 4, binding.DIF | (1 << 25))[0] == 6


def test_plan_null_out(L):
    assert L.split_dft_plan(None, 16, 1, 0) == 3


def test_forced_allocation_failure(L, monkeypatch):
    monkeypatch.setenv("SPLIT_DFT_FAIL_ALLOC", "1")
    st, h = _plan(L, 64, 2)
    assert st == 7 and h.value is None


def test_calls_with_invalid_plan(L):
    bogus = ctypes.c_void_p(0x1000)
    buf = ctypes.c_void_p(0x100000)
    assert L.split_dft_exec(None, buf, buf, buf, buf, None) == 9
    assert L.split_dft_exec(bogus, buf, buf, buf, buf, None) == 9
    assert L.split_dft_adjoint(bogus, buf, buf, buf, buf, None) == 9
    assert L.split_dft_exec_noalloc(None, buf, buf, buf, buf, None) == 9
    assert L.split_dft_exec_noalloc(bogus, buf, buf, buf, buf, None) == 9
    assert L.split_dft_exec_adjoint(bogus, buf, buf, buf, buf, buf, buf, buf, buf, None) == 9
    assert L.split_dft_exec_adjoint_ws(bogus, buf, buf, buf, buf, buf, buf, buf, buf, buf, 1 << 20, None) == 9
    assert L.split_dft_destroy(bogus) == 9
    assert L.split_dft_destroy(None) == 0
    assert L.split_dft_plan_info(bogus, None, None, None, None, None) == 9
    assert L.split_dft_workspace_bytes(None) == 0
    b = ctypes.create_string_buffer(16)
    assert L.split_dft_plan_describe(bogus, b, 16) == 9


def test_status_strings(L):
    for code in range(10):
        assert L.split_dft_status_string(code)
    assert L.split_dft_status_string(99) == b"unknown status"


@pytest.mark.parametrize("m", range(0, 17))
def test_twiddle_table_matches_oracle_bitwise(m):
    c, s = binding.twiddle_table(m)
    oc, os_ = oracle.twiddle_table_f32(m)
    assert np.array_equal(c.view(np.uint32), oc.view(np.uint32))
    assert np.array_equal(s.view(np.uint32), os_.view(np.uint32))


def test_twiddle_table_rejects_bad_args(L):
    buf = (ctypes.c_float * 4)()
    assert L.split_dft_twiddle_table(17, buf, buf) == 1
    assert L.split_dft_twiddle_table(-1, buf, buf) == 1
    assert L.split_dft_twiddle_table(2, None, buf) == 3


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2504_07264_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "split_oracle" not in text and "liboracle" not in text, f


def test_many_plan_validates_before_any_hip_call(L):
    import numpy as np
    h = ctypes.c_void_p()
    for bad in ([4, 3], [1], [1 << 17], [0], [-16]):
        a = np.asarray(bad, np.int64)
        assert L.split_dft_many_plan(ctypes.byref(h), a.ctypes.data, a.size, 0) == 1
    a = np.asarray([16, 32], np.int64)
    assert L.split_dft_many_plan(ctypes.byref(h), a.ctypes.data, 0, 0) == 2
    assert L.split_dft_many_plan(ctypes.byref(h), a.ctypes.data, 2, 1) == 6
    assert L.split_dft_many_plan(ctypes.byref(h), a.ctypes.data, 2, 9 << 8) == 6
    assert L.split_dft_many_plan(ctypes.byref(h), a.ctypes.data, 2, 1 << 31) == 6
    assert L.split_dft_many_plan(ctypes.byref(h), a.ctypes.data, 2, 9 << 25) == 6   # threshold below 2^10
    assert L.split_dft_many_plan(ctypes.byref(h), a.ctypes.data, 2, 18 << 25) == 6  # above 2^17
    assert L.split_dft_many_plan(None, a.ctypes.data, 2, 0) == 3
    assert L.split_dft_many_plan(ctypes.byref(h), None, 2, 0) == 3
    bogus = ctypes.c_void_p(0x1000)
    assert L.split_dft_many_exec(bogus, None, None, None, None, None) == 9
    buf = ctypes.c_void_p(0x100000)
    assert L.split_dft_many_exec_ws(bogus, buf, buf, buf, buf, buf, 1 << 20, None) == 9
    assert L.split_dft_many_adjoint_ws(bogus, buf, buf, buf, buf, buf, 1 << 20, None) == 9
    assert L.split_dft_many_exec_adjoint_ws(bogus, buf, buf, buf, buf, buf, buf, buf, buf, buf, 1 << 20,
                                            None) == 9
    g = ctypes.c_void_p()
    assert L.split_dft_many_graph_ws(bogus, buf, buf, buf, buf, None, None, None, None, buf, 1 << 20,
                                     ctypes.byref(g)) == 9
    assert L.split_dft_many_workspace_bytes(None) == 0 and L.split_dft_many_workspace_bytes(bogus) == 0
    assert L.split_dft_graph_launch(bogus, None) == 9
    assert L.split_dft_many_destroy(None) == 0 and L.split_dft_graph_destroy(None) == 0


def test_ragged_generator_recipe():
    from paper_2504_07264_amd import inputs
    lengths, planes = inputs.draw_ragged(50, 4, 16, 4, planes=2)
    assert len(lengths) == 50 and all(int(n) & (int(n) - 1) == 0 for n in lengths)
    assert 16 <= int(lengths.min()) and int(lengths.max()) <= 65536
    assert planes[0].numel() == int(lengths.sum()) == planes[1].numel()
