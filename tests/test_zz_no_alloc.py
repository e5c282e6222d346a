"""The no-allocation entry point split_dft_exec_noalloc, called through the C
ABI, against split_dft_exec on the same plans and inputs: bit-identical
outputs, on consecutive calls of decreasing size (so the second call runs in
a static scratch array that still holds the first call's intermediate), plus
sampled rows against the oracle's FP32 mirror of eq. (6)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2504_07264_amd import Plan, binding, inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_both(n, batch, seed, flags=0):
    """(split_dft_exec result, split_dft_exec_noalloc result, inputs) on one plan."""
    say("  no-alloc n=%d batch=%d flags=%#x" % (n, batch, flags))
    L = binding.lib()
    xr, xi = inputs.draw_planes(n, batch, "normal", seed)
    with Plan(n, batch, flags, own_workspace=True) as p:
        ar, ai = xr.cuda(), xi.cuda()
        s = torch.cuda.current_stream().cuda_stream
        ref = (torch.empty_like(ar), torch.empty_like(ai))
        got = (torch.full_like(ar, float("nan")), torch.full_like(ai, float("nan")))
        assert L.split_dft_exec(p.handle, ar.data_ptr(), ai.data_ptr(), ref[0].data_ptr(), ref[1].data_ptr(), s) == 0
        assert L.split_dft_exec_noalloc(p.handle, ar.data_ptr(), ai.data_ptr(), got[0].data_ptr(),
                                        got[1].data_ptr(), s) == 0
        torch.cuda.synchronize()
        # argument errors are reported before any launch, as for split_dft_exec
        assert L.split_dft_exec_noalloc(p.handle, ar.data_ptr(), ai.data_ptr(), got[0].data_ptr(),
                                        got[0].data_ptr(), s) == 5
        assert L.split_dft_exec_noalloc(p.handle, ar.data_ptr() + 4, ai.data_ptr(), got[0].data_ptr(),
                                        got[1].data_ptr(), s) == 4
        assert L.split_dft_exec_noalloc(p.handle, None, ai.data_ptr(), got[0].data_ptr(), got[1].data_ptr(), s) == 3
        return [t.cpu().numpy() for t in ref], [t.cpu().numpy() for t in got], (xr.numpy(), xi.numpy())


def check(n, batch, seed, rows=4):
    (rr, ri), (gr, gi), (xr, xi) = run_both(n, batch, seed)
    assert np.array_equal(gr, rr) and np.array_equal(gi, ri), "no-alloc result differs from split_dft_exec"
    idx = np.unique(np.r_[0, batch - 1, np.random.default_rng(seed).integers(0, batch, rows)])
    mr, mi = oracle.split_fft_f32(xr[idx], xi[idx])
    assert np.array_equal(gr[idx], mr) and np.array_equal(gi[idx], mi), "differs from the FP32 mirror of eq. (6)"


def test_two_calls_larger_then_smaller():
    # 2^16: the plan's own chunk is 200 transforms (100 MiB); the 64 MiB
    # scratch takes at most 128, so the call runs two chunks of 100
    n1, b1 = 1 << 16, 200
    assert binding.lib().split_dft_exec_noalloc  # exported
    assert 2 * 4 * n1 * b1 > (64 << 20)
    check(n1, b1, 41)
    # then a smaller two-pass call (2^15, one chunk), reusing the array
    check(1 << 15, 37, 42)


def test_single_pass_and_matrix_core_plans():
    # plans without a workspace run as split_dft_exec
    check(1024, 300, 43)
    (rr, ri), (gr, gi), _ = run_both(256, 96, 44, binding.BF16X3)
    assert np.array_equal(gr, rr) and np.array_equal(gi, ri)


def test_destroyed_plan_rejected():
    L = binding.lib()
    p = Plan(1 << 15, 2)
    h = p.handle
    p.close()
    plane = 4 * 2 * (1 << 15)  # bytes of one [2][2^15] plane
    buf = torch.empty(4 * plane // 4, device="cuda")
    ptr = buf.data_ptr()
    assert L.split_dft_exec_noalloc(h, ptr, ptr + plane, ptr + 2 * plane, ptr + 3 * plane, None) == 9
