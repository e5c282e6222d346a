"""Matrix-core split-precision modes at N = 256 (needs an MI355X).

These modes approximate the DFT (operands split into bf16/fp16 parts, FP32
accumulation), so the bar is the per-transform relative L2 error against the
FP64 oracle, not bit equality:
* FP16X2 and BF16X3 meet the FP32 bound 2e-7*log2(N) + 1e-7 (1.7e-6 at N=256);
* BF16X2 carries about 2^-17 relative error per split operand (bf16 hi+lo
  keeps 16 significand bits); summed over the 32-term contractions of two
  stages this is a few 1e-6, bounded here by 2e-5.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2504_07264_amd import Plan, binding, inputs

pytestmark = pytest.mark.gpu

TOL = {"fp16x2": 2e-7 * 8 + 1e-7, "bf16x3": 2e-7 * 8 + 1e-7, "bf16x2": 2e-5}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run(mode, xr, xi, adjoint=False):
    n, batch = xr.shape[1], xr.shape[0]
    say("  mfma mode=%s batch=%d adjoint=%s" % (mode, batch, adjoint))
    with Plan(n, batch, binding.PRECISIONS[mode]) as p:
        a, b = xr.cuda(), xi.cuda()
        yr, yi = (p.adjoint if adjoint else p.exec)(a, b)
        torch.cuda.synchronize()
        return yr.cpu().numpy(), yi.cpu().numpy()


@pytest.mark.parametrize("mode", ["fp16x2", "bf16x3", "bf16x2"])
def test_precision_workload_n256(mode):
    w = inputs.PREC_N256
    xr, xi = inputs.draw(w)
    yr, yi = run(mode, xr, xi)
    rr, ri = oracle.split_fft(xr.double().numpy(), xi.double().numpy())
    err = oracle.rel_l2_per_row(yr, yi, rr, ri)
    say("  %s: rel L2 max %.3e median %.3e (bound %.1e)" % (mode, err.max(), np.median(err), TOL[mode]))
    assert err.max() <= TOL[mode]
    rows = np.random.default_rng(4).choice(w.batch, 32, replace=False)
    dr, di = oracle.dft_direct(xr.double().numpy()[rows], xi.double().numpy()[rows])
    assert oracle.rel_l2_per_row(yr[rows], yi[rows], dr, di).max() <= TOL[mode]


@pytest.mark.parametrize("mode", ["fp16x2", "bf16x3", "bf16x2"])
def test_ragged_batch_and_adjoint(mode):
    xr, xi = inputs.draw_planes(256, 1001, "normal", 77)
    yr, yi = run(mode, xr, xi)
    rr, ri = oracle.split_fft(xr.double().numpy(), xi.double().numpy())
    assert oracle.rel_l2_per_row(yr, yi, rr, ri).max() <= TOL[mode]
    ar, ai = run(mode, xr, xi, adjoint=True)
    dr, di = oracle.adjoint_direct(xr.double().numpy(), xi.double().numpy())
    assert oracle.rel_l2_per_row(ar, ai, dr, di).max() <= TOL[mode]


@pytest.mark.parametrize("mode", ["fp16x2", "bf16x3", "bf16x2"])
def test_single_tone_and_delta(mode):
    n, k0 = 256, 37
    t = 2 * np.pi * ((k0 * np.arange(n)) % n) / n
    xr = torch.tensor(np.stack([np.cos(t), np.zeros(n)]), dtype=torch.float32)
    xi = torch.tensor(np.stack([np.sin(t), np.zeros(n)]), dtype=torch.float32)
    xr[1, 0] = 1.0  # row 1: delta
    yr, yi = run(mode, xr, xi)
    assert abs(yr[0, k0] - n) < 1e-3 and np.hypot(np.delete(yr[0], k0), np.delete(yi[0], k0)).max() < 1e-3
    assert np.abs(yr[1] - 1).max() < 1e-5 and np.abs(yi[1]).max() < 1e-5


def test_mode_requires_n256():
    for n in (16, 1024):
        with pytest.raises(binding.SplitDFTError) as e:
            Plan(n, 4, binding.BF16X2)
        assert e.value.status_name == "UNSUPPORTED"


@pytest.mark.parametrize("mode", ["fp16x2", "bf16x3", "bf16x2"])
def test_any_input_scale(mode):
    # rows scaled by powers of ten far outside FP16's range (and far below
    # its normal range), plus an all-zero row: each row's error stays within
    # the mode's bound (FP16X2 scales every row into range first)
    xr, xi = inputs.draw_planes(256, 12, "uniform", 78)
    scales = torch.tensor([1e-30, 1e-12, 1e-6, 1e-3, 1.0, 30.0, 1e3, 6e4, 1e6, 1e12, 1e30, 0.0])[:, None]
    xr, xi = xr * scales, xi * scales
    yr, yi = run(mode, xr, xi)
    assert np.isfinite(yr).all() and np.isfinite(yi).all()
    assert not yr[-1].any() and not yi[-1].any()
    rr, ri = oracle.split_fft(xr.double().numpy()[:-1], xi.double().numpy()[:-1])
    err = oracle.rel_l2_per_row(yr[:-1], yi[:-1], rr, ri)
    say("  %s: per-scale rel L2 %s" % (mode, np.array2string(err, precision=2)))
    assert err.max() <= TOL[mode]
