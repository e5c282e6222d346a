"""Autograd: the split DFT as a differentiable op whose backward is the
hand-written adjoint kernel (needs an MI355X).

loss = sum(wr * yr + wi * yi) is linear in x, so its gradient is
E_2N^T (wr, wi) = (C wr - S wi, S wr + C wi), independent of x.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2504_07264_amd import inputs, split_dft_autograd

pytestmark = pytest.mark.gpu


def tol(n):
    return 2e-7 * (int(n).bit_length() - 1) + 1e-7


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_gradient_matches_fp64_finite_differences():
    w = inputs.GRAD_FD_N64
    xr, xi, wr, wi = inputs.draw(w)
    say("  autograd n=%d batch=%d" % (w.n, w.batch))
    ar = xr.cuda().requires_grad_(True)
    ai = xi.cuda().requires_grad_(True)
    yr, yi = split_dft_autograd(ar, ai)
    (wr.cuda() * yr + wi.cuda() * yi).sum().backward()
    torch.cuda.synchronize()
    g_r, g_i = ar.grad.cpu().numpy(), ai.grad.cpu().numpy()

    # central differences of the FP64 loss evaluated with the direct eq. (5)
    X = [xr.double().numpy(), xi.double().numpy()]
    W = [wr.double().numpy(), wi.double().numpy()]

    def loss(a, b):
        yr_, yi_ = oracle.dft_direct(a, b)
        return (W[0] * yr_ + W[1] * yi_).sum()

    h = 1e-3
    fd = [np.zeros_like(X[0]), np.zeros_like(X[1])]
    for p in range(2):
        for b in range(w.batch):
            for n in range(w.n):
                plus = [X[0].copy(), X[1].copy()]
                minus = [X[0].copy(), X[1].copy()]
                plus[p][b, n] += h
                minus[p][b, n] -= h
                fd[p][b, n] = (loss(*plus) - loss(*minus)) / (2 * h)
    err = oracle.rel_l2_per_row(g_r, g_i, fd[0], fd[1])
    assert err.max() <= tol(w.n), err.max()
    # the FP64 direct adjoint gives the same gradient
    dr, di = oracle.adjoint_direct(W[0], W[1])
    assert oracle.rel_l2_per_row(fd[0], fd[1], dr, di).max() < 1e-9


def test_full_size_forward_and_backward_n4096():
    w = inputs.GRAD_N4096
    xr, xi, wr, wi = inputs.draw(w)
    say("  autograd n=%d batch=%d" % (w.n, w.batch))
    ar = xr.cuda().requires_grad_(True)
    ai = xi.cuda().requires_grad_(True)
    yr, yi = split_dft_autograd(ar, ai)
    (wr.cuda() * yr + wi.cuda() * yi).sum().backward()
    torch.cuda.synchronize()
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    assert np.array_equal(yr.detach().cpu().numpy(), mr) and np.array_equal(yi.detach().cpu().numpy(), mi)
    gr, gi = ar.grad.cpu().numpy(), ai.grad.cpu().numpy()
    hr, hi = oracle.split_adjoint_f32(wr.numpy(), wi.numpy())
    assert np.array_equal(gr, hr) and np.array_equal(gi, hi)
    rows = np.random.default_rng(3).choice(w.batch, 16, replace=False)
    dr, di = oracle.adjoint_direct(wr.double().numpy()[rows], wi.double().numpy()[rows])
    assert oracle.rel_l2_per_row(gr[rows], gi[rows], dr, di).max() <= tol(w.n)


def test_one_output_used_and_leading_dims():
    n = 256
    xr, xi = inputs.draw_planes(n, 6, "normal", 31)
    ar = xr.view(2, 3, n).cuda().requires_grad_(True)
    ai = xi.view(2, 3, n).cuda().requires_grad_(True)
    yr, yi = split_dft_autograd(ar, ai)
    assert yr.shape == (2, 3, n)
    yr.sum().backward()  # gradient w.r.t. yi is absent (zero)
    torch.cuda.synchronize()
    ones = np.ones((6, n), np.float32)
    hr, hi = oracle.split_adjoint_f32(ones, np.zeros_like(ones))
    assert np.array_equal(ar.grad.reshape(6, n).cpu().numpy(), hr)
    assert np.array_equal(ai.grad.reshape(6, n).cpu().numpy(), hi)


def test_views_that_start_off_alignment_and_strided_views():
    # a view starting 4 bytes into its allocation, and a transposed
    # (non-contiguous) one: the wrapper copies them to aligned, contiguous
    # operands; results and gradients equal the mirror's bits
    n, rows = 64, 10
    xr, xi = inputs.draw_planes(n, rows, "normal", 33)
    br = torch.empty(rows * n + 1, device="cuda")
    br[1:] = xr.reshape(-1).cuda()
    ar = br[1:].view(rows, n)
    assert ar.data_ptr() % 16 != 0
    ai_t = xi.cuda().t().contiguous().t()  # non-contiguous view of the same values
    assert not ai_t.is_contiguous()
    ar.requires_grad_(True)
    ai_t.requires_grad_(True)
    yr, yi = split_dft_autograd(ar, ai_t)
    (yr.sum() + 2 * yi.sum()).backward()
    torch.cuda.synchronize()
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    assert np.array_equal(yr.detach().cpu().numpy(), mr) and np.array_equal(yi.detach().cpu().numpy(), mi)
    ones = np.ones((rows, n), np.float32)
    hr, hi = oracle.split_adjoint_f32(ones, 2 * ones)
    assert np.array_equal(ar.grad.cpu().numpy(), hr) and np.array_equal(ai_t.grad.cpu().numpy(), hi)


def test_cached_plans_are_bounded():
    # the convenience entry points keep a small most-recently-used set of plans
    from paper_2504_07264_amd import binding

    n = 16
    for batch in range(1, binding.PLAN_CACHE_SIZE + 5):
        xr, xi = inputs.draw_planes(n, batch, "normal", 40 + batch)
        yr, yi = binding.split_dft(xr.cuda(), xi.cuda())
        torch.cuda.synchronize()
        mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
        assert np.array_equal(yr.cpu().numpy(), mr) and np.array_equal(yi.cpu().numpy(), mi)
        assert len(binding._plan_cache) <= binding.PLAN_CACHE_SIZE
