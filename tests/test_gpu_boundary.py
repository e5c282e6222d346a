"""Boundary behaviour on the GPU (needs an MI355X): the fused forward +
adjoint call, caller-owned workspaces, the lifetime of captured graphs, and
the convenience entry points on concurrent streams.

Every result is compared bit for bit with the oracle's FP32 mirror of eq. (6)
(forward) or of the adjoint (the transpose of eq. (5)), as in the parity
tests.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2504_07264_amd import ManyPlan, Plan, SplitDFTError, binding, inputs, split_dft, split_dft_adjoint

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def to_np(t):
    return t.detach().cpu().numpy()


def assert_bit_exact(yr, yi, mr, mi, label=""):
    badr = np.argwhere(yr != mr)
    badi = np.argwhere(yi != mi)
    assert badr.size == 0 and badi.size == 0, "%s not bit-exact: %d real and %d imag mismatches, first %s" % (
        label, len(badr), len(badi), (badr[:1].tolist(), badi[:1].tolist()))


# (n, batch, flags): persistent N=1024, the one-transform-per-thread N=16,
# the one-block 2^12 and 2^13 schedules, the 2^14 persistent schedule, N=1,
# a DIF schedule, and a ragged batch size (last block partly filled)
FUSED_CASES = [(1024, 37, 0), (16, 300, 0), (4096, 5, 0), (8192, 3, 0), (16384, 3, 0), (1, 70, 0),
               (1024, 9, binding.DIF), (256, 33, 0), (2048, 7, 0)]


@pytest.mark.parametrize("n,batch,flags", FUSED_CASES)
def test_fused_forward_adjoint_single_launch(n, batch, flags):
    xr, xi, gr, gi = inputs.draw_planes(n, batch, "normal", 61, planes=4)
    if flags & binding.DIF:
        mr, mi = oracle.split_fft_dif_f32(xr.numpy(), xi.numpy())
        hi_, hr_ = oracle.split_fft_dif_f32(gi.numpy(), gr.numpy())  # adjoint through the plane swap
    else:
        mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
        hr_, hi_ = oracle.split_adjoint_f32(gr.numpy(), gi.numpy())
    say("  fused n=%d batch=%d flags=%#x" % (n, batch, flags))
    with Plan(n, batch, flags) as p:
        d = [t.cuda() for t in (xr, xi, gr, gi)]
        yr, yi, hr, hi = p.exec_adjoint(*d)
        torch.cuda.synchronize()
        assert_bit_exact(to_np(yr), to_np(yi), mr, mi, "forward")
        assert_bit_exact(to_np(hr), to_np(hi), hr_, hi_, "adjoint")
        # in place in both directions
        p.exec_adjoint(d[0], d[1], d[2], d[3], out=(d[0], d[1], d[2], d[3]))
        torch.cuda.synchronize()
        assert_bit_exact(to_np(d[0]), to_np(d[1]), mr, mi, "forward in place")
        assert_bit_exact(to_np(d[2]), to_np(d[3]), hr_, hi_, "adjoint in place")


def test_fused_two_pass_and_matrix_core_equal_separate_calls():
    n, batch = 1 << 15, 6
    xr, xi, gr, gi = inputs.draw_planes(n, batch, "normal", 62, planes=4)
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    hr_, hi_ = oracle.split_adjoint_f32(gr.numpy(), gi.numpy())
    say("  fused two-pass n=%d batch=%d" % (n, batch))
    with Plan(n, batch) as p:
        yr, yi, hr, hi = p.exec_adjoint(*[t.cuda() for t in (xr, xi, gr, gi)])
        torch.cuda.synchronize()
        assert_bit_exact(to_np(yr), to_np(yi), mr, mi, "two-pass forward")
        assert_bit_exact(to_np(hr), to_np(hi), hr_, hi_, "two-pass adjoint")
    # the matrix-core modes run the two directions one after the other: the
    # same values as separate calls
    n, batch = 256, 40
    xr, xi, gr, gi = inputs.draw_planes(n, batch, "uniform", 63, planes=4)
    for mode in (binding.BF16X2, binding.FP16X2, binding.BF16X3):
        say("  fused matrix-core mode %d" % mode)
        with Plan(n, batch, mode) as p:
            d = [t.cuda() for t in (xr, xi, gr, gi)]
            yr, yi, hr, hi = p.exec_adjoint(*d)
            sr, si = p.exec(d[0], d[1])
            tr, ti = p.adjoint(d[2], d[3])
            torch.cuda.synchronize()
            assert_bit_exact(to_np(yr), to_np(yi), to_np(sr), to_np(si), "mode %d forward" % mode)
            assert_bit_exact(to_np(hr), to_np(hi), to_np(tr), to_np(ti), "mode %d adjoint" % mode)


def test_fused_rejects_overlap_between_directions():
    n, batch = 1024, 4
    with Plan(n, batch) as p:
        L = binding.lib()
        s = torch.cuda.current_stream().cuda_stream
        a = [torch.zeros(batch, n, device="cuda") for _ in range(8)]
        ptr = [t.data_ptr() for t in a]
        # the forward output is the adjoint's input
        assert L.split_dft_exec_adjoint(p.handle, ptr[0], ptr[1], ptr[2], ptr[3], ptr[2], ptr[5], ptr[6], ptr[7],
                                        s) == 5
        # the adjoint output partly overlaps the forward input
        assert L.split_dft_exec_adjoint(p.handle, ptr[0], ptr[1], ptr[2], ptr[3], ptr[4], ptr[5],
                                        ptr[0] + 64, ptr[7], s) == 5
        assert L.split_dft_exec_adjoint(p.handle, ptr[0], ptr[1], ptr[2], ptr[3], None, ptr[5], ptr[6], ptr[7],
                                        s) == 3
        assert L.split_dft_exec_adjoint(p.handle, ptr[0], ptr[1], ptr[2], ptr[3], ptr[4] + 4, ptr[5], ptr[6],
                                        ptr[7], s) == 4


def small_ragged(seed):
    g = np.random.default_rng(seed)
    lengths = np.repeat(1 << np.arange(4, 17), 2)
    g.shuffle(lengths)
    return lengths


def mirror_all(lengths, offs, ar, ai, adjoint=False):
    out = {}
    for k, n in enumerate(lengths):
        n = int(n)
        f = oracle.split_adjoint_f32 if adjoint else oracle.split_fft_f32
        yr, yi = f(ar[offs[k]:offs[k] + n][None], ai[offs[k]:offs[k] + n][None])
        out[k] = (yr[0], yi[0])
    return out


def check_ragged(lengths, offs, got_r, got_i, ref, label):
    bad = [k for k, (rr, ri) in ref.items()
           if not (np.array_equal(got_r[offs[k]:offs[k] + int(lengths[k])], rr)
                   and np.array_equal(got_i[offs[k]:offs[k] + int(lengths[k])], ri))]
    assert not bad, "%s: %d transforms differ, e.g. %s" % (label, len(bad), bad[:5])


def test_grouped_caller_workspace_and_graph_outliving_plan():
    lengths = small_ragged(71)
    total = int(lengths.sum())
    g = torch.Generator().manual_seed(72)
    planes = [torch.randn(total, generator=g) for _ in range(4)]
    say("  grouped caller workspace: %d transforms, %d points" % (len(lengths), total))
    p = ManyPlan(lengths)
    offs = p.offsets
    fwd = mirror_all(lengths, offs, planes[0].numpy(), planes[1].numpy())
    adj = mirror_all(lengths, offs, planes[2].numpy(), planes[3].numpy(), adjoint=True)
    ws = p.workspace_bytes()
    assert ws > 0 and p.info()["workspace_bytes"] == ws
    d = [t.cuda() for t in planes]
    out = [torch.empty(total, device="cuda") for _ in range(4)]
    L = binding.lib()
    s = torch.cuda.current_stream().cuda_stream
    # no workspace of its own: a NULL workspace is an error, before any launch
    assert L.split_dft_many_exec(p._h, d[0].data_ptr(), d[1].data_ptr(), out[0].data_ptr(), out[1].data_ptr(),
                                 s) == 3
    # an explicit torch workspace, then the binding's own per-call one
    w = torch.empty(ws // 4, device="cuda")
    yr, yi = p.exec(d[0], d[1], workspace=w)
    hr, hi = p.adjoint(d[2], d[3])
    torch.cuda.synchronize()
    check_ragged(lengths, offs, to_np(yr), to_np(yi), fwd, "exec with workspace")
    check_ragged(lengths, offs, to_np(hr), to_np(hi), adj, "adjoint with per-call workspace")
    # a graph captured on a torch workspace; the plan is destroyed first, the
    # graph still replays (the library keeps the plan's device data)
    graph = p.graph(d[0], d[1], out[0], out[1], d[2], d[3], out[2], out[3])
    p.close()
    for rep in range(3):
        for o in out:
            o.fill_(float("nan"))
        graph.launch()
        torch.cuda.synchronize()
        check_ragged(lengths, offs, to_np(out[0]), to_np(out[1]), fwd, "graph forward, plan destroyed, %d" % rep)
        check_ragged(lengths, offs, to_np(out[2]), to_np(out[3]), adj, "graph adjoint, plan destroyed, %d" % rep)
    graph.close()
    # a destroyed graph handle is rejected
    with pytest.raises(SplitDFTError):
        graph.launch()


def test_grouped_plan_owned_workspace_and_device_without_index():
    lengths = small_ragged(73)
    total = int(lengths.sum())
    g = torch.Generator().manual_seed(74)
    xr, xi = [torch.randn(total, generator=g) for _ in range(2)]
    with ManyPlan(lengths, device="cuda", own_workspace=True) as p:
        assert p.device.index == torch.cuda.current_device()
        offs = p.offsets
        L = binding.lib()
        d = [xr.cuda(), xi.cuda()]
        out = [torch.empty(total, device="cuda") for _ in range(2)]
        s = torch.cuda.current_stream().cuda_stream
        assert L.split_dft_many_exec(p._h, d[0].data_ptr(), d[1].data_ptr(), out[0].data_ptr(),
                                     out[1].data_ptr(), s) == 0
        torch.cuda.synchronize()
        check_ragged(lengths, offs, to_np(out[0]), to_np(out[1]), mirror_all(lengths, offs, xr.numpy(), xi.numpy()),
                     "plan-owned workspace")
        # a misaligned caller workspace is rejected before any launch
        w = torch.empty(p.workspace_bytes() // 4 + 4, device="cuda")
        assert L.split_dft_many_exec_ws(p._h, d[0].data_ptr(), d[1].data_ptr(), out[0].data_ptr(),
                                        out[1].data_ptr(), w.data_ptr() + 4, p.workspace_bytes(), s) == 4
        assert L.split_dft_many_exec_ws(p._h, d[0].data_ptr(), d[1].data_ptr(), out[0].data_ptr(),
                                        out[1].data_ptr(), w.data_ptr(), p.workspace_bytes() - 16, s) == 2
        assert L.split_dft_many_exec_ws(p._h, d[0].data_ptr(), d[1].data_ptr(), out[0].data_ptr(),
                                        out[1].data_ptr(), out[1].data_ptr(), p.workspace_bytes(), s) == 5


def test_convenience_entry_points_on_two_streams_two_pass():
    # the cached plan of the convenience functions is shared; each call gets
    # its own workspace, so two-pass calls on two streams cannot collide
    n, batch = 1 << 15, 24
    xs = [inputs.draw_planes(n, batch, "normal", 81 + k) for k in range(2)]
    fwd = oracle.split_fft_f32(xs[0][0].numpy(), xs[0][1].numpy())
    adj = oracle.split_adjoint_f32(xs[1][0].numpy(), xs[1][1].numpy())
    dev = [(xr.cuda(), xi.cuda()) for xr, xi in xs]
    torch.cuda.synchronize()
    say("  convenience calls n=%d batch=%d on two streams" % (n, batch))
    streams = [torch.cuda.Stream() for _ in range(2)]
    res = []
    for rep in range(3):
        with torch.cuda.stream(streams[0]):
            a = split_dft(*dev[0])
        with torch.cuda.stream(streams[1]):
            b = split_dft_adjoint(*dev[1])
        res.append((a, b))
    torch.cuda.synchronize()
    for a, b in res:
        assert_bit_exact(to_np(a[0]), to_np(a[1]), fwd[0], fwd[1], "stream 0 forward")
        assert_bit_exact(to_np(b[0]), to_np(b[1]), adj[0], adj[1], "stream 1 adjoint")
