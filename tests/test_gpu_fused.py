"""The fused two-pass schedule: both passes of a length-2^15 or 2^16 transform
in one persistent launch, each transform's intermediate handed from its
pass-1 to its pass-2 tiles through a ring of slots per XCD (eq. (6) split at
stage 8, Section III).  Bit-exact against the FP32 mirror of eq. (6) over
batches that reuse every ring slot several times, forward and adjoint, on
repeated launches, in place, on planes off a 128-byte line (rotated pass-1
tiles), for batches smaller than the number of XCDs, through a caller
workspace, through the no-allocation entry point and replayed from a HIP
graph; guard words around the outputs."""
import sys

import numpy as np
import pytest
import torch

import oracle
from guards import assert_guards_intact, guarded_empty
from paper_2504_07264_amd import Plan, SplitDFTError, inputs, variant_flag

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def fused_flags(m):
    k = 0
    while True:
        try:
            with Plan(1 << m, 1, variant_flag(k)) as p:
                d = p.describe()
        except SplitDFTError:
            return None
        if "fused" in d:
            return variant_flag(k)
        k += 1


def assert_bit_exact(yr, yi, mr, mi, what):
    yr, yi = yr.cpu().numpy().reshape(mr.shape), yi.cpu().numpy().reshape(mi.shape)
    badr, badi = np.argwhere(yr != mr), np.argwhere(yi != mi)
    assert badr.size == 0 and badi.size == 0, "%s: %d real and %d imag mismatches, first at %s" % (
        what, len(badr), len(badi), (badr[:1].tolist(), badi[:1].tolist()))


def guarded_planes(n, batch):
    bufr, yr = guarded_empty(n * batch)
    bufi, yi = guarded_empty(n * batch)
    return bufr, bufi, yr.view(batch, n), yi.view(batch, n)


@pytest.mark.parametrize("m,batch", [(15, 201), (16, 97)])
def test_fused_every_slot_reused(m, batch):
    n = 1 << m
    flags = fused_flags(m)
    assert flags is not None, "no fused schedule compiled for n = %d" % n
    xr, xi = inputs.draw_planes(n, batch, "normal", 700 + m)
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    ar, ai = oracle.split_adjoint_f32(xr.numpy(), xi.numpy())
    dr, di = xr.cuda(), xi.cuda()
    with Plan(n, batch, flags) as p:
        say("  fused n=%d batch=%d: %s" % (n, batch, p.describe()))
        for rep in range(3):
            bufr, bufi, yr, yi = guarded_planes(n, batch)
            p.exec(dr, di, yr, yi)
            torch.cuda.synchronize()
            assert_guards_intact(bufr, "yr")
            assert_guards_intact(bufi, "yi")
            assert_bit_exact(yr, yi, mr, mi, "forward, launch %d" % rep)
        bufr, bufi, gr, gi = guarded_planes(n, batch)
        p.adjoint(dr, di, gr, gi)
        torch.cuda.synchronize()
        assert_guards_intact(bufr, "gxr")
        assert_guards_intact(bufi, "gxi")
        assert_bit_exact(gr, gi, ar, ai, "adjoint")


@pytest.mark.parametrize("m", [15, 16])
def test_fused_in_place_off_line_and_small_batches(m):
    n = 1 << m
    flags = fused_flags(m)
    for batch in (1, 3, 11):
        xr, xi = inputs.draw_planes(n, batch, "normal", 800 + m + batch)
        mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
        with Plan(n, batch, flags) as p:
            say("  fused n=%d batch=%d in place" % (n, batch))
            yr, yi = xr.cuda(), xi.cuda()
            p.exec(yr, yi, yr, yi)
            torch.cuda.synchronize()
            assert_bit_exact(yr, yi, mr, mi, "in place, batch %d" % batch)
            # planes 16 bytes past a 128-byte line: rotated pass-1 tiles
            say("  fused n=%d batch=%d off-line planes" % (n, batch))
            br = torch.empty(n * batch + 32, device="cuda")
            bi = torch.empty(n * batch + 32, device="cuda")
            pr, pi = br[4:4 + n * batch].view(batch, n), bi[4:4 + n * batch].view(batch, n)
            pr.copy_(xr.view(batch, n))
            pi.copy_(xi.view(batch, n))
            bufr, bufi, yr, yi = guarded_planes(n, batch)
            p.exec(pr, pi, yr, yi)
            torch.cuda.synchronize()
            assert_guards_intact(bufr, "yr")
            assert_guards_intact(bufi, "yi")
            assert_bit_exact(yr, yi, mr, mi, "off-line planes, batch %d" % batch)


@pytest.mark.parametrize("m", [15, 16])
def test_fused_caller_workspace_and_no_allocation(m):
    n, batch = 1 << m, 37
    flags = fused_flags(m)
    xr, xi = inputs.draw_planes(n, batch, "normal", 900 + m)
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    dr, di = xr.cuda(), xi.cuda()
    with Plan(n, batch, flags) as p:
        # a workspace full of garbage: the launch clears the control block itself
        ws = torch.full(((p.workspace_bytes() + 3) // 4,), float("nan"), device="cuda")
        ws.view(torch.int32)[::7] = -1
        say("  fused n=%d batch=%d caller workspace (%d bytes)" % (n, batch, p.workspace_bytes()))
        yr, yi = p.exec(dr, di, workspace=ws)
        torch.cuda.synchronize()
        assert_bit_exact(yr, yi, mr, mi, "caller workspace")
        say("  fused n=%d batch=%d no-allocation entry point" % (n, batch))
        for rep in range(2):
            zr, zi = torch.empty_like(dr), torch.empty_like(di)
            p.exec_noalloc(dr, di, zr, zi)
            torch.cuda.synchronize()
            assert_bit_exact(zr, zi, mr, mi, "no-allocation entry point, call %d" % rep)


@pytest.mark.parametrize("m,batch", [(15, 77), (16, 40)])
def test_fused_captured_in_a_graph(m, batch):
    # the control block is cleared by a kernel, not a memset, so the fused
    # launch can be captured: every replay must equal the eager result, with
    # other work and synchronisations between the replays
    n = 1 << m
    flags = fused_flags(m)
    xr, xi = inputs.draw_planes(n, batch, "normal", 950 + m)
    say("  fused graph capture n=%d batch=%d" % (n, batch))
    with Plan(n, batch, flags) as p:
        ws = torch.empty((p.workspace_bytes() + 3) // 4, device="cuda")
        ar, ai = xr.cuda(), xi.cuda()
        er, ei = p.exec(ar, ai, workspace=ws)
        gr, gi = p.adjoint(er, ei, workspace=ws)
        torch.cuda.synchronize()
        yr, yi = torch.empty_like(ar), torch.empty_like(ai)
        hr, hi = torch.empty_like(ar), torch.empty_like(ai)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):  # warm-up on the capturing stream
            p.exec(ar, ai, yr, yi, workspace=ws)
            p.adjoint(yr, yi, hr, hi, workspace=ws)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            p.exec(ar, ai, yr, yi, workspace=ws)
            p.adjoint(yr, yi, hr, hi, workspace=ws)
        for k in range(3):
            for t in (yr, yi, hr, hi):
                t.fill_(float("nan"))
            ws.fill_(float("nan"))  # garbage in the control block and the ring
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(yr, er) and torch.equal(yi, ei), "replay %d forward" % k
            assert torch.equal(hr, gr) and torch.equal(hi, gi), "replay %d adjoint" % k
        del graph
