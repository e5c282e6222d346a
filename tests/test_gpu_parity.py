"""GPU parity of the HIP path against the CPU oracle (needs an MI355X).

Bars:
* bit-exact (==, so +0 == -0) against the oracle's FP32 structural mirror of
  eq. (6) (same factors, same operation forms, same order);
* per-transform relative L2 error <= 2e-7 * log2(N) + 1e-7 against the FP64
  oracle (O2 on every row; O1, the direct evaluation of eq. (5), on sampled
  rows or bins).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from guards import assert_guards_intact, guarded_empty
from paper_2504_07264_amd import Plan, SplitDFTError, binding, inputs, variant_flag

pytestmark = pytest.mark.gpu


def tol(n):
    m = int(n).bit_length() - 1
    return 2e-7 * m + 1e-7


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def to_np(t):
    return t.detach().cpu().numpy()


def gpu_exec(n, batch, xr, xi, flags=0, adjoint=False):
    say("  exec n=%d batch=%d flags=%#x adjoint=%s" % (n, batch, flags, adjoint))
    with Plan(n, batch, flags) as p:
        dr, di = xr.cuda(), xi.cuda()
        yr, yi = (p.adjoint if adjoint else p.exec)(dr, di)
        torch.cuda.synchronize()
        return to_np(yr), to_np(yi)


def assert_bit_exact(yr, yi, mr, mi):
    badr = np.argwhere(yr != mr)
    badi = np.argwhere(yi != mi)
    assert badr.size == 0 and badi.size == 0, (
        "not bit-exact: %d real and %d imag mismatches, first at %s"
        % (len(badr), len(badi), (badr[:1].tolist(), badi[:1].tolist())))


def assert_within_tol(yr, yi, rr, ri, n):
    err = oracle.rel_l2_per_row(yr, yi, rr, ri)
    assert err.max() <= tol(n), "max rel L2 %.3e > %.3e" % (err.max(), tol(n))
    return err


# ------------------------------------------------------- the N=16 workload
def test_small_n16_bit_exact_and_direct():
    w = inputs.SMALL_N16
    xr, xi = inputs.draw(w)
    yr, yi = gpu_exec(w.n, w.batch, xr, xi)
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    assert_bit_exact(yr, yi, mr, mi)
    rr, ri = oracle.dft_direct(xr.double().numpy(), xi.double().numpy())
    assert_within_tol(yr, yi, rr, ri, w.n)


# ------------------------------------------------------- every length, every schedule
def all_variants(m):
    out = [0]
    k = 0
    while True:
        try:
            with Plan(1 << m, 1, variant_flag(k)):
                pass
        except SplitDFTError:
            break
        out.append(variant_flag(k))
        k += 1
    return out


@pytest.mark.parametrize("m", range(0, 17))
def test_every_length_and_schedule(m):
    n = 1 << m
    # a batch that is not a multiple of any workgroup's transform count, and
    # spans several workgroups
    batch = max(3, min(1000, (1 << 19) // n)) | 1
    xr, xi = inputs.draw_planes(n, batch, "normal", 1000 + m)
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    rr, ri = oracle.split_fft(xr.double().numpy(), xi.double().numpy())
    for flags in all_variants(m):
        yr, yi = gpu_exec(n, batch, xr, xi, flags)
        assert_bit_exact(yr, yi, mr, mi)
        assert_within_tol(yr, yi, rr, ri, n)


@pytest.mark.parametrize("m", range(4, 15))
def test_persistent_schedules_many_blocks_per_workgroup(m):
    # The persistent schedules loop over blocks with a grid stride and
    # prefetch the next block: a batch of about 2^24 points gives every
    # resident workgroup several blocks, and an odd batch a ragged last block.
    n = 1 << m
    batch = ((1 << 24) // n + 3) | 1
    flags_list = []
    for flags in all_variants(m)[1:] + all_dif_variants(m)[1:]:
        with Plan(n, 1, flags) as p:
            if "persistent" in p.describe():
                flags_list.append(flags)
    if not flags_list:
        pytest.skip("no persistent schedule for n = %d" % n)
    xr, xi = inputs.draw_planes(n, batch, "normal", 3000 + m)
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    dr = di = None
    for flags in flags_list:
        dif = bool(flags & binding.DIF)
        if dif and dr is None:
            dr, di = oracle.split_fft_dif_f32(xr.numpy(), xi.numpy())
        yr, yi = gpu_exec(n, batch, xr, xi, flags)
        assert_bit_exact(yr, yi, *((dr, di) if dif else (mr, mi)))
        if not dif:
            yr, yi = gpu_exec(n, batch, xr, xi, flags, adjoint=True)
            ar, ai = oracle.split_adjoint_f32(xr.numpy(), xi.numpy())
            assert_bit_exact(yr, yi, ar, ai)


@pytest.mark.parametrize("m", [0, 1, 4, 7, 10, 12, 15, 16])
def test_adjoint_every_length(m):
    n = 1 << m
    batch = max(1, min(257, (1 << 18) // n))
    gr, gi = inputs.draw_planes(n, batch, "uniform", 2000 + m)
    yr, yi = gpu_exec(n, batch, gr, gi, adjoint=True)
    mr, mi = oracle.split_adjoint_f32(gr.numpy(), gi.numpy())
    assert_bit_exact(yr, yi, mr, mi)
    rr, ri = oracle.adjoint_direct(gr.double().numpy(), gi.double().numpy()) if n <= 4096 else \
        oracle.split_adjoint_f32(gr.numpy(), gi.numpy())
    if n <= 4096:
        assert_within_tol(yr, yi, rr, ri, n)


@pytest.mark.parametrize("m", [4, 10, 15, 16])
def test_closed_forms_exact(m):
    n = 1 << m
    batch = 3
    x = torch.zeros(batch, n)
    x[:, 0] = 1.0
    z = torch.zeros(batch, n)
    yr, yi = gpu_exec(n, batch, x, z)
    assert np.all(yr == 1.0) and np.all(yi == 0.0)
    one = torch.ones(batch, n)
    yr, yi = gpu_exec(n, batch, one, z)
    expect = np.zeros((batch, n), np.float32)
    expect[:, 0] = n
    assert np.array_equal(yr, expect) and np.all(yi == 0.0)


@pytest.mark.parametrize("m", [3, 10, 13, 16])
def test_single_tone_sign(m):
    n = 1 << m
    k0 = n // 3
    t = 2 * np.pi * ((k0 * np.arange(n)) % n) / n
    xr = torch.tensor(np.cos(t), dtype=torch.float32)[None]
    xi = torch.tensor(np.sin(t), dtype=torch.float32)[None]
    yr, yi = gpu_exec(n, 1, xr, xi)
    assert abs(yr[0, k0] - n) < 1e-4 * n
    mag = np.hypot(yr[0], yi[0])
    mag[k0] = 0
    assert mag.max() < 1e-4 * n


# ------------------------------------------------------- the N=1024 x 16384 workload
def test_headline_full_size():
    w = inputs.HEADLINE_N1024
    xr, xi = inputs.draw(w)
    say("  exec n=%d batch=%d into guarded outputs" % (w.n, w.batch))
    with Plan(w.n, w.batch) as p:
        (br, pr), (bi, pi) = guarded_empty(w.n * w.batch), guarded_empty(w.n * w.batch)
        p.exec(xr.cuda(), xi.cuda(), pr.view(w.batch, w.n), pi.view(w.batch, w.n))
        torch.cuda.synchronize()
        assert_guards_intact(br, "yr")
        assert_guards_intact(bi, "yi")
        yr, yi = to_np(pr).reshape(w.batch, w.n), to_np(pi).reshape(w.batch, w.n)
    say("  oracle mirror + FP64 on %d rows" % w.batch)
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    assert_bit_exact(yr, yi, mr, mi)
    rr, ri = oracle.split_fft(xr.double().numpy(), xi.double().numpy())
    err = assert_within_tol(yr, yi, rr, ri, w.n)
    say("  rel L2: max %.3e median %.3e" % (err.max(), np.median(err)))
    rows = np.random.default_rng(0).choice(w.batch, 64, replace=False)
    dr, di = oracle.dft_direct(xr.double().numpy()[rows], xi.double().numpy()[rows])
    assert_within_tol(yr[rows], yi[rows], dr, di, w.n)


def test_adjoint_full_size_n4096():
    w = inputs.GRAD_N4096
    xr, xi, wr, wi = inputs.draw(w)
    say("  adjoint n=%d batch=%d into guarded outputs" % (w.n, w.batch))
    with Plan(w.n, w.batch) as p:
        (br, pr), (bi, pi) = guarded_empty(w.n * w.batch), guarded_empty(w.n * w.batch)
        p.adjoint(wr.cuda(), wi.cuda(), pr.view(w.batch, w.n), pi.view(w.batch, w.n))
        torch.cuda.synchronize()
        assert_guards_intact(br, "gxr")
        assert_guards_intact(bi, "gxi")
        yr, yi = to_np(pr).reshape(w.batch, w.n), to_np(pi).reshape(w.batch, w.n)
    mr, mi = oracle.split_adjoint_f32(wr.numpy(), wi.numpy())
    assert_bit_exact(yr, yi, mr, mi)
    rows = np.random.default_rng(1).choice(w.batch, 16, replace=False)
    dr, di = oracle.adjoint_direct(wr.double().numpy()[rows], wi.double().numpy()[rows])
    assert_within_tol(yr[rows], yi[rows], dr, di, w.n)


# ------------------------------------------------------- boundary behaviour on the device
# small batches (one block per workgroup) and batches that give every
# resident workgroup of a persistent schedule several blocks
@pytest.mark.parametrize("n,batch,dif", [(1024, 37, False), (1024, 16387, False), (64, 262147, False),
                                         (8192, 2051, False), (1024, 16387, True), (16384, 1027, True),
                                         (32768, 41, True), (65536, 300, True), (512, 32771, False),
                                         (512, 32771, True), (16384, 1027, False), (16384, 3, False)])
def test_in_place_and_swapped_planes(n, batch, dif):
    xr, xi = inputs.draw_planes(n, batch, "normal", 7)
    mirror = oracle.split_fft_dif_f32 if dif else oracle.split_fft_f32
    mr, mi = mirror(xr.numpy(), xi.numpy())
    with Plan(n, batch, binding.DIF if dif else 0) as p:
        say("  in place n=%d batch=%d %s" % (n, batch, p.describe()))
        ar, ai = xr.cuda(), xi.cuda()
        p.exec(ar, ai, ar, ai)
        torch.cuda.synchronize()
        assert_bit_exact(to_np(ar), to_np(ai), mr, mi)
        br, bi = xr.cuda(), xi.cuda()
        p.exec(br, bi, bi, br)  # outputs swapped onto the inputs
        torch.cuda.synchronize()
        assert_bit_exact(to_np(bi), to_np(br), mr, mi)


def test_rejects_misaligned_and_overlapping():
    n, batch = 64, 4
    with Plan(n, batch) as p:
        big = torch.zeros(3 * n * batch + 8, device="cuda")
        a = big[: n * batch].view(batch, n)
        b = big[n * batch: 2 * n * batch].view(batch, n)
        L = binding.lib()
        s = torch.cuda.current_stream().cuda_stream
        st = L.split_dft_exec(p.handle, a.data_ptr() + 4, b.data_ptr(), a.data_ptr(), b.data_ptr(), s)
        assert st == 4
        st = L.split_dft_exec(p.handle, a.data_ptr(), b.data_ptr(), a.data_ptr() + 64, b.data_ptr(), s)
        assert st == 5
        st = L.split_dft_exec(p.handle, a.data_ptr(), b.data_ptr(), b.data_ptr(), b.data_ptr(), s)
        assert st == 5
        with pytest.raises(ValueError):
            p.exec(a[:, :32].contiguous(), b[:, :32].contiguous())
        with pytest.raises(TypeError):
            p.exec(a.double(), b.double())


def test_runs_on_a_side_stream():
    n, batch = 256, 1000
    xr, xi = inputs.draw_planes(n, batch, "uniform", 9)
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    st = torch.cuda.Stream()
    with Plan(n, batch) as p:
        dr, di = xr.cuda(), xi.cuda()
        torch.cuda.current_stream().synchronize()
        with torch.cuda.stream(st):
            yr, yi = p.exec(dr, di)
        st.synchronize()
        assert_bit_exact(to_np(yr), to_np(yi), mr, mi)


def test_batch_one_and_large_batch_small_n():
    for n, batch in ((16, 1), (2, 1), (1, 5), (16, 1 << 20)):
        xr, xi = inputs.draw_planes(n, batch, "normal", 11)
        yr, yi = gpu_exec(n, batch, xr, xi)
        mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
        assert_bit_exact(yr, yi, mr, mi)


@pytest.mark.parametrize("n,batch", [(16, (1 << 27) + 5), (1024, (1 << 21) + 3), (4096, (1 << 19) + 1),
                                     (1 << 14, (1 << 17) + 1), (1 << 16, (1 << 15) + 1)])
def test_element_offsets_beyond_int32(n, batch):
    # more than 2^31 floats per plane: every address of the schedules must be
    # formed in 64 bits; in place, with sampled rows (including the ones that
    # straddle element 2^31 and the last one) checked bit-exact
    points = n * batch
    assert points > (1 << 31)
    say("  beyond int32: n=%d batch=%d points=%d" % (n, batch, points))
    g = torch.Generator(device="cuda")
    g.manual_seed(17)
    xr = torch.randn(batch, n, device="cuda", generator=g)
    xi = torch.randn(batch, n, device="cuda", generator=g)
    edge = (1 << 31) // n
    rows = sorted({0, 1, edge - 1, edge, min(edge + 1, batch - 1), batch // 3, batch - 2, batch - 1})
    sr, si = to_np(xr[rows]), to_np(xi[rows])
    with Plan(n, batch) as p:
        p.exec(xr, xi, xr, xi)
        torch.cuda.synchronize()
    mr, mi = oracle.split_fft_f32(sr, si)
    assert_bit_exact(to_np(xr[rows]), to_np(xi[rows]), mr, mi)
    del xr, xi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("m", [14, 15, 16])
def test_two_pass_planes_off_cache_lines(m):
    # planes that start 16 bytes off a 128-byte line, each by a different
    # amount (pass 1 rotates its tiles by the input's offset; the output and
    # imaginary planes sit elsewhere): the rotated tiles must give the same bits
    n, batch = 1 << m, 37
    xr, xi = inputs.draw_planes(n, batch, "normal", 19)
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    flags = variant_flag(len(list_single_pass(m))) if m == 14 else 0  # the two-pass schedule at 2^14
    say("  two-pass off-line planes n=%d batch=%d" % (n, batch))
    pool = torch.zeros(4 * (n * batch + 64), device="cuda")
    stride = n * batch + 64

    def plane(k, off):
        return pool[k * stride + off: k * stride + off + n * batch].view(batch, n)

    ar, ai, yr, yi = plane(0, 4), plane(1, 28), plane(2, 16), plane(3, 8)
    ar.copy_(xr.cuda())
    ai.copy_(xi.cuda())
    with Plan(n, batch, flags) as p:
        assert p.describe().startswith("two-pass")
        p.exec(ar, ai, yr, yi)
        torch.cuda.synchronize()
        assert_bit_exact(to_np(yr), to_np(yi), mr, mi)
        # and in place, from the same off-line planes
        p.exec(ar, ai, ar, ai)
        torch.cuda.synchronize()
        assert_bit_exact(to_np(ar), to_np(ai), mr, mi)


def list_single_pass(m):
    out, k = [], 0
    while True:
        try:
            with Plan(1 << m, 1, variant_flag(k)) as p:
                d = p.describe()
        except SplitDFTError:
            return out
        if d.startswith("two-pass"):
            return out
        out.append(d)
        k += 1


@pytest.mark.parametrize("n,batch", [(1024, 4099), (4096, 515), (1 << 16, 600)])
def test_captured_in_a_graph(n, batch):
    # exec and adjoint captured in a torch (HIP) graph: single-pass persistent,
    # one-block-per-workgroup and chunked two-pass schedules launch nothing but
    # kernels, so every replay must equal the eager result, with other work and
    # synchronisations between the replays
    xr, xi = inputs.draw_planes(n, batch, "normal", 27)
    say("  graph capture n=%d batch=%d" % (n, batch))
    with Plan(n, batch) as p:
        ar, ai = xr.cuda(), xi.cuda()
        er, ei = p.exec(ar, ai)
        gr, gi = p.adjoint(er, ei)
        torch.cuda.synchronize()
        yr, yi = torch.empty_like(ar), torch.empty_like(ai)
        hr, hi = torch.empty_like(ar), torch.empty_like(ai)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):  # warm-up on the capturing stream
            p.exec(ar, ai, yr, yi)
            p.adjoint(yr, yi, hr, hi)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            p.exec(ar, ai, yr, yi)
            p.adjoint(yr, yi, hr, hi)
        for k in range(3):
            for t in (yr, yi, hr, hi):
                t.fill_(float("nan"))
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(yr, er) and torch.equal(yi, ei), "replay %d forward" % k
            assert torch.equal(hr, gr) and torch.equal(hi, gi), "replay %d adjoint" % k
        del graph


@pytest.mark.parametrize("n", [16, 1024, 1 << 15])
def test_subnormal_inputs_bit_exact(n):
    # inputs in the FP32 subnormal range (and a mix with normal values): the
    # kernels keep subnormals (no flush to zero), as the oracle's FP32 mirror
    # does, so the results stay bit-identical
    xr, xi = inputs.draw_planes(n, 9, "normal", 29)
    tiny = 2.0 ** -140
    xr = xr * tiny
    xi[1::2] = xi[1::2] * tiny  # odd rows: both planes subnormal; even rows: normal imaginary parts
    assert (xr.abs() < 2.0 ** -126).all() and (xr != 0).any() and torch.isfinite(xi).all()
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    yr, yi = gpu_exec(n, 9, xr, xi)
    assert_bit_exact(yr, yi, mr, mi)


def test_two_pass_chunks_and_caller_workspace():
    # more rows than one workspace chunk, in place, then with a caller workspace
    n, batch = 1 << 16, 515
    xr, xi = inputs.draw_planes(n, batch, "normal", 13)
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    say("  two-pass n=%d batch=%d" % (n, batch))
    with Plan(n, batch, own_workspace=True) as p:
        ws = p.workspace_bytes()
        assert 0 < ws <= (256 << 20)
        assert ws < 2 * 4 * n * batch  # chunked
        ar, ai = xr.cuda(), xi.cuda()
        p.exec(ar, ai, ar, ai)
        torch.cuda.synchronize()
        assert_bit_exact(to_np(ar), to_np(ai), mr, mi)
        L = binding.lib()
        w = torch.empty(ws // 4, device="cuda")
        br, bi = xr.cuda(), xi.cuda()
        yr, yi = torch.empty_like(br), torch.empty_like(bi)
        s = torch.cuda.current_stream().cuda_stream
        assert L.split_dft_exec_ws(p.handle, br.data_ptr(), bi.data_ptr(), yr.data_ptr(), yi.data_ptr(),
                                   w.data_ptr(), ws, s) == 0
        torch.cuda.synchronize()
        assert_bit_exact(to_np(yr), to_np(yi), mr, mi)
        hr, hi = oracle.split_adjoint_f32(xr.numpy(), xi.numpy())
        assert L.split_dft_adjoint_ws(p.handle, br.data_ptr(), bi.data_ptr(), yr.data_ptr(), yi.data_ptr(),
                                      w.data_ptr(), ws, s) == 0
        torch.cuda.synchronize()
        assert_bit_exact(to_np(yr), to_np(yi), hr, hi)
        # a NULL workspace means the plan's own
        yr.zero_()
        yi.zero_()
        assert L.split_dft_exec_ws(p.handle, br.data_ptr(), bi.data_ptr(), yr.data_ptr(), yi.data_ptr(),
                                   None, 0, s) == 0
        torch.cuda.synchronize()
        assert_bit_exact(to_np(yr), to_np(yi), mr, mi)
        # too small, misaligned or overlapping workspaces are rejected before any launch
        assert L.split_dft_exec_ws(p.handle, br.data_ptr(), bi.data_ptr(), yr.data_ptr(), yi.data_ptr(),
                                   w.data_ptr(), ws - 16, s) == 2
        assert L.split_dft_exec_ws(p.handle, br.data_ptr(), bi.data_ptr(), yr.data_ptr(), yi.data_ptr(),
                                   w.data_ptr() + 4, ws, s) == 4
        assert L.split_dft_exec_ws(p.handle, br.data_ptr(), bi.data_ptr(), yr.data_ptr(), yi.data_ptr(),
                                   yr.data_ptr(), ws, s) == 5
    # a plan without a workspace of its own: NULL is an error, the binding
    # allocates one per call through torch
    with Plan(n, batch) as p:
        assert p.workspace_bytes() > 0
        L = binding.lib()
        s = torch.cuda.current_stream().cuda_stream
        br, bi = xr.cuda(), xi.cuda()
        yr, yi = torch.empty_like(br), torch.empty_like(bi)
        assert L.split_dft_exec(p.handle, br.data_ptr(), bi.data_ptr(), yr.data_ptr(), yi.data_ptr(), s) == 3
        assert b"SPLIT_DFT_CALLER_WORKSPACE" in L.split_dft_last_error()
        yr, yi = p.exec(br, bi)
        torch.cuda.synchronize()
        assert_bit_exact(to_np(yr), to_np(yi), mr, mi)


def test_two_pass_calls_overlap_on_streams_with_own_workspaces():
    # one two-pass plan, two side streams, each call with its own workspace
    # tensor (the Python binding's workspace argument): both results exact
    n, batch = 1 << 15, 300
    xs = [inputs.draw_planes(n, batch, "normal", 41 + k) for k in range(2)]
    refs = [oracle.split_fft_f32(xr.numpy(), xi.numpy()) for xr, xi in xs]
    adj = oracle.split_adjoint_f32(xs[1][0].numpy(), xs[1][1].numpy())
    say("  two-pass n=%d batch=%d on two streams" % (n, batch))
    with Plan(n, batch) as p:
        ws = p.workspace_bytes()
        dev = [(xr.cuda(), xi.cuda()) for xr, xi in xs]
        torch.cuda.synchronize()
        streams = [torch.cuda.Stream() for _ in range(2)]
        outs = []
        for k, st in enumerate(streams):
            with torch.cuda.stream(st):
                w = torch.empty(ws // 4, device="cuda")
                outs.append(p.exec(dev[k][0], dev[k][1], workspace=w))
        with torch.cuda.stream(streams[1]):
            w2 = torch.empty(ws // 4, device="cuda")
            gr, gi = p.adjoint(dev[1][0], dev[1][1], workspace=w2)
        torch.cuda.synchronize()
        for (yr, yi), (mr, mi) in zip(outs, refs):
            assert_bit_exact(to_np(yr), to_np(yi), mr, mi)
        assert_bit_exact(to_np(gr), to_np(gi), adj[0], adj[1])
        with pytest.raises(SplitDFTError):
            p.exec(dev[0][0], dev[0][1], workspace=torch.empty(ws // 4 - 4, device="cuda"))
        with pytest.raises(ValueError):
            p.exec(dev[0][0], dev[0][1], workspace=torch.empty(8))


def test_single_pass_plans_need_no_workspace():
    with Plan(1024, 8) as p:
        assert p.workspace_bytes() == 0


# ------------------------------------------------------- decimation in frequency (eq. 9)
def all_dif_variants(m):
    out = [binding.DIF]
    k = 0
    while True:
        try:
            with Plan(1 << m, 1, binding.DIF | variant_flag(k)):
                pass
        except SplitDFTError:
            break
        out.append(binding.DIF | variant_flag(k))
        k += 1
    return out


@pytest.mark.parametrize("m", range(0, 17))
def test_dif_every_length(m):
    n = 1 << m
    batch = max(3, min(1000, (1 << 19) // n)) | 1
    xr, xi = inputs.draw_planes(n, batch, "normal", 3000 + m)
    mr, mi = oracle.split_fft_dif_f32(xr.numpy(), xi.numpy())
    rr, ri = oracle.split_fft(xr.double().numpy(), xi.double().numpy())
    for flags in all_dif_variants(m):
        yr, yi = gpu_exec(n, batch, xr, xi, flags)
        assert_bit_exact(yr, yi, mr, mi)
        assert_within_tol(yr, yi, rr, ri, n)
    # the adjoint through the plane exchange
    ar, ai = gpu_exec(n, batch, xr, xi, binding.DIF, adjoint=True)
    hr, hi = oracle.split_fft_dif_f32(xi.numpy(), xr.numpy())
    assert_bit_exact(ar, ai, hi, hr)


def test_plan_info_and_describe():
    with Plan(1024, 7) as p:
        info = p.info()
        assert info == {"n": 1024, "batch": 7, "log2n": 10, "ept": 16, "tpw": 4}
        assert p.workspace_bytes() == 0 and "persistent" in p.describe()
    with Plan(1 << 16, 3) as p:
        info = p.info()
        assert info["log2n"] == 16 and info["tpw"] == 0
        assert p.describe().startswith("two-pass") and p.workspace_bytes() == 3 * (1 << 16) * 2 * 4
    with Plan(256, 5, binding.PRECISIONS["bf16x2"]) as p:
        assert p.describe().startswith("mfma16x16x32 bf16x2")
    from paper_2504_07264_amd import ManyPlan
    with ManyPlan([16, 1 << 15, 64]) as mp:
        mi = mp.info()
        assert mi["count"] == 3 and mi["points"] == 16 + (1 << 15) + 64
        assert mi["workgroups"] > 0 and mi["items"] >= 1 and mi["workspace_bytes"] >= (1 << 15) * 2 * 4


@pytest.mark.parametrize("m,batch", [(15, 300), (16, 131)])
def test_dif_two_pass_workspace_paths(m, batch):
    # the DIF two-pass schedule through a caller workspace and through the
    # no-allocation entry point (whose static array holds fewer transforms than
    # the batch: several chunks), bit-exact against the DIF mirror of eq. (9)
    n = 1 << m
    xr, xi = inputs.draw_planes(n, batch, "normal", 3100 + m)
    mr, mi = oracle.split_fft_dif_f32(xr.numpy(), xi.numpy())
    with Plan(n, batch, binding.DIF) as p:
        say("  dif workspace paths n=%d batch=%d %s" % (n, batch, p.describe()))
        dr, di = xr.cuda(), xi.cuda()
        ws = torch.full(((p.workspace_bytes() + 3) // 4,), float("nan"), device="cuda")
        yr, yi = p.exec(dr, di, workspace=ws)
        torch.cuda.synchronize()
        assert_bit_exact(to_np(yr), to_np(yi), mr, mi)
        zr, zi = torch.empty_like(dr), torch.empty_like(di)
        p.exec_noalloc(dr, di, zr, zi)
        torch.cuda.synchronize()
        assert_bit_exact(to_np(zr), to_np(zi), mr, mi)
