"""Grouped execution of a ragged batch of mixed lengths (needs an MI355X).

Every transform of the batch must equal, bit for bit, the oracle's FP32
mirror of eq. (6) for its length (forward), or of the adjoint, whatever the
mix, order or launch form (direct, or replayed from a captured graph).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from guards import assert_guards_intact, guarded_empty
from paper_2504_07264_amd import ManyPlan, SplitDFTError, binding, inputs, many_flags

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def mirror_ragged(lengths, offs, ar, ai, which, adjoint=False):
    """FP32 mirror results of the transforms ``which`` (dict k -> (yr, yi))."""
    out = {}
    by_n = {}
    for k in which:
        by_n.setdefault(int(lengths[k]), []).append(k)
    for n, ks in by_n.items():
        rr = np.stack([ar[offs[k]:offs[k] + n] for k in ks])
        ri = np.stack([ai[offs[k]:offs[k] + n] for k in ks])
        yr, yi = (oracle.split_adjoint_f32 if adjoint else oracle.split_fft_f32)(rr, ri)
        for j, k in enumerate(ks):
            out[k] = (yr[j], yi[j])
    return out


def check(lengths, offs, got_r, got_i, ref, label):
    bad = []
    for k, (rr, ri) in ref.items():
        n = int(lengths[k])
        gr = got_r[offs[k]:offs[k] + n]
        gi = got_i[offs[k]:offs[k] + n]
        if not (np.array_equal(gr, rr) and np.array_equal(gi, ri)):
            bad.append((k, n))
    assert not bad, "%s: %d transforms differ from the mirror, e.g. %s" % (label, len(bad), bad[:5])


def mixed_lengths(seed, per_len=3, mmin=2, mmax=16):
    g = np.random.default_rng(seed)
    ls = np.repeat(1 << np.arange(mmin, mmax + 1), per_len)
    g.shuffle(ls)
    return ls


# (kernel build, every length in the persistent kernel, per-length threshold)
@pytest.mark.parametrize("build,one_kernel,split", [(-1, False, 0), (1, False, 0), (-1, True, 0), (1, True, 0),
                                                    (-1, False, 10), (-1, False, 15), (-1, False, 17)])
def test_mixed_lengths_forward_adjoint_both(build, one_kernel, split):
    lengths = mixed_lengths(5)
    total = int(lengths.sum())
    g = torch.Generator().manual_seed(6)
    xr, xi, gr, gi = [torch.randn(total, generator=g) for _ in range(4)]
    say("  grouped build=%d one_kernel=%s split=%d count=%d points=%d"
        % (build, one_kernel, split, len(lengths), total))
    with ManyPlan(lengths, many_flags(build, one_kernel=one_kernel, per_length_from=split)) as p:
        offs = p.offsets
        assert offs[-1] == total
        fwd = mirror_ragged(lengths, offs, xr.numpy(), xi.numpy(), range(len(lengths)))
        adj = mirror_ragged(lengths, offs, gr.numpy(), gi.numpy(), range(len(lengths)), adjoint=True)
        dx = [t.cuda() for t in (xr, xi, gr, gi)]
        yr, yi = p.exec(dx[0], dx[1])
        torch.cuda.synchronize()
        check(lengths, offs, yr.cpu().numpy(), yi.cpu().numpy(), fwd, "forward")
        hr, hi = p.adjoint(dx[2], dx[3])
        torch.cuda.synchronize()
        check(lengths, offs, hr.cpu().numpy(), hi.cpu().numpy(), adj, "adjoint")
        yr, yi, hr, hi = p.exec_adjoint(*dx)
        torch.cuda.synchronize()
        check(lengths, offs, yr.cpu().numpy(), yi.cpu().numpy(), fwd, "both/forward")
        check(lengths, offs, hr.cpu().numpy(), hi.cpu().numpy(), adj, "both/adjoint")
        # in place, forward
        ar, ai = dx[0].clone(), dx[1].clone()
        p.exec(ar, ai, ar, ai)
        torch.cuda.synchronize()
        check(lengths, offs, ar.cpu().numpy(), ai.cpu().numpy(), fwd, "in place")


def test_graph_replays_match_eager():
    lengths = mixed_lengths(7, per_len=2, mmin=4)
    total = int(lengths.sum())
    g = torch.Generator().manual_seed(8)
    planes = [torch.randn(total, generator=g).cuda() for _ in range(4)]
    outs = [torch.empty(total, device="cuda") for _ in range(4)]
    with ManyPlan(lengths) as p:
        offs = p.offsets
        fwd = mirror_ragged(lengths, offs, planes[0].cpu().numpy(), planes[1].cpu().numpy(), range(len(lengths)))
        adj = mirror_ragged(lengths, offs, planes[2].cpu().numpy(), planes[3].cpu().numpy(), range(len(lengths)),
                            adjoint=True)
        gr = p.graph(planes[0], planes[1], outs[0], outs[1], planes[2], planes[3], outs[2], outs[3])
        for rep in range(4):
            for o in outs:
                o.fill_(float("nan"))
            # eager work of the program between replays
            e = p.exec(planes[0], planes[1])
            torch.cuda.synchronize()
            check(lengths, offs, e[0].cpu().numpy(), e[1].cpu().numpy(), fwd, "eager %d" % rep)
            gr.launch()
            torch.cuda.synchronize()
            check(lengths, offs, outs[0].cpu().numpy(), outs[1].cpu().numpy(), fwd, "graph fwd %d" % rep)
            check(lengths, offs, outs[2].cpu().numpy(), outs[3].cpu().numpy(), adj, "graph adj %d" % rep)
        gr.close()


def test_ragged_workload_20000():
    # every transform of the workload, both directions, bit for bit, with
    # guard words around each of the four output planes
    lengths, (xr, xi, gr, gi) = inputs.draw_ragged(inputs.RAGGED_COUNT, inputs.RAGGED_KMIN, inputs.RAGGED_KMAX,
                                                   inputs.RAGGED_SEED)
    lengths = lengths.numpy()
    total = int(lengths.sum())
    say("  ragged workload: %d transforms, %d points, guarded outputs" % (len(lengths), total))
    with ManyPlan(lengths) as p:
        offs = p.offsets
        dx = [t.cuda() for t in (xr, xi, gr, gi)]
        guarded = [guarded_empty(total) for _ in range(4)]
        out = [g[1] for g in guarded]
        graph = p.graph(dx[0], dx[1], out[0], out[1], dx[2], dx[3], out[2], out[3])
        graph.launch()
        torch.cuda.synchronize()
        for (buf, _), name in zip(guarded, ("yr", "yi", "gxr", "gxi")):
            assert_guards_intact(buf, name)
        o = [t.cpu().numpy() for t in out]
        everything = range(len(lengths))
        say("  FP32 mirror of all %d transforms, both directions" % len(lengths))
        fwd = mirror_ragged(lengths, offs, xr.numpy(), xi.numpy(), everything)
        adj = mirror_ragged(lengths, offs, gr.numpy(), gi.numpy(), everything, adjoint=True)
        check(lengths, offs, o[0], o[1], fwd, "workload forward")
        check(lengths, offs, o[2], o[3], adj, "workload adjoint")
        rng = np.random.default_rng(9)
        which = sorted(set(rng.choice(len(lengths), 27, replace=False).tolist())
                       | {int(np.flatnonzero(lengths == (1 << k))[0]) for k in range(4, 17)})
        for k in which:
            n = int(lengths[k])
            rr, ri = oracle.split_fft(xr.numpy()[offs[k]:offs[k] + n].astype(np.float64)[None],
                                      xi.numpy()[offs[k]:offs[k] + n].astype(np.float64)[None])
            err = oracle.rel_l2_per_row(o[0][offs[k]:offs[k] + n][None], o[1][offs[k]:offs[k] + n][None], rr, ri)
            assert err.max() <= 2e-7 * (n.bit_length() - 1) + 1e-7
        graph.close()


def test_many_short_transforms():
    # only lengths 2^4 .. 2^11: everything runs in the persistent kernel, each
    # workgroup through many group items of every short length
    lengths, (xr, xi, gr, gi) = inputs.draw_ragged(60000, 4, 11, 5)
    lengths = lengths.numpy()
    total = int(lengths.sum())
    say("  short ragged batch: %d transforms, %d points" % (len(lengths), total))
    with ManyPlan(lengths) as p:
        offs = p.offsets
        dx = [t.cuda() for t in (xr, xi, gr, gi)]
        out = [torch.empty(total, device="cuda") for _ in range(4)]
        graph = p.graph(dx[0], dx[1], out[0], out[1], dx[2], dx[3], out[2], out[3])
        graph.launch()
        torch.cuda.synchronize()
        rng = np.random.default_rng(13)
        which = sorted(set(rng.choice(len(lengths), 300, replace=False).tolist())
                       | {int(np.flatnonzero(lengths == (1 << k))[-1]) for k in range(4, 12)})
        o = [t.cpu().numpy() for t in out]
        check(lengths, offs, o[0], o[1], mirror_ragged(lengths, offs, xr.numpy(), xi.numpy(), which), "forward")
        check(lengths, offs, o[2], o[3], mirror_ragged(lengths, offs, gr.numpy(), gi.numpy(), which, adjoint=True),
              "adjoint")
        graph.close()


@pytest.mark.parametrize("one_kernel", [False, True])
def test_offsets_beyond_int32(one_kernel):
    # more than 2^31 floats per plane, and transforms of every length placed
    # past element 2^31: offsets and addresses must be formed in 64 bits on
    # every route (per-length launches, the persistent kernel's items)
    rng = np.random.default_rng(21)
    head = np.full((1 << 15) + 1, 1 << 16, dtype=np.int64)
    tail = np.repeat(1 << np.arange(2, 17), 2)
    rng.shuffle(tail)
    lengths = np.concatenate([head, tail])
    flags = binding.MANY_ONE_KERNEL if one_kernel else 0
    with ManyPlan(lengths, flags=flags) as p:
        offs = p.offsets
        total = p.points
        assert total > (1 << 31)
        say("  ragged beyond int32: %d transforms, %d points, one_kernel=%s" % (len(lengths), total, one_kernel))
        g = torch.Generator(device="cuda")
        g.manual_seed(23)
        xr = torch.randn(total, device="cuda", generator=g)
        xi = torch.randn(total, device="cuda", generator=g)
        yr, yi = p.exec(xr, xi)
        torch.cuda.synchronize()
        edge = int(np.searchsorted(offs, 1 << 31, side="right")) - 1
        which = sorted({0, edge - 1, edge, edge + 1} | set(range(len(head), len(lengths))))
        segs = lambda t: {k: to_np_seg(t, offs[k], int(lengths[k])) for k in which}
        sx_r, sx_i, sy_r, sy_i = segs(xr), segs(xi), segs(yr), segs(yi)
        bad = []
        for k in which:
            mr, mi = oracle.split_fft_f32(sx_r[k][None], sx_i[k][None])
            if not (np.array_equal(sy_r[k], mr[0]) and np.array_equal(sy_i[k], mi[0])):
                bad.append((k, int(lengths[k])))
        assert not bad, "transforms differ from the mirror: %s" % bad[:5]
        del xr, xi, yr, yi
    torch.cuda.empty_cache()


def to_np_seg(t, off, n):
    return t[int(off):int(off) + n].cpu().numpy()


def test_rejects_bad_lengths_and_pointers():
    for bad in ([4, 3], [1], [1 << 17], [0]):
        with pytest.raises(SplitDFTError) as e:
            ManyPlan(bad)
        assert e.value.status_name == "INVALID_LENGTH"
    with ManyPlan([16, 64]) as p:
        a = torch.zeros(80, device="cuda")
        with pytest.raises(ValueError):
            p.exec(a[:40], a[40:])
        L = binding.lib()
        s = torch.cuda.current_stream().cuda_stream
        b = torch.zeros(4 * 80 + 4, device="cuda")
        assert L.split_dft_many_exec(p._h, b.data_ptr() + 4, b.data_ptr(), b.data_ptr(), b.data_ptr(), s) == 4
        assert L.split_dft_many_exec(p._h, b.data_ptr(), b[80:].data_ptr(), b[160:].data_ptr(),
                                     b[164:].data_ptr(), s) == 5
