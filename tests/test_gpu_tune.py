"""The autotuner on the device: it times every compiled schedule, and a
tuned plan stays bit-exact against the FP32 mirror (needs an MI355X)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_07264_amd import inputs, tune

pytestmark = pytest.mark.gpu


def test_tune_length_and_use_it(tmp_path):
    path = str(tmp_path / "tune.json")
    n, batch = 1024, 513
    best, timings = tune.tune_length(n, batch, iters=3)
    assert best in tune.schedules(n) and len(timings) == len(tune.schedules(n))
    tune.record(tune.length_key(n, batch), best, timings, path)
    assert tune.lookup(tune.length_key(n, batch), path) == best
    xr, xi = inputs.draw_planes(n, batch, "normal", 21)
    with tune.tuned_plan(n, batch, path) as p:
        yr, yi = p.exec(xr.cuda(), xi.cuda())
        torch.cuda.synchronize()
    mr, mi = oracle.split_fft_f32(xr.numpy(), xi.numpy())
    assert np.array_equal(yr.cpu().numpy(), mr) and np.array_equal(yi.cpu().numpy(), mi)


def test_tune_dif_length_and_use_it(tmp_path):
    path = str(tmp_path / "tune.json")
    n, batch = 4096, 129
    best, timings = tune.tune_length(n, batch, iters=3, dif=True)
    assert best in tune.schedules(n, True) and len(timings) == len(tune.schedules(n, True))
    tune.record(tune.length_key(n, batch, True), best, timings, path)
    xr, xi = inputs.draw_planes(n, batch, "normal", 22)
    with tune.tuned_plan(n, batch, path, dif=True) as p:
        assert p.describe().startswith("dif ")
        yr, yi = p.exec(xr.cuda(), xi.cuda())
        torch.cuda.synchronize()
    mr, mi = oracle.split_fft_dif_f32(xr.numpy(), xi.numpy())
    assert np.array_equal(yr.cpu().numpy(), mr) and np.array_equal(yi.cpu().numpy(), mi)


def test_tune_many_small(tmp_path):
    path = str(tmp_path / "tune.json")
    lengths = [16, 1 << 14, 256, 1 << 16, 64, 4096] * 3
    best, timings = tune.tune_many(lengths, iters=2)
    # kernel builds x workgroups-per-CU settings, per-length thresholds, and
    # every length in the persistent kernel
    assert best in timings and len(timings) == 11
    assert {v["one_kernel"] for v in timings.values()} == {False, True}
    assert {v["per_length_from"] for v in timings.values()} == {0, 11, 13, 14}
    tune.record(tune.ragged_key(lengths), best, timings, path)
    with tune.tuned_many_plan(lengths, path) as p:
        assert p.points == sum(lengths)
