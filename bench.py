#!/usr/bin/env python3
"""Benchmark of the split-format DFT hot path on one MI355X.

One step = the whole path on one batch: the forward transform (eq. 5 via the
factorisation of eq. 6) of 16384 rows of length 1024, followed by the adjoint
(backward) transform of an upstream gradient of the same shape.  Inputs are
resident in HBM before timing starts; buffer sets rotate (>= 1 GiB in total)
so the 256 MB Infinity Cache cannot serve repeats.

Prints ONE JSON line (rank 0):
  value      algorithmic GB/s of the step (16 B per complex point per
             direction: 8 B read + 8 B written, FP32 planar)
  roofline   the dominant kernel (the forward length-1024 kernel): algorithmic
             bytes per launch / its mean launch time from HIP events recorded
             on the launch stream during the timed region, against 8 TB/s
  cpu_baseline  the CPU oracle (FP64 factorised transform, OpenMP over rows)
             on the same step, timed on this host's cores
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "split-complex FFT GB/s + 5NlogN GFLOP/s, N=1024×16K; fwd+bwd; MFMA vs FP32"
HBM_PEAK_GBS = 8000.0
N, BATCH = 1024, 16384
ROTATE_SETS = 4

# HBM traffic of the forward length-1024 kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE counters (KiB per dispatch), scaled by the counter/byte ratio of a
# plain copy kernel.  Valid only for the kernel source it was measured on.
TRAFFIC = {
    # "sha256 of csrc/fft_lds.hip": bytes per launch
}


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2504_07264_amd", "csrc", "fft_lds.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def cpu_baseline(xr, xi, gr, gi):
    """Time the CPU oracle on the same step (forward + adjoint)."""
    import numpy as np

    import oracle

    threads = oracle.max_threads()
    a, b = xr.numpy().astype(np.float64), xi.numpy().astype(np.float64)
    c, d = gr.numpy().astype(np.float64), gi.numpy().astype(np.float64)
    rows = a.shape[0]
    # bound the sample to roughly 10-30 s of work
    t0 = time.perf_counter()
    oracle.split_fft(a[:64], b[:64])
    per_row = (time.perf_counter() - t0) / 64
    sample = int(max(64, min(rows, 10.0 / max(per_row * 2, 1e-9))))
    t0 = time.perf_counter()
    oracle.split_fft(a[:sample], b[:sample])
    # the adjoint through the plane swap: (C g_r - S g_i, S g_r + C g_i)
    oracle.split_fft(d[:sample], c[:sample])
    dt = time.perf_counter() - t0
    nbytes = 2 * 16 * N * sample
    return {
        "value": nbytes / dt / 1e9,
        "unit": "GB/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": "%d of %d rows (N=%d), FP64 factorised forward + adjoint, %.2f s" % (sample, rows, N, dt),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; the transforms are independent per row, "
              "so N GPUs would each run the same kernel on batch/N rows with no communication. "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2504_07264_amd import Plan, inputs

    assert torch.cuda.is_available(), "no GPU visible"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    w = inputs.HEADLINE_N1024
    xr, xi = inputs.draw(w)
    gr, gi = inputs.draw_planes(N, BATCH, "normal", w.seed + 100)

    sets = []
    for k in range(ROTATE_SETS):
        s = {
            "xr": xr.to(dev), "xi": xi.to(dev), "gr": gr.to(dev), "gi": gi.to(dev),
            "yr": torch.empty(BATCH, N, device=dev), "yi": torch.empty(BATCH, N, device=dev),
            "hr": torch.empty(BATCH, N, device=dev), "hi": torch.empty(BATCH, N, device=dev),
        }
        sets.append(s)
    plan = Plan(N, BATCH)
    stream = torch.cuda.current_stream(dev)

    def step(k, ev=None):
        s = sets[k % ROTATE_SETS]
        if ev is not None:
            ev[0].record(stream)
        plan.exec(s["xr"], s["xi"], s["yr"], s["yi"])
        if ev is not None:
            ev[1].record(stream)
        plan.adjoint(s["gr"], s["gi"], s["hr"], s["hi"])

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()

    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k, events[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    fwd_ms = sorted(a.elapsed_time(b) for a, b in events)
    fwd_mean_ms = sum(fwd_ms) / len(fwd_ms)
    step_bytes = 2 * 16 * N * BATCH
    launch_bytes = 16 * N * BATCH
    gbs = step_bytes / (ms_per_step * 1e-3) / 1e9
    flops = 2 * 5 * N * math.log2(N) * BATCH
    achieved = launch_bytes / (fwd_mean_ms * 1e-3) / 1e9
    traffic = TRAFFIC.get(kernel_source_hash())

    info = plan.info()
    out = {
        "metric": METRIC,
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "split_fft_n1024_b16384 forward + adjoint",
            "n": N,
            "batch": BATCH,
            "inputs": "FP32 planar N(0,1), seeds 1 (x) and 101 (upstream gradient)",
            "schedule": "%d elements/thread, %d transforms/workgroup" % (info["ept"], info["tpw"]),
            "rotating_buffer_sets": ROTATE_SETS,
        },
        "gflops_5nlogn": round(flops / (ms_per_step * 1e-3) / 1e9, 1),
        "forward_kernel_us": {"mean": round(fwd_mean_ms * 1e3, 2), "median": round(fwd_ms[len(fwd_ms) // 2] * 1e3, 2),
                              "p10": round(fwd_ms[len(fwd_ms) // 10] * 1e3, 2),
                              "p90": round(fwd_ms[(9 * len(fwd_ms)) // 10] * 1e3, 2)},
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
        },
        "device": torch.cuda.get_device_name(dev),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(xr, xi, gr, gi)
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
