#!/usr/bin/env python3
"""Benchmark of the split-format DFT hot path on one MI355X.

One step = the whole path on one batch: the forward transform (eq. 5 via the
factorisation of eq. 6) of 16384 rows of length 1024, followed by the adjoint
(backward) transform of an upstream gradient of the same shape.  Inputs are
resident in HBM before timing starts; buffer sets rotate (>= 1 GiB in total)
so the 256 MB Infinity Cache cannot serve repeats.  The kernel schedule is
the autotuner's choice, timed on this device before the timed region.

Prints ONE JSON line (rank 0):
  value      algorithmic GB/s of the step (16 B per complex point per
             direction: 8 B read + 8 B written, FP32 planar), from the host
             clock around the timed steps
  roofline   the dominant kernel (the length-1024 kernel, which both the
             forward and the adjoint launch): algorithmic bytes per launch /
             its mean time per launch, from HIP events recorded on the launch
             stream at both ends of the timed region (which holds nothing
             else), against 8 TB/s
  kernel_us_per_launch  median, p10 and p90 of >= 100 launches, each between
             two HIP events (a second timed region)
  cpu_baseline  the CPU oracle (FP64 factorised transform, OpenMP over rows)
             on the same step, timed on this host's cores
Side reports: the fused forward + adjoint launch, matrix cores against FP32
(time and error per mode), the copy ceiling, DIF, N=4096 forward + adjoint,
the two-pass lengths and the ragged batch (default and tuned schedules).
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
PREWARM_S = 1.0
MIN_ITERS = 100  # timed iterations per side measurement


def stats_us(us):
    """Median, p10, p90 and mean of a list of microsecond timings (n: how
    many timed groups)."""
    t = sorted(us)

    def q(f):
        return t[min(len(t) - 1, max(0, int(round(f * (len(t) - 1)))))]

    return {"median": round(q(0.5), 2), "p10": round(q(0.1), 2), "p90": round(q(0.9), 2),
            "mean": round(sum(t) / len(t), 2), "n": len(t)}


def event_times(fn, iters, stream, group: int = 4):
    """Run fn(k) for k < iters * group, back to back, with a HIP event recorded
    on `stream` before the first call and after every `group` calls; returns
    the microseconds per call of each group (an event between every call
    would keep consecutive kernels from overlapping and add its own time)."""
    import torch

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(iters + 1)]
    ev[0].record(stream)
    for j in range(iters):
        for k in range(j * group, (j + 1) * group):
            fn(k)
        ev[j + 1].record(stream)
    torch.cuda.synchronize()
    return [ev[j].elapsed_time(ev[j + 1]) * 1e3 / group for j in range(iters)]


# HBM traffic of the forward length-1024 kernel: rocprofv3 FETCH_SIZE and
# WRITE_SIZE per dispatch, scaled by what the same counters read for a plain
# copy of known size.  The summary records the kernel source it was measured
# on; for any other source the traffic is reported as null.
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "split_fft_n1024_b16384_hbm_traffic.md")


def code_hash(texts) -> str:
    """sha256 of source texts with line comments, trailing blanks and blank
    lines removed (a comment edit does not change it)."""
    import re

    code = []
    for text in texts:
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines()]
        code.append("\n".join(ln for ln in lines if ln.strip()))
    return hashlib.sha256("\n".join(code).encode()).hexdigest()


def kernel_source_hash() -> str:
    """code_hash of the forward kernel's device source (fft_lds.hip, then the
    stage code it includes, fft_device.h)."""
    texts = []
    for name in ("fft_lds.hip", "fft_device.h"):
        with open(os.path.join(ROOT, "paper_2504_07264_amd", "csrc", name)) as f:
            texts.append(f.read())
    return code_hash(texts)


def measured_traffic():
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line:
            k, v = line.strip().split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return int(float(fields["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def device_info(dev):
    """Name, architecture, CU count, HIP version and (best effort, from sysfs)
    the current and highest shader / memory clock levels of the device."""
    import torch

    props = torch.cuda.get_device_properties(dev)
    info = {"name": props.name, "arch": getattr(props, "gcnArchName", None), "cus": props.multi_processor_count,
            "hip": getattr(torch.version, "hip", None)}
    try:
        pci = "%04x:%02x:%02x.0" % (props.pci_domain_id, props.pci_bus_id, props.pci_device_id)
    except AttributeError:
        return info
    for key, fname in (("sclk", "pp_dpm_sclk"), ("mclk", "pp_dpm_mclk")):
        try:
            with open("/sys/bus/pci/devices/%s/%s" % (pci, fname)) as f:
                levels = [ln.split(":", 1)[1].strip() for ln in f.read().splitlines() if ":" in ln]
        except OSError:
            continue
        cur = [lv.rstrip("*").strip() for lv in levels if lv.endswith("*")]
        info[key] = {"current": cur[0] if cur else None, "max": levels[-1].rstrip("*").strip() if levels else None}
    return info


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline(xr, xi, gr, gi, budget_s: float = 2.0):
    """Time the CPU oracle (FP64 factorised transform, OpenMP over rows) on
    the same step: forward of x and adjoint of g over all rows, repeated
    until about ``budget_s`` seconds of wall time (times the thread count in
    CPU time) have passed."""
    import numpy as np

    import oracle

    threads = oracle.max_threads()
    a, b = xr.numpy().astype(np.float64), xi.numpy().astype(np.float64)
    c, d = gr.numpy().astype(np.float64), gi.numpy().astype(np.float64)
    rows = a.shape[0]
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.split_fft(a, b)
        # the adjoint through the plane swap: (C g_r - S g_i, S g_r + C g_i)
        oracle.split_fft(d, c)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            break
    nbytes = 2 * 16 * N * rows * reps
    # single thread, on a quarter of the rows
    sub = rows // 4
    t0 = time.perf_counter()
    oracle.split_fft(a[:sub], b[:sub], 1)
    oracle.split_fft(d[:sub], c[:sub], 1)
    dt1 = time.perf_counter() - t0
    # the direct definition (O1, O(N^2)) on 64 sampled rows, all threads
    idx = np.random.default_rng(0).choice(rows, 64, replace=False)
    t0 = time.perf_counter()
    oracle.dft_direct(a[idx], b[idx])
    dto1 = time.perf_counter() - t0
    return {
        "value": round(nbytes / dt / 1e9, 3),
        "unit": "GB/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": "all %d rows (N=%d), FP64 factorised forward + adjoint, %d repetitions in %.2f s wall"
                  % (rows, N, reps, dt),
        "host_cpu": host_cpu_model(),
        "os_cpu_count": os.cpu_count(),
        "single_thread": {"value": round(2 * 16 * N * sub / dt1 / 1e9, 3), "unit": "GB/s",
                          "sample": "%d rows forward + adjoint, one thread, %.2f s" % (sub, dt1)},
        "direct_o1": {"value": round(16 * N * 64 / dto1 / 1e9, 4), "unit": "GB/s",
                      "sample": "64 sampled rows, FP64 direct evaluation of eq. (5), %d threads, %.2f s"
                                % (threads, dto1)},
    }


COUNTER_WORKLOADS = ("n1024", "two_pass", "two_pass_fused", "n16384", "n8192", "l2_handover")


def counters_run(workload: str = "n1024", reps: int = 5):
    """Launch the kernels of one workload ``reps`` times, each launch followed
    by a plain device copy of 128 MiB read and 128 MiB written, for
    hardware-counter collection: the copy's FETCH_SIZE / WRITE_SIZE per
    dispatch calibrate the counters against known bytes.

    n1024     the forward length-1024 kernel, 16384 rows (the headline)
    two_pass  forward N=2^15 x 512 and N=2^16 x 256 (both passes each)
    two_pass_fused  the same through the fused two-pass schedule (one launch
              each, intermediate handed over through a per-XCD ring)
    n16384    forward N=2^14 x 1024 (single pass)
    n8192     forward N=2^13 x 2048 (single pass)
    l2_handover  the L2 hand-over model (every configuration once, with the
              copy kernel on the same bytes as its calibration)
    """
    if workload == "l2_handover":
        print(json.dumps({"counters_run": 1, "workload": workload, "result": l2_handover(reps=1)}), flush=True)
        return
    import torch

    from paper_2504_07264_amd import Plan, inputs

    dev = torch.device("cuda", 0)
    src = torch.randn(2, N * BATCH, device=dev)
    dst = torch.empty_like(src)
    if workload == "n1024":
        shapes = [(N, BATCH)]
    elif workload in ("two_pass", "two_pass_fused"):
        shapes = [(1 << 15, 512), (1 << 16, 256)]
    elif workload == "n16384":
        shapes = [(1 << 14, 1024)]
    elif workload == "n8192":
        shapes = [(1 << 13, 2048)]
    else:
        raise SystemExit("unknown counters workload %r (one of %s)" % (workload, ", ".join(COUNTER_WORKLOADS)))
    report = []
    for n, batch in shapes:
        if (n, batch) == (N, BATCH):
            xr, xi = inputs.draw(inputs.HEADLINE_N1024)
        else:
            xr, xi = inputs.draw_planes(n, batch, "normal", 30 + int(math.log2(n)))
        xr, xi = xr.to(dev), xi.to(dev)
        yr, yi = torch.empty_like(xr), torch.empty_like(xi)
        flags = fused_schedule_flags(int(math.log2(n))) if workload == "two_pass_fused" else 0
        with Plan(n, batch, flags, own_workspace=True) as plan:
            for _ in range(reps):
                plan.exec(xr, xi, yr, yi)
                torch.cuda.synchronize()
                dst.copy_(src)
                torch.cuda.synchronize()
            report.append({"n": n, "batch": batch, "schedule": plan.describe()})
        del xr, xi, yr, yi
    print(json.dumps({"counters_run": reps, "workload": workload, "plans": report,
                      "copy_bytes_each_way": src.numel() * 4}), flush=True)


# executed 16x16x32 matrix-core instructions per length-256 transform (two
# 16-point stages x two output planes x products per split mode)
MFMA_PER_TRANSFORM = {"bf16x2": 2 * 2 * 3, "fp16x2": 2 * 2 * 3, "bf16x3": 2 * 2 * 6}
MFMA_FLOPS = 2 * 16 * 16 * 32
MFMA_PEAK_TFLOPS = 2500.0  # dense bf16 / fp16
ERROR_ROWS = 512  # sampled rows for the error of each precision mode


def tol(n: int) -> float:
    """The FP32 accuracy bound: relative L2 error per transform <= 2e-7 log2 N + 1e-7."""
    return 2e-7 * math.log2(n) + 1e-7


def rel_error_fp64(xr, xi, yr, yi, rows):
    """Relative L2 error per row (both planes together) of (yr, yi) against
    numpy's FP64 FFT of the same FP32 inputs, over the sampled rows: the
    forward DFT of eq. (1), whose real and imaginary parts are eq. (5)."""
    import numpy as np

    x = xr[rows].astype(np.float64) + 1j * xi[rows].astype(np.float64)
    ref = np.fft.fft(x, axis=1)
    got = yr[rows].astype(np.float64) + 1j * yi[rows].astype(np.float64)
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    return {"max": float("%.3g" % err.max()), "median": float("%.3g" % np.median(err)), "rows": int(len(rows))}


def mfma_vs_fp32(iters: int = MIN_ITERS, sets: int = 4):
    """Forward N=256 x 65536 (uniform[-1, 1], seed 3) in FP32 and in the three
    matrix-core split-precision modes: launch time (median, p10, p90 of HIP
    event intervals) and the relative L2 error of sampled rows against an FP64
    FFT (outside the timed region)."""
    import numpy as np
    import torch

    from paper_2504_07264_amd import Plan, binding, inputs

    w = inputs.PREC_N256
    xr, xi = inputs.draw(w)
    dev = torch.device("cuda", 0)
    bufs = [(xr.to(dev), xi.to(dev), torch.empty_like(xr, device=dev), torch.empty_like(xi, device=dev))
            for _ in range(sets)]
    stream = torch.cuda.current_stream(dev)
    rows = np.sort(np.random.default_rng(7).choice(w.batch, ERROR_ROWS, replace=False))
    xr_np, xi_np = xr.numpy(), xi.numpy()
    out = {"workload": "split_fft_n256_b65536_uniform forward", "n": w.n, "batch": w.batch,
           "error": "relative L2 per transform against an FP64 FFT, %d sampled rows; FP32 bound %.2e"
                    % (ERROR_ROWS, tol(w.n))}
    nbytes = 16 * w.n * w.batch
    for name in ("fp32", "bf16x2", "fp16x2", "bf16x3"):
        with Plan(w.n, w.batch, binding.PRECISIONS[name]) as plan:
            for k in range(5):
                plan.exec(*bufs[k % sets])
            us = stats_us(event_times(lambda k: plan.exec(*bufs[k % sets]), iters, stream))
            a, b, c, d = bufs[0]
            plan.exec(a, b, c, d)
            torch.cuda.synchronize()
            err = rel_error_fp64(xr_np, xi_np, c.cpu().numpy(), d.cpu().numpy(), rows)
            err["within_fp32_bound"] = err["max"] <= tol(w.n)
            rec = {"us": us, "GBps": round(nbytes / us["median"] / 1e3, 1), "schedule": plan.describe(),
                   "rel_l2_error": err}
            if name in MFMA_PER_TRANSFORM:
                tflops = MFMA_PER_TRANSFORM[name] * MFMA_FLOPS * w.batch / us["median"] / 1e6
                rec["mfma_tflops"] = round(tflops, 1)
                rec["mfma_utilisation"] = round(tflops / MFMA_PEAK_TFLOPS, 4)
            out[name] = rec
    for name in ("bf16x2", "fp16x2", "bf16x3"):
        out[name]["time_vs_fp32"] = round(out[name]["us"]["median"] / out["fp32"]["us"]["median"], 3)
    return out


def bench_lib():
    """The benchmark's HBM streaming kernels (libsplitdft_bench.so)."""
    import ctypes

    from paper_2504_07264_amd import build

    if not os.path.exists(build.BENCH_LIB_PATH):
        raise RuntimeError("libsplitdft_bench.so is missing; build with `python -m paper_2504_07264_amd.build`")
    L = ctypes.CDLL(build.BENCH_LIB_PATH)
    L.splitdft_bench_stream.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p]
    L.splitdft_bench_stream.restype = ctypes.c_int
    L.splitdft_bench_l2_control_bytes.argtypes = []
    L.splitdft_bench_l2_control_bytes.restype = ctypes.c_int64
    L.splitdft_bench_l2_handover.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int] * 6 + [ctypes.c_void_p]
    L.splitdft_bench_l2_handover.restype = ctypes.c_int
    return L


# (tiles per transform, ring slots per XCD, self mode, workgroups)
L2_CONFIGS = ((4, 4, 0, 512), (4, 8, 0, 512), (4, 12, 0, 512), (4, 8, 1, 512), (4, 2, 1, 512),
              (8, 4, 0, 512), (8, 8, 0, 512), (8, 8, 1, 512))


def l2_handover(reps: int = 3, per_xcd: int = 128):
    """The L2 hand-over model of a two-pass transform (csrc/bench_l2.hip):
    transforms of 4 tiles (256 KiB, the size of a 2^15 transform) and 8 tiles
    (512 KiB, 2^16), 128 per XCD, every pass-2 tile gathering from every
    pass-1 tile through a ring of slots per XCD, against a 16-byte copy of the
    same bytes.  Each launch is timed alone (its control block is cleared
    before it) and its output checked against the permuted input."""
    import torch

    L = bench_lib()
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    s = stream.cuda_stream
    cb = L.splitdft_bench_l2_control_bytes()
    ctl = torch.zeros((cb + 3) // 4, dtype=torch.int32, device=dev)
    gen = torch.Generator(device=dev).manual_seed(11)
    sink = torch.zeros(1, device=dev)
    out = {"model": "pass-1 tiles of 64 KiB handed to pass-2 tiles through a per-XCD ring in L2; no arithmetic",
           "transforms_per_xcd": per_xcd}

    def event_us(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        rc = fn()
        b.record(stream)
        torch.cuda.synchronize()
        if rc != 0:
            raise RuntimeError("launch failed: hipError %d" % rc)
        return a.elapsed_time(b) * 1e3

    for tiles in sorted({c[0] for c in L2_CONFIGS}):
        tf = tiles * 16384
        n = 8 * per_xcd * tf
        x = torch.randn(n, device=dev, generator=gen)
        y = torch.empty_like(x)
        moved = 2 * n * 4
        copy = [event_us(lambda: L.splitdft_bench_stream(x.data_ptr(), y.data_ptr(), n, 0, sink.data_ptr(), s))
                for _ in range(reps + 1)][1:]
        rec = {"bytes_in": n * 4, "copy_us": round(sorted(copy)[len(copy) // 2], 1)}
        rec["copy_GBps"] = round(moved / rec["copy_us"] / 1e3)
        want = x.view(-1, tiles, tiles, 16384 // tiles).transpose(1, 2)
        for (t, slots, self_mode, grid) in L2_CONFIGS:
            if t != tiles:
                continue
            ring = torch.empty(8 * slots * tf, device=dev)
            times, correct, timeouts = [], True, 0
            for _ in range(reps):
                ctl.zero_()
                y.zero_()
                times.append(event_us(lambda: L.splitdft_bench_l2_handover(
                    x.data_ptr(), y.data_ptr(), ring.data_ptr(), ctl.data_ptr(), grid, per_xcd, tiles, slots,
                    self_mode, 1 << 16, s)))
                tail = ctl[-3:].tolist()
                timeouts += tail[0] + tail[1]
                correct &= bool(torch.equal(y, x) if self_mode else torch.equal(y.view_as(want), want))
            us = sorted(times)[len(times) // 2]
            rec["slots%d%s" % (slots, "_self" if self_mode else "")] = {
                "ring_MiB_per_xcd": slots * tf * 4 / 2**20, "workgroups": grid, "us": round(us, 1),
                "GBps_in_out": round(moved / us / 1e3), "vs_copy": round(us / rec["copy_us"], 2),
                "correct": correct, "timeouts": timeouts}
            del ring
        out["tiles%d" % tiles] = rec
        del x, y
    return out


def copy_ceiling(iters: int = MIN_ITERS, sets: int = 4):
    """The achievable HBM rate for the headline kernel's bytes (128 MiB read
    and 128 MiB written per launch): 16-byte nontemporal streaming kernels
    (copy with four and with one vector per thread, the planar copy of two
    64 MiB planes into two as the transform streams them, read-only,
    write-only), torch's copy_ and the HIP runtime's device-to-device memcpy,
    each timed as the median of HIP-event intervals."""
    import ctypes

    import torch

    dev = torch.device("cuda", 0)
    src = [torch.randn(2 * N * BATCH, device=dev) for _ in range(sets)]
    dst = [torch.empty_like(src[0]) for _ in range(sets)]
    sink = torch.zeros(1, device=dev)
    nfl = src[0].numel()
    nbytes = nfl * 4
    stream = torch.cuda.current_stream(dev)
    s = stream.cuda_stream
    out = {"bytes_each_way": nbytes}

    def timed(fn, moved):
        for k in range(5):
            fn(k)
        us = stats_us(event_times(fn, iters, stream))
        return {"us": us, "GBps": round(moved / us["median"] / 1e3, 1)}

    L = bench_lib()

    def probe(mode):
        def fn(k):
            rc = L.splitdft_bench_stream(src[k % sets].data_ptr(), dst[k % sets].data_ptr(), nfl, mode,
                                         sink.data_ptr(), s)
            if rc != 0:
                raise RuntimeError("streaming kernel launch failed: hipError %d" % rc)
        return fn

    out["nt_float4_copy"] = timed(probe(0), 2 * nbytes)
    out["nt_float4_copy_one_vector_per_thread"] = timed(probe(4), 2 * nbytes)
    out["nt_float4_planar_copy"] = timed(probe(3), 2 * nbytes)
    out["nt_float4_read"] = timed(probe(1), nbytes)
    out["nt_float4_write"] = timed(probe(2), nbytes)
    out["torch_copy"] = timed(lambda k: dst[k % sets].copy_(src[k % sets]), 2 * nbytes)
    try:
        hip = ctypes.CDLL("libamdhip64.so", mode=ctypes.RTLD_GLOBAL)
        hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                       ctypes.c_void_p]
        hip.hipMemcpyAsync.restype = ctypes.c_int
        d2d = 3  # hipMemcpyDeviceToDevice
        out["hip_memcpy_d2d"] = timed(lambda k: hip.hipMemcpyAsync(dst[k % sets].data_ptr(),
                                                                   src[k % sets].data_ptr(), nbytes, d2d, s),
                                      2 * nbytes)
    except OSError:
        out["hip_memcpy_d2d"] = None
    return out


def dif_n1024(iters: int = MIN_ITERS, sets: int = 4, rounds: int = 5):
    """Forward N=1024 x 16384 through the decimation-in-frequency schedule
    (eq. 9), same inputs as the headline: launch time statistics, timed in
    rounds interleaved with the default (DIT) schedule on the same buffers, so
    that both see the same clocks."""
    import torch

    from paper_2504_07264_amd import Plan, binding, inputs

    w = inputs.HEADLINE_N1024
    xr, xi = inputs.draw(w)
    dev = torch.device("cuda", 0)
    bufs = [(xr.to(dev), xi.to(dev), torch.empty_like(xr, device=dev), torch.empty_like(xi, device=dev))
            for _ in range(sets)]
    stream = torch.cuda.current_stream(dev)
    with Plan(w.n, w.batch, binding.DIF) as plan, Plan(w.n, w.batch) as dit:
        for k in range(5):
            plan.exec(*bufs[k % sets])
            dit.exec(*bufs[k % sets])
        t_dif, t_dit = [], []
        for _ in range(rounds):
            t_dif += event_times(lambda k: plan.exec(*bufs[k % sets]), iters // rounds, stream)
            t_dit += event_times(lambda k: dit.exec(*bufs[k % sets]), iters // rounds, stream)
        us, us_dit = stats_us(t_dif), stats_us(t_dit)
        return {"workload": "split_fft_n1024_b16384 forward, decimation in frequency (eq. 9)", "us": us,
                "GBps": round(16 * w.n * w.batch / us["median"] / 1e3, 1), "schedule": plan.describe(),
                "dit_same_rounds_us": us_dit, "time_vs_dit": round(us["median"] / us_dit["median"], 3),
                "from": "%d rounds, each %d groups of 4 launches of the DIF and then of the DIT schedule"
                        % (rounds, iters // rounds)}


def fused_schedule_flags(m: int):
    """Plan flags of the compiled fused two-pass schedule of length 2^m, or None."""
    from paper_2504_07264_amd import Plan, SplitDFTError, variant_flag

    k = 0
    while True:
        try:
            with Plan(1 << m, 1, variant_flag(k)) as p:
                if "fused" in p.describe():
                    return variant_flag(k)
        except SplitDFTError:
            return None
        k += 1


def two_pass_large(iters: int = MIN_ITERS, sets: int = 4):
    """Forward N=2^15 x 512 and N=2^16 x 256 (2^24 points each): launch time
    statistics over rotating buffer sets, for the default schedule and the
    fused two-pass schedule (both passes in one launch through a per-XCD ring)."""
    import torch

    from paper_2504_07264_amd import Plan, inputs

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    res = {}
    for m in (15, 16):
        n, batch = 1 << m, (1 << 24) >> m
        xr, xi = inputs.draw_planes(n, batch, "normal", 30 + m)
        bufs = [(xr.to(dev), xi.to(dev), torch.empty(batch, n, device=dev), torch.empty(batch, n, device=dev))
                for _ in range(sets)]
        for name, flags in (("default", 0), ("fused", fused_schedule_flags(m))):
            if flags is None:
                continue
            with Plan(n, batch, flags, own_workspace=True) as plan:
                for k in range(3):
                    plan.exec(*bufs[k % sets])
                us = stats_us(event_times(lambda k: plan.exec(*bufs[k % sets]), iters, stream))
                rec = {"us": us, "GBps": round(16 * n * batch / us["median"] / 1e3, 1), "schedule": plan.describe()}
            if name == "default":
                res["n%d_b%d" % (n, batch)] = rec
            else:
                res["n%d_b%d" % (n, batch)]["fused"] = rec
        del bufs
    res["note"] = "forward only; GB/s counts 16 B per point, the two passes move twice that"
    return res


def single_pass_large(iters: int = MIN_ITERS, sets: int = 4):
    """Forward N=2^13 x 2048 and N=2^14 x 1024 (2^24 points each, the longest
    single-pass lengths): launch time statistics over rotating buffer sets."""
    import torch

    from paper_2504_07264_amd import Plan, inputs

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    res = {}
    for m in (13, 14):
        n, batch = 1 << m, (1 << 24) >> m
        xr, xi = inputs.draw_planes(n, batch, "normal", 30 + m)
        bufs = [(xr.to(dev), xi.to(dev), torch.empty(batch, n, device=dev), torch.empty(batch, n, device=dev))
                for _ in range(sets)]
        with Plan(n, batch) as plan:
            for k in range(3):
                plan.exec(*bufs[k % sets])
            us = stats_us(event_times(lambda k: plan.exec(*bufs[k % sets]), iters, stream))
            res["n%d_b%d" % (n, batch)] = {"us": us, "GBps": round(16 * n * batch / us["median"] / 1e3, 1),
                                          "frac_of_8TBps": round(16 * n * batch / us["median"] / 1e3 / HBM_PEAK_GBS, 4),
                                          "schedule": plan.describe()}
        del bufs
    return res


def grad_n4096(iters: int = MIN_ITERS, sets: int = 3):
    """Forward + adjoint (the autograd step's two kernels) at N=4096 x 4096,
    as two launches and as one fused launch."""
    import torch

    from paper_2504_07264_amd import Plan, inputs

    w = inputs.GRAD_N4096
    xr, xi, wr, wi = inputs.draw(w)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    bufs = [tuple(t.to(dev) for t in (xr, xi, wr, wi)) + tuple(torch.empty(w.batch, w.n, device=dev)
                                                             for _ in range(4)) for _ in range(sets)]
    with Plan(w.n, w.batch) as plan:
        def step(k):
            a, b, c, d, yr, yi, gr, gi = bufs[k % sets]
            plan.exec(a, b, yr, yi)
            plan.adjoint(c, d, gr, gi)

        def fused(k):
            a, b, c, d, yr, yi, gr, gi = bufs[k % sets]
            plan.exec_adjoint(a, b, c, d, out=(yr, yi, gr, gi))

        for k in range(3):
            step(k)
            fused(k)
        two = stats_us(event_times(step, iters, stream))
        one = stats_us(event_times(fused, iters, stream))
        nbytes = 2 * 16 * w.n * w.batch
        return {"workload": "split_fft_n4096_b4096 forward + adjoint", "schedule": plan.describe(),
                "two_launches_us": two, "two_launches_GBps": round(nbytes / two["median"] / 1e3, 1),
                "fused_us": one, "fused_GBps": round(nbytes / one["median"] / 1e3, 1)}


def ragged_grouped(iters: int = MIN_ITERS // 2):
    """20000 transforms of lengths 2^4..2^16, forward + adjoint, replayed from
    a captured HIP graph: the default schedule and the autotuner's choice
    (grouped-kernel build, workgroups per CU, per-length threshold), timed on
    this device just before."""
    import torch

    from paper_2504_07264_amd import ManyPlan, inputs, tune

    lengths, planes = inputs.draw_ragged(inputs.RAGGED_COUNT, inputs.RAGGED_KMIN, inputs.RAGGED_KMAX,
                                         inputs.RAGGED_SEED)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    total = int(lengths.sum())
    xr, xi, gr, gi = [t.to(dev) for t in planes]
    del planes
    out = [torch.empty(total, device=dev) for _ in range(4)]
    lens = [int(v) for v in lengths.tolist()]
    t0 = time.perf_counter()
    best, timings = tune.tune_many(lens, iters=5)
    tune_s = time.perf_counter() - t0
    res = {"workload": "20000 transforms, lengths 2^4..2^16 (k uniform, seed 4), forward + adjoint, one graph",
           "points": total, "tune_s": round(tune_s, 2),
           "tune_candidates_us": {str(k): v["us"] for k, v in timings.items()}}
    for name, flags in (("default", 0), ("tuned", best)):
        with ManyPlan(lens, flags) as plan:
            g = plan.graph(xr, xi, out[0], out[1], gr, gi, out[2], out[3])
            for _ in range(3):
                g.launch()
            us = stats_us(event_times(lambda k: g.launch(), iters, stream, group=1))
            info = plan.info()
            g.close()
        res[name] = {"flags": int(flags), "ms_per_launch": round(us["median"] / 1e3, 4), "us": us,
                     "GBps": round(32 * total / us["median"] / 1e3, 1), "workgroups": info["workgroups"],
                     "items": info["items"]}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mfma", action="store_true", help="skip the matrix-core comparison")
    ap.add_argument("--no-extra", action="store_true", help="skip the side reports")
    ap.add_argument("--no-tune", action="store_true", help="use the default schedule for the headline")
    ap.add_argument("--l2-handover", action="store_true",
                    help="only the L2 hand-over model of a two-pass transform (one JSON line)")
    ap.add_argument("--counters", nargs="?", const="n1024", default=None, choices=COUNTER_WORKLOADS,
                    help="only launch one workload's kernels and a calibration copy (for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only; the transforms are independent per row, "
              "so N GPUs would each run the same kernel on batch/N rows with no communication. "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.counters:
        counters_run(args.counters)
        return
    if args.l2_handover:
        print(json.dumps({"l2_handover": l2_handover()}), flush=True)
        return

    import torch

    from paper_2504_07264_amd import Plan, inputs, tune

    assert torch.cuda.is_available(), "no GPU visible"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    w = inputs.HEADLINE_N1024
    xr, xi = inputs.draw(w)
    gr, gi = inputs.draw_planes(N, BATCH, "normal", w.seed + 100)

    # the autotuner's schedule for this length and batch, timed here
    tuned = None
    flags = 0
    if not args.no_tune:
        t0 = time.perf_counter()
        flags, timings = tune.tune_length(N, BATCH, iters=20)
        tuned = {"flags": int(flags), "tune_s": round(time.perf_counter() - t0, 2),
                 "candidates_us": {timings[f]["schedule"]: timings[f]["us"] for f in timings},
                 "finalists_us": {timings[f]["schedule"]: timings[f]["final_us"] for f in timings
                                  if "final_us" in timings[f]}}
        torch.cuda.empty_cache()

    sets = []
    for k in range(ROTATE_SETS):
        s = {
            "xr": xr.to(dev), "xi": xi.to(dev), "gr": gr.to(dev), "gi": gi.to(dev),
            "yr": torch.empty(BATCH, N, device=dev), "yi": torch.empty(BATCH, N, device=dev),
            "hr": torch.empty(BATCH, N, device=dev), "hi": torch.empty(BATCH, N, device=dev),
        }
        sets.append(s)
    plan = Plan(N, BATCH, flags)
    stream = torch.cuda.current_stream(dev)

    def step(k):
        s = sets[k % ROTATE_SETS]
        plan.exec(s["xr"], s["xi"], s["yr"], s["yi"])
        plan.adjoint(s["gr"], s["gi"], s["hr"], s["hi"])

    def launch(k):
        # launch k of the step sequence: forward for even k, adjoint for odd
        s = sets[(k // 2) % ROTATE_SETS]
        if k % 2 == 0:
            plan.exec(s["xr"], s["xi"], s["yr"], s["yi"])
        else:
            plan.adjoint(s["gr"], s["gi"], s["hr"], s["hi"])

    def fused_step(k):
        s = sets[k % ROTATE_SETS]
        plan.exec_adjoint(s["xr"], s["xi"], s["gr"], s["gi"], out=(s["yr"], s["yi"], s["hr"], s["hi"]))

    # Untimed: the GPU raises its clocks over the first few hundred
    # milliseconds of sustained work, so run steps for at least PREWARM_S
    # seconds before the W warmup steps and the timed region.
    t_pre = time.perf_counter()
    k = 0
    while time.perf_counter() - t_pre < PREWARM_S:
        for _ in range(20):
            step(k)
            k += 1
        torch.cuda.synchronize()
    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()

    # The timed region holds only the kernel's launches (forward and adjoint
    # run the same kernel); one event pair on the launch stream at its two
    # ends gives the mean time per launch (an event pair around each launch
    # would idle the stream between launches and add its dispatch time).
    e_start, e_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_start.record(stream)
    for k in range(args.steps):
        step(k)
    e_end.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    launches = 2 * args.steps
    launch_ms = e_start.elapsed_time(e_end) / launches
    step_bytes = 2 * 16 * N * BATCH
    launch_bytes = 16 * N * BATCH
    gbs = step_bytes / (ms_per_step * 1e-3) / 1e9
    flops = 2 * 5 * N * math.log2(N) * BATCH
    achieved = launch_bytes / (launch_ms * 1e-3) / 1e9
    traffic = measured_traffic()

    # a second timed region for the distribution: an event after every launch
    per_launch = stats_us(event_times(launch, MIN_ITERS, stream, group=10))
    two_launch_steps = stats_us(event_times(step, MIN_ITERS, stream, group=5))
    fused_steps = stats_us(event_times(fused_step, MIN_ITERS, stream, group=5))

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
            "schedule": plan.describe(),
            "schedule_from": "autotuner" if tuned else "default",
            "rotating_buffer_sets": ROTATE_SETS,
        },
        "gflops_5nlogn": round(flops / (ms_per_step * 1e-3) / 1e9, 1),
        "kernel_us_per_launch": {"mean": round(launch_ms * 1e3, 2), "launches": launches,
                                 "from": "HIP events at both ends of the timed region, launch stream",
                                 "distribution": per_launch,
                                 "distribution_from": "a second region: %d groups of 10 back-to-back launches, "
                                                      "one HIP event after each group" % MIN_ITERS},
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
        },
        "step_us": {"two_launches": two_launch_steps, "fused_one_launch": fused_steps,
                    "fused_GBps": round(step_bytes / fused_steps["median"] / 1e3, 1),
                    "from": "%d groups of 5 back-to-back steps, one HIP event after each group" % MIN_ITERS},
        "tuned": tuned,
        "device": device_info(dev),
    }
    del sets
    plan.close()
    torch.cuda.empty_cache()
    if not args.no_mfma:
        out["mfma_vs_fp32"] = mfma_vs_fp32()
        torch.cuda.empty_cache()
    if not args.no_extra:
        out["copy_ceiling"] = copy_ceiling()
        torch.cuda.empty_cache()
        out["dif_n1024"] = dif_n1024()
        torch.cuda.empty_cache()
        out["grad_n4096"] = grad_n4096()
        torch.cuda.empty_cache()
        out["single_pass_large"] = single_pass_large()
        torch.cuda.empty_cache()
        out["two_pass_large"] = two_pass_large()
        torch.cuda.empty_cache()
        out["ragged_grouped"] = ragged_grouped()
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(xr, xi, gr, gi)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
