"""Autotuner for kernel schedules.

Every length has several compiled schedules (elements per thread, transforms
per workgroup, LDS exchange form, 16-byte staging, two-pass tiling), and the
grouped kernel has two builds and a workgroups-per-CU setting.  The tuner
times each candidate on the current device with HIP events over rotating
buffers and records the fastest in a JSON cache keyed by the device (name,
CU count) and the library build; plans created with ``schedule="tuned"``
(``tuned_plan``) look the choice up there.

Command line:
    python -m paper_2504_07264_amd.tune --lengths 16,256,1024,4096,65536 \\
        --points 16777216 [--ragged 20000] [--cache PATH]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import threading

import torch

from . import binding
from .binding import ManyPlan, Plan, SplitDFTError, many_flags, variant_flag

_cache_lock = threading.Lock()


def cache_path() -> str:
    p = os.environ.get("SPLIT_DFT_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "splitdft", "tune.json")


def device_key(device=None) -> str:
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    props = torch.cuda.get_device_properties(dev)
    with open(binding.LIB_PATH, "rb") as f:
        lib_hash = hashlib.sha256(f.read()).hexdigest()[:16]
    arch = getattr(props, "gcnArchName", "gfx")
    return "%s|%s|cu%d|lib%s" % (props.name, arch, props.multi_processor_count, lib_hash)


def load_cache(path=None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(data: dict, path=None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(fn, iters: int, warmup: int = 3, group: int = 4) -> float:
    """Median microseconds per call of fn(k) over ``iters`` groups of
    ``group`` back-to-back calls, one HIP event after each group (so that
    consecutive kernels overlap as they do in use)."""
    for k in range(warmup):
        fn(k)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(iters + 1)]
    ev[0].record()
    for j in range(iters):
        for k in range(j * group, (j + 1) * group):
            fn(k)
        ev[j + 1].record()
    torch.cuda.synchronize()
    t = sorted(ev[j].elapsed_time(ev[j + 1]) / group for j in range(iters))
    return t[len(t) // 2] * 1e3


def schedules(n: int, dif: bool = False):
    """Flag values of every compiled FP32 schedule for length n (of the
    decimation-in-frequency factorisation when dif)."""
    base = binding.DIF if dif else 0
    out = []
    k = 0
    while True:
        try:
            with Plan(n, 1, base | variant_flag(k)):
                pass
        except SplitDFTError:
            return out
        out.append(base | variant_flag(k))
        k += 1


def tune_length(n: int, batch: int, iters: int = 20, sets: int = 3, dif: bool = False, finalists: int = 4,
                rounds: int = 5):
    """Time every compiled schedule for (n, batch); returns (best flags,
    timings).  A first pass times each schedule once; the fastest
    ``finalists`` and the default schedule are then timed again in
    ``rounds`` interleaved rounds (so that drift of the device's clocks hits
    them alike), and the best median over the rounds wins."""
    dev = torch.device("cuda", torch.cuda.current_device())
    bufs = [tuple(torch.randn(batch, n, device=dev) for _ in range(4)) for _ in range(sets)]
    timings = {}
    for flags in schedules(n, dif):
        with Plan(n, batch, flags) as p:
            us = _time(lambda k: p.exec(*bufs[k % sets]), iters, group=8)
            timings[flags] = {"us": round(us, 2), "schedule": p.describe()}
    default = binding.DIF if dif else 0
    with Plan(n, batch, default) as p:
        desc = p.describe()
    # the default schedule's flag value among the compiled ones
    default_flags = next((f for f in timings if timings[f]["schedule"] == desc), None)
    top = sorted(timings, key=lambda f: timings[f]["us"])[:finalists]
    if default_flags is not None and default_flags not in top:
        top.append(default_flags)
    plans = {f: Plan(n, batch, f) for f in top}
    try:
        rounds_us = {f: [] for f in top}
        for _ in range(rounds):
            for f in top:
                p = plans[f]
                rounds_us[f].append(_time(lambda k: p.exec(*bufs[k % sets]), iters, group=8))
    finally:
        for p in plans.values():
            p.close()
    for f in top:
        t = sorted(rounds_us[f])
        timings[f]["final_us"] = round(t[len(t) // 2], 2)
    best = min(top, key=lambda f: timings[f]["final_us"])
    return best, timings


def tune_many(lengths, iters: int = 5):
    """Time the grouped kernel builds, workgroups-per-CU settings and the
    split between per-length launches and the persistent kernel (threshold, or
    every length in the persistent kernel) on a forward + adjoint graph of the
    ragged batch; returns (best flags, timings)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    total = int(sum(int(n) for n in lengths))
    planes = [torch.randn(total, device=dev) for _ in range(8)]
    candidates = [(b, w, False, 0) for b in range(2) for w in (0, 1)]
    candidates += [(0, 0, False, t) for t in (11, 13, 14)]
    candidates += [(b, w, True, 0) for b in range(2) for w in (0, 1)]
    timings = {}
    for build, wpc, one_kernel, split in candidates:
        flags = many_flags(build, wpc, one_kernel, split)
        with ManyPlan(lengths, flags) as p:
            g = p.graph(*planes)
            us = _time(lambda k: g.launch(), iters, warmup=1, group=1)
            g.close()
            timings[flags] = {"us": round(us, 1), "workgroups": p.info()["workgroups"], "one_kernel": one_kernel,
                              "per_length_from": split}
    best = min(timings, key=lambda f: timings[f]["us"])
    return best, timings


def ragged_key(lengths) -> str:
    h = hashlib.sha256(torch.as_tensor(list(lengths), dtype=torch.int64).numpy().tobytes()).hexdigest()[:16]
    return "ragged:%d:%s" % (len(lengths), h)


def record(key: str, flags: int, timings: dict, path=None) -> None:
    with _cache_lock:
        data = load_cache(path)
        dk = device_key()
        data.setdefault(dk, {})[key] = {"flags": int(flags),
                                        "timings": {str(k): v for k, v in timings.items()}}
        save_cache(data, path)


def lookup(key: str, path=None):
    """Tuned flags for ``key`` on this device and library build, or None."""
    data = load_cache(path)
    entry = data.get(device_key(), {}).get(key)
    return None if entry is None else int(entry["flags"])


def length_key(n: int, batch: int, dif: bool = False) -> str:
    return "%s:%d:%d" % ("length-dif" if dif else "length", n, batch)


def tuned_plan(n: int, batch: int, path=None, dif: bool = False) -> Plan:
    """A plan with the cached fastest schedule (default schedule if untuned)."""
    flags = lookup(length_key(n, batch, dif), path)
    return Plan(n, batch, (binding.DIF if dif else 0) if flags is None else flags)


def tuned_many_plan(lengths, path=None) -> ManyPlan:
    flags = lookup(ragged_key(lengths), path)
    return ManyPlan(lengths, 0 if flags is None else flags)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--lengths", default="16,256,1024,4096,65536")
    ap.add_argument("--points", type=int, default=1 << 24, help="points per length (batch = points / n)")
    ap.add_argument("--ragged", type=int, default=0, help="also tune the ragged workload of this many transforms")
    ap.add_argument("--cache", default=None)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--dif", action="store_true", help="tune the decimation-in-frequency schedules")
    ap.add_argument("--all", action="store_true",
                    help="print every schedule's time (first pass and, for the finalists, the rounds' median)")
    args = ap.parse_args(argv)
    for n in [int(x) for x in args.lengths.split(",") if x]:
        batch = max(1, args.points // n)
        if args.dif and not schedules(n, True):
            continue
        best, t = tune_length(n, batch, args.iters, dif=args.dif)
        record(length_key(n, batch, args.dif), best, t, args.cache)
        line = {"n": n, "batch": batch, "dif": args.dif, "best_flags": best, "best": t[best], "candidates": len(t)}
        if args.all:
            line["schedules"] = [dict(t[f], flags=f) for f in sorted(t)]
        print(json.dumps(line), flush=True)
    if args.ragged:
        from . import inputs

        _, lengths = inputs.ragged_lengths(args.ragged, inputs.RAGGED_KMIN, inputs.RAGGED_KMAX, inputs.RAGGED_SEED)
        lengths = [int(v) for v in lengths.tolist()]
        best, t = tune_many(lengths)
        record(ragged_key(lengths), best, t, args.cache)
        print(json.dumps({"ragged": args.ragged, "best_flags": best, "timings": t}), flush=True)


if __name__ == "__main__":
    main()
