"""Benchmark: keys/s of the exact-splitting samplesort on one MI355X.

One step = one complete sort (every step of the method: tile sort, splitter
search, partitioning, multiway merges) of N = 2^28 int64 keys already resident
in HBM, into a separate output array.  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--dist uniform]
                    [--log2n 28] [--all-dists] [--no-cpu-baseline]

The roofline object reports the dominant kernel: its algorithmic HBM bytes per
launch (every key read once and written once: 16 bytes per int64 key) divided
by its mean launch time, timed with HIP events recorded by the library on the
stream the kernel runs on, during the timed steps.  The CPU baseline is the
sequential oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GKeys/s and % HBM roofline at N=2^28 int64; batched p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def generators():
    import workloads as W

    return {
        "uniform": lambda n: W.uniform_i64(n, seed=2),
        "mod1000": lambda n: W.mod1000_i64(n, seed=3),
        "sorted": lambda n: W.sorted_i64(n),
        "reverse": lambda n: W.reverse_i64(n),
        "swapped1pct": lambda n: W.swapped_i64(n, seed=6),
    }


def time_sort(pss, torch, keys_dev, out, ws, steps: int, warmup: int, profile: bool):
    for _ in range(warmup):
        pss.sort(keys_dev, out=out, workspace=ws)
    torch.cuda.synchronize()
    if profile:
        pss.profile(True)
        pss.profile_read()  # drop anything recorded so far
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        pss.sort(keys_dev, out=out, workspace=ws)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernels = None
    if profile:
        kernels = pss.profile_read()
        pss.profile(False)
    return wall, ev0.elapsed_time(ev1) / 1e3, kernels


def cpu_baseline(log2n: int = 25):
    """The oracle as it stands (sequential C, one thread) on a bounded sample
    of the same workload: 2^log2n uniform int64 keys, n_B = n_P = 48."""
    import oracle
    import workloads as W

    n = 1 << log2n
    keys = W.uniform_i64(n, seed=2)
    oracle.build()
    t0 = time.perf_counter()
    oracle.pses(keys, 48, 48)
    dt = time.perf_counter() - t0
    return {"value": n / dt / 1e9, "unit": "GKeys/s", "cores": 1, "kind": "oracle",
            "sample": f"2^{log2n} uniform int64 keys (seed 2), n_B = n_P = 48, single thread, "
                      f"{dt:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--dist", default="uniform", choices=list(generators()))
    ap.add_argument("--all-dists", action="store_true",
                    help="also time the other four int64 distributions")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-only", action="store_true",
                    help="only time a plain device-to-device copy of the keys (bandwidth and "
                         "counter calibration), print its line and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU path is a design, not part of this build)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd import _lib

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    _lib.load()  # fail loudly when the HIP library is missing

    n = 1 << args.log2n
    gens = generators()
    keys = gens[args.dist](n)
    keys_dev = torch.from_numpy(keys).cuda()
    out = torch.empty_like(keys_dev)
    ws = torch.empty(_lib.workspace_bytes(_lib.I64, _lib.VAL_NONE, n), dtype=torch.uint8,
                     device="cuda")
    plan = _lib.plan(_lib.I64, _lib.VAL_NONE, n)

    # plain copy of the same bytes: the achievable read+write bandwidth here
    for _ in range(2):
        out.copy_(keys_dev)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        out.copy_(keys_dev)
    torch.cuda.synchronize()
    copy_s = (time.perf_counter() - t0) / reps
    copy_gbs = 2 * 8 * n / copy_s / 1e9
    if args.copy_only:
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n,
                          "copy_ms": round(copy_s * 1e3, 4), "copy_gbs": round(copy_gbs, 1)}))
        return 0

    wall, ev_s, kernels = time_sort(pss, torch, keys_dev, out, ws, args.steps, args.warmup,
                                    profile=True)
    assert pss.device_check(0) == 0
    ms_per_step = wall / args.steps * 1e3
    gkeys = n / (wall / args.steps) / 1e9

    # dominant kernel family by total time
    dom_name, dom = max(kernels.items(), key=lambda kv: kv[1]["ms"])
    per_launch_ms = dom["ms"] / dom["launches"]
    per_launch_bytes = dom["bytes"] / dom["launches"]
    achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
    roofline = {
        "bound": "hbm",
        "kernel": dom_name,
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None,
        "bytes_per_launch": per_launch_bytes,
        "mean_launch_ms": round(per_launch_ms, 4),
    }
    # whole-sort view against the method's 2 data passes (16 B/key each)
    algo_bytes = 2 * 2 * 8 * n
    line = {
        "metric": METRIC,
        "value": round(gkeys, 3),
        "unit": "GKeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": f"single-array sort, N=2^{args.log2n} int64 keys, {args.dist} "
                        "distribution, keys only, ascending, out of place",
            "n": n,
            "distribution": args.dist,
            "plan": plan,
        },
        "roofline": roofline,
        "sort_roofline_2pass_frac": round(algo_bytes / (wall / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
        "hip_event_ms_per_step": round(ev_s / args.steps * 1e3, 4),
        "copy_gbs": round(copy_gbs, 1),
        "kernels": {k: {"launches": v["launches"] // args.steps,
                        "ms_per_step": round(v["ms"] / args.steps, 4)} for k, v in kernels.items()},
    }
    if args.all_dists:
        per = {}
        for name, g in gens.items():
            if name == args.dist:
                per[name] = round(gkeys, 3)
                continue
            k = g(n)
            keys_dev.copy_(torch.from_numpy(k))
            del k
            w, _, _ = time_sort(pss, torch, keys_dev, out, ws, max(3, args.steps // 2), 1, False)
            per[name] = round(n / (w / max(3, args.steps // 2)) / 1e9, 3)
        line["distributions_gkeys_per_s"] = per
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
