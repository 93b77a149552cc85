"""Autotuner of the batched segmented sort.

Two choices are tuned together:

* the tile classes: a segment of at most `small_max_2k` keys is sorted by one
  128-thread workgroup (2048-key tile), one of at most `small_max_4k` keys by
  a 256-thread workgroup (4096-key tile), anything longer by 512-thread
  workgroups on 8192-key tiles followed by merge passes;
* the runs merged per pass (`fan_log2`): 32 runs (five merge rounds in LDS,
  the keys-only merge with gap sentinels) or 64 runs (six rounds, one pass
  fewer for segments of 33-64 tiles or 1025-4096 tiles).

Which choice is fastest depends on the size mix, so the tuner times every
candidate on a synthetic batch shaped like the caller's (same key type,
payload, segment count and total size, segment sizes log-uniform over the
observed range) and keeps the fastest.  Results are cached in a JSON file
keyed by GPU architecture, key type, payload, and the size bucket (log2 of
total keys and of segment count).  Every candidate sorts identically; only
the speed differs.
"""
from __future__ import annotations

import json
import os
import threading
import time

import numpy as np

CACHE_PATH = os.environ.get(
    "PSS_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json"))
CANDIDATES = [(a, b, f) for f in (5, 6) for a in (0, 512, 1024, 2048) for b in (0, 2048, 4096)
              if a <= b]
_lock = threading.Lock()


def _arch() -> str:
    try:
        import torch

        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def bucket_key(kt: int, vt: int, n: int, n_segs: int) -> str:
    lg = lambda x: int(np.log2(max(int(x), 1)))  # noqa: E731
    return f"{_arch()}/k{kt}/v{vt}/n{lg(n)}/s{lg(n_segs)}"


def _load() -> dict:
    try:
        with open(CACHE_PATH) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def cached(kt: int, vt: int, n: int, n_segs: int) -> dict | None:
    """Cached best tuning for this shape bucket, or None."""
    return _load().get(bucket_key(kt, vt, n, n_segs))


def tune(kt: int, vt: int, n: int, n_segs: int, lo_log2: float = 6.0, hi_log2: float = 20.0,
         reps: int = 3, seed: int = 99, store: bool = True) -> dict:
    """Time every candidate on a synthetic batch and return (and cache) the
    fastest as {"small_max_2k": .., "small_max_4k": .., "fan_log2": .., "ms": ..}."""
    import torch

    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd import _lib

    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp2(rng.uniform(lo_log2, hi_log2, size=n_segs))).astype(np.int64)
    sizes = np.maximum((sizes * (n / max(sizes.sum(), 1))).astype(np.int64), 0)
    offs = np.zeros(n_segs + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    total = int(offs[-1])
    width = _lib.KEY_BYTES[kt]
    raw = rng.integers(0, 2**63, size=total, dtype=np.int64)
    keys = torch.from_numpy(raw if width == 8 else (raw >> 33).astype(np.int32)).cuda()
    vals = torch.arange(total, dtype=torch.int32, device="cuda") if vt else None
    d_offs = torch.from_numpy(offs).cuda()
    max_len = int(sizes.max()) if sizes.size else 0
    results = []
    for a, b, f in CANDIDATES:
        tu = _lib.Tuning(a, b, max_len, f, 0)
        pss.segmented_sort(keys, d_offs, vals, key_type=kt, tuning=tu)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            pss.segmented_sort(keys, d_offs, vals, key_type=kt, tuning=tu)
        torch.cuda.synchronize()
        results.append(((time.perf_counter() - t0) / reps * 1e3, a, b, f))
    ms, a, b, f = min(results)
    default = next(t for t, x, y, z in results if (x, y, z) == (2048, 4096, 5))
    best = {"small_max_2k": a, "small_max_4k": b, "fan_log2": f, "ms": round(ms, 4),
            "default_ms": round(default, 4),
            "candidates": [{"small_max_2k": x, "small_max_4k": y, "fan_log2": z, "ms": round(t, 4)}
                           for t, x, y, z in results]}
    if store:
        with _lock:
            cache = _load()
            cache[bucket_key(kt, vt, total, n_segs)] = best
            tmp = CACHE_PATH + f".tmp{os.getpid()}"
            with open(tmp, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
            os.replace(tmp, CACHE_PATH)
    return best


if __name__ == "__main__":
    # python -m paper_2305_05245_amd.autotune [cache.json]: tune two batch
    # shapes, int64 keys only and u64 keys with uint32 values: the 4096-array
    # batch (sizes 2^6..2^20) and 1024 arrays of 2^17..2^19 keys (segments of
    # 17-64 tiles, where 64 runs per pass save a whole pass)
    import sys

    import workloads as W

    if len(sys.argv) > 1:
        CACHE_PATH = sys.argv[1]
    for segs, lo, hi in ((4096, 6.0, 20.0), (1024, 17.0, 19.0)):
        sizes = W.segment_sizes_loguniform(segs, lo, hi, seed=12)
        total = int(sizes.sum())
        for kt, vt in ((3, 0), (2, 1)):
            best = tune(kt, vt, total, sizes.size, lo_log2=lo, hi_log2=hi)
            print(json.dumps({"key": kt, "val": vt, "n": total, "segs": int(sizes.size),
                              "lo_log2": lo, "hi_log2": hi, **best}), flush=True)
