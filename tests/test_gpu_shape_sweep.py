"""Seeded sweeps over the shapes that vary most: batched segmented sorts
(segment counts, size mixes with empty segments and exact tile multiples,
key types, payloads, tile-class thresholds and 32 or 64 runs per pass) and
the paper's single level (n_B, n_P, sizes).  Every segment, or the whole
output, is compared element by element with numpy's stable sort of the keys'
order bits; a stable sort is unique, so values must equal its argsort."""
import numpy as np
import pytest

from gpu_util import announce, gpu_sort, order_bits
from test_gpu_segmented import gpu_segmented

pytestmark = pytest.mark.gpu

DTYPES = [np.uint32, np.int32, np.uint64, np.int64, np.float32, np.float64]
TUNINGS = [(2048, 4096, 5), (0, 0, 5), (512, 2048, 6), (2048, 4096, 6), (0, 4096, 5)]


def random_keys(rng, dtype, n, dup):
    if dup:
        raw = rng.integers(0, 4, size=n).astype(np.uint64)
    else:
        raw = rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)
    if np.dtype(dtype).itemsize == 4:
        return (raw >> np.uint64(32)).astype(np.uint32).view(dtype) if not dup else \
            raw.astype(np.uint32).view(dtype)
    return raw.view(dtype)


def stable_expect(keys, vals):
    perm = np.argsort(order_bits(keys), kind="stable")
    return keys[perm], (vals[perm] if vals is not None else None)


@pytest.mark.parametrize("seed", range(24))
def test_segmented_shape_sweep(seed):
    rng = np.random.default_rng(2000 + seed)
    dtype = np.dtype(DTYPES[seed % len(DTYPES)])
    n_segs = int(rng.integers(1, 300))
    pick = rng.random(n_segs)
    sizes = np.where(pick < 0.1, 0,
             np.where(pick < 0.2, 4096 * rng.integers(1, 5, size=n_segs),
              np.where(pick < 0.3, 8192 * rng.integers(1, 5, size=n_segs),
                       np.rint(np.exp2(rng.uniform(0, 17, size=n_segs))).astype(np.int64))))
    if seed % 4 == 0:
        sizes[rng.integers(0, n_segs)] = int(rng.integers(1 << 18, 1 << 21))  # one long segment
    sizes = sizes.astype(np.int64)
    offs = np.zeros(n_segs + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    n = int(offs[-1])
    keys = random_keys(rng, dtype, n, seed % 3 == 0)
    kv = seed % 2 == 1
    vals = np.arange(n, dtype=np.uint32) if kv else None
    a, b, f = TUNINGS[seed % len(TUNINGS)]
    announce("seg-sweep", seed, dtype.name, n_segs, n, "kv" if kv else "keys", a, b, f)
    gk, gv = gpu_segmented(keys, offs, vals, tuning={"small_max_2k": a, "small_max_4k": b,
                                                      "fan_log2": f})
    for i in range(n_segs):
        lo, hi = int(offs[i]), int(offs[i + 1])
        if hi == lo:
            continue
        ek, ev = stable_expect(keys[lo:hi], vals[lo:hi] if kv else None)
        assert gk[lo:hi].view(np.uint8).tobytes() == ek.view(np.uint8).tobytes(), i
        if kv:
            assert np.array_equal(gv[lo:hi], ev), i


@pytest.mark.parametrize("seed", range(16))
def test_single_level_shape_sweep(seed):
    rng = np.random.default_rng(3000 + seed)
    dtype = np.dtype(DTYPES[seed % len(DTYPES)])
    n = int(np.exp2(rng.uniform(4, 22)))
    n_b = int(rng.integers(1, 200))
    n_p = int(rng.integers(1, 300))
    keys = random_keys(rng, dtype, n, seed % 3 == 0)
    kv = seed % 2 == 1
    vals = np.arange(n, dtype=np.uint32) if kv else None
    announce("level-sweep", seed, dtype.name, n, n_b, n_p, "kv" if kv else "keys")
    gk, gv = gpu_sort(keys, vals, n_blocks=n_b, n_parts=n_p)
    ek, ev = stable_expect(keys, vals)
    assert gk.view(np.uint8).tobytes() == ek.view(np.uint8).tobytes()
    if kv:
        assert np.array_equal(gv, ev)
