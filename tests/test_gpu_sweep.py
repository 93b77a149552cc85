"""A seeded sweep over sizes, key types, key mixes and payloads: 64 cases of
log-uniform size up to 2^23 (so every plan shape from one tile to several
passes, tile sizes of keys-only and key-value sorts, ragged tails), each
compared element by element with numpy's stable sort of the keys' order bits
(IEEE totalOrder for floats, written independently of the library's key map).
A stable sort is unique, so the values must equal numpy's stable argsort."""
import numpy as np
import pytest

from gpu_util import announce, gpu_sort, order_bits

pytestmark = pytest.mark.gpu

DTYPES = [np.uint32, np.int32, np.uint64, np.int64, np.float32, np.float64]


def case(seed: int):
    rng = np.random.default_rng(1000 + seed)
    dtype = np.dtype(DTYPES[seed % len(DTYPES)])
    n = int(np.exp2(rng.uniform(0.0, 23.0)))
    kind = ("uniform", "few", "runs")[seed % 3]
    if kind == "few":  # heavy duplicates
        raw = rng.integers(0, 5, size=n).astype(np.uint64)
    elif kind == "runs":  # presorted runs of random length
        raw = np.sort(rng.integers(0, 1 << 62, size=n, dtype=np.uint64))
        cut = rng.integers(0, max(n, 1), size=8)
        for c in cut:
            raw[c:] = raw[c:][::-1].copy() if c % 2 else raw[c:]
    else:
        raw = rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)
    keys = raw.astype(np.uint64).view(np.uint64)
    if dtype.itemsize == 4:
        keys = (keys >> np.uint64(32)).astype(np.uint32).view(dtype)
    else:
        keys = keys.view(dtype)
    if dtype.kind == "f":
        keys = keys.copy()
        bits = keys.view(np.uint64 if dtype.itemsize == 8 else np.uint32)
        # keep NaNs of every payload: totalOrder places them by their bits
        if kind == "few":
            keys[:] = np.array([-0.0, 0.0, 1.5, -np.inf, np.nan], dtype=dtype)[raw.astype(np.int64) % 5]
        del bits
    kv = seed % 2 == 1
    return dtype, n, kind, keys, kv


@pytest.mark.parametrize("seed", range(64))
def test_sweep_against_numpy_stable_sort(seed):
    dtype, n, kind, keys, kv = case(seed)
    announce("sweep", seed, dtype.name, n, kind, "kv" if kv else "keys")
    vals = np.arange(n, dtype=np.uint32) if kv else None
    gk, gv = gpu_sort(keys, vals)
    perm = np.argsort(order_bits(keys), kind="stable")
    assert gk.view(np.uint8).tobytes() == keys[perm].view(np.uint8).tobytes()
    if kv:
        assert np.array_equal(gv, perm.astype(np.uint32))
