"""Pins of the oracle's record sort (Table 1: Pair, 16-byte records, and
Particle, 96-byte records, sorted by a key field): against the plain definition
(records ordered by (key, input index), the key order from the independent
definitions in refdefs), on Pair- and Particle-shaped records and odd layouts."""
from __future__ import annotations

import numpy as np
import pytest

import refdefs

LAYOUTS = [  # (record bytes, key offset, key type)
    (16, 0, "u64"),    # Pair: key, index
    (96, 0, "u64"),    # Particle: key, 11 doubles
    (96, 88, "f64"),
    (12, 4, "i32"),
    (4, 0, "f32"),
    (40, 8, "i64"),
]
NP = {"u64": np.uint64, "f64": np.float64, "i32": np.int32, "f32": np.float32, "i64": np.int64}


def make_records(rng, n, rb, off, kt, dup):
    rec = rng.integers(0, 256, size=(n, rb), dtype=np.uint8)
    dt = np.dtype(NP[kt])
    if dup:
        keys = rng.integers(0, 3, size=n).astype(dt)
    elif dt.kind == "f":
        keys = rng.standard_normal(n).astype(dt)
    else:
        keys = rng.integers(np.iinfo(dt).min, np.iinfo(dt).max, size=n, dtype=dt, endpoint=True)
    rec[:, off:off + dt.itemsize] = keys.view(np.uint8).reshape(n, dt.itemsize)
    return rec, keys


def expected(rec, keys):
    return rec[refdefs.stable_order(keys)]


@pytest.mark.parametrize("rb,off,kt", LAYOUTS)
@pytest.mark.parametrize("dup", [False, True])
def test_records_plain_definition(oracle_lib, rb, off, kt, dup):
    rng = np.random.default_rng(rb * 100 + off + dup)
    for n in (0, 1, 2, 7, 100, 1000):
        rec, keys = make_records(rng, n, rb, off, kt, dup)
        got = oracle_lib.sort_records(rec, kt, off, n_blocks=int(rng.integers(1, 9)),
                                      n_parts=int(rng.integers(1, 9)))
        assert np.array_equal(got, expected(rec, keys)), (n, rb, off, kt, dup)


def test_records_bad_layout(oracle_lib):
    rec = np.zeros((4, 8), dtype=np.uint8)
    with pytest.raises(RuntimeError):
        oracle_lib.sort_records(rec, "u64", 4)   # key runs past the record
