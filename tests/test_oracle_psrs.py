"""Pins of the oracle's PSRS variant (regular-sampling pivots, Section 2.3):
hand-worked examples, the one-block closed form, the load-balance bound of
regular sampling on distinct keys, the value-partition property, and the
Duplicate3 saturation that motivates exact splitting (Fig. 3)."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import refdefs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def check_worked_examples(oracle_lib, lib=None):
    for c in load("psrs_regular_sampling_worked.json")["cases"]:
        keys = np.array(c["keys"], dtype=np.uint32)
        r = oracle_lib.psrs(keys, c["n_blocks"], c["n_parts"], lib=lib)
        assert r.samples.tolist() == c["samples"], c["name"]
        assert r.pivots.tolist() == c["pivots"], c["name"]
        assert r.split.tolist() == c["split"], c["name"]
        assert r.offsets.tolist() == c["offsets"], c["name"]
        assert r.keys.tolist() == sorted(c["keys"]), c["name"]


def check_single_block_closed_form(oracle_lib, rng, lib=None):
    """n_B = 1: the samples are the block's elements at floor(jN/n_P), so
    P_k = S[floor(k (n_P-1) / n_P)] = S[k-1] is the element of 0-based rank
    floor(kN/n_P); with distinct keys |{x <= P_k}| = floor(kN/n_P) + 1."""
    for n, n_p in ((1, 2), (7, 3), (100, 7), (1000, 64), (513, 512)):
        keys = rng.permutation(np.arange(10 * n, dtype=np.int64))[:n]
        r = oracle_lib.psrs(keys, 1, n_p, lib=lib)
        srt = np.sort(keys)
        ranks = [k * n // n_p for k in range(1, n_p)]
        assert r.pivots.tolist() == srt[ranks].tolist()
        assert r.offsets[1:-1].tolist() == [x + 1 for x in ranks]


def test_worked_examples(oracle_lib):
    check_worked_examples(oracle_lib)


def test_single_block_closed_form(oracle_lib):
    check_single_block_closed_form(oracle_lib, np.random.default_rng(21))


@pytest.mark.parametrize("n_b,n_p,m", [(2, 2, 5), (4, 8, 3), (16, 16, 4), (48, 48, 2), (7, 5, 9)])
def test_regular_sampling_bound_on_distinct_keys(oracle_lib, n_b, n_p, m):
    """Blocks of L = n_P m distinct keys: a block with a_b samples <= P_k holds
    between a_b m and (a_b + 1) m elements <= P_k, and consecutive pivots are
    at most ceil(n_B (n_P-1) / n_P) <= n_B samples apart, so no partition
    exceeds 2 n_B m = 2N/n_P (the load-balance guarantee of regular sampling)."""
    rng = np.random.default_rng(n_b * 1000 + n_p)
    n = n_b * n_p * m
    for _ in range(5):
        keys = rng.permutation(n).astype(np.uint64)
        r = oracle_lib.psrs(keys, n_b, n_p)
        assert r.sizes.max() <= 2 * n // n_p
        assert r.keys.tolist() == list(range(n))


@pytest.mark.parametrize("dtype", [np.uint32, np.int32, np.int64, np.float32, np.float64])
def test_value_partition_and_stable_output(oracle_lib, dtype):
    """Partition k of the output holds exactly the keys x with P_k < x <=
    P_{k+1} (Section 2), and the output is the stable sort."""
    rng = np.random.default_rng(5)
    for _ in range(6):
        n = int(rng.integers(1, 800))
        if dtype in (np.float32, np.float64):
            keys = rng.standard_normal(n).astype(dtype)
            keys[rng.random(n) < 0.3] = dtype(0.5)
            keys[rng.random(n) < 0.05] = -0.0
        else:
            keys = rng.integers(-20 if np.issubdtype(dtype, np.signedinteger) else 0, 40,
                                size=n).astype(dtype)
        n_b, n_p = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        vals = np.arange(n, dtype=np.uint32)
        r = oracle_lib.psrs(keys, n_b, n_p, vals=vals)
        perm = refdefs.stable_order(keys)
        assert r.keys.view(np.uint8).tobytes() == keys[perm].view(np.uint8).tobytes()
        assert np.array_equal(r.vals, perm)
        ok = refdefs.order_keys(r.keys)
        pk = refdefs.order_keys(r.pivots) if n_p > 1 else np.zeros(0, dtype=np.int64)
        for k in range(n_p):
            part = ok[int(r.offsets[k]):int(r.offsets[k + 1])]
            if k > 0:
                assert (part > pk[k - 1]).all()
            if k < n_p - 1:
                assert (part <= pk[k]).all()
        # per block, the split positions are the upper bounds of the pivots
        for b, (lo, hi) in enumerate(refdefs.block_bounds(n, n_b)):
            blk = np.sort(refdefs.order_keys(keys[lo:hi]))
            want = [0] + [int(np.searchsorted(blk, p, side="right")) for p in pk] + [hi - lo]
            assert r.split[b].tolist() == want


def test_duplicate3_saturates_but_exact_splitting_does_not(oracle_lib):
    """Keys from {0, 1, 2} (the paper's Duplicate3): a pivot-only partition has
    at most 3 non-empty parts whatever the pivots, so one holds >= N/3; exact
    splitting keeps every part at floor or ceil of N/n_P (Fig. 3)."""
    rng = np.random.default_rng(8)
    n, n_b, n_p = 3000, 16, 16
    keys = rng.integers(0, 3, size=n).astype(np.uint64)
    r = oracle_lib.psrs(keys, n_b, n_p)
    sizes = r.sizes
    assert np.count_nonzero(sizes) <= 3
    assert sizes.max() >= n / 3
    assert set(r.pivots.tolist()) <= {0, 1, 2}
    e = oracle_lib.pses(keys, n_b, n_p)
    assert np.diff(e.offsets.astype(np.int64)).max() == -(-n // n_p)
    assert np.array_equal(r.keys, e.keys)


def test_all_equal_and_edge_cases(oracle_lib):
    keys = np.full(100, 7, dtype=np.int32)
    r = oracle_lib.psrs(keys, 4, 5)
    assert r.pivots.tolist() == [7] * 4
    assert r.sizes.tolist() == [100, 0, 0, 0, 0]
    r = oracle_lib.psrs(np.zeros(0, dtype=np.uint64), 3, 4)
    assert r.keys.size == 0 and r.offsets.tolist() == [0] * 5 and r.samples.size == 0
    r = oracle_lib.psrs(np.array([3, 1, 2], dtype=np.int64), 2, 1)
    assert r.keys.tolist() == [1, 2, 3] and r.offsets.tolist() == [0, 3] and r.samples.size == 0
    r = oracle_lib.psrs(np.array([3, 1, 2], dtype=np.int64), 5, 8)
    assert r.keys.tolist() == [1, 2, 3] and r.offsets[-1] == 3
