"""Pins of the CPU oracle against what the paper and mathematics fix.

* the paper's worked examples (Fig. 1, Fig. 3(b), Fig. 3(a)) from tests/golden;
* IEEE 754-2019 totalOrder on a hand-written table of special encodings;
* brute force over every sequence of length <= 6 on {0, 1, 2} and every
  (n_B, n_P) up to N + 1: output, pivots (Eq. 1), counts (Eq. 2), split table
  and offsets against direct O(N^2)-style counting;
* random inputs of every key type against a library stable sort, with the
  invariants the paper states (equal partition sizes, offsets r_k);
* closed forms of the split table for all-equal, ascending and descending input.
"""
import itertools
import json
import os

import numpy as np
import pytest

import refdefs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ------------------------------------------------------------- worked examples
def test_fig1_worked_example(oracle_lib):
    g = load("fig1_parallel_sort.json")
    keys = np.array(g["keys"], dtype=np.uint32)
    r = oracle_lib.pses(keys, g["n_blocks"], g["n_parts"])
    assert r.blocks.tolist() == g["sorted_blocks"]
    assert r.pivots.tolist() == g["pivots"]
    assert r.keys.tolist() == g["output"]
    # partitions of each sorted block, as drawn in Fig. 1
    L = -(-keys.size // g["n_blocks"])
    for k, key in ((0, "partition_0_by_block"), (1, "partition_1_by_block")):
        for b in range(g["n_blocks"]):
            blk = r.blocks[b * L:(b + 1) * L]
            seg = blk[int(r.split[b, k]):int(r.split[b, k + 1])].tolist()
            assert seg == g[key][b]


def test_fig3b_exact_splitting_example(oracle_lib):
    g = load("fig3b_pses_duplicates.json")
    keys = np.array(g["keys"], dtype=np.uint32)
    r = oracle_lib.pses(keys, g["n_blocks"], g["n_parts"])
    assert r.blocks.tolist() == g["sorted_blocks"]
    assert r.pivots.tolist() == g["pivots"]
    assert r.counts.tolist() == g["counts"]
    lt, le = oracle_lib.rank_counts(keys, g["pivots"][0])
    assert [lt] == g["count_less_than_pivot"] and [le] == g["count_less_equal_pivot"]
    L = -(-keys.size // g["n_blocks"])
    for k, key in ((0, "partition_0_by_block"), (1, "partition_1_by_block")):
        for b in range(g["n_blocks"]):
            blk = r.blocks[b * L:(b + 1) * L]
            assert blk[int(r.split[b, k]):int(r.split[b, k + 1])].tolist() == g[key][b]
    sizes = np.diff(r.offsets).tolist()
    assert sizes == g["partition_sizes"]
    assert r.keys.tolist() == g["output"]


def test_fig3a_pivot_only_partitioning_is_imbalanced(oracle_lib):
    """Fig. 3(a): with a pivot alone (no c_k), some partition gets >= 5 of 6
    elements whatever the pivot; exact splitting (above) gives 3 and 3."""
    g = load("fig3a_psrs_counterexample.json")
    keys = np.array(g["keys"], dtype=np.uint32)
    sizes = []
    for p in sorted(set(g["keys"])):
        left = int(np.count_nonzero(keys <= p))
        sizes.append(max(left, keys.size - left))
        if p == 1:
            assert [left, keys.size - left] == g["pivot_only_partition_sizes"]
    assert min(sizes) >= g["max_partition_lower_bound_any_pivot"]
    r = oracle_lib.pses(keys, g["n_blocks"], g["n_parts"])
    assert np.diff(r.offsets).max() == 3


# ------------------------------------------------------------------ totalOrder
@pytest.mark.parametrize("name,dtype", [("totalorder_f64.json", "f64"),
                                        ("totalorder_f32.json", "f32")])
def test_total_order_table(oracle_lib, name, dtype):
    g = load(name)
    bits = [int(h, 16) for h in g["ascending_bits_hex"]]
    for i, a in enumerate(bits):
        for j, b in enumerate(bits):
            expect = (i > j) - (i < j)
            assert oracle_lib.compare(dtype, a, b) == expect, (hex(a), hex(b))


def test_total_order_sort_of_specials(oracle_lib):
    g = load("totalorder_f64.json")
    bits = np.array([int(h, 16) for h in g["ascending_bits_hex"]], dtype=np.uint64)
    rng = np.random.default_rng(0)
    for n_b, n_p in ((1, 1), (3, 4), (5, 7), (22, 22)):
        shuffled = bits[rng.permutation(bits.size)]
        r = oracle_lib.pses(shuffled.view(np.float64), n_b, n_p)
        assert r.keys.view(np.uint64).tolist() == bits.tolist()


def test_integer_orders(oracle_lib):
    assert oracle_lib.compare("i32", 0xFFFFFFFF, 0) == -1          # -1 < 0
    assert oracle_lib.compare("u32", 0xFFFFFFFF, 0) == 1
    assert oracle_lib.compare("i64", 1 << 63, (1 << 63) - 1) == -1   # min < max
    assert oracle_lib.compare("u64", 1 << 63, (1 << 63) - 1) == 1


# ------------------------------------------------------------- brute force
def check_against_definitions(oracle_lib, keys, n_b, n_p, vals=None):
    n = keys.size
    r = oracle_lib.pses(keys, n_b, n_p, vals=vals)
    perm = refdefs.stable_order(keys)
    assert r.keys.view(np.uint8).tobytes() == keys[perm].view(np.uint8).tobytes()
    if vals is not None:
        assert np.array_equal(r.vals, vals[perm])
    piv, cnt, valid = refdefs.expected_pivots_counts(keys, n_p)
    for k in range(n_p - 1):
        assert int(r.counts[k]) == cnt[k]
        if valid[k]:
            assert r.pivots[k:k + 1].view(np.uint8).tobytes() == \
                np.asarray(piv[k], dtype=keys.dtype).reshape(1).view(np.uint8).tobytes()
    assert np.array_equal(r.split, refdefs.expected_split(keys, n_b, n_p))
    assert r.offsets.tolist() == [k * n // n_p for k in range(n_p + 1)]
    # step 1: each block sorted and a permutation of its slice
    for lo, hi in refdefs.block_bounds(n, n_b):
        seg = keys[lo:hi]
        assert r.blocks[lo:hi].view(np.uint8).tobytes() == \
            seg[refdefs.stable_order(seg)].view(np.uint8).tobytes()
    return r


def test_bruteforce_small_sequences(oracle_lib):
    cases = 0
    for n in range(0, 7):
        for tup in itertools.product(range(3), repeat=n):
            keys = np.array(tup, dtype=np.uint32)
            for n_b in range(1, n + 2):
                for n_p in range(1, n + 2):
                    check_against_definitions(oracle_lib, keys, n_b, n_p)
                    cases += 1
    assert cases > 30000


def test_bruteforce_stability_with_values(oracle_lib):
    for n in range(1, 7):
        for tup in itertools.product(range(2), repeat=n):
            keys = np.array(tup, dtype=np.int64)
            vals = np.arange(n, dtype=np.uint32)
            for n_b in range(1, n + 2):
                for n_p in range(1, n + 2):
                    r = check_against_definitions(oracle_lib, keys, n_b, n_p, vals=vals)
                    # ties in input order: vals increase within equal keys
                    for v in np.unique(keys):
                        sel = r.vals[r.keys == v]
                        assert np.all(np.diff(sel.astype(np.int64)) > 0)


def test_selection_tree_equals_linear_head_scan(oracle_lib):
    rng = np.random.default_rng(5)
    for _ in range(40):
        n = int(rng.integers(0, 400))
        keys = rng.integers(0, 7, size=n).astype(np.uint32)
        vals = np.arange(n, dtype=np.uint32)
        n_b, n_p = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        a = oracle_lib.pses(keys, n_b, n_p, vals=vals, merge_kind=0)
        b = oracle_lib.pses(keys, n_b, n_p, vals=vals, merge_kind=1)
        assert np.array_equal(a.keys, b.keys) and np.array_equal(a.vals, b.vals)


# ------------------------------------------------------------ random inputs
def random_keys(rng, dtype, n):
    if dtype == np.float64:
        pool = np.concatenate([rng.standard_normal(8),
                               np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1.0])])
        x = pool[rng.integers(0, pool.size, n)] if rng.random() < 0.5 else rng.standard_normal(n)
        bits = x.view(np.uint64).copy()
        k = rng.random(n) < 0.02
        bits[k] = np.uint64(0xFFF8000000000000)
        return bits.view(np.float64)
    if dtype == np.float32:
        x = rng.standard_normal(n).astype(np.float32)
        x[rng.random(n) < 0.05] = -0.0
        x[rng.random(n) < 0.02] = np.nan
        return x
    info = np.iinfo(dtype)
    if rng.random() < 0.3:
        return rng.integers(0, 5, size=n).astype(dtype)
    return rng.integers(info.min, info.max, size=n, dtype=dtype, endpoint=True)


@pytest.mark.parametrize("dtype", [np.uint32, np.int32, np.uint64, np.int64,
                                   np.float32, np.float64])
def test_random_inputs_all_types(oracle_lib, dtype):
    rng = np.random.default_rng(11)
    for _ in range(12):
        n = int(rng.integers(0, 2500))
        keys = random_keys(rng, dtype, n)
        n_b, n_p = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        vals = np.arange(n, dtype=np.uint32) if rng.random() < 0.5 else None
        r = check_against_definitions(oracle_lib, keys, n_b, n_p, vals=vals)
        sizes = np.diff(r.offsets)
        assert set(sizes.tolist()) <= {n // n_p, -(-n // n_p)}


# ---------------------------------------------------------- closed forms
def clamp(x, lo, hi):
    return max(lo, min(x, hi))


@pytest.mark.parametrize("kind", ["equal", "iota", "reverse"])
def test_split_table_closed_forms(oracle_lib, kind):
    for n, n_b, n_p in ((1000, 7, 13), (999, 10, 3), (64, 64, 64), (5, 4, 9), (4096, 33, 65)):
        if kind == "equal":
            keys = np.full(n, 42, dtype=np.int64)
        elif kind == "iota":
            keys = np.arange(n, dtype=np.int64)
        else:
            keys = np.arange(n - 1, -1, -1, dtype=np.int64)
        r = oracle_lib.pses(keys, n_b, n_p)
        L = -(-n // n_b)
        for b in range(n_b):
            lo, hi = min(b * L, n), min((b + 1) * L, n)
            ln = hi - lo
            for k in range(n_p + 1):
                rk = k * n // n_p
                if kind in ("equal", "iota"):
                    expect = clamp(rk - lo, 0, ln)
                else:
                    expect = clamp(rk - (n - lo - ln), 0, ln)
                assert int(r.split[b, k]) == expect, (n, n_b, n_p, b, k)


def test_short_and_empty_blocks(oracle_lib):
    # N = 5, n_B = 4: block length ceil(5/4) = 2, sizes 2, 2, 1, 0
    r = oracle_lib.pses(np.array([9, 3, 7, 1, 5], dtype=np.uint32), 4, 3)
    assert r.split[:, -1].tolist() == [2, 2, 1, 0]
    assert r.keys.tolist() == [1, 3, 5, 7, 9]


def test_more_partitions_than_elements(oracle_lib):
    keys = np.array([3, 1, 2], dtype=np.int32)
    r = oracle_lib.pses(keys, 2, 8)
    assert r.offsets.tolist() == [k * 3 // 8 for k in range(9)]
    assert r.keys.tolist() == [1, 2, 3]


def test_empty_input(oracle_lib):
    r = oracle_lib.pses(np.zeros(0, dtype=np.uint64), 3, 4)
    assert r.keys.size == 0 and r.offsets.tolist() == [0] * 5
    assert r.counts.tolist() == [0, 0, 0]
