"""The oracle's pins must catch plausible mistakes.

Each case copies pses_oracle.c, plants one mistake of the kind the pins are
meant to catch (a dropped term, a wrong sign or index, a wrong tie-break, a
transposed operand), compiles the copy with gcc into a temporary directory and
runs a compact version of the pin suite against it.  The test passes only if
every planted mistake makes at least one pin fail.  Mistakes are planted in the
oracle, on the CPU; the real oracle is untouched.
"""
import itertools
import json
import os
import subprocess

import numpy as np
import pytest

import oracle
import refdefs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pses_oracle.c")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

MUTANTS = {
    "r_k rounded up": (
        "const uint64_t r = (uint64_t)(((u128)k * n) / n_p);\n    if (r == 0) { piv[k] = 0;",
        "const uint64_t r = (uint64_t)(((u128)k * n + n_p - 1) / n_p);\n    if (r == 0) { piv[k] = 0;"),
    "Eq. 2 off by one": ("ck[k] = r - lt;", "ck[k] = r - lt + 1;"),
    "Eq. 2 uses <= count": ("ck[k] = r - lt;", "ck[k] = le - r;"),
    "selection tree tie to higher run": ("  return a < b;\n}", "  return a > b;\n}"),
    "totalOrder negative not reversed": ("  return cmp_u64(mb, ma);", "  return cmp_u64(ma, mb);"),
    "totalOrder sign inverted": ("if (sa != sb) return sa ? -1 : 1;", "if (sa != sb) return sa ? 1 : -1;"),
    "int32 compared unsigned": (
        "case 1: return cmp_i64((int32_t)(uint32_t)a, (int32_t)(uint32_t)b);",
        "case 1: return cmp_u64(a & 0xffffffffu, b & 0xffffffffu);"),
    "block length floor": ("uint64_t L = n / n_b + (n % n_b != 0);", "uint64_t L = n / n_b + 1;"),
    "lower bound uses <=": (
        "if (oracle_compare(dtype, blk[mid].bits, v) < 0) lo = mid + 1;",
        "if (oracle_compare(dtype, blk[mid].bits, v) <= 0) lo = mid + 1;"),
    "block sort unstable on ties": (
        "if (oracle_compare(dtype, src[i].bits, src[j].bits) <= 0) dst[o++] = src[i++];",
        "if (oracle_compare(dtype, src[i].bits, src[j].bits) < 0) dst[o++] = src[i++];"),
    "pivot search strict": (
        "blk[b][mid].bits) >= r) hi = mid;", "blk[b][mid].bits) > r) hi = mid;"),
    "pivot is max over blocks": (
        "if (!have || oracle_compare(dtype, cand, best) < 0) best = cand;",
        "if (!have || oracle_compare(dtype, cand, best) > 0) best = cand;"),
    "equal copies taken from every block": (
        "const uint64_t take = eq_b < remaining ? eq_b : remaining;\n        remaining -= take;",
        "const uint64_t take = eq_b < ck[k] ? eq_b : ck[k];\n        remaining -= 0;"),
    "split ignores c_k": ("v = lt_b + take;", "v = lt_b;"),
    "tree replay keeps loser": (
        "    t->node[node] = run_beats(t, r, l) ? r : l;\n  }\n}",
        "    t->node[node] = run_beats(t, l, r) ? r : l;\n  }\n}"),
    "merge reads segment end as start": ("seg[b] = blk[b] + a;", "seg[b] = blk[b] + (a ? a - 1 : 0);"),
}


def pin_suite(lib) -> None:
    """Compact pins: worked examples, totalOrder table, brute force, closed
    forms and random inputs.  Raises on the first failed pin."""
    with open(os.path.join(GOLDEN, "fig1_parallel_sort.json")) as f:
        g1 = json.load(f)
    r = oracle.pses(np.array(g1["keys"], dtype=np.uint32), 2, 2, lib=lib)
    assert r.keys.tolist() == g1["output"] and r.pivots.tolist() == g1["pivots"]
    with open(os.path.join(GOLDEN, "fig3b_pses_duplicates.json")) as f:
        g3 = json.load(f)
    r = oracle.pses(np.array(g3["keys"], dtype=np.uint32), 2, 2, lib=lib)
    assert r.counts.tolist() == g3["counts"] and r.keys.tolist() == g3["output"]
    assert r.split[:, 1].tolist() == [2, 1]
    with open(os.path.join(GOLDEN, "totalorder_f64.json")) as f:
        bits = [int(h, 16) for h in json.load(f)["ascending_bits_hex"]]
    for i, a in enumerate(bits):
        for j, b in enumerate(bits):
            assert oracle.compare("f64", a, b, lib=lib) == (i > j) - (i < j)
    for n in range(0, 6):
        for tup in itertools.product(range(3), repeat=n):
            keys = np.array(tup, dtype=np.uint32)
            vals = np.arange(n, dtype=np.uint32)
            for n_b in range(1, n + 2):
                for n_p in range(1, n + 2):
                    r = oracle.pses(keys, n_b, n_p, vals=vals, lib=lib)
                    perm = refdefs.stable_order(keys)
                    assert np.array_equal(r.keys, keys[perm]) and np.array_equal(r.vals, perm)
                    _, cnt, _ = refdefs.expected_pivots_counts(keys, n_p)
                    assert r.counts.tolist() == cnt
                    assert np.array_equal(r.split, refdefs.expected_split(keys, n_b, n_p))
    rng = np.random.default_rng(3)
    for dtype in (np.int32, np.float64):
        for _ in range(4):
            n = int(rng.integers(1, 600))
            keys = rng.integers(-3, 3, size=n).astype(dtype)
            if dtype == np.float64:
                keys[rng.random(n) < 0.2] = -0.0
            n_b, n_p = int(rng.integers(1, 50)), int(rng.integers(1, 50))
            r = oracle.pses(keys, n_b, n_p, lib=lib)
            perm = refdefs.stable_order(keys)
            assert r.keys.view(np.uint8).tobytes() == keys[perm].view(np.uint8).tobytes()
            assert np.array_equal(r.split, refdefs.expected_split(keys, n_b, n_p))


def test_real_oracle_passes_compact_pins(oracle_lib):
    pin_suite(oracle_lib._load())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name!r} not unique"
    mutated = src.replace(old, new)
    (tmp_path / "pses_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "pses_oracle.h")).read())
    (tmp_path / "pses_oracle.c").write_text(mutated)
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(so),
                           str(tmp_path / "pses_oracle.c")])
    lib = oracle.bind(str(so))
    with pytest.raises((AssertionError, RuntimeError)):
        pin_suite(lib)
