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
from test_oracle_psrs import check_single_block_closed_form, check_worked_examples

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
    "merge reads segment end as start": (
        "seg[b] = blk[b] + a;\n      seg_len[b] = e - a;\n    }\n    rc = merge_kind",
        "seg[b] = blk[b] + (a ? a - 1 : 0);\n      seg_len[b] = e - a;\n    }\n    rc = merge_kind"),
    # PSRS (regular-sampling pivots)
    "psrs sample positions shifted down": (
        "smp[ns++] = blk[b][(uint64_t)(((u128)j * blen[b]) / n_p)];",
        "smp[ns++] = blk[b][(uint64_t)(((u128)(j - 1) * blen[b]) / n_p)];"),
    "psrs samples left unsorted": ("rc = merge_sort_stable(dtype, smp, ns);", "rc = ORACLE_OK;"),
    "psrs pivot index divided first": (
        "piv[k] = ns ? smp[(uint64_t)(((u128)k * ns) / n_p)].bits : 0;",
        "piv[k] = ns ? smp[(uint64_t)k * (ns / n_p)].bits : 0;"),
    "psrs partition by lower bound": (
        "? count_less_equal(dtype, blk[b], blen[b], piv[k]) : 0;",
        "? count_less(dtype, blk[b], blen[b], piv[k]) : 0;"),
    "records copied in input order": (
        "(const unsigned char *)records + (uint64_t)perm[j] * record_bytes, record_bytes);",
        "(const unsigned char *)records + (uint64_t)j * record_bytes, record_bytes);"),
    "records keyed at offset 0": (
        "memcpy(keys + i * kb, (const unsigned char *)records + i * record_bytes + key_offset, kb);",
        "memcpy(keys + i * kb, (const unsigned char *)records + i * record_bytes, kb);"),
    "psrs merge tie to higher block": (
        "rc = merge_selection_tree(dtype, seg, seg_len, n_b, merged + off[k]);\n    if (rc) goto done;\n  }\n\n  for (uint64_t i = 0; i < n; ++i) {\n    store_bits(keys_out, i, kb, merged[i].bits);\n    if (vals) vals_out[i] = merged[i].val;\n  }\n  if (samples_out)",
        "for (uint32_t h = 0; h < n_b / 2; ++h) { const elem_t *t = seg[h]; seg[h] = seg[n_b - 1 - h]; seg[n_b - 1 - h] = t; uint64_t u = seg_len[h]; seg_len[h] = seg_len[n_b - 1 - h]; seg_len[n_b - 1 - h] = u; }\n    rc = merge_selection_tree(dtype, seg, seg_len, n_b, merged + off[k]);\n    if (rc) goto done;\n  }\n\n  for (uint64_t i = 0; i < n; ++i) {\n    store_bits(keys_out, i, kb, merged[i].bits);\n    if (vals) vals_out[i] = merged[i].val;\n  }\n  if (samples_out)"),
}


def psrs_pins(lib) -> None:
    """Compact pins of the PSRS variant: hand-worked examples, the one-block
    closed form, and the stable output with values on duplicate-heavy keys."""
    check_worked_examples(oracle, lib=lib)
    rng = np.random.default_rng(4)
    check_single_block_closed_form(oracle, rng, lib=lib)
    for _ in range(4):
        n = int(rng.integers(1, 400))
        keys = rng.integers(0, 5, size=n).astype(np.int64)
        vals = np.arange(n, dtype=np.uint32)
        r = oracle.psrs(keys, int(rng.integers(2, 20)), int(rng.integers(2, 20)), vals=vals, lib=lib)
        perm = refdefs.stable_order(keys)
        assert np.array_equal(r.keys, keys[perm]) and np.array_equal(r.vals, perm)


def record_pins(lib) -> None:
    """Compact record-sort pins: Particle-shaped records with the key at the
    end, against (key, index) order."""
    rng = np.random.default_rng(9)
    for n in (5, 300):
        rec = rng.integers(0, 256, size=(n, 96), dtype=np.uint8)
        keys = rng.integers(0, 4, size=n).astype(np.float64)
        rec[:, 88:96] = keys.view(np.uint8).reshape(n, 8)
        got = oracle.sort_records(rec, "f64", 88, 3, 3, lib=lib)
        assert np.array_equal(got, rec[refdefs.stable_order(keys)])


def pin_suite(lib) -> None:
    """Compact pins: worked examples, totalOrder table, brute force, closed
    forms and random inputs.  Raises on the first failed pin."""
    record_pins(lib)
    psrs_pins(lib)
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
