"""GPU parity: libpss on the device against the CPU oracle, bit for bit.

Small and medium sizes compare every output element with the oracle (and, in
the paper's single-level mode, every intermediate: sorted blocks, pivots P_k,
counts c_k, split table, offsets).  The full-size configurations (2^28 int64,
2^27 float64, five distributions each) are compared element by element with
their exact sorted output: the oracle's at full N for uniform int64 and for
normal floats with specials, closed forms or numpy's sort of the order bits
for the others, plus sampled ranks counted one by one by the oracle.  Every
sort runs on a workspace poisoned with 0xAB and checks the device error word.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import (KEY_OF_DTYPE, announce, from_device, gpu_sort, is_sorted, order_bits,
                      to_device)

pytestmark = pytest.mark.gpu

ALL_DTYPES = [np.uint32, np.int32, np.uint64, np.int64, np.float32, np.float64]
SIZES = [0, 1, 2, 3, 17, 1000, 8191, 8192, 8193, 16389, 100003, 262145, 1 << 20]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2305_05245_amd as pss

    pss._lib.load()


def seeded_keys(dtype, n, seed, kind="uniform"):
    rng = np.random.default_rng(seed)
    dtype = np.dtype(dtype)
    if kind == "dup":
        return rng.integers(0, 3, size=n).astype(dtype)
    if kind == "equal":
        return np.full(n, 7, dtype=dtype)
    if kind == "iota":
        return np.arange(n).astype(dtype)
    if kind == "reverse":
        return np.arange(n)[::-1].astype(dtype)
    if dtype == np.float64:
        x = rng.standard_normal(n)
        bits = x.view(np.uint64)
        sel = rng.random(n) < 0.01
        pats = np.array([0x8000000000000000, 0x7FF0000000000000, 0xFFF0000000000000,
                         0x7FF8000000000000, 0xFFF8000000000000, 0x7FF0000000000001, 0],
                        dtype=np.uint64)
        bits[sel] = pats[rng.integers(0, pats.size, int(sel.sum()))]
        return x
    if dtype == np.float32:
        x = rng.standard_normal(n).astype(np.float32)
        bits = x.view(np.uint32)
        sel = rng.random(n) < 0.01
        pats = np.array([0x80000000, 0x7F800000, 0xFF800000, 0x7FC00000, 0xFFC00000, 0],
                        dtype=np.uint32)
        bits[sel] = pats[rng.integers(0, pats.size, int(sel.sum()))]
        return x
    info = np.iinfo(dtype)
    return rng.integers(info.min, info.max, size=n, dtype=dtype, endpoint=True)


def oracle_sort(keys, vals=None):
    nb = 16 if keys.size > 64 else 3
    r = oracle.pses(keys, nb, nb, vals=vals)
    return r.keys, r.vals


def same_bits(a, b):
    return a.view(np.uint8).tobytes() == b.view(np.uint8).tobytes()


# ------------------------------------------------------------ automatic plan
@pytest.mark.parametrize("dtype", ALL_DTYPES, ids=lambda d: np.dtype(d).name)
def test_auto_sort_all_sizes(dtype):
    for i, n in enumerate(SIZES):
        keys = seeded_keys(dtype, n, 100 + i)
        announce("auto", np.dtype(dtype).name, n)
        got, _ = gpu_sort(keys)
        exp, _ = oracle_sort(keys)
        assert same_bits(got, exp), (np.dtype(dtype).name, n)


@pytest.mark.parametrize("kind", ["dup", "equal", "iota", "reverse"])
@pytest.mark.parametrize("dtype", [np.int32, np.uint64, np.float64], ids=lambda d: np.dtype(d).name)
def test_auto_sort_structured(dtype, kind):
    for n in (8193, 100003, 1 << 20):
        keys = seeded_keys(dtype, n, 7, kind)
        announce("auto-structured", np.dtype(dtype).name, kind, n)
        got, _ = gpu_sort(keys)
        exp, _ = oracle_sort(keys)
        assert same_bits(got, exp), (kind, n)


@pytest.mark.parametrize("dtype", [np.uint64, np.int32, np.float64, np.uint32],
                         ids=lambda d: np.dtype(d).name)
@pytest.mark.parametrize("kind", ["uniform", "dup"])
def test_auto_key_value_stable(dtype, kind):
    # 4095 / 4096 / 4097 / 12289: edges of the 4096-key tiles key-value sorts use
    for n in (1, 4095, 4096, 4097, 5000, 8192, 12289, 70001, 600000):
        keys = seeded_keys(dtype, n, 31, kind)
        vals = np.arange(n, dtype=np.uint32)
        announce("auto-kv", np.dtype(dtype).name, kind, n)
        gk, gv = gpu_sort(keys, vals)
        ek, ev = oracle_sort(keys, vals)
        assert same_bits(gk, ek) and np.array_equal(gv, ev), (kind, n)


def test_key_value_fan64_passes():
    """Key-value sorts take 4096-key tiles, 4096-key partitions and up to 64
    runs a pass: 2^18 keys (64 tiles, one pass of 64 runs), 2^18 + 1 (two
    passes), 2^24 (two passes of 64), uniform and three-valued keys, against
    the oracle (keys and the stable values)."""
    for n in (1 << 18, (1 << 18) + 1, 1 << 24):
        for kind in ("uniform", "dup"):
            keys = seeded_keys(np.uint64, n, 41, kind)
            vals = np.arange(n, dtype=np.uint32)
            announce("auto-kv-fan64", kind, n)
            gk, gv = gpu_sort(keys, vals)
            ek, ev = oracle_sort(keys, vals)
            assert same_bits(gk, ek) and np.array_equal(gv, ev), (kind, n)


def test_four_merge_passes():
    """2^28 + 3 int64 keys: 2^15 + 1 tiles, so the plan takes four merge
    passes of 16 runs (and the tile sort's output starts in the workspace).
    int64 keys sort uniquely: the output must equal numpy's sort."""
    n = (1 << 28) + 3
    keys = W.uniform_i64(n, seed=21)
    announce("auto-4-pass", n)
    got, _ = gpu_sort(keys)
    assert np.array_equal(got, np.sort(keys))


def test_medium_sizes_three_passes():
    # 2^24 keys: 2048 tiles, three merge passes
    keys = W.uniform_i64(1 << 24, seed=2)
    announce("auto-2^24-i64")
    got, _ = gpu_sort(keys)
    exp, _ = oracle_sort(keys)
    assert same_bits(got, exp)


# ------------------------------------------------------- paper single level
def check_paper(keys, n_b, n_p):
    import torch

    import paper_2305_05245_amd as pss

    announce("paper", keys.dtype.name, keys.size, n_b, n_p)
    ref = oracle.pses(keys, n_b, n_p)
    d = to_device(keys)
    res = pss.splitters(d, n_b, n_p, key_type=KEY_OF_DTYPE[keys.dtype])
    torch.cuda.synchronize()
    assert same_bits(from_device(res["sorted_blocks"], keys.dtype), ref.blocks), "step 1"
    assert np.array_equal(res["split"].cpu().numpy().astype(np.uint64), ref.split), "step 3"
    assert np.array_equal(res["offsets"].cpu().numpy().astype(np.uint64), ref.offsets), "offsets"
    assert np.array_equal(res["counts"].cpu().numpy().astype(np.uint64), ref.counts), "c_k"
    piv = from_device(res["pivots"], keys.dtype)
    valid = ref.counts > 0
    assert same_bits(piv[valid], ref.pivots[valid]), "P_k"
    got, _ = gpu_sort(keys, n_blocks=n_b, n_parts=n_p)
    assert same_bits(got, ref.keys), "output"


def test_paper_config1_int32_64x64():
    """N = 2^20 int32 uniform over the full range, n_B = n_P = 64."""
    check_paper(W.uniform_i32(1 << 20, seed=1), 64, 64)


@pytest.mark.parametrize("n,n_b,n_p", [
    (100003, 7, 13), (5, 4, 9), (1000, 1, 1), (1000, 1, 50), (1000, 50, 1),
    (50000, 300, 3), (70000, 3, 300), (20000, 2048, 5), (30000, 64, 4096),
    (40000, 2, 2), (16384 * 3 + 1, 3, 3), (1 << 18, 100, 7),
])
@pytest.mark.parametrize("kind", ["uniform", "dup", "equal", "reverse"])
def test_paper_shapes(n, n_b, n_p, kind):
    dtype = {"uniform": np.int64, "dup": np.uint32, "equal": np.float64, "reverse": np.int32}[kind]
    check_paper(seeded_keys(dtype, n, n + n_b, kind), n_b, n_p)


def test_paper_float_specials():
    check_paper(W.normal_specials_f64(200000, seed=11, fraction=0.01), 33, 65)


def test_paper_key_value():
    keys = seeded_keys(np.uint64, 123457, 3, "dup")
    vals = np.arange(keys.size, dtype=np.uint32)
    announce("paper-kv")
    gk, gv = gpu_sort(keys, vals, n_blocks=37, n_parts=19)
    ref = oracle.pses(keys, 37, 19, vals=vals)
    assert same_bits(gk, ref.keys) and np.array_equal(gv, ref.vals)


# --------------------------------------------------------------- full size
C2 = {
    "uniform": lambda n: W.uniform_i64(n, seed=2),
    "mod1000": lambda n: W.mod1000_i64(n, seed=3),
    "sorted": lambda n: W.sorted_i64(n),
    "reverse": lambda n: W.reverse_i64(n),
    "swapped1pct": lambda n: W.swapped_i64(n, seed=6),
}
C3 = {
    "uniform01": lambda n: W.uniform01_f64(n, seed=7),
    "normal": lambda n: W.normal_f64(n, seed=8),
    "allequal": lambda n: W.allequal_f64(n),
    "organpipe": lambda n: W.organpipe_f64(n),
    "normal_specials": lambda n: W.normal_specials_f64(n, seed=11),
}


def expected_full(dist: str, keys: np.ndarray) -> np.ndarray:
    """The exact sorted output of a full-size input.

    uniform int64 (2^28) and normal with specials (2^27 f64) come from the
    oracle, element by element.  The inputs that are permutations of 0..N-1
    (sorted, reverse, 1% transpositions) sort to 0..N-1; all-equal sorts to
    itself; organ pipe min(i, N-1-i) holds each value below N/2 twice (N
    even); mod 1000 sorts to each value v repeated as often as it occurs
    (counted by bincount).  The two remaining float inputs (uniform [0,1),
    normal) sort to their order bits sorted by numpy, mapped back to the
    same bits, so the multiset comparison is exact."""
    n = keys.size
    if dist in ("uniform", "normal_specials"):
        return oracle.pses(keys, 16, 16).keys
    if dist in ("sorted", "reverse", "swapped1pct"):
        return np.arange(n, dtype=np.int64)
    if dist == "allequal":
        return keys.copy()
    if dist == "organpipe":
        assert n % 2 == 0
        return np.repeat(np.arange(n // 2, dtype=np.float64), 2)
    if dist == "mod1000":
        return np.repeat(np.arange(1000, dtype=np.int64), np.bincount(keys, minlength=1000))
    # uniform01, normal: sort the totalOrder bits and map them back
    o = np.sort(order_bits(keys))
    return np.where(o < 0, o ^ np.int64(0x7FFFFFFFFFFFFFFF), o).view(np.float64)


def check_full(dist: str, keys: np.ndarray, samples: int = 4, seed: int = 0):
    announce("full", dist, keys.dtype.name, keys.size)
    got, _ = gpu_sort(keys)
    assert got.size == keys.size
    assert is_sorted(got), "not ascending"
    exp = expected_full(dist, keys)
    assert same_bits(got, exp), "differs from the exact sorted output"
    # independent of the above: sampled ranks by the oracle's direct count
    rng = np.random.default_rng(seed)
    for r in rng.integers(0, keys.size, size=samples).tolist() + [0, keys.size - 1]:
        lt, le = oracle.rank_counts(keys, got[r])
        assert lt <= r < le, f"rank {r} holds the wrong key"


@pytest.mark.parametrize("dist", list(C2))
def test_full_size_int64_2p28(dist):
    check_full(dist, C2[dist](1 << 28))


@pytest.mark.parametrize("dist", list(C3))
def test_full_size_float64_2p27(dist):
    check_full(dist, C3[dist](1 << 27))


@pytest.mark.parametrize("dist", ["uniform", "mod1000"])
def test_full_size_key_value_2p28(dist):
    """The key-value workload at full size: 2^28 int64 keys with the values
    0..N-1 (passes of 64, 32 and 32 runs).  A stable sort is unique: the
    values must equal numpy's stable argsort of the keys, and the keys the
    input in that order."""
    keys = C2[dist](1 << 28)
    vals = np.arange(keys.size, dtype=np.uint32)
    announce("full-kv", dist, keys.size)
    gk, gv = gpu_sort(keys, vals)
    perm = np.argsort(keys, kind="stable")
    assert np.array_equal(gv, perm.astype(np.uint32)), "values differ from the stable order"
    del perm
    assert np.array_equal(gk, keys[gv]), "keys differ from the input in the values' order"


@pytest.mark.parametrize("dist", list(C2))
def test_c2_distributions_exact_at_2p22(dist):
    keys = C2[dist](1 << 22)
    announce("c2-exact", dist)
    got, _ = gpu_sort(keys)
    exp, _ = oracle_sort(keys)
    assert same_bits(got, exp)


@pytest.mark.parametrize("dist", list(C3))
def test_c3_distributions_exact_at_2p22(dist):
    keys = C3[dist](1 << 22)
    announce("c3-exact", dist)
    got, _ = gpu_sort(keys)
    exp, _ = oracle_sort(keys)
    assert same_bits(got, exp)


@pytest.mark.parametrize("name", ["UniformInt", "UniformFloat", "AlmostSorted", "Duplicate3"])
def test_paper_inputs_at_1e7(name):
    """Table 1's four scalar inputs at the paper's N = 10^7, automatic plan,
    against the oracle run with the paper's 48 blocks and partitions."""
    gen = {"UniformInt": W.uniform_u32, "UniformFloat": W.uniform01_f32,
           "AlmostSorted": W.almost_sorted_u32, "Duplicate3": W.duplicate3_u32}[name]
    keys = gen(10 ** 7)
    announce("paper input", name, keys.size)
    got, _ = gpu_sort(keys)
    ref = oracle.pses(keys, 48, 48)
    assert same_bits(got, ref.keys)


def test_maximum_size_u32():
    """The largest supported n, 2^31 - 1 uint32 keys (seed 21), automatic
    plan (four merge passes): ascending and the same multiset, checked on the
    device, and sampled ranks by the oracle's direct count on the host."""
    import torch

    import paper_2305_05245_amd as pss

    n = (1 << 31) - 1
    keys = W.uniform_u32(n, seed=21)
    announce("maximum size", n)
    d = torch.from_numpy(keys.view(np.int32)).cuda()
    out, _ = pss.sort(d, key_type="u32")
    torch.cuda.synchronize()
    assert pss.device_check() == 0

    def signature(t):
        x = t.to(torch.int64) & 0xFFFFFFFF
        m1 = (x ^ (x >> 17)) * (0x9E3779B97F4A7C15 - (1 << 64))
        m1 = m1 ^ (m1 >> 29)
        m2 = (x + 0x632BE59BD9B4E019) * (0xBF58476D1CE4E5B9 - (1 << 64))
        m2 = m2 ^ (m2 >> 32)
        return int(m1.sum()), int(m2.sum())

    x = out.to(torch.int64) & 0xFFFFFFFF
    assert bool((x[1:] >= x[:-1]).all()), "not ascending"
    del x
    assert signature(out) == signature(d), "not a permutation"
    rng = np.random.default_rng(21)
    for r in rng.integers(0, n, size=2).tolist() + [0, n - 1]:
        v = np.uint32(int(out[r].item()) & 0xFFFFFFFF)
        lt, le = oracle.rank_counts(keys, v)
        assert lt <= r < le, f"rank {r} holds the wrong key"
