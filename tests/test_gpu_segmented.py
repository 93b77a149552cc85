"""GPU parity of the batched segmented sort: every segment of the output must
equal the oracle's sort of that segment alone, bit for bit (stable payload
where given), for every tile class and tuning; at the full batched size
(4096 segments, 2^6..2^20 keys each) every segment against numpy's sort of
it and sampled segments against the oracle; segments above 2^23 keys (three
merge passes) against the oracle.  Every call runs on a workspace poisoned
with 0xAB and checks the device error word."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import KEY_OF_DTYPE, announce, from_device, poisoned_workspace, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available()


def keys_for(dtype, n, seed):
    rng = np.random.default_rng(seed)
    dtype = np.dtype(dtype)
    if dtype.kind == "f":
        x = rng.standard_normal(n).astype(dtype)
        x[rng.random(n) < 0.02] = -0.0
        return x
    info = np.iinfo(dtype)
    if seed % 3 == 0:
        return rng.integers(0, 4, size=n).astype(dtype)
    return rng.integers(info.min, info.max, size=n, dtype=dtype, endpoint=True)


def oracle_segmented(keys, offs, vals=None):
    out = np.empty_like(keys)
    vout = None if vals is None else np.empty_like(vals)
    for i in range(offs.size - 1):
        lo, hi = int(offs[i]), int(offs[i + 1])
        if hi == lo:
            continue
        nb = 4 if hi - lo > 16 else 1
        r = oracle.pses(keys[lo:hi], nb, nb, vals=None if vals is None else vals[lo:hi])
        out[lo:hi] = r.keys
        if vals is not None:
            vout[lo:hi] = r.vals
    return out, vout


def gpu_segmented(keys, offs, vals=None, tuning=None, max_seg_len=None):
    """Segmented sort on the device with a poisoned workspace; the device
    error word must stay clear."""
    import torch

    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd import _lib

    dk = to_device(keys)
    dv = to_device(vals.astype(np.uint32)) if vals is not None else None
    d_offs = torch.from_numpy(offs.astype(np.int64)).cuda()
    kt = KEY_OF_DTYPE[keys.dtype]
    vt = _lib.VAL_U32 if vals is not None else _lib.VAL_NONE
    tu = pss._resolve_tuning(tuning, _lib.KEY_NAMES[kt], vt, keys.size, offs.size - 1,
                             max_seg_len if max_seg_len is not None else
                             (int(np.max(np.diff(offs))) if offs.size > 1 else 0))
    ws = poisoned_workspace(_lib.segmented_workspace_bytes(_lib.KEY_NAMES[kt], vt, keys.size,
                                                           offs.size - 1, tu))
    out, vout = pss.segmented_sort(dk, d_offs, dv, key_type=kt, tuning=tu, workspace=ws)
    torch.cuda.synchronize()
    assert pss.device_check() == 0, "device error word set"
    return from_device(out, keys.dtype), (from_device(vout, np.uint32) if vout is not None else None)


MIXED = [0, 1, 2, 17, 100, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193, 20000,
         0, 5, 300001, 70000, 1 << 20]


def mixed_offsets(seed):
    rng = np.random.default_rng(seed)
    sizes = np.array(MIXED + rng.integers(0, 9000, size=40).tolist(), dtype=np.int64)
    rng.shuffle(sizes)
    offs = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    return offs


def same(a, b):
    return a.view(np.uint8).tobytes() == b.view(np.uint8).tobytes()


@pytest.mark.parametrize("dtype", [np.uint32, np.int32, np.uint64, np.int64, np.float32, np.float64],
                         ids=lambda d: np.dtype(d).name)
def test_segmented_mixed_sizes_all_types(dtype):
    offs = mixed_offsets(1)
    keys = keys_for(dtype, int(offs[-1]), 7)
    announce("segmented-mixed", np.dtype(dtype).name, offs.size - 1, int(offs[-1]))
    got, _ = gpu_segmented(keys, offs)
    exp, _ = oracle_segmented(keys, offs)
    assert same(got, exp)


@pytest.mark.parametrize("dtype", [np.uint64, np.int32, np.float64], ids=lambda d: np.dtype(d).name)
def test_segmented_key_value_stable(dtype):
    offs = mixed_offsets(2)
    keys = keys_for(dtype, int(offs[-1]), 9)  # seed 9: three-valued keys (many ties)
    vals = np.arange(keys.size, dtype=np.uint32)
    announce("segmented-kv", np.dtype(dtype).name)
    gk, gv = gpu_segmented(keys, offs, vals)
    ek, ev = oracle_segmented(keys, offs, vals)
    assert same(gk, ek) and np.array_equal(gv, ev)


@pytest.mark.parametrize("tuning", [{"small_max_2k": 0, "small_max_4k": 0},
                                    {"small_max_2k": 512, "small_max_4k": 2048},
                                    {"small_max_2k": 2048, "small_max_4k": 4096},
                                    {"small_max_2k": 1024, "small_max_4k": 4096},
                                    {"small_max_2k": 2048, "small_max_4k": 4096, "fan_log2": 6},
                                    {"small_max_2k": 0, "small_max_4k": 0, "fan_log2": 6}],
                         ids=["all8k", "512-2k", "2k-4k", "1k-4k", "2k-4k-fan64", "all8k-fan64"])
def test_segmented_every_tuning_same_output(tuning):
    offs = mixed_offsets(3)
    keys = keys_for(np.int64, int(offs[-1]), 11)
    announce("segmented-tuning", tuning)
    got, _ = gpu_segmented(keys, offs, tuning=tuning)
    exp, _ = oracle_segmented(keys, offs)
    assert same(got, exp)


def test_segmented_equals_one_sort_per_array():
    import torch

    import paper_2305_05245_amd as pss

    offs = mixed_offsets(4)
    keys = keys_for(np.int64, int(offs[-1]), 13)
    announce("segmented-vs-per-array")
    got, _ = gpu_segmented(keys, offs)
    dk = to_device(keys)
    for i in range(offs.size - 1):
        lo, hi = int(offs[i]), int(offs[i + 1])
        if hi > lo:
            one, _ = pss.sort(dk[lo:hi].contiguous(), key_type="i64")
            torch.cuda.synchronize()
            assert same(got[lo:hi], from_device(one, np.int64)), i


def test_segmented_loguniform_batch_exact():
    sizes = W.segment_sizes_loguniform(512, 6.0, 18.0, seed=12)
    offs = W.segment_offsets(sizes).astype(np.int64)
    keys = W.uniform_i64(int(offs[-1]), seed=13)
    announce("segmented-loguniform-512", int(offs[-1]))
    got, _ = gpu_segmented(keys, offs)
    exp, _ = oracle_segmented(keys, offs)
    assert same(got, exp)


def test_segmented_full_batch_4096_segments():
    """4096 segments of round(2^U), U ~ U[6, 20] int64 keys (about 4.4e8 keys):
    every segment equals numpy's sort of that segment's input (int64 keys:
    the exact sorted output), and sampled segments equal the oracle's."""
    sizes = W.segment_sizes_loguniform(4096, 6.0, 20.0, seed=12)
    offs = W.segment_offsets(sizes).astype(np.int64)
    n = int(offs[-1])
    keys = W.uniform_i64(n, seed=13)
    announce("segmented-full", n)
    got, _ = gpu_segmented(keys, offs)
    for i in range(offs.size - 1):
        lo, hi = int(offs[i]), int(offs[i + 1])
        assert np.array_equal(got[lo:hi], np.sort(keys[lo:hi])), i
    rng = np.random.default_rng(0)
    for i in rng.choice(offs.size - 1, size=8, replace=False).tolist():
        lo, hi = int(offs[i]), int(offs[i + 1])
        if hi - lo <= (1 << 18):
            r = oracle.pses(keys[lo:hi], 4, 4)
            assert same(got[lo:hi], r.keys), i


@pytest.mark.parametrize("fan", [5, 6], ids=["fan32", "fan64"])
@pytest.mark.parametrize("kv", [False, True], ids=["keys", "key-value"])
def test_segmented_three_merge_passes(kv, fan):
    """Keys only, segments above 2^23 keys take three merge passes of 32 runs
    (2^11+ tiles of 8192 keys) with the segment's data ending in the output or
    the workspace by the parity of its own pass count: segments of 2^23 + 1
    and 2^24 keys (three passes), 2^23 (two), 2^20 + 3 (two) and short ones
    (none or one), mixed, against the oracle segment by segment.  With 64
    runs per pass the same segments take two passes (2^24: 2048 tiles =
    64 x 32) and 2^20 + 3 one pass fewer, so the parities differ.  Key-value
    batches use 4096-key tiles: 2^23 + 1 and 2^24 keys take three passes of
    32 runs and two of 64, 2^20 + 3 two passes either way."""
    sizes = np.array([1000, (1 << 23) + 1, 5, (1 << 20) + 3, 1 << 24, 8193, 1 << 23, 0, 77],
                     dtype=np.int64)
    offs = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    keys = np.concatenate([W.request_keys(int(s), i % 2 == 1, seed=40 + i)
                           for i, s in enumerate(sizes)]).view(np.uint64)
    vals = np.arange(keys.size, dtype=np.uint32) if kv else None
    announce("segmented-3-pass", "kv" if kv else "keys", "fan", 1 << fan, int(offs[-1]))
    gk, gv = gpu_segmented(keys, offs, vals, tuning={"small_max_2k": 2048, "small_max_4k": 4096,
                                                     "fan_log2": fan})
    ek, ev = oracle_segmented(keys, offs, vals)
    assert same(gk, ek)
    if kv:
        assert np.array_equal(gv, ev)


def test_segmented_invalid_offsets_reported():
    import torch

    import paper_2305_05245_amd as pss

    keys = keys_for(np.int64, 1000, 5)
    bad = np.array([0, 600, 400, 1000], dtype=np.int64)   # decreasing
    announce("segmented-invalid-offsets")
    dk = to_device(keys)
    pss.segmented_sort(dk, torch.from_numpy(bad).cuda(), key_type="i64")
    assert pss.device_check(0) & 16
