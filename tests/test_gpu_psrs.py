"""GPU parity of the regular-sampling (PSRS) variant against the oracle, bit
for bit: sorted blocks, sorted samples, pivots, split table, offsets,
partition sizes and the sorted output (stable with values), on shapes that
cover ragged and empty blocks, more partitions than keys, one partition, the
three co-rank kernels (up to 32, up to 64 and more than 64 blocks), heavy
duplicates (partitions far larger than one merge chunk) and float specials."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import KEY_OF_DTYPE, announce, from_device, to_device
from test_gpu_parity import same_bits, seeded_keys

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2305_05245_amd as pss

    pss._lib.load()


def check_psrs(keys, n_b, n_p, vals=None):
    import torch

    import paper_2305_05245_amd as pss

    announce("psrs", keys.dtype.name, keys.size, n_b, n_p, "kv" if vals is not None else "")
    kt = KEY_OF_DTYPE[keys.dtype]
    ref = oracle.psrs(keys, n_b, n_p, vals=vals)
    d = to_device(keys)
    res = pss.psrs_splitters(d, n_b, n_p, key_type=kt)
    torch.cuda.synchronize()
    assert same_bits(from_device(res["sorted_blocks"], keys.dtype), ref.blocks), "step 1"
    assert same_bits(from_device(res["samples"], keys.dtype), ref.samples), "samples"
    assert same_bits(from_device(res["pivots"], keys.dtype), ref.pivots), "P_k"
    assert np.array_equal(res["split"].cpu().numpy().astype(np.uint64), ref.split), "split"
    assert np.array_equal(res["offsets"].cpu().numpy().astype(np.uint64), ref.offsets), "offsets"
    dv = to_device(vals) if vals is not None else None
    out, vout, sizes = pss.psrs_sort(d, dv, n_blocks=n_b, n_parts=n_p, key_type=kt)
    torch.cuda.synchronize()
    assert same_bits(from_device(out, keys.dtype), ref.keys), "output"
    assert np.array_equal(sizes.cpu().numpy(), ref.sizes), "partition sizes"
    if vals is not None:
        assert np.array_equal(from_device(vout, np.uint32), ref.vals), "values"
    assert pss.device_check() == 0
    return ref


@pytest.mark.parametrize("n,n_b,n_p", [
    (100003, 7, 13), (5, 4, 3), (5, 4, 9), (1000, 1, 1), (1000, 1, 50), (1000, 50, 1),
    (50000, 300, 3), (70000, 3, 300), (20000, 2048, 5), (40000, 2, 2), (60000, 48, 48),
    (16384 * 3 + 1, 3, 3), (1 << 18, 100, 7), (1 << 18, 33, 64),
])
@pytest.mark.parametrize("kind", ["uniform", "dup", "equal", "reverse"])
def test_psrs_shapes(n, n_b, n_p, kind):
    dtype = {"uniform": np.int64, "dup": np.uint32, "equal": np.float64, "reverse": np.int32}[kind]
    check_psrs(seeded_keys(dtype, n, n + n_b, kind), n_b, n_p)


def test_psrs_float_specials_and_types():
    check_psrs(W.normal_specials_f64(200000, seed=11, fraction=0.01), 33, 65)
    check_psrs(seeded_keys(np.float32, 90001, 4), 17, 31)
    check_psrs(seeded_keys(np.uint64, 90001, 5), 64, 64)


def test_psrs_key_value_stable():
    keys = seeded_keys(np.uint64, 123457, 3, "dup")
    check_psrs(keys, 37, 19, vals=np.arange(keys.size, dtype=np.uint32))
    keys = seeded_keys(np.int32, 80000, 6)
    check_psrs(keys, 100, 10, vals=np.arange(keys.size, dtype=np.uint32)[::-1].copy())


def test_psrs_duplicate3_imbalance_at_2p22():
    """Duplicate3 at 2^22 keys, n_B = n_P = 256: at most three non-empty
    partitions, each hundreds of merge chunks long; the output equals the
    exact-splitting sort's."""
    import torch

    import paper_2305_05245_amd as pss

    keys = W.duplicate3_u32(1 << 22, seed=16).astype(np.uint64)
    ref = check_psrs(keys, 256, 256)
    assert np.count_nonzero(ref.sizes) <= 3 and ref.sizes.max() >= keys.size // 3
    d = to_device(keys)
    a, _, _ = pss.psrs_sort(d, n_blocks=256, n_parts=256, key_type="u64")
    b, _ = pss.sort(d, n_blocks=256, n_parts=256, key_type="u64")
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_psrs_empty_and_errors():
    import torch

    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd import PssError

    announce("psrs empty/errors")
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    out, _, sizes = pss.psrs_sort(e, n_blocks=4, n_parts=5, key_type="i64")
    torch.cuda.synchronize()
    assert out.numel() == 0 and sizes.cpu().tolist() == [0] * 5
    x = torch.zeros(100, dtype=torch.int64, device="cuda")
    with pytest.raises(PssError):
        pss.psrs_sort(x, n_blocks=0, n_parts=4)
    with pytest.raises(PssError):
        pss.psrs_sort(x, n_blocks=4, n_parts=0)


@pytest.mark.parametrize("n,n_b,n_p", [(100003, 7, 13), (50000, 300, 3), (20000, 2048, 5),
                                       (1 << 18, 100, 7), (5, 4, 9), (1 << 20, 64, 64)])
@pytest.mark.parametrize("kind", ["uniform", "dup"])
def test_merge_by_sort(n, n_b, n_p, kind):
    """Step 4 by sorting each gathered chunk (Section 2.2) gives the same
    output as the merge, for exact-splitting and regular-sampling pivots,
    keys only and stable key-value."""
    import torch

    import paper_2305_05245_amd as pss

    dtype = np.int64 if kind == "uniform" else np.uint32
    keys = seeded_keys(dtype, n, n + 7 * n_b, kind)
    vals = np.arange(n, dtype=np.uint32)
    kt = KEY_OF_DTYPE[keys.dtype]
    announce("merge by sort", keys.dtype.name, n, n_b, n_p)
    ref = oracle.pses(keys, n_b, n_p, vals=vals)
    pss.set_merge_method("sort")
    try:
        d, dv = to_device(keys), to_device(vals)
        k1, _ = pss.sort(d, n_blocks=n_b, n_parts=n_p, key_type=kt)
        k2, v2 = pss.sort(d, dv, n_blocks=n_b, n_parts=n_p, key_type=kt)
        k3, v3, _ = pss.psrs_sort(d, dv, n_blocks=n_b, n_parts=n_p, key_type=kt)
        torch.cuda.synchronize()
    finally:
        pss.set_merge_method("pairwise")
    for k in (k1, k2, k3):
        assert same_bits(from_device(k, keys.dtype), ref.keys)
    for v in (v2, v3):
        assert np.array_equal(from_device(v, np.uint32), ref.vals)
    assert pss.device_check() == 0


@pytest.mark.parametrize("n,n_b,n_p", [(1 << 22, 16, 16), ((1 << 22) + 12345, 37, 29),
                                       (1 << 23, 64, 64), ((1 << 21) + 7, 5, 100),
                                       ((1 << 23) + 4321, 100, 77), (1 << 24, 256, 256)])
@pytest.mark.parametrize("kind", ["uniform", "dup"])
def test_single_level_sampled_search(n, n_b, n_p, kind):
    """At most 256 blocks of at least 2^16 keys: the partition search of the
    single level starts from the blocks' merged samples (up to 64 blocks in
    the one-lane-per-run kernel, more in the one with per-run counts in LDS;
    block lengths that are not multiples of the sample stride included).  Sorted output (PSES and
    PSRS, keys only and stable key-value) against the oracle; pss_splitters
    keeps the full search, so its intermediates check that path too."""
    import torch

    import paper_2305_05245_amd as pss
    from test_gpu_parity import check_paper

    dtype = np.int64 if kind == "uniform" else np.uint32
    keys = seeded_keys(dtype, n, n + 3 * n_b, kind)
    vals = np.arange(n, dtype=np.uint32)
    kt = KEY_OF_DTYPE[keys.dtype]
    if n_b <= 128:
        check_paper(keys, n_b, n_p)
        ref = oracle.pses(keys, n_b, n_p, vals=vals)
    else:
        # the PSES oracle's pivot search grows with n_B^2 (over a minute
        # here); the sorted output is unique, so the PSRS oracle's serves
        ref = oracle.psrs(keys, n_b, n_p, vals=vals)
        announce("sampled single level", n, n_b, n_p)
        k0, _ = pss.sort(to_device(keys), n_blocks=n_b, n_parts=n_p, key_type=kt)
        torch.cuda.synchronize()
        assert same_bits(from_device(k0, keys.dtype), ref.keys)
    announce("sampled single level kv", n, n_b, n_p)
    d, dv = to_device(keys), to_device(vals)
    k1, v1 = pss.sort(d, dv, n_blocks=n_b, n_parts=n_p, key_type=kt)
    torch.cuda.synchronize()
    assert same_bits(from_device(k1, keys.dtype), ref.keys)
    assert np.array_equal(from_device(v1, np.uint32), ref.vals)
    check_psrs(keys, n_b, n_p, vals=vals)
