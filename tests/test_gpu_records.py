"""GPU parity of the record sort (Table 1's Pair and Particle: fixed-size
records sorted stably by a key field) against the oracle, byte for byte, on
Pair- and Particle-shaped layouts, keys at other offsets and of other types,
duplicate-heavy keys, sizes spanning many tiles, and the argument checks."""
import numpy as np
import pytest

import oracle
from gpu_util import announce

pytestmark = pytest.mark.gpu

NP = {"u64": np.uint64, "f64": np.float64, "i32": np.int32, "f32": np.float32, "i64": np.int64,
      "u32": np.uint32}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2305_05245_amd as pss

    pss._lib.load()


def make_records(n, rb, off, kt, dup, seed):
    rng = np.random.default_rng(seed)
    rec = rng.integers(0, 256, size=(n, rb), dtype=np.uint8)
    dt = np.dtype(NP[kt])
    if dup:
        keys = rng.integers(0, 3, size=n).astype(dt)
    elif dt.kind == "f":
        keys = rng.standard_normal(n).astype(dt)
    else:
        keys = rng.integers(np.iinfo(dt).min, np.iinfo(dt).max, size=n, dtype=dt, endpoint=True)
    rec[:, off:off + dt.itemsize] = keys.view(np.uint8).reshape(n, dt.itemsize)
    return rec


def check(n, rb, off, kt, dup, seed=1):
    import torch

    import paper_2305_05245_amd as pss

    announce("records", n, rb, off, kt, "dup" if dup else "")
    rec = make_records(n, rb, off, kt, dup, seed)
    want = oracle.sort_records(rec, kt, off)
    d = torch.from_numpy(rec).cuda()
    got = pss.sort_records(d, kt, key_offset=off)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)
    assert pss.device_check() == 0


@pytest.mark.parametrize("rb,off,kt", [(16, 0, "u64"), (96, 0, "u64"), (96, 88, "f64"),
                                       (12, 4, "i32"), (4, 0, "f32"), (40, 8, "i64"),
                                       (8, 4, "u32"), (4096, 4088, "u64")])
@pytest.mark.parametrize("n", [0, 1, 7, 8193, 100003])
def test_record_layouts(rb, off, kt, n):
    if rb * n > 64 << 20:
        n = (64 << 20) // rb
    check(n, rb, off, kt, dup=False, seed=n + rb)


@pytest.mark.parametrize("rb", [16, 96])
def test_records_duplicates_stable(rb):
    check(300001, rb, 0, "u64", dup=True, seed=rb)


def test_pair_and_particle_multi_pass():
    """Pair at 2^22 and Particle at 2^21 records: two or more merge passes."""
    check(1 << 22, 16, 0, "u64", dup=False, seed=5)
    check(1 << 21, 96, 0, "u64", dup=False, seed=6)


def test_record_argument_errors():
    import torch

    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd import PssError

    announce("records errors")
    x = torch.zeros((100, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(PssError):
        pss.sort_records(x, "u64", key_offset=12)      # key past the record end
    with pytest.raises(PssError):
        pss.sort_records(x, "u64", key_offset=4)       # misaligned key
    y = torch.zeros((100, 10), dtype=torch.uint8, device="cuda")
    with pytest.raises(PssError):
        pss.sort_records(y, "u32", key_offset=0)       # record size not a multiple of 4
    with pytest.raises(PssError):
        pss.sort_records(x, "u64", key_offset=0, out=x)  # in place
