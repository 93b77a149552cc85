"""No sort writes outside its own buffers.

Every buffer a sort is handed (workspace, outputs, partition sizes) sits
between two guard bands of poisoned bytes in one larger allocation; after the
sort, every guard byte must still hold the poison and the inputs must be
unchanged.  Shapes: twelve sorts of the kinds (four key types, keys only and
key-value, uniform and mod-1000 keys, 2^18 to 2^22 keys) that are otherwise
run on four streams at once, here one after another on one stream, ragged
small sizes and the paper's single level; batched segmented sorts with empty,
tile-sized and multi-pass segments under three tunings; the regular-sampling
variant; and record sorts with keys at the start, inside and at the end of a
record."""
import numpy as np
import pytest

from gpu_util import KEY_OF_DTYPE, POISON, announce, from_device, order_bits, to_device

pytestmark = pytest.mark.gpu

GUARD = 1 << 20  # bytes of poison on each side of every buffer


def _keys(rng, dtype, n, dup):
    if dup:
        raw = rng.integers(0, 1000, size=n).astype(np.uint64)
    else:
        raw = rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)
    if np.dtype(dtype).itemsize == 4:
        raw = (raw >> np.uint64(32)).astype(np.uint32) if not dup else raw.astype(np.uint32)
    return raw.view(dtype)


def _cases():
    rng = np.random.default_rng(77)
    out = []
    for s, dtype in enumerate([np.int64, np.uint64, np.float64, np.int32]):
        for j in range(3):
            n = int(rng.integers(1 << 18, 1 << 22))
            out.append((dtype, n, j == 1, (s + j) % 2 == 1, 0, 0))
    out += [(np.int64, 1, False, False, 0, 0), (np.uint32, 4097, True, True, 0, 0),
            (np.float32, 8193, False, False, 0, 0), (np.int64, 12289, False, True, 0, 0),
            (np.int64, 300_001, False, False, 37, 19), (np.uint64, 200_003, True, True, 64, 64)]
    return out


CASES = _cases()


class Guarded:
    """A device buffer of `nbytes` with GUARD poisoned bytes on each side."""

    def __init__(self, nbytes: int):
        import torch

        self.nbytes = int(nbytes)
        self.all = torch.full((self.nbytes + 2 * GUARD,), POISON, dtype=torch.uint8, device="cuda")
        self.inner = self.all[GUARD:GUARD + self.nbytes]

    def ptr(self) -> int:
        return self.all.data_ptr() + GUARD

    def guards_intact(self) -> bool:
        import torch

        lo, hi = self.all[:GUARD], self.all[GUARD + self.nbytes:]
        return bool((lo == POISON).all()) and bool((hi == POISON).all())


@pytest.mark.parametrize("case", range(len(CASES)))
def test_sort_writes_only_its_buffers(case):
    import torch

    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd import _lib

    dtype, n, dup, kv, nb, np_ = CASES[case]
    rng = np.random.default_rng(1000 + case)
    keys = _keys(rng, dtype, n, dup)
    vals = rng.permutation(n).astype(np.uint32) if kv else None
    kt = _lib.KEY_NAMES[KEY_OF_DTYPE[np.dtype(dtype)]]
    vt = _lib.VAL_U32 if kv else _lib.VAL_NONE
    announce("guards", np.dtype(dtype).name, n, "dup" if dup else "uniform",
             "kv" if kv else "keys", nb, np_)
    dk = to_device(keys)
    dv = to_device(vals) if kv else None
    kbytes = keys.itemsize * n
    ws = Guarded(max(_lib.workspace_bytes(kt, vt, n, nb, np_), 256))
    ko = Guarded(kbytes)
    vo = Guarded(4 * n) if kv else None
    ctx = pss._context(0)
    ctx.sort(kt, vt, dk.data_ptr(), ko.ptr(), dv.data_ptr() if kv else 0, vo.ptr() if kv else 0,
             n, nb, np_, ws.ptr(), ws.nbytes, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert pss.device_check() == 0
    assert ws.guards_intact(), "write outside the workspace"
    assert ko.guards_intact(), "write outside the key output"
    if kv:
        assert vo.guards_intact(), "write outside the value output"
    assert from_device(dk, dtype).tobytes() == keys.tobytes(), "input keys changed"
    if kv:
        assert np.array_equal(from_device(dv, np.uint32), vals), "input values changed"
    perm = np.argsort(order_bits(keys), kind="stable")
    got = ko.inner.cpu().numpy().view(dtype)
    assert got.tobytes() == keys[perm].tobytes()
    if kv:
        assert np.array_equal(vo.inner.cpu().numpy().view(np.uint32), vals[perm])


SEG_CASES = [
    (np.int64, [0, 1, 4096, 4097, 8192, 100_000, 0, (1 << 20) + 3, 17, 1 << 21], False, None),
    (np.uint64, [5, 0, 2048, 2049, (1 << 19) + 1, 4095, 12_289, 0], True,
     {"small_max_2k": 2048, "small_max_4k": 4096, "fan_log2": 6}),
    (np.float32, "loguniform", True, {"small_max_2k": 0, "small_max_4k": 0}),
]


@pytest.mark.parametrize("case", range(len(SEG_CASES)))
def test_segmented_sort_writes_only_its_buffers(case):
    import torch

    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd import _lib

    dtype, sizes, kv, tuning = SEG_CASES[case]
    rng = np.random.default_rng(2000 + case)
    if sizes == "loguniform":
        sizes = np.rint(np.exp2(rng.uniform(0, 16, size=300))).astype(np.int64).tolist()
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    n = int(offs[-1])
    keys = _keys(rng, dtype, n, case == 1)
    vals = rng.permutation(n).astype(np.uint32) if kv else None
    kt = _lib.KEY_NAMES[KEY_OF_DTYPE[np.dtype(dtype)]]
    vt = _lib.VAL_U32 if kv else _lib.VAL_NONE
    tu = _lib.Tuning.from_dict(tuning, max(sizes)) if tuning is not None else None
    announce("segmented guards", np.dtype(dtype).name, len(sizes), n, "kv" if kv else "keys", tuning)
    dk = to_device(keys)
    dv = to_device(vals) if kv else None
    d_offs = torch.from_numpy(offs).cuda()
    ws = Guarded(max(_lib.segmented_workspace_bytes(kt, vt, n, len(sizes), tu), 256))
    ko = Guarded(keys.itemsize * n)
    vo = Guarded(4 * n) if kv else None
    ctx = pss._context(0)
    ctx.segmented_sort(kt, vt, dk.data_ptr(), ko.ptr(), dv.data_ptr() if kv else 0,
                       vo.ptr() if kv else 0, n, d_offs.data_ptr(), len(sizes), tu, ws.ptr(),
                       ws.nbytes, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert pss.device_check() == 0
    assert ws.guards_intact(), "write outside the workspace"
    assert ko.guards_intact(), "write outside the key output"
    if kv:
        assert vo.guards_intact(), "write outside the value output"
    assert from_device(dk, dtype).tobytes() == keys.tobytes(), "input keys changed"
    assert np.array_equal(d_offs.cpu().numpy(), offs), "segment offsets changed"
    gk = ko.inner.cpu().numpy().view(dtype)
    gv = vo.inner.cpu().numpy().view(np.uint32) if kv else None
    for i in range(len(sizes)):
        lo, hi = int(offs[i]), int(offs[i + 1])
        perm = np.argsort(order_bits(keys[lo:hi]), kind="stable")
        assert gk[lo:hi].tobytes() == keys[lo:hi][perm].tobytes(), i
        if kv:
            assert np.array_equal(gv[lo:hi], vals[lo:hi][perm]), i


@pytest.mark.parametrize("n,n_b,n_p,kv", [(300_001, 37, 19, False), (200_003, 64, 64, True)])
def test_psrs_sort_writes_only_its_buffers(n, n_b, n_p, kv):
    import torch

    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd import _lib

    rng = np.random.default_rng(n)
    keys = _keys(rng, np.uint64, n, dup=kv)
    vals = np.arange(n, dtype=np.uint32) if kv else None
    vt = _lib.VAL_U32 if kv else _lib.VAL_NONE
    announce("psrs guards", n, n_b, n_p, "kv" if kv else "keys")
    dk = to_device(keys)
    dv = to_device(vals) if kv else None
    ws = Guarded(max(_lib.psrs_workspace_bytes(_lib.U64, vt, n, n_b, n_p), 256))
    ko = Guarded(8 * n)
    vo = Guarded(4 * n) if kv else None
    sizes = Guarded(8 * n_p)
    pss._context(0).psrs_sort(_lib.U64, vt, dk.data_ptr(), ko.ptr(), dv.data_ptr() if kv else 0,
                              vo.ptr() if kv else 0, n, n_b, n_p, sizes.ptr(), ws.ptr(), ws.nbytes,
                              torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert pss.device_check() == 0
    for name, g in (("workspace", ws), ("key output", ko), ("partition sizes", sizes)) + \
            ((("value output", vo),) if kv else ()):
        assert g.guards_intact(), f"write outside the {name}"
    assert from_device(dk, np.uint64).tobytes() == keys.tobytes(), "input keys changed"
    gk = ko.inner.cpu().numpy().view(np.uint64)
    assert np.array_equal(gk, np.sort(keys))
    assert int(sizes.inner.cpu().numpy().view(np.uint64).sum()) == n
    if kv:
        gv = vo.inner.cpu().numpy().view(np.uint32)
        assert np.array_equal(keys[gv], gk), "values do not carry their keys"
        assert np.array_equal(np.sort(gv), vals)


@pytest.mark.parametrize("n,rb,off", [(100_003, 16, 0), (50_001, 96, 8), (4097, 24, 16)])
def test_record_sort_writes_only_its_buffers(n, rb, off):
    import torch

    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd import _lib

    rng = np.random.default_rng(rb)
    rec = rng.integers(0, 256, size=(n, rb), dtype=np.uint8)
    keys = rng.integers(0, 50, size=n).astype(np.uint64)  # duplicates: stability shows
    rec[:, off:off + 8] = keys.view(np.uint8).reshape(n, 8)
    announce("record guards", n, rb, off)
    d_in = torch.from_numpy(rec.reshape(-1).copy()).cuda()
    ws = Guarded(max(_lib.records_workspace_bytes(_lib.U64, n), 256))
    out = Guarded(n * rb)
    pss._context(0).sort_records(_lib.U64, d_in.data_ptr(), out.ptr(), n, rb, off, ws.ptr(),
                                 ws.nbytes, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert pss.device_check() == 0
    assert ws.guards_intact(), "write outside the workspace"
    assert out.guards_intact(), "write outside the record output"
    assert np.array_equal(d_in.cpu().numpy(), rec.reshape(-1)), "input records changed"
    perm = np.argsort(keys, kind="stable")
    assert np.array_equal(out.inner.cpu().numpy().reshape(n, rb), rec[perm])
