"""No sort writes outside its own buffers.

Every buffer a sort is handed (workspace, key output, value output) sits
between two guard bands of poisoned bytes in one larger allocation; after the
sort, every guard byte must still hold the poison and the inputs must be
unchanged.  Shapes: the twelve sorts (four key types, keys only and key-value,
uniform and mod-1000 keys, 2^18 to 2^22 keys) that are otherwise run on four
streams at once, here one after another on one stream, plus ragged small
sizes and the paper's single level."""
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
