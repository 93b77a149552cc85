"""Helpers for the GPU parity tests: moving seeded numpy inputs to the device
and back, and exact property checks usable at any size."""
from __future__ import annotations

import sys

import numpy as np

KEY_OF_DTYPE = {np.dtype(np.uint32): "u32", np.dtype(np.int32): "i32",
                np.dtype(np.uint64): "u64", np.dtype(np.int64): "i64",
                np.dtype(np.float32): "f32", np.dtype(np.float64): "f64"}


def announce(*parts) -> None:
    """Name the case before any GPU work, so a fault can be attributed."""
    print("[case]", *parts, file=sys.stderr, flush=True)


def to_device(a: np.ndarray):
    import torch

    a = np.ascontiguousarray(a)
    view = {4: np.int32, 8: np.int64}[a.dtype.itemsize]
    return torch.from_numpy(a.view(view).copy()).cuda()


def from_device(t, dtype) -> np.ndarray:
    return t.cpu().numpy().view(dtype)


POISON = 0xAB


def poisoned_workspace(nbytes: int):
    """A device workspace whose every byte is 0xAB, so that a kernel reading
    scratch memory it has not written first yields a mismatch instead of
    whatever an earlier call left there."""
    import torch

    return torch.full((max(int(nbytes), 256),), POISON, dtype=torch.uint8, device="cuda")


def gpu_sort(keys: np.ndarray, vals: np.ndarray | None = None, n_blocks: int = 0, n_parts: int = 0):
    """Sort on the device through the C ABI, with a poisoned workspace; the
    device error word must stay clear."""
    import torch

    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd import _lib

    kt = KEY_OF_DTYPE[keys.dtype]
    dk = to_device(keys)
    dv = to_device(vals.astype(np.uint32)) if vals is not None else None
    ws = poisoned_workspace(_lib.workspace_bytes(_lib.KEY_NAMES[kt],
                                                 _lib.VAL_U32 if vals is not None else _lib.VAL_NONE,
                                                 keys.size, n_blocks, n_parts))
    out, vout = pss.sort(dk, dv, n_blocks=n_blocks, n_parts=n_parts, key_type=kt, workspace=ws)
    torch.cuda.synchronize()
    assert pss.device_check() == 0, "device error word set"
    ko = from_device(out, keys.dtype)
    vo = from_device(vout, np.uint32) if vout is not None else None
    return ko, vo


def order_bits(keys: np.ndarray) -> np.ndarray:
    """Signed integers ordered like the keys (floats: IEEE totalOrder), written
    independently of the library's key map."""
    k = np.ascontiguousarray(keys)
    if k.dtype == np.float64:
        s = k.view(np.int64)
        return np.where(s < 0, s ^ np.int64(0x7FFFFFFFFFFFFFFF), s)
    if k.dtype == np.float32:
        s = k.view(np.int32).astype(np.int64)
        return np.where(s < 0, s ^ np.int64(0x7FFFFFFF), s)
    if k.dtype == np.uint64:
        return (k ^ np.uint64(1 << 63)).view(np.int64)
    return k.astype(np.int64)


def is_sorted(keys: np.ndarray) -> bool:
    o = order_bits(keys)
    return bool(np.all(o[1:] >= o[:-1]))


def multiset_signature(keys: np.ndarray) -> tuple:
    """Order-independent signature of the multiset of key bit patterns: count,
    and two sums of different 64-bit mixes (mod 2^64)."""
    b = np.ascontiguousarray(keys).view({4: np.uint32, 8: np.uint64}[keys.dtype.itemsize])
    x = b.astype(np.uint64)
    with np.errstate(over="ignore"):
        m1 = (x ^ (x >> np.uint64(31))) * np.uint64(0x9E3779B97F4A7C15)
        m1 ^= m1 >> np.uint64(29)
        m2 = (x + np.uint64(0x632BE59BD9B4E019)) * np.uint64(0xBF58476D1CE4E5B9)
        m2 ^= m2 >> np.uint64(32)
        return (int(x.size), int(m1.sum(dtype=np.uint64)), int(m2.sum(dtype=np.uint64)))
