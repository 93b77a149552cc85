"""Independent plain definitions used by the tests to pin the oracle.

These are written from the problem statement, not from the oracle: the sorted
output is the stable ascending sort under the key order; the order of floats is
IEEE totalOrder, expressed here through the signed-integer form of the bit
pattern (a negative pattern has its magnitude bits inverted), which differs
from both the oracle's predicate and the GPU library's key map.
"""
from __future__ import annotations

import numpy as np


def order_keys(keys: np.ndarray) -> np.ndarray:
    """int64/uint64 array whose numeric order is the key order of `keys`."""
    k = np.ascontiguousarray(keys)
    if k.dtype == np.float64:
        s = k.view(np.int64)
        return np.where(s < 0, s ^ np.int64(0x7FFFFFFFFFFFFFFF), s)
    if k.dtype == np.float32:
        s = k.view(np.int32).astype(np.int64)
        return np.where(s < 0, s ^ np.int64(0x7FFFFFFF), s)
    if k.dtype in (np.uint64,):
        return k
    return k.astype(np.int64)


def stable_order(keys: np.ndarray) -> np.ndarray:
    """Permutation that sorts `keys` ascending, ties by input index."""
    return np.argsort(order_keys(keys), kind="stable")


def block_bounds(n: int, n_blocks: int):
    L = -(-n // n_blocks) if n else 0
    return [(min(b * L, n), min((b + 1) * L, n)) for b in range(n_blocks)]


def expected_split(keys: np.ndarray, n_blocks: int, n_parts: int) -> np.ndarray:
    """s[b][k] = number of elements of block b among the r_k first elements of
    the stable sorted order (r_k = floor(k N / n_P)); ties therefore go to the
    lowest block, earliest position first."""
    n = keys.size
    perm = stable_order(keys)
    pos_in_sorted = np.empty(n, dtype=np.int64)
    pos_in_sorted[perm] = np.arange(n)
    out = np.zeros((n_blocks, n_parts + 1), dtype=np.uint64)
    for b, (lo, hi) in enumerate(block_bounds(n, n_blocks)):
        p = np.sort(pos_in_sorted[lo:hi])
        for k in range(n_parts + 1):
            r = k * n // n_parts
            out[b, k] = np.searchsorted(p, r, side="left")
    return out


def expected_pivots_counts(keys: np.ndarray, n_parts: int):
    """Canonical P_k = element of rank r_k - 1 and c_k = r_k - |{x < P_k}|,
    with |{x < P_k}| counted directly."""
    n = keys.size
    ok = order_keys(keys)
    srt = np.sort(ok, kind="stable")
    perm = stable_order(keys)
    piv, cnt, valid = [], [], []
    for k in range(1, n_parts):
        r = k * n // n_parts
        if r == 0:
            piv.append(None)
            cnt.append(0)
            valid.append(False)
            continue
        v = srt[r - 1]
        lt = int(np.count_nonzero(ok < v))
        le = int(np.count_nonzero(ok <= v))
        assert lt <= r <= le
        piv.append(keys[perm[r - 1]])
        cnt.append(r - lt)
        valid.append(True)
    return piv, cnt, valid
