"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and lays out arrays: it holds none of the
sorting method's arithmetic, so both the oracle and the GPU library can be fed
the same bytes.  Every generator is deterministic in its seed.

The shapes follow the paper's inputs (Table 1 of arXiv 2305.05245: uniform
integers, uniform floats in [0, 1), almost-sorted integers, three distinct
values, key-index pairs) scaled to the configurations this project measures.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _raw64(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniformly random 64-bit words."""
    return rng.bit_generator.random_raw(n).astype(np.uint64, copy=False)


# ----------------------------------------------------------------- integers
def uniform_i32(n: int, seed: int = 1) -> np.ndarray:
    """Uniform over the whole int32 range."""
    return (_raw64(_rng(seed), n) >> np.uint64(32)).astype(np.uint32).view(np.int32)


def uniform_u32(n: int, seed: int = 1) -> np.ndarray:
    return (_raw64(_rng(seed), n) >> np.uint64(32)).astype(np.uint32)


def uniform_i64(n: int, seed: int = 2) -> np.ndarray:
    """Uniform over the whole int64 range."""
    return _raw64(_rng(seed), n).view(np.int64)


def uniform_u64(n: int, seed: int = 2) -> np.ndarray:
    return _raw64(_rng(seed), n)


def mod1000_i64(n: int, seed: int = 3) -> np.ndarray:
    """Uniform 64-bit words reduced mod 1000: heavy duplicates in [0, 999]."""
    return (_raw64(_rng(seed), n) % np.uint64(1000)).astype(np.int64)


def sorted_i64(n: int, seed: int = 4) -> np.ndarray:
    return np.arange(n, dtype=np.int64)


def reverse_i64(n: int, seed: int = 5) -> np.ndarray:
    return np.arange(n - 1, -1, -1, dtype=np.int64)


def swapped_i64(n: int, seed: int = 6, fraction: float = 0.01) -> np.ndarray:
    """0..n-1 with floor(fraction*n) transpositions of uniformly drawn position
    pairs, applied one after another."""
    a = np.arange(n, dtype=np.int64)
    m = int(fraction * n)
    if n < 2 or m == 0:
        return a
    rng = _rng(seed)
    i = rng.integers(0, n, size=m)
    j = rng.integers(0, n, size=m)
    _apply_transpositions(a, i, j)
    return a


def _apply_transpositions(a: np.ndarray, i: np.ndarray, j: np.ndarray, chunk: int = 1 << 12):
    # Transpositions are applied strictly in order.  A chunk whose position
    # pairs touch no position twice can be applied at once; others fall back to
    # a plain loop.
    for s in range(0, i.size, chunk):
        ii, jj = i[s:s + chunk], j[s:s + chunk]
        touched = np.concatenate([ii, jj])
        if np.unique(touched).size == touched.size:
            a[ii], a[jj] = a[jj].copy(), a[ii].copy()
        else:
            for x, y in zip(ii.tolist(), jj.tolist()):
                a[x], a[y] = a[y], a[x]


def duplicate3_u32(n: int, seed: int = 16) -> np.ndarray:
    """Uniform over {0, 1, 2} (the paper's Duplicate3)."""
    return (_raw64(_rng(seed), n) % np.uint64(3)).astype(np.uint32)


def almost_sorted_u32(n: int, seed: int = 17) -> np.ndarray:
    """0..n-1 with floor(sqrt(n)) random transpositions (the paper's
    AlmostSorted)."""
    a = np.arange(n, dtype=np.uint32)
    m = int(np.sqrt(n))
    if n < 2 or m == 0:
        return a
    rng = _rng(seed)
    _apply_transpositions(a, rng.integers(0, n, size=m), rng.integers(0, n, size=m))
    return a


# ------------------------------------------------------------------- floats
def uniform01_f64(n: int, seed: int = 7) -> np.ndarray:
    return _rng(seed).random(n)


def normal_f64(n: int, seed: int = 8) -> np.ndarray:
    return _rng(seed).standard_normal(n)


def allequal_f64(n: int, seed: int = 9) -> np.ndarray:
    return np.full(n, 1.0, dtype=np.float64)


def organpipe_f64(n: int, seed: int = 10) -> np.ndarray:
    i = np.arange(n, dtype=np.int64)
    return np.minimum(i, n - 1 - i).astype(np.float64)


SPECIAL_NAN_BITS = (0x7FF8000000000000, 0xFFF8000000000000, 0x7FF0000000000001)


def normal_specials_f64(n: int, seed: int = 11, fraction: float = 0.001) -> np.ndarray:
    """Standard normal with floor(fraction*n) positions (drawn without
    replacement) overwritten in equal thirds by -0.0, +inf and NaN; the NaNs
    are split over a positive quiet, a negative quiet and a signalling
    pattern."""
    rng = _rng(seed)
    x = rng.standard_normal(n)
    m = int(fraction * n)
    if m == 0:
        return x
    pos = rng.choice(n, size=m, replace=False)
    t = m // 3
    x[pos[:t]] = -0.0
    x[pos[t:2 * t]] = np.inf
    bits = x.view(np.uint64)
    nan_pos = pos[2 * t:]
    pats = np.array(SPECIAL_NAN_BITS, dtype=np.uint64)
    bits[nan_pos] = pats[np.arange(nan_pos.size) % 3]
    return x


def uniform01_f32(n: int, seed: int = 18) -> np.ndarray:
    return _rng(seed).random(n, dtype=np.float32)


# ------------------------------------------------------------- key + value
def index_values(n: int) -> np.ndarray:
    """The payload used for key-value sorts: each element's input index."""
    return np.arange(n, dtype=np.uint32)


# --------------------------------------------------------- segmented batch
def segment_sizes_loguniform(n_segs: int = 4096, lo_exp: float = 6.0, hi_exp: float = 20.0,
                             seed: int = 12) -> np.ndarray:
    """Segment sizes round(2**U), U ~ Uniform[lo_exp, hi_exp]."""
    u = _rng(seed).uniform(lo_exp, hi_exp, size=n_segs)
    return np.rint(np.exp2(u)).astype(np.int64)


def segment_offsets(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(sizes.size + 1, dtype=np.uint64)
    np.cumsum(sizes, out=off[1:])
    return off


# ------------------------------------------------------------ serving load
def serving_requests(n_req: int, rate_per_s: float, seed_arrival: int = 14,
                     seed_size: int = 15, seed_keys: int = 16,
                     mu_log2: float = 16.0, sigma: float = 1.5,
                     lo: int = 1 << 10, hi: int = 1 << 24):
    """Poisson arrivals (exponential gaps), lognormal sizes clipped to
    [lo, hi], and per request a flag choosing uniform (False) or
    duplicate-heavy {0, 1, 2} (True) keys.  Returns (arrival_s, sizes, dup)."""
    gaps = _rng(seed_arrival).exponential(1.0 / rate_per_s, size=n_req)
    arrival = np.cumsum(gaps)
    sz = _rng(seed_size).lognormal(mean=mu_log2 * np.log(2.0), sigma=sigma, size=n_req)
    sizes = np.clip(np.rint(sz), lo, hi).astype(np.int64)
    dup = _rng(seed_keys).random(n_req) < 0.5
    return arrival, sizes, dup


def request_keys(size: int, dup: bool, seed: int) -> np.ndarray:
    """uint64 keys for one request: uniform or over {0, 1, 2}."""
    w = _raw64(_rng(seed), size)
    return w % np.uint64(3) if dup else w
