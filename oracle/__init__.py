"""Oracle: TEST INFRASTRUCTURE ONLY.

A plain, sequential CPU implementation of the paper's four-step parallel
samplesort with exact splitting (PSES; arXiv 2305.05245, Section 2, Section 2.3
Eq. 1 and Eq. 2), and of the same steps with regular-sampling pivots (PSRS,
Section 2.3), written in C (``pses_oracle.c``) and wrapped here with ctypes
and numpy.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import this package; the GPU library never does.

Everything here works on raw key bits: floats are compared by IEEE totalOrder
written out from its definition, never by a floating-point compare.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pses_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

# key-type codes of the oracle (same numbering as the public library's enum)
DTYPES = {
    "u32": (0, np.uint32),
    "i32": (1, np.int32),
    "u64": (2, np.uint64),
    "i64": (3, np.int64),
    "f32": (4, np.float32),
    "f64": (5, np.float64),
}
BITS_VIEW = {4: np.uint32, 8: np.uint64}

ERRORS = {
    1: "bad arguments",
    2: "out of memory",
    10: "Eq. 1 violated",
    11: "c_k out of range",
    12: "sum of split positions != r_k",
    13: "split positions not monotone",
    14: "offset O_k != r_k",
    15: "partition size not floor/ceil(N/n_P)",
    16: "no pivot candidate",
    17: "sorted indices are not a permutation",
}


def build(force: bool = False) -> str:
    """Compile pses_oracle.c with gcc into liboracle.so (next to the source)."""
    with _lock:
        if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
        ):
            tmp = _LIB_PATH + f".tmp{os.getpid()}"
            subprocess.check_call(
                ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                 "-o", tmp, _SRC]
            )
            os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_HP_SRC = os.path.join(_HERE, "pses_host_parallel.c")
_HP_PATH = os.path.join(_HERE, "libhostpar.so")
_hp = None


def build_host_parallel(force: bool = False) -> str:
    """Compile the OpenMP host baseline (pses_host_parallel.c, which includes
    the oracle's source) into libhostpar.so."""
    with _lock:
        newest = max(os.path.getmtime(_HP_SRC), os.path.getmtime(_SRC))
        if force or not os.path.exists(_HP_PATH) or os.path.getmtime(_HP_PATH) < newest:
            tmp = _HP_PATH + f".tmp{os.getpid()}"
            subprocess.check_call(
                ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
                 "-o", tmp, _HP_SRC]
            )
            os.replace(tmp, _HP_PATH)
    return _HP_PATH


def host_parallel_pses(keys: np.ndarray, n_blocks: int, n_parts: int) -> np.ndarray:
    """The host baseline: the oracle's steps with their loops over blocks,
    pivots and partitions shared among OpenMP threads (keys only)."""
    global _hp
    if _hp is None:
        build_host_parallel()
        lib = ctypes.CDLL(_HP_PATH)
        lib.host_parallel_pses.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p,
                                           ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
        lib.host_parallel_pses.restype = ctypes.c_int
        lib.host_parallel_threads.restype = ctypes.c_int
        _hp = lib
    keys = np.ascontiguousarray(keys)
    name = {np.dtype(v[1]): k for k, v in DTYPES.items()}[keys.dtype]
    out = np.empty_like(keys)
    rc = _hp.host_parallel_pses(dtype_code(name), keys.size, keys.ctypes.data_as(ctypes.c_void_p),
                                n_blocks, n_parts, out.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise RuntimeError(f"host_parallel_pses failed: {rc}")
    return out


def host_parallel_threads() -> int:
    host_parallel_pses(np.zeros(1, dtype=np.int64), 1, 1)  # loads the library
    return int(_hp.host_parallel_threads())


def bind(path: str):
    """ctypes handle for a compiled oracle at `path` (the default build, or a
    mutated copy compiled by the tests that check the pins catch mistakes)."""
    lib = ctypes.CDLL(path)
    u64, u32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
    lib.oracle_compare.argtypes = [ctypes.c_int, u64, u64]
    lib.oracle_compare.restype = ctypes.c_int
    lib.oracle_pses.argtypes = [ctypes.c_int, u64, vp, vp, u32, u32, vp, vp,
                                vp, vp, vp, vp, vp, ctypes.c_int]
    lib.oracle_pses.restype = ctypes.c_int
    lib.oracle_psrs.argtypes = [ctypes.c_int, u64, vp, vp, u32, u32, vp, vp,
                                vp, vp, vp, vp, vp, vp]
    lib.oracle_psrs.restype = ctypes.c_int
    lib.oracle_sort_records.argtypes = [ctypes.c_int, u64, vp, u32, u32, u32, u32, vp]
    lib.oracle_sort_records.restype = ctypes.c_int
    lib.oracle_rank_counts.argtypes = [ctypes.c_int, u64, vp, u64, vp, vp]
    lib.oracle_rank_counts.restype = None
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = bind(_LIB_PATH)
    return _lib


def dtype_code(dtype: str) -> int:
    return DTYPES[dtype][0]


def to_bits(x) -> int:
    """Raw bits of one numpy scalar as a Python int (zero-extended)."""
    a = np.asarray(x)
    return int(a.view(BITS_VIEW[a.dtype.itemsize]))


def compare(dtype: str, a_bits: int, b_bits: int, lib=None) -> int:
    """Step O0: -1, 0, +1 for the key order of `dtype` on raw bits."""
    return int((lib or _load()).oracle_compare(dtype_code(dtype), a_bits, b_bits))


@dataclass
class PsesResult:
    keys: np.ndarray          # sorted output
    vals: np.ndarray | None   # payload in output order (stable by input index)
    blocks: np.ndarray        # step 1: concatenation of the sorted blocks
    pivots: np.ndarray        # step 2: canonical P_1..P_{n_P-1} (raw key dtype)
    counts: np.ndarray        # step 2: c_1..c_{n_P-1} (uint64)
    split: np.ndarray         # step 3: [n_B, n_P+1] uint64 boundaries
    offsets: np.ndarray       # step 4: O_0..O_{n_P} (uint64)


def pses(keys: np.ndarray, n_blocks: int, n_parts: int, vals: np.ndarray | None = None,
         merge_kind: int = 0, lib=None) -> PsesResult:
    """Run the whole sequential method on host arrays.  Raises on any violated
    invariant (Eq. 1, Eq. 2 range, split sums, offsets, partition sizes)."""
    keys = np.ascontiguousarray(keys)
    name = {np.dtype(v[1]): k for k, v in DTYPES.items()}[keys.dtype]
    code = dtype_code(name)
    n = keys.size
    out = np.empty_like(keys)
    blocks = np.empty_like(keys)
    pivots = np.zeros(max(n_parts - 1, 0), dtype=keys.dtype)
    counts = np.zeros(max(n_parts - 1, 0), dtype=np.uint64)
    split = np.zeros((n_blocks, n_parts + 1), dtype=np.uint64)
    offsets = np.zeros(n_parts + 1, dtype=np.uint64)
    vin = vout = None
    if vals is not None:
        vin = np.ascontiguousarray(vals, dtype=np.uint32)
        assert vin.size == n
        vout = np.empty_like(vin)

    def p(a):
        return None if a is None else a.ctypes.data_as(ctypes.c_void_p)

    rc = (lib or _load()).oracle_pses(code, n, p(keys), p(vin), n_blocks, n_parts, p(out), p(vout),
                             p(blocks), p(pivots) if pivots.size else None,
                             p(counts) if counts.size else None, p(split), p(offsets),
                             merge_kind)
    if rc != 0:
        raise RuntimeError(f"oracle_pses failed: {ERRORS.get(rc, rc)}")
    return PsesResult(out, vout, blocks, pivots, counts, split, offsets)


@dataclass
class PsrsResult:
    keys: np.ndarray          # sorted output
    vals: np.ndarray | None   # payload in output order (stable by input index)
    blocks: np.ndarray        # step 1: concatenation of the sorted blocks
    samples: np.ndarray       # step 2: the sorted regular samples S
    pivots: np.ndarray        # step 2: P_1..P_{n_P-1} (raw key dtype)
    split: np.ndarray         # step 3: [n_B, n_P+1] uint64 boundaries
    offsets: np.ndarray       # step 4: O_0..O_{n_P} (uint64), O_k = |{x <= P_k}|

    @property
    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64))


def psrs(keys: np.ndarray, n_blocks: int, n_parts: int, vals: np.ndarray | None = None,
         lib=None) -> PsrsResult:
    """The four steps with PSRS (regular-sampling) pivots on host arrays."""
    keys = np.ascontiguousarray(keys)
    name = {np.dtype(v[1]): k for k, v in DTYPES.items()}[keys.dtype]
    code = dtype_code(name)
    n = keys.size
    out = np.empty_like(keys)
    blocks = np.empty_like(keys)
    samples = np.zeros(max(n_blocks * (n_parts - 1), 1), dtype=keys.dtype)
    ns = ctypes.c_uint64()
    pivots = np.zeros(max(n_parts - 1, 0), dtype=keys.dtype)
    split = np.zeros((n_blocks, n_parts + 1), dtype=np.uint64)
    offsets = np.zeros(n_parts + 1, dtype=np.uint64)
    vin = vout = None
    if vals is not None:
        vin = np.ascontiguousarray(vals, dtype=np.uint32)
        assert vin.size == n
        vout = np.empty_like(vin)

    def p(a):
        return None if a is None else a.ctypes.data_as(ctypes.c_void_p)

    rc = (lib or _load()).oracle_psrs(code, n, p(keys), p(vin), n_blocks, n_parts, p(out), p(vout),
                                      p(blocks), p(samples), ctypes.byref(ns),
                                      p(pivots) if pivots.size else None, p(split), p(offsets))
    if rc != 0:
        raise RuntimeError(f"oracle_psrs failed: {ERRORS.get(rc, rc)}")
    return PsrsResult(out, vout, blocks, samples[:ns.value].copy(), pivots, split, offsets)


def sort_records(records: np.ndarray, key_dtype: str, key_offset: int, n_blocks: int = 16,
                 n_parts: int = 16, lib=None) -> np.ndarray:
    """Records (a 2-D uint8 array, one row per record) sorted stably by the key
    of type `key_dtype` at byte `key_offset` of each row."""
    rec = np.ascontiguousarray(records, dtype=np.uint8)
    n, rb = rec.shape
    out = np.empty_like(rec)
    rc = (lib or _load()).oracle_sort_records(dtype_code(key_dtype), n,
                                              rec.ctypes.data_as(ctypes.c_void_p), rb, key_offset,
                                              n_blocks, n_parts,
                                              out.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise RuntimeError(f"oracle_sort_records failed: {ERRORS.get(rc, rc)}")
    return out


def rank_counts(keys: np.ndarray, v, lib=None) -> tuple[int, int]:
    """|{x < v}| and |{x <= v}| over `keys` by a linear pass (Eq. 1's counts)."""
    keys = np.ascontiguousarray(keys)
    name = {np.dtype(t[1]): k for k, t in DTYPES.items()}[keys.dtype]
    lt = ctypes.c_uint64()
    le = ctypes.c_uint64()
    (lib or _load()).oracle_rank_counts(dtype_code(name), keys.size,
                               keys.ctypes.data_as(ctypes.c_void_p),
                               to_bits(np.asarray(v, dtype=keys.dtype)),
                               ctypes.byref(lt), ctypes.byref(le))
    return int(lt.value), int(le.value)
