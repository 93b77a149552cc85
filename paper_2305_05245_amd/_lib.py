"""ctypes binding of libpss (include/pss.h): argument marshalling only.

Every step of the sort runs in the HIP kernels of libpss.so.  There is no CPU
fallback: if the library has not been built, loading it raises.
"""
from __future__ import annotations

import ctypes
import json
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
# PSS_LIB may name another build of the library (e.g. to compare two builds)
LIB_PATH = os.environ.get("PSS_LIB") or os.path.join(HERE, "libpss.so")

# pss_key_t
U32, I32, U64, I64, F32, F64 = 0, 1, 2, 3, 4, 5
KEY_NAMES = {"u32": U32, "i32": I32, "u64": U64, "i64": I64, "f32": F32, "f64": F64}
KEY_BYTES = {U32: 4, I32: 4, U64: 8, I64: 8, F32: 4, F64: 8}
# pss_val_t
VAL_NONE, VAL_U32 = 0, 1
# PSS_NOALLOC_SCRATCH_BYTES: the scratch array of pss_sort_noalloc
NOALLOC_SCRATCH_BYTES = 64 << 20
# pss_inject_t
INJECT_NONE, INJECT_LAUNCH, INJECT_ALLOC = 0, 1, 2
# pss_status
(OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_OOM, ERR_HIP, ERR_WORKSPACE, ERR_BUDGET, ERR_BUSY,
 ERR_CANCELLED) = range(9)



class Request(ctypes.Structure):
    """pss_request (include/pss.h): one serving request, device pointers."""

    _fields_ = [("key", ctypes.c_int), ("val", ctypes.c_int), ("keys_in", ctypes.c_void_p),
                ("keys_out", ctypes.c_void_p), ("vals_in", ctypes.c_void_p),
                ("vals_out", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("arrival_ns", ctypes.c_uint64)]


class Stats(ctypes.Structure):
    """pss_stats (include/pss.h)."""

    _fields_ = [(f, ctypes.c_uint64) for f in ("submitted", "completed", "rejected", "cancelled",
                                               "failed", "batches", "keys_completed")] + \
               [(f, ctypes.c_double) for f in ("keys_per_s", "latency_p50_ms", "latency_p99_ms",
                                               "latency_mean_ms", "latency_max_ms",
                                               "mean_batch_requests", "mean_batch_keys")] + \
               [(f, ctypes.c_uint64) for f in ("budget_in_use", "queued")]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


# Names and signatures of every entry point in include/pss.h.
_c = ctypes
_vp, _u64, _u32, _sz, _int = _c.c_void_p, _c.c_uint64, _c.c_uint32, _c.c_size_t, _c.c_int
SIGNATURES = {
    "pss_create": (_int, [_int, _c.POINTER(_vp)]),
    "pss_destroy": (None, [_vp]),
    "pss_status_string": (_c.c_char_p, [_int]),
    "pss_last_error": (_c.c_char_p, [_vp]),
    "pss_validate": (_int, [_int, _int, _vp, _vp, _vp, _vp, _u64, _u32, _u32, _sz]),
    "pss_workspace_bytes": (_int, [_vp, _int, _int, _u64, _u32, _u32, _c.POINTER(_sz)]),
    "pss_plan_describe": (_int, [_int, _int, _u64, _u32, _u32, _c.c_char_p, _sz]),
    "pss_sort": (_int, [_vp, _int, _int, _vp, _vp, _vp, _vp, _u64, _u32, _u32, _vp, _sz, _vp]),
    "pss_device_check": (_int, [_vp, _c.POINTER(_u32)]),
    "pss_segmented_graph_create": (_int, [_vp, _int, _int, _vp, _vp, _vp, _vp, _u64, _vp, _u32,
                                          _vp, _vp, _sz, _c.POINTER(_vp)]),
    "pss_graph_launch": (_int, [_vp, _vp]),
    "pss_graph_destroy": (None, [_vp]),
    "pss_segmented_workspace_bytes": (_int, [_vp, _int, _int, _u64, _u32, _vp, _c.POINTER(_sz)]),
    "pss_segmented_sort": (_int, [_vp, _int, _int, _vp, _vp, _vp, _vp, _u64, _vp, _u32, _vp, _vp,
                                  _sz, _vp]),
    "pss_profile_enable": (_int, [_vp, _int]),
    "pss_profile_read": (_int, [_vp, _c.c_char_p, _sz]),
    "pss_profile_only": (_int, [_vp, _c.c_char_p]),
    "pss_server_create": (_int, [_vp, _sz, _u32, _vp, _c.POINTER(_vp)]),
    "pss_submit": (_int, [_vp, _c.POINTER(Request), _c.POINTER(_u64)]),
    "pss_poll": (_int, [_vp, _u64, _c.POINTER(_int), _c.POINTER(_int)]),
    "pss_wait": (_int, [_vp, _u64, _c.POINTER(_int)]),
    "pss_cancel": (_int, [_vp, _u64]),
    "pss_server_stats": (_int, [_vp, _c.POINTER(Stats)]),
    "pss_server_reset_stats": (_int, [_vp]),
    "pss_server_destroy": (None, [_vp]),
    "pss_splitters": (_int, [_vp, _int, _vp, _u64, _u32, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                             _vp]),
    "pss_set_merge_method": (_int, [_vp, _int]),
    "pss_records_workspace_bytes": (_int, [_vp, _int, _u64, _c.POINTER(_sz)]),
    "pss_sort_records": (_int, [_vp, _int, _vp, _vp, _u64, _u32, _u32, _vp, _sz, _vp]),
    "pss_psrs_workspace_bytes": (_int, [_vp, _int, _int, _u64, _u32, _u32, _c.POINTER(_sz)]),
    "pss_psrs_sort": (_int, [_vp, _int, _int, _vp, _vp, _vp, _vp, _u64, _u32, _u32, _vp, _vp, _sz,
                             _vp]),
    "pss_psrs_splitters": (_int, [_vp, _int, _vp, _u64, _u32, _u32, _vp, _vp, _vp, _vp, _vp, _vp,
                                  _sz, _vp]),
    "pss_debug_inject": (_int, [_int, _c.c_int64]),
    "pss_sort_noalloc": (_int, [_vp, _int, _int, _vp, _vp, _vp, _vp, _u64, _u32, _u32, _vp]),
}

_lock = threading.Lock()
_lib = None


class PssError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libpss.so (once).  Raises FileNotFoundError if it is not built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise FileNotFoundError(
                    f"{path} is missing: build the HIP library first "
                    "(python -m paper_2305_05245_amd.build)")
            lib = ctypes.CDLL(path)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def debug_inject(what: int, after: int = 0) -> None:
    """pss_debug_inject: arm the (after+1)-th next operation of a kind to fail
    (INJECT_LAUNCH, INJECT_ALLOC); INJECT_NONE or after < 0 disarms."""
    check(load().pss_debug_inject(what, after))


def status_string(status: int) -> str:
    return load().pss_status_string(status).decode()


def last_error(ctx=None) -> str:
    return (load().pss_last_error(ctx) or b"").decode()


def check(status: int, ctx=None) -> None:
    if status != OK:
        raise PssError(status, last_error(ctx))


def validate(key: int, val: int, keys_in: int, keys_out: int, vals_in: int, vals_out: int,
             n: int, n_blocks: int = 0, n_parts: int = 0, ws_bytes: int | None = None) -> int:
    """pss_validate: the argument check of pss_sort (no device access)."""
    ws = ctypes.c_size_t(-1).value if ws_bytes is None else ws_bytes
    return load().pss_validate(key, val, keys_in or None, keys_out or None, vals_in or None,
                               vals_out or None, n, n_blocks, n_parts, ws)


def workspace_bytes(key: int, val: int, n: int, n_blocks: int = 0, n_parts: int = 0) -> int:
    out = ctypes.c_size_t()
    check(load().pss_workspace_bytes(None, key, val, n, n_blocks, n_parts, ctypes.byref(out)))
    return int(out.value)


def records_workspace_bytes(key: int, n: int) -> int:
    out = ctypes.c_size_t()
    check(load().pss_records_workspace_bytes(None, key, n, ctypes.byref(out)))
    return int(out.value)


def psrs_workspace_bytes(key: int, val: int, n: int, n_blocks: int, n_parts: int) -> int:
    out = ctypes.c_size_t()
    check(load().pss_psrs_workspace_bytes(None, key, val, n, n_blocks, n_parts, ctypes.byref(out)))
    return int(out.value)


def psrs_sample_count(n: int, n_blocks: int, n_parts: int) -> int:
    """Number of regular samples of the PSRS variant: n_P - 1 from each
    non-empty block of ceil(n / n_B) keys."""
    if n == 0 or n_parts < 2:
        return 0
    L = -(-n // n_blocks)
    return -(-n // L) * (n_parts - 1)


def plan(key: int, val: int, n: int, n_blocks: int = 0, n_parts: int = 0) -> dict:
    buf = ctypes.create_string_buffer(4096)
    check(load().pss_plan_describe(key, val, n, n_blocks, n_parts, buf, len(buf)))
    return json.loads(buf.value.decode())


class Tuning(ctypes.Structure):
    """pss_tuning: which segments use the 2048- and 4096-key tile sorts, a
    bound on the longest segment (bounds the merge passes launched), and the
    runs merged per pass (fan_log2: 5 or 6, 0 = 5)."""

    _fields_ = [("small_max_2k", ctypes.c_uint32), ("small_max_4k", ctypes.c_uint32),
                ("max_seg_len", ctypes.c_uint64), ("fan_log2", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {"small_max_2k": self.small_max_2k, "small_max_4k": self.small_max_4k,
                "max_seg_len": self.max_seg_len, "fan_log2": self.fan_log2 or 5}

    @classmethod
    def from_dict(cls, d: dict | None, max_seg_len: int = 0) -> "Tuning":
        d = d or {}
        return cls(int(d.get("small_max_2k", 2048)), int(d.get("small_max_4k", 4096)),
                   int(d.get("max_seg_len", max_seg_len)), int(d.get("fan_log2", 0)), 0)


def segmented_workspace_bytes(key: int, val: int, n: int, n_segs: int,
                              tuning: Tuning | None = None) -> int:
    out = ctypes.c_size_t()
    check(load().pss_segmented_workspace_bytes(None, key, val, n, n_segs,
                                               ctypes.byref(tuning) if tuning else None,
                                               ctypes.byref(out)))
    return int(out.value)


class Graph:
    """An instantiated HIP graph of one segmented-sort launch sequence."""

    def __init__(self, lib, handle):
        self.lib = lib
        self.handle = handle

    def launch(self, stream: int) -> None:
        check(self.lib.pss_graph_launch(self.handle, stream or None))

    def close(self) -> None:
        if self.handle:
            self.lib.pss_graph_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One pss_ctx bound to a HIP device.

    A pss_ctx may be used by one thread at a time (include/pss.h), while
    Python code may share a Context between threads: every call into the
    library, together with the read of the context's last error message,
    holds the context's lock."""

    def __init__(self, device: int = 0):
        self.lib = load()
        h = ctypes.c_void_p()
        check(self.lib.pss_create(device, ctypes.byref(h)))
        self.handle = h
        self.device = device
        self._mu = threading.RLock()

    def _call(self, name: str, *args) -> None:
        with self._mu:
            check(getattr(self.lib, name)(self.handle, *args), self.handle)

    def close(self):
        if self.handle:
            with self._mu:
                self.lib.pss_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sort(self, key: int, val: int, keys_in: int, keys_out: int, vals_in: int, vals_out: int,
             n: int, n_blocks: int, n_parts: int, ws: int, ws_bytes: int, stream: int) -> None:
        self._call("pss_sort", key, val, keys_in or None, keys_out or None,
                   vals_in or None, vals_out or None, n, n_blocks, n_parts,
                   ws or None, ws_bytes, stream or None)

    def sort_noalloc(self, key: int, val: int, keys_in: int, keys_out: int, vals_in: int,
                     vals_out: int, n: int, n_blocks: int, n_parts: int, stream: int) -> None:
        """pss_sort_noalloc: pss_sort on the library's fixed scratch array
        (no workspace argument, no allocation)."""
        self._call("pss_sort_noalloc", key, val, keys_in or None, keys_out or None,
                   vals_in or None, vals_out or None, n, n_blocks, n_parts, stream or None)

    def profile(self, on: bool) -> None:
        self._call("pss_profile_enable", 1 if on else 0)

    def profile_only(self, family: str | None) -> None:
        """Time only this kernel family's launches while profiling (None: all)."""
        self._call("pss_profile_only", family.encode() if family else None)

    def profile_read(self) -> dict:
        buf = ctypes.create_string_buffer(1 << 16)
        self._call("pss_profile_read", buf, len(buf))
        return json.loads(buf.value.decode())

    def segmented_sort(self, key: int, val: int, keys_in: int, keys_out: int, vals_in: int,
                       vals_out: int, n: int, seg_offsets: int, n_segs: int,
                       tuning: Tuning | None, ws: int, ws_bytes: int, stream: int) -> None:
        self._call("pss_segmented_sort", key, val, keys_in or None, keys_out or None,
                   vals_in or None, vals_out or None, n, seg_offsets or None,
                   n_segs, ctypes.byref(tuning) if tuning else None,
                   ws or None, ws_bytes, stream or None)

    def segmented_graph(self, key: int, val: int, keys_in: int, keys_out: int, vals_in: int,
                        vals_out: int, n: int, seg_offsets: int, n_segs: int,
                        tuning: Tuning | None, ws: int, ws_bytes: int) -> "Graph":
        h = ctypes.c_void_p()
        self._call("pss_segmented_graph_create", key, val, keys_in or None, keys_out or None,
                   vals_in or None, vals_out or None, n, seg_offsets or None, n_segs,
                   ctypes.byref(tuning) if tuning else None, ws or None, ws_bytes,
                   ctypes.byref(h))
        return Graph(self.lib, h)

    def device_check(self) -> int:
        """Synchronise the device and return (and clear) the error word."""
        code = ctypes.c_uint32()
        self._call("pss_device_check", ctypes.byref(code))
        return int(code.value)

    def set_merge_method(self, method: int) -> None:
        self._call("pss_set_merge_method", method)

    def sort_records(self, key: int, records_in: int, records_out: int, n: int,
                     record_bytes: int, key_offset: int, ws: int, ws_bytes: int,
                     stream: int) -> None:
        self._call("pss_sort_records", key, records_in or None, records_out or None,
                   n, record_bytes, key_offset, ws or None, ws_bytes,
                   stream or None)

    def psrs_sort(self, key: int, val: int, keys_in: int, keys_out: int, vals_in: int,
                  vals_out: int, n: int, n_blocks: int, n_parts: int, part_sizes: int, ws: int,
                  ws_bytes: int, stream: int) -> None:
        self._call("pss_psrs_sort", key, val, keys_in or None, keys_out or None,
                   vals_in or None, vals_out or None, n, n_blocks, n_parts,
                   part_sizes or None, ws or None, ws_bytes, stream or None)

    def psrs_splitters(self, key: int, keys_in: int, n: int, n_blocks: int, n_parts: int,
                       sorted_blocks: int, samples: int, pivots: int, split: int, offsets: int,
                       ws: int, ws_bytes: int, stream: int) -> None:
        self._call("pss_psrs_splitters", key, keys_in or None, n, n_blocks, n_parts,
                   sorted_blocks or None, samples or None, pivots or None,
                   split or None, offsets or None, ws or None, ws_bytes,
                   stream or None)

    def splitters(self, key: int, keys_in: int, n: int, n_blocks: int, n_parts: int,
                  sorted_blocks: int, pivots: int, counts: int, split: int, offsets: int,
                  ws: int, ws_bytes: int, stream: int) -> None:
        self._call("pss_splitters", key, keys_in or None, n, n_blocks, n_parts,
                   sorted_blocks or None, pivots or None, counts or None,
                   split or None, offsets or None, ws or None, ws_bytes,
                   stream or None)
