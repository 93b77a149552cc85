"""pss: parallel samplesort with exact splitting (PSES) for AMD MI355X.

Python face of libpss (include/pss.h).  PyTorch supplies device memory and the
current HIP stream; every step of the sort runs in the library's HIP kernels.

    import paper_2305_05245_amd as pss
    out, _ = pss.sort(keys)                      # automatic multi-level plan
    out, vals = pss.sort(keys, vals)             # stable key-value sort
    out, _ = pss.sort(keys, n_blocks=64, n_parts=64)   # the paper's single level
    info = pss.splitters(keys, 64, 64)           # steps 1-3 (pivots, c_k, split)
    out, _, sizes = pss.psrs_sort(keys, n_blocks=64, n_parts=64)  # regular-sampling pivots
    out = pss.sort_records(particles, "u64", key_offset=0)       # records [n, 96] uint8
"""
from __future__ import annotations

import threading

import torch

from . import _lib
from ._lib import PssError, Tuning, plan, validate, workspace_bytes  # noqa: F401

__all__ = ["sort", "sort_noalloc", "segmented_sort", "splitters", "psrs_sort", "psrs_splitters", "sort_records", "set_merge_method", "device_check", "Tuning", "key_type_of", "plan", "workspace_bytes", "PssError",
           "Workspace"]

_DTYPE_KEY = {
    torch.int32: _lib.I32,
    torch.int64: _lib.I64,
    torch.float32: _lib.F32,
    torch.float64: _lib.F64,
}
for _name, _code in (("uint32", _lib.U32), ("uint64", _lib.U64)):
    if hasattr(torch, _name):
        _DTYPE_KEY[getattr(torch, _name)] = _code

_ctx_lock = threading.Lock()
_contexts: dict[int, _lib.Context] = {}


def _context(device: int) -> _lib.Context:
    with _ctx_lock:
        c = _contexts.get(device)
        if c is None:
            c = _lib.Context(device)
            _contexts[device] = c
        return c


class Workspace:
    """Grow-only device scratch buffer (caller-owned memory handed to the
    library as `ws`), one per (device, stream).

    Work queued on one stream runs in order, so a buffer that only that
    stream uses is never read by one sort while another writes it, and when
    it grows, the caching allocator hands the old block out again only to
    work ordered after the sorts already queued on the same stream."""

    _lock = threading.Lock()
    _per_stream: dict[tuple[int, int], "Workspace"] = {}

    def __init__(self, device: int):
        self.device = device
        self.buf = torch.empty(0, dtype=torch.uint8, device=f"cuda:{device}")

    @classmethod
    def get(cls, device: int, nbytes: int) -> torch.Tensor:
        """The current stream's buffer on `device`, grown to nbytes."""
        key = (device, _stream_handle(device))
        with cls._lock:
            ws = cls._per_stream.get(key)
            if ws is None:
                ws = cls._per_stream[key] = cls(device)
            if ws.buf.numel() < nbytes:
                ws.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8,
                                     device=f"cuda:{device}")
            return ws.buf


def key_type_of(t: torch.Tensor, key_type: str | int | None = None) -> int:
    if key_type is not None:
        return _lib.KEY_NAMES[key_type] if isinstance(key_type, str) else int(key_type)
    try:
        return _DTYPE_KEY[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported key dtype {t.dtype}") from None


def _stream_handle(device: int) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def sort(keys: torch.Tensor, vals: torch.Tensor | None = None, n_blocks: int = 0,
         n_parts: int = 0, key_type: str | int | None = None, out: torch.Tensor | None = None,
         vals_out: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """Sort a 1-D device tensor ascending (floats by IEEE totalOrder); with
    `vals` (uint32 payload, any 4-byte dtype) the sort is stable.  Returns
    (sorted_keys, sorted_vals or None).  Asynchronous on the current stream."""
    if not keys.is_cuda or keys.dim() != 1 or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous 1-D device tensor")
    kt = key_type_of(keys, key_type)
    if keys.element_size() != _lib.KEY_BYTES[kt]:
        raise ValueError("key dtype width does not match key_type")
    dev = keys.device.index if keys.device.index is not None else torch.cuda.current_device()
    n = keys.numel()
    vt = _lib.VAL_NONE
    if vals is not None:
        if not vals.is_cuda or vals.numel() != n or vals.element_size() != 4 or not vals.is_contiguous():
            raise ValueError("vals must be a contiguous device tensor of n 4-byte elements")
        vt = _lib.VAL_U32
    if out is None:
        out = torch.empty_like(keys)
    if vals is not None and vals_out is None:
        vals_out = torch.empty_like(vals)
    need = _lib.workspace_bytes(kt, vt, n, n_blocks, n_parts)
    ws = workspace if workspace is not None else Workspace.get(dev, need)
    ctx = _context(dev)
    ctx.sort(kt, vt, keys.data_ptr(), out.data_ptr(),
             vals.data_ptr() if vals is not None else 0,
             vals_out.data_ptr() if vals is not None else 0,
             n, n_blocks, n_parts, ws.data_ptr(), ws.numel(), _stream_handle(dev))
    return out, (vals_out if vals is not None else None)


def sort_noalloc(keys: torch.Tensor, out: torch.Tensor, vals: torch.Tensor | None = None,
                 vals_out: torch.Tensor | None = None, n_blocks: int = 0, n_parts: int = 0,
                 key_type: str | int | None = None):
    """`sort` on the library's fixed scratch array instead of a workspace: the
    call allocates no device memory (for graph capture and loops that must not
    allocate), so the caller passes the outputs.  Sorts whose workspace would
    exceed NOALLOC_SCRATCH_BYTES (64 MiB) raise PssError (ERR_WORKSPACE).
    Calls that overlap on one device share the array and must not run
    concurrently."""
    if not keys.is_cuda or keys.dim() != 1 or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous 1-D device tensor")
    kt = key_type_of(keys, key_type)
    if keys.element_size() != _lib.KEY_BYTES[kt]:
        raise ValueError("key dtype width does not match key_type")
    if out is None or out.shape != keys.shape or out.dtype != keys.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous tensor shaped like keys")
    n = keys.numel()
    vt = _lib.VAL_NONE
    if vals is not None:
        if (not vals.is_cuda or vals.numel() != n or vals.element_size() != 4
                or not vals.is_contiguous()):
            raise ValueError("vals must be a contiguous device tensor of n 4-byte elements")
        if (vals_out is None or vals_out.numel() != n or vals_out.element_size() != 4
                or not vals_out.is_contiguous()):
            raise ValueError("vals_out must be a contiguous tensor of n 4-byte elements")
        vt = _lib.VAL_U32
    dev = keys.device.index if keys.device.index is not None else torch.cuda.current_device()
    _context(dev).sort_noalloc(kt, vt, keys.data_ptr(), out.data_ptr(),
                               vals.data_ptr() if vals is not None else 0,
                               vals_out.data_ptr() if vals is not None else 0,
                               n, n_blocks, n_parts, _stream_handle(dev))
    return out, (vals_out if vals is not None else None)


def profile(on: bool, device: int = 0, only: str | None = None) -> None:
    """Turn per-launch event timing of the library on or off; `only` limits
    it to one kernel family (e.g. "merge"), None times every launch."""
    ctx = _context(device)
    ctx.profile_only(only)
    ctx.profile(on)


def profile_read(device: int = 0) -> dict:
    """Per kernel family: launches, total ms and algorithmic bytes since the
    last read (waits for the recorded events)."""
    return _context(device).profile_read()


def segmented_sort(keys: torch.Tensor, seg_offsets, vals: torch.Tensor | None = None,
                   key_type: str | int | None = None, tuning: "Tuning | dict | None" = None,
                   max_seg_len: int | None = None, out: torch.Tensor | None = None,
                   vals_out: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """Sort every segment [seg_offsets[i], seg_offsets[i+1]) of a 1-D device
    tensor independently (stable with `vals`).  seg_offsets: a device int64
    tensor of n_segs + 1 offsets, or a host sequence (copied to the device;
    its longest segment then bounds the merge passes launched).  `tuning`
    chooses the small-segment tile sorts (see autotune.py); None = defaults,
    or the autotuner's cached choice when one exists.  Returns (keys, vals)."""
    if not keys.is_cuda or keys.dim() != 1 or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous 1-D device tensor")
    kt = key_type_of(keys, key_type)
    dev = keys.device.index if keys.device.index is not None else torch.cuda.current_device()
    n = keys.numel()
    if isinstance(seg_offsets, torch.Tensor) and seg_offsets.is_cuda:
        offs = seg_offsets.to(torch.int64).contiguous()
    else:
        import numpy as np

        host = np.asarray(seg_offsets, dtype=np.int64)
        if max_seg_len is None and host.size > 1:
            max_seg_len = int(np.max(np.diff(host)))
        offs = torch.from_numpy(host).to(keys.device)
    n_segs = offs.numel() - 1
    vt = _lib.VAL_NONE
    if vals is not None:
        if not vals.is_cuda or vals.numel() != n or vals.element_size() != 4:
            raise ValueError("vals must be a device tensor of n 4-byte elements")
        vt = _lib.VAL_U32
    tu = _resolve_tuning(tuning, kt, vt, n, n_segs, max_seg_len)
    if out is None:
        out = torch.empty_like(keys)
    if vals is not None and vals_out is None:
        vals_out = torch.empty_like(vals)
    need = _lib.segmented_workspace_bytes(kt, vt, n, n_segs, tu)
    ws = workspace if workspace is not None else Workspace.get(dev, need)
    _context(dev).segmented_sort(kt, vt, keys.data_ptr(), out.data_ptr(),
                                 vals.data_ptr() if vals is not None else 0,
                                 vals_out.data_ptr() if vals is not None else 0,
                                 n, offs.data_ptr(), n_segs, tu, ws.data_ptr(), ws.numel(),
                                 _stream_handle(dev))
    return out, (vals_out if vals is not None else None)


def _resolve_tuning(tuning, kt, vt, n, n_segs, max_seg_len):
    if isinstance(tuning, _lib.Tuning):
        tu = tuning
    else:
        d = tuning
        if d is None:
            from . import autotune

            d = autotune.cached(kt, vt, n, n_segs)
        tu = _lib.Tuning.from_dict({k: v for k, v in (d or {}).items() if k != "max_seg_len"})
    if max_seg_len is not None and tu.max_seg_len == 0:
        tu = _lib.Tuning(tu.small_max_2k, tu.small_max_4k, int(max_seg_len), tu.fan_log2, 0)
    return tu


def device_check(device: int = 0) -> int:
    """Synchronise `device` and return (and clear) the library's device error
    word: 0 when every kernel found its invariants intact."""
    return _context(device).device_check()


def splitters(keys: torch.Tensor, n_blocks: int, n_parts: int,
              key_type: str | int | None = None) -> dict:
    """Steps 1-3 of the paper's method on the device: sorted blocks, canonical
    pivots P_k, counts c_k (Eq. 2), the split table [n_B, n_P+1] and the
    offsets O_k of the merged partitions."""
    if not keys.is_cuda or keys.dim() != 1 or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous 1-D device tensor")
    kt = key_type_of(keys, key_type)
    dev = keys.device.index if keys.device.index is not None else torch.cuda.current_device()
    n = keys.numel()
    d = keys.device
    res = {
        "sorted_blocks": torch.empty_like(keys),
        "pivots": torch.zeros(max(n_parts - 1, 0), dtype=keys.dtype, device=d),
        "counts": torch.zeros(max(n_parts - 1, 0), dtype=torch.int64, device=d),
        "split": torch.zeros((n_blocks, n_parts + 1), dtype=torch.int64, device=d),
        "offsets": torch.zeros(n_parts + 1, dtype=torch.int64, device=d),
    }
    need = _lib.workspace_bytes(kt, _lib.VAL_NONE, n, n_blocks, n_parts)
    ws = Workspace.get(dev, need)
    ctx = _context(dev)

    def ptr(t):
        return t.data_ptr() if t.numel() else 0

    ctx.splitters(kt, keys.data_ptr(), n, n_blocks, n_parts, ptr(res["sorted_blocks"]),
                  ptr(res["pivots"]), ptr(res["counts"]), ptr(res["split"]), ptr(res["offsets"]),
                  ws.data_ptr(), ws.numel(), _stream_handle(dev))
    return res


def psrs_sort(keys: torch.Tensor, vals: torch.Tensor | None = None, n_blocks: int = 64,
              n_parts: int = 64, key_type: str | int | None = None,
              out: torch.Tensor | None = None, vals_out: torch.Tensor | None = None,
              workspace: torch.Tensor | None = None):
    """The paper's single level with regular-sampling (PSRS) pivots instead of
    exact splitting: same output as `sort`, partition sizes that follow the
    data.  Returns (sorted_keys, sorted_vals or None, partition_sizes [n_P]
    int64 device tensor)."""
    if not keys.is_cuda or keys.dim() != 1 or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous 1-D device tensor")
    kt = key_type_of(keys, key_type)
    if keys.element_size() != _lib.KEY_BYTES[kt]:
        raise ValueError("key dtype width does not match key_type")
    dev = keys.device.index if keys.device.index is not None else torch.cuda.current_device()
    n = keys.numel()
    vt = _lib.VAL_NONE
    if vals is not None:
        if not vals.is_cuda or vals.numel() != n or vals.element_size() != 4 or not vals.is_contiguous():
            raise ValueError("vals must be a contiguous device tensor of n 4-byte elements")
        vt = _lib.VAL_U32
    if out is None:
        out = torch.empty_like(keys)
    if vals is not None and vals_out is None:
        vals_out = torch.empty_like(vals)
    sizes = torch.empty(n_parts, dtype=torch.int64, device=keys.device)
    need = _lib.psrs_workspace_bytes(kt, vt, n, n_blocks, n_parts)
    ws = workspace if workspace is not None else Workspace.get(dev, need)
    _context(dev).psrs_sort(kt, vt, keys.data_ptr(), out.data_ptr(),
                            vals.data_ptr() if vals is not None else 0,
                            vals_out.data_ptr() if vals is not None else 0, n, n_blocks, n_parts,
                            sizes.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(dev))
    return out, (vals_out if vals is not None else None), sizes


def psrs_splitters(keys: torch.Tensor, n_blocks: int, n_parts: int,
                   key_type: str | int | None = None) -> dict:
    """Steps 1-3 with regular-sampling pivots on the device: sorted blocks,
    sorted samples S, pivots P_k = S[floor(k |S| / n_P)], the split table
    [n_B, n_P+1] (keys <= P_k per block) and offsets |{x <= P_k}|."""
    if not keys.is_cuda or keys.dim() != 1 or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous 1-D device tensor")
    kt = key_type_of(keys, key_type)
    dev = keys.device.index if keys.device.index is not None else torch.cuda.current_device()
    n = keys.numel()
    d = keys.device
    res = {
        "sorted_blocks": torch.empty_like(keys),
        "samples": torch.empty(_lib.psrs_sample_count(n, n_blocks, n_parts), dtype=keys.dtype,
                               device=d),
        "pivots": torch.zeros(max(n_parts - 1, 0), dtype=keys.dtype, device=d),
        "split": torch.zeros((n_blocks, n_parts + 1), dtype=torch.int64, device=d),
        "offsets": torch.zeros(n_parts + 1, dtype=torch.int64, device=d),
    }
    ws = Workspace.get(dev, _lib.psrs_workspace_bytes(kt, _lib.VAL_NONE, n, n_blocks, n_parts))

    def ptr(t):
        return t.data_ptr() if t.numel() else 0

    _context(dev).psrs_splitters(kt, keys.data_ptr(), n, n_blocks, n_parts,
                                 ptr(res["sorted_blocks"]), ptr(res["samples"]),
                                 ptr(res["pivots"]), ptr(res["split"]), ptr(res["offsets"]),
                                 ws.data_ptr(), ws.numel(), _stream_handle(dev))
    return res


def sort_records(records: torch.Tensor, key_type: str | int, key_offset: int = 0,
                 out: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """Sort fixed-size records by a key field, stable.  `records` is a
    contiguous device tensor whose first dimension indexes the records (e.g. a
    [n, record_bytes] uint8 tensor, or a structured view of the same bytes);
    the key of type `key_type` sits at byte `key_offset` of each record.
    Returns the sorted records (same shape and dtype)."""
    if not records.is_cuda or not records.is_contiguous() or records.dim() < 1:
        raise ValueError("records must be a contiguous device tensor, one record per row")
    kt = _lib.KEY_NAMES[key_type] if isinstance(key_type, str) else int(key_type)
    n = records.shape[0]
    rb = records.element_size()
    for d in records.shape[1:]:
        rb *= d
    dev = records.device.index if records.device.index is not None else torch.cuda.current_device()
    if out is None:
        out = torch.empty_like(records)
    need = _lib.records_workspace_bytes(kt, n)
    ws = workspace if workspace is not None else Workspace.get(dev, need)
    _context(dev).sort_records(kt, records.data_ptr(), out.data_ptr(), n, rb, key_offset,
                               ws.data_ptr(), ws.numel(), _stream_handle(dev))
    return out


MERGE_METHODS = {"pairwise": 0, "sort": 1}


def set_merge_method(method: str, device: int = 0) -> None:
    """Step 4 of the paper's single level on `device`: "pairwise" stable merge
    rounds (default) or "sort" (gather each chunk and sort it, Section 2.2)."""
    _context(device).set_merge_method(MERGE_METHODS[method])
