"""Resident batch buffers plus one captured HIP graph of the segmented sort.

A ``SegmentedGraph`` owns device buffers for up to ``n_cap`` keys (and uint32
payloads) in up to ``seg_cap`` segments, captures the library's segmented-sort
launch sequence over them once (pss_segmented_graph_create), and replays it
for every batch that fits.  Loading a batch copies the requests' device
tensors into the input buffer (one concatenation on the device) and the
offsets, padded with the batch total, into the offsets buffer.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib

_WIDTH_DTYPE = {4: torch.int32, 8: torch.int64}


class SegmentedGraph:
    def __init__(self, n_cap: int, seg_cap: int, key_type: str = "u64", with_vals: bool = True,
                 device: int = 0, tuning: dict | None = None):
        from . import _context

        self.kt = _lib.KEY_NAMES[key_type]
        self.vt = _lib.VAL_U32 if with_vals else _lib.VAL_NONE
        self.n_cap, self.seg_cap, self.device = int(n_cap), int(seg_cap), device
        d = torch.device(f"cuda:{device}")
        dt = _WIDTH_DTYPE[_lib.KEY_BYTES[self.kt]]
        self.keys_in = torch.zeros(self.n_cap, dtype=dt, device=d)
        self.keys_out = torch.empty_like(self.keys_in)
        self.vals_in = torch.zeros(self.n_cap, dtype=torch.int32, device=d) if with_vals else None
        self.vals_out = torch.empty_like(self.vals_in) if with_vals else None
        self.offsets = torch.zeros(self.seg_cap + 1, dtype=torch.int64, device=d)
        self.offsets_host = torch.zeros(self.seg_cap + 1, dtype=torch.int64, pin_memory=True)
        t = tuning or {}
        self.tuning = _lib.Tuning.from_dict(t)
        need = _lib.segmented_workspace_bytes(self.kt, self.vt, self.n_cap, self.seg_cap, self.tuning)
        self.ws = torch.empty(max(need, 256), dtype=torch.uint8, device=d)
        torch.cuda.synchronize(d)
        self.graph = _context(device).segmented_graph(
            self.kt, self.vt, self.keys_in.data_ptr(), self.keys_out.data_ptr(),
            self.vals_in.data_ptr() if with_vals else 0, self.vals_out.data_ptr() if with_vals else 0,
            self.n_cap, self.offsets.data_ptr(), self.seg_cap, self.tuning, self.ws.data_ptr(),
            self.ws.numel())
        self.resident_bytes = sum(x.numel() * x.element_size() for x in
                                  (self.keys_in, self.keys_out, self.offsets, self.ws)
                                  if x is not None)
        if with_vals:
            self.resident_bytes += 2 * self.n_cap * 4

    def load(self, keys: list, vals: list | None, stream: torch.cuda.Stream) -> np.ndarray:
        """Copy a batch (lists of 1-D device tensors) into the resident buffers
        on `stream`; return the host offsets of the batch (len(keys) + 1)."""
        sizes = np.fromiter((k.numel() for k in keys), dtype=np.int64, count=len(keys))
        offs = np.zeros(len(keys) + 1, dtype=np.int64)
        np.cumsum(sizes, out=offs[1:])
        total = int(offs[-1])
        if len(keys) > self.seg_cap or total > self.n_cap:
            raise ValueError("batch exceeds the graph's capacity")
        with torch.cuda.stream(stream):
            if total:
                torch.cat(keys, out=self.keys_in[:total])
                if self.vals_in is not None:
                    torch.cat(vals, out=self.vals_in[:total])
            oh = self.offsets_host.numpy()
            oh[: offs.size] = offs
            oh[offs.size:] = total
            self.offsets.copy_(self.offsets_host, non_blocking=True)
        return offs

    def run(self, stream: torch.cuda.Stream) -> None:
        self.graph.launch(stream.cuda_stream)
