"""Python face of the library's serving loop (pss_server_* in include/pss.h).

    srv = Server(hbm_budget_bytes=64 << 30, max_streams=4)
    t = srv.submit(keys, out, vals, vals_out, key_type="u64")   # device tensors
    status = srv.wait(t)          # PSS_OK (0) once out / vals_out hold the result
    print(srv.stats())            # keys/s, p50 / p99 latency from arrival, batches

Queueing, admission against the budget, batching, the sorts and the copies
all happen in libpss; this class only marshals arguments and keeps each
request's tensors alive until its result has been collected.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib


class Server:
    def __init__(self, hbm_budget_bytes: int = 64 << 30, max_streams: int = 4,
                 tuning: "dict | _lib.Tuning | None" = None, device: int = 0):
        from . import _context

        self.lib = _lib.load()
        self.device = device
        ctx = _context(device)
        tu = tuning
        if isinstance(tuning, dict):
            tu = _lib.Tuning.from_dict({k: v for k, v in tuning.items() if k != "max_seg_len"})
        h = ctypes.c_void_p()
        _lib.check(self.lib.pss_server_create(ctx.handle, int(hbm_budget_bytes), int(max_streams),
                                              ctypes.byref(tu) if tu is not None else None,
                                              ctypes.byref(h)))
        self.handle = h
        self._live: dict[int, tuple] = {}

    # -- requests -------------------------------------------------------
    def submit_raw(self, key: int, val: int, keys_in: int, keys_out: int, vals_in: int,
                   vals_out: int, n: int, arrival_ns: int = 0) -> int:
        """Submit by device address (the caller keeps the memory alive)."""
        r = _lib.Request()
        r.key, r.val, r.keys_in, r.keys_out = key, val, keys_in or None, keys_out or None
        r.vals_in, r.vals_out, r.n, r.arrival_ns = vals_in or None, vals_out or None, n, arrival_ns
        ticket = ctypes.c_uint64()
        _lib.check(self.lib.pss_submit(self.handle, ctypes.byref(r), ctypes.byref(ticket)))
        return int(ticket.value)

    def submit(self, keys: torch.Tensor, out: torch.Tensor, vals: torch.Tensor | None = None,
               vals_out: torch.Tensor | None = None, key_type: str | int | None = None,
               arrival_ns: int = 0) -> int:
        """Queue one sort of a 1-D device tensor into `out` (stable with
        uint32 `vals` into `vals_out`).  Returns the ticket.  The tensors
        are held until the result is collected with poll() or wait()."""
        from . import key_type_of

        for t in (keys, out) + ((vals, vals_out) if vals is not None else ()):
            if t is None or not t.is_cuda or t.dim() != 1 or not t.is_contiguous():
                raise ValueError("request arrays must be contiguous 1-D device tensors")
        kt = key_type_of(keys, key_type)
        n = keys.numel()
        if out.numel() != n or keys.element_size() != _lib.KEY_BYTES[kt]:
            raise ValueError("keys / out sizes or widths do not match")
        vt = _lib.VAL_NONE
        if vals is not None:
            if vals_out is None or vals.numel() != n or vals_out.numel() != n or \
                    vals.element_size() != 4 or vals_out.element_size() != 4:
                raise ValueError("vals / vals_out must hold n 4-byte elements")
            vt = _lib.VAL_U32
        tk = self.submit_raw(kt, vt, keys.data_ptr(), out.data_ptr(),
                             vals.data_ptr() if vals is not None else 0,
                             vals_out.data_ptr() if vals is not None else 0, n, arrival_ns)
        self._live[tk] = (keys, out, vals, vals_out)
        return tk

    def poll(self, ticket: int) -> tuple[bool, int | None]:
        done, status = ctypes.c_int(), ctypes.c_int()
        _lib.check(self.lib.pss_poll(self.handle, ticket, ctypes.byref(done), ctypes.byref(status)))
        if done.value:
            self._live.pop(ticket, None)
            return True, int(status.value)
        return False, None

    def wait(self, ticket: int) -> int:
        st = ctypes.c_int()
        _lib.check(self.lib.pss_wait(self.handle, ticket, ctypes.byref(st)))
        self._live.pop(ticket, None)
        return int(st.value)

    def cancel(self, ticket: int) -> int:
        """PSS_OK if the request was withdrawn, PSS_ERR_BUSY if already launched."""
        st = self.lib.pss_cancel(self.handle, ticket)
        if st not in (_lib.OK, _lib.ERR_BUSY):
            _lib.check(st)
        return int(st)

    # -- accounting ------------------------------------------------------
    def stats(self) -> dict:
        s = _lib.Stats()
        _lib.check(self.lib.pss_server_stats(self.handle, ctypes.byref(s)))
        return s.as_dict()

    def reset_stats(self) -> None:
        _lib.check(self.lib.pss_server_reset_stats(self.handle))

    def close(self) -> None:
        if self.handle:
            self.lib.pss_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
