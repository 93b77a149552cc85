"""Serving loop (pss_server_*): every request's result is the same whether it
is sorted alone or batched with others, and equals the stable sort of its
input; budget admission, cancellation and the error paths behave as
documented."""
from __future__ import annotations

import time

import numpy as np
import pytest

import workloads as W
from gpu_util import announce, order_bits, to_device

pytestmark = pytest.mark.gpu


def _stable(keys: np.ndarray):
    o = np.argsort(order_bits(keys), kind="stable")
    return keys[o], o.astype(np.uint32)


def _mixed_requests(n_req: int, seed: int):
    """The serving workload's shape (lognormal sizes, half uniform and half
    duplicate-heavy u64 keys with their input index as value), sizes clipped
    to 2^18 so the test stays short, plus keys-only requests of other types
    interleaved to exercise batching by type."""
    _, sizes, dup = W.serving_requests(n_req, 1000.0, seed_arrival=seed, seed_size=seed + 1,
                                       seed_keys=seed + 2, mu_log2=12.0, hi=1 << 18)
    reqs = []
    for i, (s, d) in enumerate(zip(sizes, dup)):
        if i % 7 == 3:
            reqs.append(("f64", W.normal_specials_f64(int(s), seed=seed * 100 + i), None))
        elif i % 7 == 5:
            reqs.append(("u32", W.duplicate3_u32(int(s), seed=seed * 100 + i), None))
        else:
            reqs.append(("u64", W.request_keys(int(s), bool(d), seed=seed * 100 + i),
                         W.index_values(int(s))))
    return reqs


def _run(srv, reqs, together: bool):
    import torch

    outs, tickets = [], []
    for kt, k, v in reqs:
        dk = to_device(k)
        ok = torch.empty_like(dk)
        dv = to_device(v) if v is not None else None
        ov = torch.empty_like(dv) if v is not None else None
        tk = srv.submit(dk, ok, dv, ov, key_type=kt)
        outs.append((ok, ov))
        if together:
            tickets.append(tk)
        else:
            assert srv.wait(tk) == 0
    for tk in tickets:
        assert srv.wait(tk) == 0
    res = []
    for (kt, k, v), (ok, ov) in zip(reqs, outs):
        res.append((ok.cpu().numpy().view(k.dtype),
                    ov.cpu().numpy().view(np.uint32) if ov is not None else None))
    return res


def test_each_result_same_alone_and_in_the_mix():
    import torch  # noqa: F401

    from paper_2305_05245_amd.serving import Server

    reqs = _mixed_requests(48, seed=31)
    announce("serving mix", len(reqs), "requests", sum(k.size for _, k, _ in reqs), "keys")
    with Server(hbm_budget_bytes=3 << 28, max_streams=3) as srv:
        mixed = _run(srv, reqs, together=True)
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0 and st["rejected"] == 0
        assert 0 < st["latency_p50_ms"] <= st["latency_p99_ms"] <= st["latency_max_ms"]
        assert st["keys_completed"] == sum(k.size for _, k, _ in reqs)
        assert st["batches"] >= 1 and st["keys_per_s"] > 0
        announce("serving alone", len(reqs), "requests")
        alone = _run(srv, reqs, together=False)
    for i, ((kt, k, v), (mk, mv), (ak, av)) in enumerate(zip(reqs, mixed, alone)):
        ek, eo = _stable(k)
        assert np.array_equal(mk.view(np.uint8), ak.view(np.uint8)), i
        assert np.array_equal(mk.view(np.uint8), ek.view(np.uint8)), i
        if v is not None:
            assert np.array_equal(mv, av), i
            assert np.array_equal(mv, eo), i


def test_budget_rejects_oversize_and_serves_the_rest():
    import torch

    from paper_2305_05245_amd import PssError, _lib
    from paper_2305_05245_amd.serving import Server

    announce("serving budget")
    with Server(hbm_budget_bytes=64 << 20, max_streams=2) as srv:   # 32 MiB per stream
        big = torch.zeros(1 << 21, dtype=torch.int64, device="cuda")
        with pytest.raises(PssError) as e:
            srv.submit(big, torch.empty_like(big), key_type="u64")
        assert e.value.status == _lib.ERR_BUDGET
        k = W.request_keys(100_000, False, seed=5)
        dk = to_device(k)
        out = torch.empty_like(dk)
        assert srv.wait(srv.submit(dk, out, key_type="u64")) == 0
        assert np.array_equal(out.cpu().numpy().view(np.uint64), np.sort(k))
        st = srv.stats()
        assert st["rejected"] == 1 and st["completed"] == 1


def test_cancel_queued_request():
    import torch

    from paper_2305_05245_amd import _lib
    from paper_2305_05245_amd.serving import Server

    announce("serving cancel")
    with Server(hbm_budget_bytes=1 << 30, max_streams=1) as srv:
        kb = to_device(W.request_keys(1 << 22, False, seed=6))
        vb = torch.arange(1 << 22, dtype=torch.int32, device="cuda")
        ob, ovb = torch.empty_like(kb), torch.empty_like(vb)
        ks = W.request_keys(5000, True, seed=7)
        dk = to_device(ks)
        out = torch.zeros_like(dk)
        t_big = srv.submit(kb, ob, vb, ovb, key_type="u64")
        t_small = srv.submit(dk, out, key_type="u64")
        c = srv.cancel(t_small)
        assert c in (_lib.OK, _lib.ERR_BUSY)
        assert srv.wait(t_big) == 0
        r = srv.wait(t_small)
        if c == _lib.OK:
            assert r == _lib.ERR_CANCELLED
            assert not out.any().item()            # never written
            assert srv.stats()["cancelled"] == 1
        else:
            assert r == _lib.OK
            assert np.array_equal(out.cpu().numpy().view(np.uint64), np.sort(ks))
        # a finished, uncollected request can no longer be cancelled
        t = srv.submit(dk, out, key_type="u64")
        deadline = time.time() + 30
        while srv.stats()["completed"] < (2 if c == _lib.OK else 3) and time.time() < deadline:
            time.sleep(0.001)
        assert srv.cancel(t) == _lib.ERR_BUSY
        assert srv.wait(t) == 0


def test_request_errors_and_empty_request():
    import torch

    from paper_2305_05245_amd import PssError, _lib
    from paper_2305_05245_amd.serving import Server

    announce("serving errors")
    with Server(hbm_budget_bytes=64 << 20, max_streams=1) as srv:
        x = torch.zeros(1000, dtype=torch.int64, device="cuda")
        with pytest.raises(PssError) as e:        # in == out
            srv.submit_raw(_lib.U64, _lib.VAL_NONE, x.data_ptr(), x.data_ptr(), 0, 0, 1000)
        assert e.value.status == _lib.ERR_INVALID
        with pytest.raises(PssError):              # unknown key type
            srv.submit_raw(9, _lib.VAL_NONE, x.data_ptr(), x.data_ptr() + 8000, 0, 0, 1)
        with pytest.raises(PssError):              # unknown ticket
            srv.wait(123456)
        e0 = torch.empty(0, dtype=torch.int64, device="cuda")
        t = srv.submit(e0, torch.empty_like(e0), key_type="i64")
        assert srv.poll(t) == (True, 0)
