"""Serving loop (pss_server_*): every request's result is the same whether it
is sorted alone or batched with others, and equals the oracle's sort of its
input, over the serving workload's whole size range (2^10 to 2^24 keys);
requests that arrive while the workers are busy share batches; a failed
launch fails only its own batch; budget admission, cancellation and the
error paths behave as documented."""
from __future__ import annotations

import time

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import announce, to_device

pytestmark = pytest.mark.gpu


def _oracle(keys: np.ndarray, vals: np.ndarray | None):
    """The request's exact result: the oracle's sort (stable by input index)."""
    nb = 4 if keys.size > 64 else 1
    r = oracle.pses(keys, nb, nb, vals=vals)
    return r.keys, r.vals


def _mixed_requests(n_req: int, seed: int):
    """The serving workload's shape: lognormal sizes (median 2^16, sigma 1.5)
    clipped to [2^10, 2^24], half uniform and half duplicate-heavy u64 keys
    with their input index as value.  Requests of 2^23 + 1 and 2^24 keys are
    added (each takes three merge passes in its batch), and keys-only requests
    of other types are interleaved to exercise batching by type."""
    _, sizes, dup = W.serving_requests(n_req, 1000.0, seed_arrival=seed, seed_size=seed + 1,
                                       seed_keys=seed + 2)
    sizes = sizes.tolist()
    sizes[5] = (1 << 23) + 1
    sizes[11] = 1 << 24
    reqs = []
    for i, (s, d) in enumerate(zip(sizes, dup)):
        if i % 7 == 3:
            reqs.append(("f64", W.normal_specials_f64(int(s), seed=seed * 100 + i), None))
        elif i % 7 == 6:
            reqs.append(("u32", W.duplicate3_u32(int(s), seed=seed * 100 + i), None))
        else:
            reqs.append(("u64", W.request_keys(int(s), bool(d), seed=seed * 100 + i),
                         W.index_values(int(s))))
    return reqs


def _stage(reqs):
    """Inputs and outputs of every request on the device, before any submit."""
    import torch

    staged = []
    for kt, k, v in reqs:
        dk = to_device(k)
        dv = to_device(v) if v is not None else None
        staged.append((kt, dk, torch.empty_like(dk), dv,
                       torch.empty_like(dv) if dv is not None else None))
    torch.cuda.synchronize()
    return staged


def _collect(reqs, staged):
    return [(ok.cpu().numpy().view(k.dtype),
             ov.cpu().numpy().view(np.uint32) if ov is not None else None)
            for (kt, k, v), (_, _, ok, _, ov) in zip(reqs, staged)]


def _submit_held(srv, hold):
    """Submit each large request once the previous one has left the queue,
    so that each occupies a worker of its own."""
    tickets = []
    for kt, dk, ok, dv, ov in hold:
        tickets.append(srv.submit(dk, ok, dv, ov, key_type=kt))
        deadline = time.time() + 10
        while srv.stats()["queued"] and time.time() < deadline:
            pass
    return tickets


def _run_mixed(srv, reqs, holders):
    """Occupy every worker with one large request, then submit all others at
    once: they queue while the workers are busy, so later batches take many
    requests each."""
    staged = _stage(reqs)
    hold = _stage(holders)
    tickets = _submit_held(srv, hold)
    tickets += [srv.submit(dk, ok, dv, ov, key_type=kt) for kt, dk, ok, dv, ov in staged]
    status = [srv.wait(t) for t in tickets]
    assert status == [0] * len(tickets)
    return _collect(reqs, staged), _collect(holders, hold)


def _run_alone(srv, reqs):
    staged = _stage(reqs)
    for kt, dk, ok, dv, ov in staged:
        assert srv.wait(srv.submit(dk, ok, dv, ov, key_type=kt)) == 0
    return _collect(reqs, staged)


def test_each_result_same_alone_and_in_the_mix():
    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd.serving import Server

    reqs = _mixed_requests(40, seed=31)
    holders = [("u64", W.request_keys(1 << 23, False, seed=900 + i), W.index_values(1 << 23))
               for i in range(3)]
    total = sum(k.size for _, k, _ in reqs) + sum(k.size for _, k, _ in holders)
    announce("serving mix", len(reqs), "requests +", len(holders), "holders", total, "keys")
    with Server(hbm_budget_bytes=3 << 30, max_streams=3) as srv:
        mixed, held = _run_mixed(srv, reqs, holders)
        st = srv.stats()
        assert st["completed"] == len(reqs) + len(holders)
        assert st["failed"] == 0 and st["rejected"] == 0
        assert 0 < st["latency_p50_ms"] <= st["latency_p99_ms"] <= st["latency_max_ms"]
        assert st["keys_completed"] == total
        assert st["keys_per_s"] > 0
        # continuous batching: requests that arrived while the workers were
        # busy shared batches
        assert st["mean_batch_requests"] > 1.0, st
        assert st["batches"] < len(reqs) + len(holders)
        assert st["budget_in_use"] == 0 and st["queued"] == 0
        announce("serving alone", len(reqs), "requests")
        srv.reset_stats()
        alone = _run_alone(srv, reqs)
        assert srv.stats()["mean_batch_requests"] == 1.0
    assert pss.device_check() == 0
    for i, ((kt, k, v), (mk, mv), (ak, av)) in enumerate(zip(reqs, mixed, alone)):
        ek, ev = _oracle(k, v)
        assert np.array_equal(mk.view(np.uint8), ak.view(np.uint8)), i
        assert np.array_equal(mk.view(np.uint8), ek.view(np.uint8)), i
        if v is not None:
            assert np.array_equal(mv, av), i
            assert np.array_equal(mv, ev), i
    for i, ((kt, k, v), (hk, hv)) in enumerate(zip(holders, held)):
        ek, ev = _oracle(k, v)
        assert np.array_equal(hk, ek) and np.array_equal(hv, ev), i


def test_injected_launch_fault_fails_one_batch_only():
    """A launch armed to fail (pss_debug_inject) fails the batch it falls in:
    every request of that batch reports PSS_ERR_HIP, every other request
    finishes with the oracle's result, the budget in use returns to 0 and the
    server keeps serving."""
    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd import _lib
    from paper_2305_05245_amd.serving import Server

    reqs = [("u64", W.request_keys(n, i % 2 == 0, seed=500 + i), W.index_values(n))
            for i, n in enumerate([3000, 70000, 1 << 17, 9000, 1 << 16, 40000, 123457, 5000,
                                   1 << 18, 777, 60000, 1 << 15])]
    holders = [("u64", W.request_keys(1 << 22, False, seed=950), W.index_values(1 << 22))]
    announce("serving injected fault", len(reqs), "requests")
    with Server(hbm_budget_bytes=1 << 30, max_streams=1) as srv:
        staged = _stage(reqs)
        hold = _stage(holders)
        try:
            # one worker: the holder's batch runs alone first (about 15
            # launches), then the rest in one or more batches (at least 11
            # launches more); the 20th launch fails
            _lib.debug_inject(_lib.INJECT_LAUNCH, 19)
            tickets = _submit_held(srv, hold)
            tickets += [srv.submit(dk, ok, dv, ov, key_type=kt) for kt, dk, ok, dv, ov in staged]
            status = [srv.wait(t) for t in tickets]
        finally:
            _lib.debug_inject(_lib.INJECT_NONE)
        st = srv.stats()
        failed = [i for i, s in enumerate(status) if s != 0]
        assert failed, "the armed launch did not fail any request"
        assert all(status[i] == _lib.ERR_HIP for i in failed)
        assert st["failed"] == len(failed)
        assert st["completed"] == len(tickets) - len(failed)
        assert st["budget_in_use"] == 0 and st["queued"] == 0
        # still serving: one more request after the fault
        extra = _stage([reqs[0]])
        kt, dk, ok, dv, ov = extra[0]
        assert srv.wait(srv.submit(dk, ok, dv, ov, key_type=kt)) == 0
        assert np.array_equal(_collect([reqs[0]], extra)[0][0], _oracle(*reqs[0][1:])[0])
    assert pss.device_check() == 0
    results = _collect(holders, hold) + _collect(reqs, staged)
    for i, ((kt, k, v), (gk, gv)) in enumerate(zip(holders + reqs, results)):
        if status[i] == 0:
            ek, ev = _oracle(k, v)
            assert np.array_equal(gk, ek) and np.array_equal(gv, ev), i


def test_injected_allocation_fault_at_server_creation():
    """An allocation armed to fail makes pss_server_create report
    PSS_ERR_BUDGET and release what it had allocated; the next server works."""
    import torch

    from paper_2305_05245_amd import PssError, _lib
    from paper_2305_05245_amd.serving import Server

    announce("serving allocation fault")
    try:
        _lib.debug_inject(_lib.INJECT_ALLOC, 2)   # the third allocation fails
        with pytest.raises(PssError) as e:
            Server(hbm_budget_bytes=256 << 20, max_streams=2)
        assert e.value.status == _lib.ERR_BUDGET
    finally:
        _lib.debug_inject(_lib.INJECT_NONE)
    k = W.request_keys(10000, True, seed=8)
    with Server(hbm_budget_bytes=256 << 20, max_streams=2) as srv:
        dk = to_device(k)
        out = torch.empty_like(dk)
        assert srv.wait(srv.submit(dk, out, key_type="u64")) == 0
        assert np.array_equal(out.cpu().numpy().view(np.uint64), _oracle(k, None)[0])


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
        assert np.array_equal(out.cpu().numpy().view(np.uint64), _oracle(k, None)[0])
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
            assert np.array_equal(out.cpu().numpy().view(np.uint64), _oracle(ks, None)[0])
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
