"""Captured segmented-sort graphs: every replay, with the program's own eager
work and synchronisations between replays, must equal the eager segmented
sort of the same batch and the stable per-segment order."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from gpu_util import announce, to_device

pytestmark = pytest.mark.gpu


def _batch(seed: int, n_segs: int, lo_exp: float, hi_exp: float, dup_every: int):
    sizes = W.segment_sizes_loguniform(n_segs, lo_exp, hi_exp, seed=seed)
    keys = [W.request_keys(int(s), dup=(i % dup_every == 0), seed=seed * 1000 + i)
            for i, s in enumerate(sizes)]
    return sizes, keys


def _expected(keys):
    """Per segment: stable order of the uint64 keys and their segment-local
    input indices."""
    ek, ev = [], []
    for k in keys:
        o = np.argsort(k, kind="stable")
        ek.append(k[o])
        ev.append(o.astype(np.uint32))
    return np.concatenate(ek), np.concatenate(ev)


def test_graph_replays_equal_eager_and_stable_order():
    import torch

    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd.segmented import SegmentedGraph

    announce("graph capture", "n_cap=2^20", "seg_cap=256", "u64+u32")
    g = SegmentedGraph(1 << 20, 256, "u64", with_vals=True)
    stream = torch.cuda.Stream()
    cases = [(21, 200, 6, 13), (22, 37, 8, 15), (21, 200, 6, 13), (23, 256, 6, 12), (24, 1, 19, 19.9)]
    side = torch.from_numpy(W.uniform_i64(300_000, seed=9)).cuda()
    for rep, (seed, n_segs, lo, hi) in enumerate(cases):
        sizes, keys = _batch(seed, n_segs, lo, hi, dup_every=2)
        total = int(sizes.sum())
        assert total <= g.n_cap
        announce("graph replay", rep, "seed", seed, "segs", n_segs, "keys", total)
        dk = [to_device(k) for k in keys]
        dv = [torch.arange(k.size, dtype=torch.int32, device="cuda") for k in keys]
        offs = g.load(dk, dv, stream)
        g.run(stream)
        stream.synchronize()
        got_k = g.keys_out[:total].cpu().numpy().view(np.uint64)
        got_v = g.vals_out[:total].cpu().numpy().view(np.uint32)

        # eager run of the same batch on the default stream
        ek, ev = pss.segmented_sort(torch.cat(dk), offs, vals=torch.cat(dv), key_type="u64")
        torch.cuda.synchronize()
        assert np.array_equal(got_k, ek.cpu().numpy().view(np.uint64))
        assert np.array_equal(got_v, ev.cpu().numpy().view(np.uint32))

        xk, xv = _expected(keys)
        assert np.array_equal(got_k, xk)
        assert np.array_equal(got_v, xv)

        # unrelated eager work between replays
        pss.sort(side)
        torch.cuda.synchronize()
        assert pss.device_check(0) == 0
    g.graph.close()
