"""pss_sort_noalloc (the allocation-free entry point, on the library's fixed
scratch array) gives exactly pss_sort's output, through the C ABI, on two
calls in a row with the second smaller than the first; requests that do not
fit the scratch array are refused before anything is launched."""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, to_device

pytestmark = pytest.mark.gpu


def _noalloc(ctx, kt, vt, dk, dv, n_blocks=0, n_parts=0):
    import torch

    out = torch.empty_like(dk)
    vout = torch.empty_like(dv) if dv is not None else None
    ctx.sort_noalloc(kt, vt, dk.data_ptr(), out.data_ptr(), dv.data_ptr() if dv is not None else 0,
                     vout.data_ptr() if vout is not None else 0, dk.numel(), n_blocks, n_parts,
                     torch.cuda.current_stream().cuda_stream)
    return out, vout


def _with_workspace(ctx, kt, vt, dk, dv, n_blocks=0, n_parts=0):
    import torch

    from paper_2305_05245_amd import _lib

    out = torch.empty_like(dk)
    vout = torch.empty_like(dv) if dv is not None else None
    ws = torch.empty(max(_lib.workspace_bytes(kt, vt, dk.numel(), n_blocks, n_parts), 256),
                     dtype=torch.uint8, device=dk.device)
    ctx.sort(kt, vt, dk.data_ptr(), out.data_ptr(), dv.data_ptr() if dv is not None else 0,
             vout.data_ptr() if vout is not None else 0, dk.numel(), n_blocks, n_parts,
             ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
    return out, vout


def _largest_fitting(kt, vt, n_blocks=0, n_parts=0):
    """Largest n whose workspace fits the scratch array (bisection on the
    library's own workspace size)."""
    from paper_2305_05245_amd import _lib

    lo, hi = 0, 1 << 30
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if _lib.workspace_bytes(kt, vt, mid, n_blocks, n_parts) <= _lib.NOALLOC_SCRATCH_BYTES:
            lo = mid
        else:
            hi = mid
    return lo


@pytest.mark.parametrize("case", ["i64", "u64+u32", "f64-paper"])
def test_noalloc_equals_pss_sort_two_calls(case):
    import torch

    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd import _lib

    ctx = pss._context(0)
    kt = {"i64": _lib.I64, "u64+u32": _lib.U64, "f64-paper": _lib.F64}[case]
    vt = _lib.VAL_U32 if case == "u64+u32" else _lib.VAL_NONE
    nb = np_ = 64 if case == "f64-paper" else 0
    n_max = _largest_fitting(kt, vt, nb, np_)
    assert n_max > 1_000_000
    for call, n in enumerate((n_max, 100_003)):       # the second call is smaller
        announce("noalloc", case, "call", call, "n", n)
        if case == "i64":
            keys = W.uniform_i64(n, seed=60 + call)
        elif case == "u64+u32":
            keys = W.request_keys(n, call == 1, seed=60 + call)
        else:
            keys = W.normal_specials_f64(n, seed=60 + call, fraction=0.01)
        dk = to_device(keys)
        dv = to_device(W.index_values(n)) if vt == _lib.VAL_U32 else None
        a_k, a_v = _noalloc(ctx, kt, vt, dk, dv, nb, np_)
        b_k, b_v = _with_workspace(ctx, kt, vt, dk, dv, nb, np_)
        torch.cuda.synchronize()
        assert torch.equal(a_k, b_k), (case, call)
        if dv is not None:
            assert torch.equal(a_v, b_v), (case, call)
    assert pss.device_check() == 0


def test_noalloc_torch_wrapper_equals_sort():
    """The torch-facing pss.sort_noalloc: caller-given outputs, the same
    result as pss.sort, key-value included."""
    import torch

    import paper_2305_05245_amd as pss

    n = 300_001
    announce("noalloc torch wrapper", n)
    dk = to_device(W.uniform_i64(n, seed=70))
    dv = torch.arange(n, dtype=torch.int32, device="cuda")
    ko, vo = torch.empty_like(dk), torch.empty_like(dv)
    pss.sort_noalloc(dk, ko, dv, vo)
    ek, ev = pss.sort(dk, dv)
    torch.cuda.synchronize()
    assert torch.equal(ko, ek) and torch.equal(vo, ev)
    with pytest.raises(ValueError):
        pss.sort_noalloc(dk, None)
    assert pss.device_check() == 0


def test_noalloc_refuses_requests_above_the_scratch_array():
    import torch

    import paper_2305_05245_amd as pss
    from paper_2305_05245_amd import PssError, _lib

    ctx = pss._context(0)
    n = _largest_fitting(_lib.I64, _lib.VAL_NONE) + 1
    announce("noalloc refusal", n)
    dk = torch.zeros(n, dtype=torch.int64, device="cuda")
    out = torch.full_like(dk, 7)
    with pytest.raises(PssError) as e:
        ctx.sort_noalloc(_lib.I64, _lib.VAL_NONE, dk.data_ptr(), out.data_ptr(), 0, 0, n, 0, 0,
                         torch.cuda.current_stream().cuda_stream)
    assert e.value.status == _lib.ERR_WORKSPACE
    torch.cuda.synchronize()
    assert bool((out == 7).all())      # nothing was launched
