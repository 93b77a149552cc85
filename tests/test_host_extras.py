"""Host-side checks of the regular-sampling, record and merge-method entry
points and of bench.py's command-line contract (no GPU needed)."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2305_05245_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


@pytest.mark.parametrize("n,n_b,n_p", [(0, 4, 3), (5, 4, 3), (5, 4, 9), (1000, 1, 50), (1000, 50, 1),
                                       (12, 3, 3), (100003, 7, 13), (20000, 2048, 5)])
def test_psrs_sample_count_matches_the_oracle(oracle_lib, n, n_b, n_p):
    keys = np.arange(n, dtype=np.uint32)[::-1].copy()
    assert _lib.psrs_sample_count(n, n_b, n_p) == oracle_lib.psrs(keys, n_b, n_p).samples.size


def test_psrs_and_record_workspaces(lib):
    a = _lib.psrs_workspace_bytes(_lib.I64, _lib.VAL_NONE, 1 << 20, 64, 64)
    b = _lib.psrs_workspace_bytes(_lib.I64, _lib.VAL_NONE, 1 << 22, 64, 64)
    assert 0 < a < b
    assert _lib.psrs_workspace_bytes(_lib.I64, _lib.VAL_NONE, 1 << 20, 64, 64) >= \
        _lib.workspace_bytes(_lib.I64, _lib.VAL_NONE, 1 << 20, 64, 64)
    r1 = _lib.records_workspace_bytes(_lib.U64, 1 << 20)
    r2 = _lib.records_workspace_bytes(_lib.U64, 1 << 21)
    assert 0 < r1 < r2
    # keys, indices, sorted keys and permutation come on top of the key-value sort's workspace
    assert r1 >= _lib.workspace_bytes(_lib.U64, _lib.VAL_U32, 1 << 20) + (1 << 20) * 24
    with pytest.raises(_lib.PssError):
        _lib.psrs_workspace_bytes(_lib.I64, _lib.VAL_NONE, 1000, 0, 4)     # PSRS needs n_B > 0
    with pytest.raises(_lib.PssError):
        _lib.psrs_workspace_bytes(_lib.I64, _lib.VAL_NONE, 1 << 30, 2048, 1 << 20)  # > 2^27 samples
    with pytest.raises(_lib.PssError):
        _lib.records_workspace_bytes(9, 100)                                 # unknown key type


def test_null_context_is_rejected(lib):
    vp = ctypes.c_void_p
    assert lib.pss_psrs_sort(None, _lib.I64, _lib.VAL_NONE, vp(8), vp(4096), None, None, 10, 2, 2,
                             None, vp(8192), 1 << 20, None) == _lib.ERR_INVALID
    assert lib.pss_psrs_splitters(None, _lib.I64, vp(8), 10, 2, 2, None, None, None, None, None,
                                  vp(8192), 1 << 20, None) == _lib.ERR_INVALID
    assert lib.pss_sort_records(None, _lib.U64, vp(8), vp(4096), 10, 16, 0, vp(8192), 1 << 20,
                                None) == _lib.ERR_INVALID
    assert lib.pss_set_merge_method(None, 1) == _lib.ERR_INVALID


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_kernel_source_digest_ignores_comments(tmp_path):
    sys.path.insert(0, ROOT)
    import bench

    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("int f(int x) {\n  return x + 1;  // add one\n}\n/* block */\n")
    b.write_text("int f(int x)   {\n\n  return x + 1;\n}\n")
    c.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.kernel_source_digest(str(a)) == bench.kernel_source_digest(str(b))
    assert bench.kernel_source_digest(str(a)) != bench.kernel_source_digest(str(c))


def test_measured_traffic_is_read_only_for_the_source_it_was_taken_on():
    """bench.py reads the merge kernel's HBM traffic from the committed counter
    summary only while its source digest matches the kernel source; when it
    does, the figure lies between the algorithmic bytes and twice them."""
    import bench

    t = bench.measured_traffic("merge", 28, "uniform")
    if t is not None:
        assert 16 * (1 << 28) <= t <= 32 * (1 << 28)
    assert bench.measured_traffic("tile_sort", 28, "uniform") is None
    assert bench.measured_traffic("merge", 27, "uniform") is None


def test_small_case_cpu_child_prints_one_json_object():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-child", "oracle_small"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    import json

    res = json.loads(r.stdout.strip().splitlines()[-1])
    assert res["n"] == 1 << 20 and res["runs"] == 5 and res["ascending"] and res["seconds"] > 0
