"""Host code of the library under the sanitizers (CPU only, no GPU).

* The argument checks, planning and workspace arithmetic of pss_api.hip, and
  the fault-injection counters, built for the host with the address and
  undefined-behaviour sanitizers (hipcc, host side only; the kernel
  launchers are replaced by stubs that are never reached).
* The serving loop's request queue (pss_queue.hpp) under a fake executor
  that sorts each batch with the CPU oracle: admission by budget, continuous
  batching, failure of one batch, cancellation and shutdown, built once with
  the address + undefined-behaviour sanitizers and once with the thread
  sanitizer.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2305_05245_amd", "csrc")
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_abi_under_asan_ubsan(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    base = [HIPCC, "--offload-arch=gfx950", "--cuda-host-only", "-O1", "-g", "-std=c++17", "-fPIC",
            *san, "-I", os.path.join(ROOT, "include")]
    objs = []
    for src, extra in ((os.path.join(CSRC, "pss_api.hip"), []),
                       (os.path.join(NATIVE, "kernel_stubs.cpp"), ["-x", "hip"]),
                       (os.path.join(NATIVE, "host_abi_sanitize.cpp"), [])):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run(base + extra + ["-c", src, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "host_abi")
    _run([HIPCC, "-fsanitize=address", "-fsanitize=undefined", *objs, "-o", exe])
    r = _run([exe])
    assert "host ABI checks passed" in r.stdout


@pytest.mark.parametrize("sanitizer", ["address,undefined", "thread"])
@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_serving_queue_fake_executor(tmp_path, sanitizer):
    flags = ["-O1", "-g", f"-fsanitize={sanitizer}", "-fno-sanitize-recover=all"]
    oracle_obj = str(tmp_path / "oracle.o")
    _run(["gcc", *flags, "-c", os.path.join(ROOT, "oracle", "pses_oracle.c"), "-o", oracle_obj])
    exe = str(tmp_path / "serving_queue")
    _run(["g++", "-std=c++17", *flags, "-I", os.path.join(ROOT, "include"),
          os.path.join(NATIVE, "serving_queue_fake.cpp"), oracle_obj, "-o", exe, "-lpthread"])
    r = _run([exe])
    assert "serving queue checks passed" in r.stdout
