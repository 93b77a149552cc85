"""The benchmark's host baseline (the oracle's steps with their loops over
blocks, pivots and partitions run by OpenMP threads, n_B = n_P = threads as
in the paper's Section 3) gives the oracle's output exactly."""
import numpy as np
import pytest

import oracle
import workloads as W


@pytest.mark.parametrize("n,nb", [(0, 1), (1, 1), (1000, 7), (100003, 16), (1 << 20, 8),
                                  (5, 13)])
@pytest.mark.parametrize("make", [lambda n: W.uniform_i64(n, seed=2),
                                  lambda n: W.mod1000_i64(n, seed=3),
                                  lambda n: W.normal_specials_f64(n, seed=11, fraction=0.01),
                                  lambda n: W.duplicate3_u32(n, seed=16)],
                         ids=["uniform_i64", "mod1000", "f64_specials", "dup3_u32"])
def test_host_baseline_equals_oracle(n, nb, make):
    keys = make(n)
    got = oracle.host_parallel_pses(keys, nb, nb)
    exp = oracle.pses(keys, nb, nb).keys
    assert got.view(np.uint8).tobytes() == exp.view(np.uint8).tobytes()


def test_host_baseline_threads():
    assert oracle.host_parallel_threads() >= 1
