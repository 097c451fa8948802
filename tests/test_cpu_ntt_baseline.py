"""The CPU NTT baseline that the benchmark times gives the oracle's bits."""
import numpy as np
import pytest

import baseline
import oracle
import workloads as W


@pytest.mark.parametrize("n,m", [(1, 1), (2, 1), (5, 3), (64, 64), (65, 1), (100, 37), (1000, 999), (4096, 2048),
                                 (5000, 17)])
@pytest.mark.parametrize("order", ["paper", "linear"])
def test_cpu_ntt_matches_oracle(n, m, order):
    g = W.rng(n * 7 + m)
    x = W.bernoulli_bits(g, n, 0.4)
    y = W.bernoulli_bits(g, n + m - 1, 0.5)
    code, want = oracle.extract("toeplitz", x, y, n, m, order)
    assert code == 0
    assert np.array_equal(baseline.toeplitz(x, y, n, m, order), want)
