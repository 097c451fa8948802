"""The paper's QKD privacy-amplification shapes (Toeplitz n = 1.738e9, m = 41,378,264,
and the improved Circulant variant, both run as two pieces of 2^30): sampled output
words against the oracle's rows, GF(2) bilinearity of the whole Toeplitz output, and
the whole Circulant output against the one 2^31 transform over the 64-bit field."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import show_case, to_dev, to_host

pytestmark = pytest.mark.gpu


def sampled_words(nw, seed):
    g = W.rng(seed)
    return sorted({0, nw // 2, nw - 1} | {int(v) for v in g.integers(0, nw, 2)})


def test_qkd_toeplitz():
    import torch

    import paper_2402_09481_amd as P
    ctx = P.Context(0)
    job = W.qkd_toeplitz()
    show_case("qkd toeplitz")
    x, y = to_dev(job.x), to_dev(job.y)
    z = to_host(ctx.extract("toeplitz", x, y, job.n, job.m, sync=True))
    assert z.size == W.nwords(job.m)
    r = job.m & 63
    assert r == 0 or int(z[-1]) >> r == 0  # tail bits zero
    for w in sampled_words(z.size, 1):
        cnt = min(64, job.m - 64 * w)
        want = oracle.toeplitz_rows(job.x, job.y, job.n, job.m, 64 * w, cnt)
        assert int(z[w]) == int(want[0]), w
    x2 = to_dev(W.bernoulli_bits(W.rng(2), job.n, 0.5))
    a = ctx.extract("toeplitz", x2, y, job.n, job.m, sync=True)
    b = ctx.extract("toeplitz", torch.bitwise_xor(x, x2), y, job.n, job.m, sync=True)
    assert torch.equal(torch.bitwise_xor(torch.from_numpy(z.view(np.int64)).cuda(), a), b)
    ctx.close()


def test_qkd_improved_circulant():
    import paper_2402_09481_amd as P
    ctx = P.Context(0)
    job = W.qkd_circulant(P.next_na_set)
    show_case("qkd circulant", job.n, job.m)
    x, y = to_dev(job.x), to_dev(job.y)
    z = to_host(ctx.extract("circulant", x, y, job.n, job.m, sync=True))  # two pieces of 2^30
    for w in sampled_words(z.size, 3):
        cnt = min(64, job.m - 64 * w)
        want = oracle.circulant_rows(job.x, job.y, job.n, job.m, 64 * w, cnt)
        assert int(z[w]) == int(want[0]), w
    # the whole output equals the one transform of 2^31 over 2^64 - 2^32 + 1
    z1 = to_host(ctx.extract("circulant", x, y, job.n, job.m, sync=True, single_transform=True))
    assert np.array_equal(z, z1)
    ctx.close()
