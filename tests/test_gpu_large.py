"""GPU parity at the full Toeplitz size (n = 2^30, m = 2^29): the library's default
plan (two pieces, transforms of 2^30 over 3*2^30+1) against the oracle on
sampled output words computed one row at a time, GF(2) bilinearity of the whole
output, and the whole output of the one-transform plan (length 2^31 over the
64-bit field) — the same integers, so the same bits."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import show_case, to_dev, to_host

pytestmark = pytest.mark.gpu

N_LARGE, M_LARGE = 1 << 30, 1 << 29


@pytest.fixture(scope="module")
def large():
    import paper_2402_09481_amd as P
    import torch
    ctx = P.Context(0)
    show_case("toeplitz_large: generating inputs")
    job = W.toeplitz_large()
    x, y = to_dev(job.x), to_dev(job.y)
    show_case("toeplitz_large: extracting")
    z = ctx.extract("toeplitz", x, y, job.n, job.m, sync=True)
    torch.cuda.synchronize()
    yield ctx, job, x, y, z
    del x, y, z
    ctx.close()
    torch.cuda.empty_cache()


def test_large_sampled_words(large):
    ctx, job, x, y, z = large
    zh = to_host(z)
    assert zh.size == M_LARGE // 64
    g = W.rng(11)
    nw = zh.size
    words = sorted({0, 1, nw // 2 - 1, nw // 2, nw - 2, nw - 1} | {int(v) for v in g.integers(0, nw, 4)})
    for w in words:
        show_case("toeplitz_large word", w)
        want = oracle.toeplitz_rows(job.x, job.y, job.n, job.m, 64 * w, 64, job.seed_order)
        assert int(zh[w]) == int(want[0]), "word %d" % w


def test_large_bilinear(large):
    import torch
    ctx, job, x, y, z = large
    show_case("toeplitz_large bilinearity")
    x2 = to_dev(W.bernoulli_bits(W.rng(99), job.n, 0.5))
    z2 = ctx.extract("toeplitz", x2, y, job.n, job.m, sync=True)
    z3 = ctx.extract("toeplitz", torch.bitwise_xor(x, x2), y, job.n, job.m, sync=True)
    assert torch.equal(torch.bitwise_xor(z, z2), z3)
    del x2, z2, z3


def test_large_two_piece_equals_64bit_transform(large):
    import torch

    import paper_2402_09481_amd as P
    ctx, job, x, y, z = large
    os.environ["EXT_FORCE_FIELD"] = "gl"
    try:
        cgl = P.Context(0)
    finally:
        del os.environ["EXT_FORCE_FIELD"]
    show_case("toeplitz_large: 64-bit single transform")
    z64 = cgl.extract("toeplitz", x, y, job.n, job.m, sync=True)
    assert torch.equal(z, z64)
    del z64
    cgl.close()
    torch.cuda.empty_cache()
