"""GPU parity on the 32-bit field 3*2^30+1 at a size that selects it by default
(Toeplitz n = 2^28 + 12345, m = 2^27 + 77: transform length 2^29): sampled
output words against oracle rows, the whole output against the 64-bit field's
(the coefficients are the same integers, so the bits must agree), and GF(2)
bilinearity."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import show_case, to_dev, to_host

pytestmark = pytest.mark.gpu

N_P0, M_P0 = (1 << 28) + 12345, (1 << 27) + 77


@pytest.fixture(scope="module")
def p0case():
    import torch

    import paper_2402_09481_amd as P
    ctx = P.Context(0)
    assert ctx._lib.ext_plan_length(0, N_P0, M_P0, None) == 1 << 29
    g = W.rng(2828)
    show_case("p0 case: generating inputs")
    x = W.bernoulli_bits(g, N_P0, 0.4)
    y = W.bernoulli_bits(g, N_P0 + M_P0 - 1, 0.5)
    xd, yd = to_dev(x), to_dev(y)
    show_case("p0 case: extracting")
    z = ctx.extract("toeplitz", xd, yd, N_P0, M_P0, sync=True)
    torch.cuda.synchronize()
    yield ctx, x, y, xd, yd, z
    del xd, yd, z
    ctx.close()
    torch.cuda.empty_cache()


def test_p0_selected_and_sampled_words(p0case):
    ctx, x, y, xd, yd, z = p0case
    import ctypes
    word_bits = ctypes.c_int32()
    assert ctx._lib.ext_plan_length(0, N_P0, M_P0, ctypes.byref(word_bits)) == 1 << 29 and word_bits.value == 32
    zh = to_host(z)
    nw = zh.size
    g = W.rng(12)
    words = sorted({0, 1, nw // 2, nw - 2, nw - 1} | {int(v) for v in g.integers(0, nw, 5)})
    for w in words:
        show_case("p0 word", w)
        cnt = min(64, M_P0 - 64 * w)
        want = oracle.toeplitz_rows(x, y, N_P0, M_P0, 64 * w, cnt, "paper")
        assert int(zh[w]) == int(want[0]), "word %d" % w


def test_p0_equals_64bit_field(p0case):
    import torch

    import paper_2402_09481_amd as P
    ctx, x, y, xd, yd, z = p0case
    os.environ["EXT_FORCE_FIELD"] = "gl"
    try:
        cgl = P.Context(0)
    finally:
        del os.environ["EXT_FORCE_FIELD"]
    show_case("p0 vs gl")
    z2 = cgl.extract("toeplitz", xd, yd, N_P0, M_P0, sync=True)
    assert torch.equal(z, z2)
    cgl.close()


def test_p0_bilinear(p0case):
    import torch
    ctx, x, y, xd, yd, z = p0case
    show_case("p0 bilinearity")
    x2 = to_dev(W.bernoulli_bits(W.rng(77), N_P0, 0.5))
    z2 = ctx.extract("toeplitz", x2, yd, N_P0, M_P0, sync=True)
    z3 = ctx.extract("toeplitz", torch.bitwise_xor(xd, x2), yd, N_P0, M_P0, sync=True)
    assert torch.equal(torch.bitwise_xor(z, z2), z3)
