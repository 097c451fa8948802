"""The piece schedule over the 64-bit field: the defining sum over input
positions split into pieces, each a Toeplitz extraction with its own seed
window, the pieces' products added in the transform domain before one inverse.
It runs every shape longer than one transform of 2^32, among them the paper's
QRNG shapes (n = 6.5e9, section "Cryptomite for randomness extraction in
(Q)RNG").

* small and medium sizes with forced piece sizes (2 to 7 pieces, ragged last
  pieces, m below and above the piece size, both Toeplitz seed orders, Dodis and
  Circulant, the Dodis degenerate input) against the oracle's whole output;
* the QRNG Toeplitz and Circulant shapes at their sizes: sampled output words
  against the schoolbook oracle rows, GF(2) bilinearity of the whole output, and
  the whole output against the same extraction with another piece count;
* shapes whose one transform of 2^27 would run over 15*2^27+1, which the default
  plan runs as two pieces of at most 2^26 over the lazy field 7*2^26+1: the whole
  output against the oracle's GF(2)[t] product and against the one transform."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import gpu_extract, show_case, to_dev, to_host

pytestmark = pytest.mark.gpu


def _ctx(piece_bits=None):
    import paper_2402_09481_amd as P
    if piece_bits is None:
        return P.Context(0)
    os.environ["EXT_PIECE_BITS"] = str(int(piece_bits))
    try:
        return P.Context(0)
    finally:
        del os.environ["EXT_PIECE_BITS"]


@pytest.fixture(scope="module")
def ctx4k():
    c = _ctx(4096)
    yield c
    c.close()


def _seed_len(kind, n, m):
    return {"toeplitz": n + m - 1, "circulant": n + 1, "dodis": n}[kind]


@pytest.mark.parametrize("kind,n,m,order", [
    ("toeplitz", 4097, 1, "paper"),        # two pieces, the second of one bit
    ("toeplitz", 4097, 4097, "linear"),
    ("toeplitz", 12288, 777, "paper"),     # exactly three pieces
    ("toeplitz", 20000, 6000, "linear"),   # five pieces, m above the piece size
    ("toeplitz", 28671, 28671, "paper"),   # seven pieces, m = n
    ("dodis", 8219, 8000, "paper"),
    ("dodis", 20029, 3, "paper"),
    ("circulant", 16420, 9000, "paper"),   # 16421 is prime with primitive root 2
])
def test_pieces_small_against_oracle(ctx4k, kind, n, m, order):
    if kind != "toeplitz":
        assert oracle.is_na_prime(n if kind == "dodis" else n + 1)
    g = W.rng(n + m)
    x = W.bernoulli_bits(g, n, 0.4)
    y = W.bernoulli_bits(g, _seed_len(kind, n, m), 0.5)
    if kind == "dodis":
        x[0] = (int(x[0]) | 1) & ~2
    show_case("pieces", kind, n, m, order)
    code, z = gpu_extract(ctx4k, kind, x, y, n, m, order)
    assert code == 0
    assert np.array_equal(z, oracle.extract(kind, x, y, n, m, order)[1])


def test_pieces_dodis_degenerate(ctx4k):
    n = 8219
    for x in (np.zeros(W.nwords(n), np.uint64), W.mask_tail(np.full(W.nwords(n), ~np.uint64(0)), n)):
        y = W.bernoulli_bits(W.rng(3), n, 0.5)
        code, z = gpu_extract(ctx4k, "dodis", x, y, n, 5000)
        assert code == oracle.EDEGENERATE and not z.any()


def test_pieces_medium_against_product():
    c = _ctx(1 << 20)
    g = W.rng(31)
    n, m = (1 << 22) + 12345, (1 << 21) + 1
    x, y = W.bernoulli_bits(g, n, 0.3), W.bernoulli_bits(g, n + m - 1, 0.5)
    show_case("pieces medium", n, m)
    code, z = gpu_extract(c, "toeplitz", x, y, n, m)
    assert code == 0
    assert np.array_equal(z, oracle.toeplitz_product(x, y, n, m)[1])
    c.close()


def _qrng_check(kind, n, m, x, y, other_piece_bits, words):
    """Sampled words against the oracle rows, bilinearity, and the same output with
    another piece count."""
    import torch
    c = _ctx()
    show_case("qrng %s n=%d m=%d: extraction" % (kind, n, m))
    z = c.extract(kind, x, y, n, m, sync=True)
    zh = to_host(z)
    xh, yh = to_host(x), to_host(y)
    nw = zh.size
    for w in words(nw):
        show_case("qrng %s word %d" % (kind, w))
        cnt = min(64, m - 64 * w)
        if kind == "toeplitz":
            want = oracle.toeplitz_rows(xh, yh, n, m, 64 * w, cnt)
        else:
            want = oracle.circulant_rows(xh, yh, n, m, 64 * w, cnt)
        assert int(zh[w]) & ((1 << cnt) - 1) == int(want[0]), (kind, w)
    show_case("qrng %s bilinearity" % kind)
    x2 = W.bernoulli_bits_device(n, 0.5, 999)
    z2 = c.extract(kind, x2, y, n, m, sync=True)
    z3 = c.extract(kind, torch.bitwise_xor(x, x2), y, n, m, sync=True)
    assert torch.equal(torch.bitwise_xor(z, z2), z3)
    del x2, z2, z3
    c.close()
    torch.cuda.empty_cache()
    show_case("qrng %s: pieces of %d bits" % (kind, other_piece_bits))
    c2 = _ctx(other_piece_bits)
    z4 = c2.extract(kind, x, y, n, m, sync=True)
    assert torch.equal(z, z4)
    c2.close()
    del z, z4
    torch.cuda.empty_cache()


def test_qrng_toeplitz_shape():
    import torch
    n, m, x, y = W.qrng_toeplitz_device()
    assert (n, m) == (6_500_000_000, 581_294_933)
    _qrng_check("toeplitz", n, m, x, y, 1_000_000_000,
                lambda nw: sorted({0, nw // 2, nw - 1, int(W.rng(5).integers(0, nw))}))
    del x, y
    torch.cuda.empty_cache()


def test_qrng_circulant_shape():
    import torch
    n_in, m, x, y = W.qrng_circulant_device(oracle.closest_na)
    assert n_in + 1 == 6_500_000_069 and m == 516_294_932
    _qrng_check("circulant", n_in, m, x, y, 1_500_000_000,
                lambda nw: sorted({0, nw // 3, nw - 1, int(W.rng(6).integers(0, nw))}))
    del x, y
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind,n,m,order", [
    ("toeplitz", 1 << 24, 1 << 23, "paper"),   # one transform of 2^25 over the lazy field, halved
    ("toeplitz", 1 << 26, 1 << 25, "paper"),
    ("toeplitz", (1 << 26) - 333, (1 << 25) - 7, "linear"),
    ("dodis", None, 1 << 24, "paper"),        # n: the next prime >= 2^26 - 2^20 with primitive root 2
    ("circulant", None, (1 << 24) + 5, "paper"),
])
def test_two_pieces_over_the_lazy_field(kind, n, m, order):
    import ctypes

    import paper_2402_09481_amd as P
    if n is None:
        p = oracle.next_na((1 << 26) - (1 << 20))
        n = p if kind == "dodis" else p - 1
    c = _ctx()
    wb = ctypes.c_int32()
    k = {"toeplitz": 0, "circulant": 1, "dodis": 2}[kind]
    L2 = 1 << 24 if n == 1 << 24 else 1 << 26
    assert c._lib.ext_plan_length(k, n, m, ctypes.byref(wb)) == L2 and wb.value == 32  # two pieces
    g = W.rng(n ^ m)
    x = W.bernoulli_bits(g, n, 0.45)
    y = W.bernoulli_bits(g, _seed_len(kind, n, m), 0.5)
    show_case("lazy two-piece", kind, n, m, order)
    code, z = gpu_extract(c, kind, x, y, n, m, order)
    assert code == 0
    want = oracle.extract_product(kind, x, y, n, m, order)[1]
    assert np.array_equal(z, want)
    # the one transform (2^27 over 15*2^27+1, or 2^25 over the lazy field) gives the same bits
    zt = c.extract(kind, to_dev(x), to_dev(y), n, m, seed_order=order, sync=True, single_transform=True)
    assert np.array_equal(to_host(zt), want)
    if kind == "dodis":
        for xd in (np.zeros(W.nwords(n), np.uint64), W.mask_tail(np.full(W.nwords(n), ~np.uint64(0)), n)):
            code, z = gpu_extract(c, kind, xd, y, n, m)
            assert code == oracle.EDEGENERATE and not z.any()
    c.close()

