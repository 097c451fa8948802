"""Pins of the oracle's GF(2)[t] product route (oracle/gf2x.c), the full-vector
check for the large workloads. It is pinned to what the mathematics fixes, not
to itself:

* the 64 x 64-bit carry-less product against a shift-and-XOR loop written here
  in Python, with the CPU instruction and with the library's own software loop;
* whole products against Python-integer carry-less multiplication (every size
  from one word to past the Karatsuba threshold, odd and unbalanced sizes);
* closed forms over GF(2): squaring spreads the bits (a(t)^2 = sum a_i t^(2i)),
  (1 + t)^(2^k) = 1 + t^(2^k), multiplication by t^k is a shift — at sizes with
  several Karatsuba levels;
* ring laws at size: commutativity, associativity, distributivity;
* each extractor against the schoolbook oracle (bit loop and packed rows), both
  Toeplitz seed orders, Dodis and Circulant over primes with primitive root 2,
  and the split of the defining sum into shares of input positions.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def clmul_py(a: int, b: int) -> int:
    r = 0
    while b:
        if b & 1:
            r ^= a
        a <<= 1
        b >>= 1
    return r


def to_int(words) -> int:
    return int.from_bytes(np.asarray(words, dtype="<u8").tobytes(), "little")


def from_int(v: int, nw: int) -> np.ndarray:
    return np.frombuffer(v.to_bytes(8 * nw, "little"), dtype="<u8").copy()


EDGE = [0, 1, 2, 3, (1 << 63), (1 << 64) - 1, 0x8000000000000001, 0x5555555555555555, 0xAAAAAAAAAAAAAAAA]


@pytest.mark.parametrize("software", [False, True])
def test_clmul64_against_shift_and_xor(software):
    g = W.rng(7)
    have = oracle.gf2_force_software(software)
    try:
        pairs = [(a, b) for a in EDGE for b in EDGE]
        pairs += [(int(a), int(b)) for a, b in g.integers(0, 1 << 64, (500, 2), dtype=np.uint64)]
        for a, b in pairs:
            assert oracle.clmul64(a, b) == clmul_py(a, b), (hex(a), hex(b))
    finally:
        oracle.gf2_force_software(False)
    assert software or have or True


@pytest.mark.parametrize("software", [False, True])
def test_product_against_python_integers(software):
    g = W.rng(8)
    oracle.gf2_force_software(software)
    try:
        sizes = [(1, 1), (1, 5), (2, 2), (3, 7), (31, 31), (32, 32), (33, 33), (33, 17), (64, 64), (65, 65),
                 (97, 40), (129, 129), (200, 3)]
        if not software:
            sizes += [(513, 513), (1000, 999), (4097, 4097)]
        for na, nb in sizes:
            a = g.integers(0, 1 << 64, na, dtype=np.uint64)
            b = g.integers(0, 1 << 64, nb, dtype=np.uint64)
            got = oracle.gf2_mul(a, b)
            assert to_int(got) == clmul_py(to_int(a), to_int(b)), (na, nb)
    finally:
        oracle.gf2_force_software(False)


def spread(words: np.ndarray) -> np.ndarray:
    """a(t)^2 over GF(2): bit i moves to bit 2i."""
    bits = W.unpack_bits(words, 64 * words.size)
    out = np.zeros(2 * bits.size, np.uint8)
    out[::2] = bits
    return W.pack_bits(out)


@pytest.mark.parametrize("nw", [40, 1 << 12, (1 << 14) + 3, 1 << 17])
def test_square_spreads_bits(nw):
    a = W.rng(nw).integers(0, 1 << 64, nw, dtype=np.uint64)
    assert np.array_equal(oracle.gf2_mul(a, a), spread(a))


@pytest.mark.parametrize("k", [6, 10, 13, 16, 19])
def test_frobenius_binomial(k):
    # (1 + t)^(2^k) = 1 + t^(2^k): k squarings of 1 + t
    p = np.array([3], np.uint64)
    for _ in range(k):
        p = oracle.gf2_mul(p, p)
        p = p[: max(1, ((int(to_int(p)).bit_length() + 63) >> 6))]
    assert to_int(p) == 1 | (1 << (1 << k))


@pytest.mark.parametrize("shift", [0, 1, 63, 64, 4097, 70001])
def test_times_monomial_is_shift(shift):
    a = W.rng(shift + 1).integers(0, 1 << 64, 3000, dtype=np.uint64)
    mono = W.pack_bits(np.eye(1, shift + 1, shift, dtype=np.uint8)[0])
    assert to_int(oracle.gf2_mul(a, mono)) == to_int(a) << shift


def test_ring_laws_at_size():
    g = W.rng(77)
    a, b, c = (g.integers(0, 1 << 64, k, dtype=np.uint64) for k in (5000, 3001, 4096))
    ab = oracle.gf2_mul(a, b)
    assert np.array_equal(ab, oracle.gf2_mul(b, a))
    left = oracle.gf2_mul(ab, c)
    right = oracle.gf2_mul(a, oracle.gf2_mul(b, c))
    assert to_int(left) == to_int(right)
    bc = b.copy()
    bc2 = np.zeros(b.size, np.uint64)
    bc2[: 3001] = c[:3001]
    lhs = oracle.gf2_mul(a, np.bitwise_xor(bc, bc2))
    rhs = np.bitwise_xor(oracle.gf2_mul(a, bc), oracle.gf2_mul(a, bc2))
    assert np.array_equal(lhs, rhs)


TOEPLITZ_SHAPES = [(1, 1), (5, 3), (63, 63), (64, 1), (65, 64), (100, 37), (129, 128), (1000, 500), (4096, 2048),
                   (20011, 777), (65536, 30000), (65601, 65601)]


@pytest.mark.parametrize("order", ["paper", "linear"])
def test_toeplitz_product_equals_schoolbook(order):
    g = W.rng(21)
    for n, m in TOEPLITZ_SHAPES:
        x = W.bernoulli_bits(g, n, 0.4)
        y = W.bernoulli_bits(g, n + m - 1, 0.5)
        want = oracle.extract("toeplitz", x, y, n, m, order)[1]
        assert np.array_equal(oracle.toeplitz_product(x, y, n, m, order)[1], want), (n, m)
        if n <= 129:  # the bit-by-bit loop as well
            assert np.array_equal(oracle.toeplitz(x, y, n, m, order)[1], want)


def test_toeplitz_shares_add_up():
    g = W.rng(22)
    n, m = 70000, 20001
    x, y = W.bernoulli_bits(g, n, 0.3), W.bernoulli_bits(g, n + m - 1, 0.5)
    want = oracle.extract("toeplitz", x, y, n, m, "paper")[1]
    seen = []
    for blk in (64, 640, 6400, 64000):
        got = oracle.toeplitz_product(x, y, n, m, "paper", block_bits=blk, progress=lambda d, t: seen.append(d))[1]
        assert np.array_equal(got, want), blk
    assert seen[-1] == n


def test_toeplitz_product_ignores_tail_bits():
    g = W.rng(23)
    n, m = 1000, 333
    x, y = W.bernoulli_bits(g, n, 0.5), W.bernoulli_bits(g, n + m - 1, 0.5)
    want = oracle.toeplitz_product(x, y, n, m)[1]
    xd, yd = x.copy(), y.copy()
    xd[-1] |= np.uint64(~((1 << (n & 63)) - 1) & ((1 << 64) - 1))
    yd[-1] |= np.uint64(~((1 << ((n + m - 1) & 63)) - 1) & ((1 << 64) - 1))
    assert np.array_equal(oracle.toeplitz_product(xd, yd, n, m)[1], want)


def test_dodis_and_circulant_products_equal_schoolbook():
    g = W.rng(24)
    primes = [p for p in (3, 5, 11, 13, 19, 29, 37, 59, 61, 67, 83, 101, 131, 1019, 4099, 65587) if oracle.is_na_prime(p)]
    assert len(primes) >= 12
    for n in primes:
        for m in sorted({1, max(1, n // 3), n - 1}):
            x = W.bernoulli_bits(g, n, 0.4)
            y = W.bernoulli_bits(g, n, 0.5)
            if oracle.check("dodis", n, m, x) == oracle.OK:
                want = oracle.extract("dodis", x, y, n, m)[1]
                assert np.array_equal(oracle.dodis_product(x, y, n, m)[1], want), ("dodis", n, m)
            want = oracle.extract("circulant", x, y, n - 1, m)[1]
            assert np.array_equal(oracle.circulant_product(x, y, n - 1, m)[1], want), ("circulant", n, m)
    # Dodis at full output length through the bit-by-bit loop
    x, y = W.bernoulli_bits(g, 13, 0.5), W.bernoulli_bits(g, 13, 0.5)
    if oracle.check("dodis", 13, 13, x) == oracle.OK:
        assert np.array_equal(oracle.dodis_product(x, y, 13, 13)[1], oracle.dodis(x, y, 13, 13)[1])


def test_products_report_preconditions():
    assert oracle.dodis_product(np.zeros(1, np.uint64), np.ones(1, np.uint64), 11, 5)[0] == oracle.EDEGENERATE
    assert oracle.circulant_product(np.zeros(1, np.uint64), np.ones(1, np.uint64), 11, 5)[0] == oracle.ENOTNA
    assert oracle.toeplitz_product(np.zeros(1, np.uint64), np.ones(1, np.uint64), 5, 6)[0] == oracle.EINVAL
