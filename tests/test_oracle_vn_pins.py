"""Pins for the Von Neumann oracle: hand-worked values from the definition,
the exact uniformity of the output under the input model of eq. (2) (computed
by enumeration with exact rationals), the exact expected output length for
i.i.d. input, the output length in closed form, and concatenation of blocks
of even length."""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def vn_list(bits):
    """The oracle on a list of 0/1 values; returns (code, list of output bits)."""
    n = len(bits)
    words = W.pack_bits(np.array(bits, np.uint8)) if n else np.zeros(1, np.uint64)
    code, z, m = oracle.von_neumann(words, n)
    if code:
        return code, None
    return code, [int(b) for b in W.unpack_bits(z, m)]


def test_worked_values():
    rows = 0
    for line in open(os.path.join(GOLD, "von_neumann_worked.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        inp, want = (s.strip() for s in line.split("|"))
        code, out = vn_list([int(c) for c in inp])
        if want == "DEGENERATE":
            assert code == oracle.EDEGENERATE, inp
        elif want == "INVALID":
            assert code == oracle.EINVAL, inp
        else:
            assert code == oracle.OK and out == [int(c) for c in want], (inp, out)
        rows += 1
    assert rows == 12


def output_distribution(n, pair_dist, vn):
    """Exact distribution of vn's output for independent pairs, pair j drawn from
    pair_dist[j] = {(a, b): probability}; a trailing odd bit is 0 or 1 w.p. 1/2."""
    dist = {}
    npairs = n // 2
    for combo in itertools.product(*[list(pair_dist[j].items()) for j in range(npairs)]):
        pr = Fraction(1)
        bits = []
        for (ab, q) in combo:
            pr *= q
            bits += list(ab)
        for tail in ([0, 1] if n % 2 else [None]):
            b = bits + ([tail] if tail is not None else [])
            out = vn(b)
            key = tuple(out) if out is not None else ()
            dist[key] = dist.get(key, Fraction(0)) + pr * (Fraction(1, 2) if n % 2 else 1)
    return dist


def symmetric_pair(a00, a11):
    """An exchangeable pair distribution: Pr(01) = Pr(10)."""
    c = (1 - a00 - a11) / 2
    return {(0, 0): a00, (1, 1): a11, (0, 1): c, (1, 0): c}


def iid_pair(p):
    """Both bits i.i.d. with Pr(bit = 0) = p (eq. (2) with equal p_i)."""
    q = 1 - p
    return {(0, 0): p * p, (1, 1): q * q, (0, 1): p * q, (1, 0): q * p}


def uniform_given_length(dist):
    by_len = {}
    for out, pr in dist.items():
        by_len.setdefault(len(out), {})[out] = pr
    for m, d in by_len.items():
        if len(d) != 2 ** m or len(set(d.values())) != 1:
            return False
    return True


def oracle_vn(bits):
    code, out = vn_list(bits)
    return out if code == oracle.OK else []


def test_output_uniform_under_the_input_model():
    # pairs independent, each exchangeable with its own law (eq. (2): equal
    # marginals inside a pair); the output given its length is exactly uniform
    laws = [symmetric_pair(Fraction(1, 5), Fraction(1, 3)), iid_pair(Fraction(3, 10)),
            symmetric_pair(Fraction(1, 2), Fraction(1, 10)), iid_pair(Fraction(2, 3)),
            symmetric_pair(Fraction(1, 7), Fraction(4, 7))]
    for n in (8, 9, 10):
        assert uniform_given_length(output_distribution(n, laws, oracle_vn)), n


def test_uniformity_pin_catches_plausible_mistakes():
    laws = [iid_pair(Fraction(1, 5)), iid_pair(Fraction(3, 4)), iid_pair(Fraction(2, 5)), iid_pair(Fraction(1, 3))]

    def shifted_pairs(b):  # pairs (x_{2j+1}, x_{2j+2})
        return [b[i] for i in range(1, len(b) - 1, 2) if b[i] != b[i + 1]]

    def emits_on_equal(b):
        return [b[2 * j] for j in range(len(b) // 2) if b[2 * j] == b[2 * j + 1]]

    assert uniform_given_length(output_distribution(8, laws, oracle_vn))
    assert not uniform_given_length(output_distribution(8, laws, shifted_pairs))
    assert not uniform_given_length(output_distribution(8, laws, emits_on_equal))


def test_expected_length_iid():
    # E[m] = floor(n/2) * 2p(1-p) exactly (the paper's m ~ p(1-p)n counts ~n/2 pairs twice)
    for n in (6, 7):
        for p in (Fraction(1, 4), Fraction(3, 10), Fraction(1, 2)):
            dist = output_distribution(n, [iid_pair(p)] * (n // 2), oracle_vn)
            em = sum(len(o) * pr for o, pr in dist.items())
            assert em == (n // 2) * 2 * p * (1 - p)
            assert sum(dist.values()) == 1


def test_length_closed_form_and_blocks():
    g = W.rng(91)
    for n in [2, 3, 63, 64, 65, 127, 128, 129, 1000, 4095, 4096, 4097, 77777]:
        for p in (0.5, 0.2929, 0.05, 0.999):
            x = W.bernoulli_bits(g, n, p)
            code, z, m = oracle.von_neumann(x, n)
            X = int.from_bytes(np.asarray(x, np.uint64).tobytes(), "little") & ((1 << n) - 1)
            npairs = n // 2
            even = int("01" * npairs, 2) if npairs else 0  # bits 0, 2, 4, ...
            want_m = bin((X ^ (X >> 1)) & even).count("1")
            assert m == want_m, (n, p)
            assert code == (oracle.OK if want_m else oracle.EDEGENERATE)
            # blocks of even length: VN(a || b) = VN(a) || VN(b)
            if n >= 130:
                cut = 64 * ((n // 2) // 64)
                xa = W.pack_bits(W.unpack_bits(x, n)[:cut])
                xb = W.pack_bits(W.unpack_bits(x, n)[cut:])
                ca, za, ma = oracle.von_neumann(xa, cut)
                cb, zb, mb = oracle.von_neumann(xb, n - cut)
                got = W.unpack_bits(z, m) if m else np.zeros(0, np.uint8)
                parts = [W.unpack_bits(za, ma) if ma else np.zeros(0, np.uint8),
                         W.unpack_bits(zb, mb) if mb else np.zeros(0, np.uint8)]
                assert np.array_equal(got, np.concatenate(parts))


def test_tail_bits_and_odd_length():
    g = W.rng(5)
    x = W.bernoulli_bits(g, 301, 0.5)
    x_dirty = x.copy()
    x_dirty[-1] |= np.uint64(((1 << 64) - 1) ^ ((1 << 45) - 1))  # bits 301.. (beyond n) must be ignored
    a = oracle.von_neumann(x, 301)
    b = oracle.von_neumann(x_dirty, 301)
    c = oracle.von_neumann(x, 300)  # the odd last bit belongs to no pair
    assert a[2] == b[2] == c[2] and np.array_equal(a[1], b[1]) and np.array_equal(a[1], c[1])
    z, m = a[1], a[2]
    if m & 63:
        assert int(z[-1]) >> (m & 63) == 0
