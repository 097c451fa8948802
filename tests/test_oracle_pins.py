"""Pins for the oracle: every check here compares it with something other than
itself — the matrices as the paper prints them, the paper's own implementation
route (embedding + cyclic convolution), exact big-integer convolution, the
Circulant two-universality theorem, hand-derived worked values, and
brute-force order computations for the prime utilities."""
import itertools
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def bits(words, n):
    return W.unpack_bits(words, n).astype(np.int64)


def rand_bits(g, n, p=0.5):
    return (g.random(n) < p).astype(np.uint8)


# ------------------------------------------------------------ matrices as printed

def toep_matrix_printed(y, n, m):
    """toep(y) of eq. toep, m rows and n columns, built the way it is drawn: the
    first column is y_0 .. y_{m-1}, the first row is y_0, y_{N-1}, y_{N-2}, ..., y_m,
    and every diagonal is constant."""
    N = n + m - 1
    T = np.zeros((m, n), np.int64)
    T[:, 0] = y[:m]
    T[0, 0] = y[0]
    for j in range(1, n):
        T[0, j] = y[N - j]
    for i in range(1, m):
        for j in range(1, n):
            T[i, j] = T[i - 1, j - 1]
    return T


def circ_matrix_printed(a):
    """circ(a) of eq. circ-matrix: row 0 is a, each next row is the previous one
    shifted right by one position (cyclically)."""
    n = len(a)
    C = np.zeros((n, n), np.int64)
    C[0] = a
    for i in range(1, n):
        C[i] = np.roll(C[i - 1], 1)
    return C


@pytest.mark.parametrize("n,m", [(1, 1), (2, 1), (2, 2), (5, 3), (7, 7), (13, 4), (64, 64), (65, 63), (100, 37)])
def test_toeplitz_matches_printed_matrix(n, m):
    g = W.rng(n * 1000 + m)
    for _ in range(6):
        x, y = rand_bits(g, n), rand_bits(g, n + m - 1)
        want = toep_matrix_printed(y.astype(np.int64), n, m) @ x.astype(np.int64) % 2
        code, z = oracle.toeplitz(W.pack_bits(x), W.pack_bits(y), n, m, "paper")
        assert code == 0
        assert (bits(z, m) == want).all()
        zr = oracle.toeplitz_rows(W.pack_bits(x), W.pack_bits(y), n, m, 0, m, "paper")
        assert (bits(zr, m) == want).all()


@pytest.mark.parametrize("n_in,m", [(2, 1), (2, 2), (4, 4), (10, 5), (12, 12), (18, 9), (60, 59), (82, 40)])
def test_circulant_matches_printed_matrix(n_in, m):
    assert oracle.is_na_prime(n_in + 1)
    g = W.rng(n_in * 7 + m)
    for _ in range(6):
        x, y = rand_bits(g, n_in), rand_bits(g, n_in + 1)
        xp = np.concatenate([x, [0]]).astype(np.int64)  # x' = [x, 0]
        want = (circ_matrix_printed(xp) @ y.astype(np.int64) % 2)[:m]
        code, z = oracle.circulant(W.pack_bits(x), W.pack_bits(y), n_in, m)
        assert code == 0 and (bits(z, m) == want).all()
        zr = oracle.circulant_rows(W.pack_bits(x), W.pack_bits(y), n_in, m, 0, m)
        assert (bits(zr, m) == want).all()


@pytest.mark.parametrize("n,m", [(3, 3), (5, 2), (11, 11), (13, 7), (59, 30), (61, 61), (83, 1)])
def test_dodis_matches_printed_matrix(n, m):
    g = W.rng(n * 13 + m)
    for _ in range(6):
        x = rand_bits(g, n)
        x[0], x[1] = 1, 0  # never degenerate
        y = rand_bits(g, n)
        want = (circ_matrix_printed(x.astype(np.int64)) @ y.astype(np.int64) % 2)[:m]
        code, z = oracle.dodis(W.pack_bits(x), W.pack_bits(y), n, m)
        assert code == 0 and (bits(z, m) == want).all()
        zr = oracle.dodis_rows(W.pack_bits(x), W.pack_bits(y), n, m, 0, m)
        assert (bits(zr, m) == want).all()


def test_dodis_unit_seed_golden():
    rows = [l.split() for l in open(os.path.join(GOLD, "dodis_n5_unit_seeds.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for xs, k, zs in rows:
        x = np.array([int(c) for c in xs], np.uint8)
        y = np.zeros(5, np.uint8)
        y[int(k)] = 1
        code, z = oracle.dodis(W.pack_bits(x), W.pack_bits(y), 5, 5)
        assert code == 0
        assert "".join(str(b) for b in bits(z, 5)) == zs


# ------------------------------------------------------------ the paper's implementation route

def cyclic_conv_int(u, v):
    """Exact integer cyclic convolution (numpy integer convolve, then wrap)."""
    L = len(u)
    full = np.convolve(u.astype(np.int64), v.astype(np.int64))
    w = full[:L].copy()
    w[: len(full) - L] += full[L:]
    return w


@pytest.mark.parametrize("n,m", [(1, 1), (3, 2), (8, 8), (16, 5), (33, 17), (64, 64), (100, 61), (257, 128)])
def test_toeplitz_equals_embedding_alg2(n, m):
    """Alg. 2 (Toeplitz implementation): u' = x padded; v'[i] = y_i for i < m and
    v'[L-n+1+i] = y_{m+i} for i = 0 .. n-2 (the printed loop runs to n-1, which
    reads y_N and writes v'[L], both out of range); w = cyclic conv(u', v');
    output = first m entries of w mod 2. Any L >= n + m - 1 gives the same bits."""
    g = W.rng(n * 31 + m)
    N = n + m - 1
    for L in sorted({1 << (N - 1).bit_length(), 2 * (1 << (N - 1).bit_length()), 1 << (2 * n).bit_length()}):
        if L < N:
            continue
        x, y = rand_bits(g, n), rand_bits(g, N)
        u = np.zeros(L, np.int64)
        v = np.zeros(L, np.int64)
        u[:n] = x
        v[:m] = y[:m]
        for i in range(n - 1):
            v[L - n + 1 + i] = y[m + i]
        want = cyclic_conv_int(u, v)[:m] % 2
        code, z = oracle.toeplitz(W.pack_bits(x), W.pack_bits(y), n, m, "paper")
        assert code == 0 and (bits(z, m) == want).all()


@pytest.mark.parametrize("n,m", [(3, 3), (5, 5), (11, 6), (13, 13), (29, 10), (53, 53), (101, 50)])
def test_dodis_equals_alg1_with_fold(n, m):
    """Alg. 1 (Dodis implementation): u'[i] = x_{(n-i) mod n}, v' = y, integer
    convolution; the indices of the R(x) * y form are taken mod n, so output i is
    w_i + w_{i+n} (mod 2). Without that fold the printed algorithm differs."""
    assert oracle.is_na_prime(n)
    g = W.rng(n * 17 + m)
    differs = 0
    for _ in range(8):
        x = rand_bits(g, n)
        x[0], x[-1] = 1, 0
        y = rand_bits(g, n)
        u = np.array([x[(n - i) % n] for i in range(n)], np.int64)
        w = np.convolve(u, y.astype(np.int64))  # length 2n - 1
        w = np.concatenate([w, [0]])
        want = (w[:m] + w[n: n + m]) % 2
        code, z = oracle.dodis(W.pack_bits(x), W.pack_bits(y), n, m)
        assert code == 0 and (bits(z, m) == want).all()
        differs += int((w[:m] % 2 != want).any())
    assert differs > 0


def test_circulant_is_dodis_on_padded_input():
    """Circulant uses the Dodis implementation with x padded by one 0 bit."""
    g = W.rng(5)
    for n in (5, 11, 13, 59, 61, 83, 101, 1019):
        assert oracle.is_na_prime(n)
        for m in (1, n // 2, n - 1):
            x = rand_bits(g, n - 1)
            y = rand_bits(g, n)
            xp = np.concatenate([x, [0]]).astype(np.uint8)
            if xp.sum() == 0:
                xp[0] = x[0] = 1
            c1, z1 = oracle.circulant(W.pack_bits(x), W.pack_bits(y), n - 1, m)
            c2, z2 = oracle.dodis(W.pack_bits(xp), W.pack_bits(y), n, m)
            assert c1 == 0 and c2 == 0 and (z1 == z2).all()


# ------------------------------------------------------------ exact integer convolution

def kronecker_conv(a, b):
    """Exact integer linear convolution via one big-integer product: pack each
    coefficient into a field wide enough that no field overflows."""
    width = max(len(a), len(b)).bit_length() + 2
    A = int("".join(format(int(t), "0%db" % width) for t in a[::-1]), 2)
    B = int("".join(format(int(t), "0%db" % width) for t in b[::-1]), 2)
    C = A * B
    mask = (1 << width) - 1
    out = []
    for _ in range(len(a) + len(b) - 1):
        out.append(C & mask)
        C >>= width
    return out


@pytest.mark.parametrize("n,m", [(64, 32), (1000, 999), (4096, 2048), (5000, 1234)])
def test_toeplitz_linear_is_convolution_parity(n, m):
    """Linear seed order: z_i is the parity of coefficient i + n - 1 of the
    integer product x(t) s(t)."""
    g = W.rng(n + 3 * m)
    x, s = rand_bits(g, n), rand_bits(g, n + m - 1)
    c = kronecker_conv(x, s)
    want = np.array([c[i + n - 1] & 1 for i in range(m)], np.int64)
    code, z = oracle.toeplitz(W.pack_bits(x), W.pack_bits(s), n, m, "linear")
    assert code == 0 and (bits(z, m) == want).all()
    zr = oracle.toeplitz_rows(W.pack_bits(x), W.pack_bits(s), n, m, 0, m, "linear")
    assert (bits(zr, m) == want).all()


def test_seed_orders_are_a_rotation():
    """s_k = y_{(k + m) mod N} turns the paper's seed order into the linear one."""
    g = W.rng(77)
    for n, m in [(1, 1), (7, 3), (64, 1), (65, 65), (300, 123)]:
        N = n + m - 1
        x, y = rand_bits(g, n), rand_bits(g, N)
        s = np.array([y[(k + m) % N] for k in range(N)], np.uint8)
        _, zp = oracle.toeplitz(W.pack_bits(x), W.pack_bits(y), n, m, "paper")
        _, zl = oracle.toeplitz(W.pack_bits(x), W.pack_bits(s), n, m, "linear")
        assert (zp == zl).all()


# ------------------------------------------------------------ structure and linearity

@pytest.mark.parametrize("kind", ["toeplitz", "circulant", "dodis"])
def test_bilinear_over_gf2(kind):
    g = W.rng(hash(kind) & 0xFFFF)
    n = {"toeplitz": 777, "circulant": 786, "dodis": 787}[kind]  # 787 is prime with primitive root 2
    m = 300
    nseed = {"toeplitz": n + m - 1, "circulant": n + 1, "dodis": n}[kind]
    x1, x2 = rand_bits(g, n), rand_bits(g, n)
    y1, y2 = rand_bits(g, nseed), rand_bits(g, nseed)
    x1[0], x1[1], x2[0], x2[1] = 1, 0, 0, 1
    f = lambda a, b: oracle.extract(kind, W.pack_bits(a), W.pack_bits(b), n, m)[1]
    # x1, x2 and x1 ^ x2 all have a 1 and a 0 in their first two bits, so none is
    # degenerate for Dodis
    assert (f(x1, y1) ^ f(x2, y1) == f(x1 ^ x2, y1)).all()
    assert (f(x1, y1) ^ f(x1, y2) == f(x1, y1 ^ y2)).all()


def test_dodis_shift_equivariance():
    """Rotating x and y by the same amount leaves Dodis unchanged; rotating y alone
    by k rotates the full (m = n) output by k."""
    n = 61
    g = W.rng(61)
    x, y = rand_bits(g, n), rand_bits(g, n)
    x[0], x[1] = 1, 0
    z = bits(oracle.dodis(W.pack_bits(x), W.pack_bits(y), n, n)[1], n)
    for k in (1, 5, 60):
        z2 = bits(oracle.dodis(W.pack_bits(np.roll(x, k)), W.pack_bits(np.roll(y, k)), n, n)[1], n)
        assert (z == z2).all()
        z3 = bits(oracle.dodis(W.pack_bits(x), W.pack_bits(np.roll(y, k)), n, n)[1], n)
        assert (z3 == np.roll(z, k)).all()


def gf2_rank(M):
    M = (np.array(M) % 2).astype(np.uint8)
    r = 0
    rows, cols = M.shape
    for c in range(cols):
        piv = next((i for i in range(r, rows) if M[i, c]), None)
        if piv is None:
            continue
        M[[r, piv]] = M[[piv, r]]
        for i in range(rows):
            if i != r and M[i, c]:
                M[i] ^= M[r]
        r += 1
    return r


@pytest.mark.parametrize("n", [3, 5, 11, 13])
def test_circulant_rank_lemma(n):
    """circ(d') has GF(2) rank >= n - 1 for every d' other than 0^n and 1^n when n is
    prime with primitive root 2 (the row-rank lemma of the Circulant proof)."""
    for d in itertools.product([0, 1], repeat=n):
        if sum(d) in (0, n):
            continue
        assert gf2_rank(circ_matrix_printed(np.array(d))) >= n - 1


@pytest.mark.parametrize("n,m", [(5, 1), (5, 2), (5, 4), (11, 3), (11, 10), (13, 6)])
def test_circulant_two_universal_exact(n, m):
    """For every x != x~ exactly 2^(n-m) of the 2^n seeds collide (the
    two-universality theorem). By linearity a collision of x and x~ is a zero output
    for d = x XOR x~, so every nonzero d in {0,1}^(n-1) is checked against all seeds."""
    Y = np.array(list(itertools.product([0, 1], repeat=n)), np.uint8)  # 2^n x n
    Yw = [W.pack_bits(row) for row in Y]
    for d in itertools.product([0, 1], repeat=n - 1):
        if not any(d):
            continue
        dw = W.pack_bits(np.array(d, np.uint8))
        zeros = 0
        for yw in Yw:
            _, z = oracle.circulant(dw, yw, n - 1, m)
            zeros += int(not z.any())
        assert zeros == 2 ** (n - m)
        if n > 5 and sum(d) > 3:
            break  # the small cases are exhaustive; larger n spot-check a few d


# ------------------------------------------------------------ primes with primitive root 2

def order_of_two(v):
    k, t = 1, 2 % v
    while t != 1:
        t = t * 2 % v
        k += 1
        if k > v:
            return None
    return k


def test_na_primes_bruteforce():
    for v in range(0, 3000):
        is_p = v >= 2 and all(v % d for d in range(2, int(v ** 0.5) + 1))
        want = is_p and v > 2 and order_of_two(v) == v - 1
        assert oracle.is_na_prime(v) == want, v


def test_na_worked_example_golden():
    kv = dict(l.split() for l in open(os.path.join(GOLD, "na_primes_worked_example.txt")) if l.strip() and not l.startswith("#"))
    kv = {k: int(v) for k, v in kv.items()}
    assert oracle.closest_na(kv["n1"] + 1) == kv["closest_na_of_n1_plus_1"]
    assert kv["n1"] + kv["toeplitz_m"] - 1 == kv["toeplitz_seed_bits"]
    assert kv["toeplitz_seed_bits"] - kv["closest_na_of_n1_plus_1"] == kv["circulant_seed_saving"]
    assert oracle.next_na(1 << 20) == kv["next_na_of_2pow20"] == W.DODIS_N


# ------------------------------------------------------------ packed rows vs bit loop, preconditions

def test_rows_match_bits_ragged():
    g = W.rng(99)
    for n, m in [(63, 1), (64, 63), (65, 65), (127, 64), (129, 100), (1000, 513)]:
        x, y = rand_bits(g, n), rand_bits(g, n + m - 1)
        for order in ("paper", "linear"):
            _, z = oracle.toeplitz(W.pack_bits(x), W.pack_bits(y), n, m, order)
            for i0, cnt in [(0, m), (m - 1, 1), (m // 3, m - m // 3)]:
                zr = oracle.toeplitz_rows(W.pack_bits(x), W.pack_bits(y), n, m, i0, cnt, order)
                assert (bits(zr, cnt) == bits(z, m)[i0: i0 + cnt]).all()


def test_input_tail_bits_ignored():
    g = W.rng(3)
    n, m = 70, 30
    x, y = rand_bits(g, n), rand_bits(g, n + m - 1)
    xw, yw = W.pack_bits(x), W.pack_bits(y)
    xw2, yw2 = xw.copy(), yw.copy()
    xw2[-1] |= np.uint64(0xFFFF000000000000)
    yw2[-1] |= np.uint64(1 << 63)
    assert (oracle.toeplitz(xw, yw, n, m)[1] == oracle.toeplitz(xw2, yw2, n, m)[1]).all()


def test_preconditions():
    z = W.pack_bits(np.zeros(11, np.uint8))
    o = W.pack_bits(np.ones(11, np.uint8))
    assert oracle.check("toeplitz", 10, 0) == oracle.EINVAL
    assert oracle.check("toeplitz", 10, 11) == oracle.EINVAL
    assert oracle.check("toeplitz", 10, 10) == oracle.OK
    assert oracle.check("circulant", 10, 10) == oracle.OK      # n = 11
    assert oracle.check("circulant", 10, 11) == oracle.EINVAL
    assert oracle.check("circulant", 11, 5) == oracle.ENOTNA   # 12 is not prime
    assert oracle.check("dodis", 7, 3) == oracle.ENOTNA        # 2 has order 3 mod 7
    assert oracle.check("dodis", 11, 3, z) == oracle.EDEGENERATE
    assert oracle.check("dodis", 11, 3, o) == oracle.EDEGENERATE
    assert oracle.dodis(z, z, 11, 3)[0] == oracle.EDEGENERATE


def test_dodis_and_circulant_equal_toeplitz_reduction():
    """Dodis(x, y) = linear-order Toeplitz(rev(x), y || y_{0..m-2}) and Circulant(x, y) =
    the same with x' = [x, 0]: both sides are XOR_j x_j y_{(i+j) mod n}. The GPU path
    computes these two extractors this way (transform length n + m - 1)."""
    g = W.rng(123)
    for n in (3, 5, 11, 13, 59, 61, 83, 787, 1019):
        assert oracle.is_na_prime(n)
        for m in sorted({1, n // 3 or 1, n - 1, n}):
            x, y = rand_bits(g, n), rand_bits(g, n)
            x[0], x[1] = 1, 0
            s = np.concatenate([y, y[: m - 1]])
            _, zd = oracle.dodis(W.pack_bits(x), W.pack_bits(y), n, m)
            _, zt = oracle.toeplitz(W.pack_bits(x[::-1].copy()), W.pack_bits(s), n, m, "linear")
            assert (zd == zt).all(), (n, m)
            if m <= n - 1:
                xc = x[: n - 1]
                xp = np.concatenate([xc, [0]]).astype(np.uint8)
                _, zc = oracle.circulant(W.pack_bits(xc), W.pack_bits(y), n - 1, m)
                _, zt2 = oracle.toeplitz(W.pack_bits(xp[::-1].copy()), W.pack_bits(s), n, m, "linear")
                assert (zc == zt2).all(), (n, m)
