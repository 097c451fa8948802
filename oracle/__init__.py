"""Oracle for the convolution extractors and the Von Neumann extractor — TEST
INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package. It shares no code with the GPU library (``paper_2402_09481_amd``)
and never imports it.

What it computes is the plain definition of each extractor as a GF(2)
matrix-vector product (see ``oracle.c`` for the formulas and the passages they
follow), plus its own primality / primitive-root utilities written from the
definition of a prime with 2 as a primitive root. Preconditions follow the
paper: Toeplitz needs 1 <= m <= n; Circulant needs n = n_in + 1 prime with
primitive root 2 and 1 <= m <= n - 1 (full row rank bound of the Circulant
proof); Dodis et al. needs n prime with primitive root 2, 1 <= m <= n and
x not all-zero and not all-one (precondition stated with the Dodis
implementation). Von Neumann needs n >= 2 (one pair) and reports EDEGENERATE
when no pair differs, the error case of its implementation (Alg. 3), which
prints no return value: here the output is returned and the error raised only
for an empty output. On a failed precondition the functions return the error
code and no output.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

OK = 0
EINVAL = -1
ENOTNA = -2
EDEGENERATE = -3

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRCS = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "gf2x.c")]
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c and gf2x.c with gcc into liboracle.so next to them."""
    stale = not os.path.exists(_SO) or any(os.path.getmtime(_SO) < os.path.getmtime(s) for s in _SRCS)
    if force or stale:
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-pthread", "-o", tmp] + _SRCS)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u64 = ctypes.c_uint64
        lib.oracle_toeplitz_bits.argtypes = [u64p, u64, u64p, u64, ctypes.c_int, u64p]
        lib.oracle_dodis_bits.argtypes = [u64p, u64p, u64, u64, u64p]
        lib.oracle_circulant_bits.argtypes = [u64p, u64, u64p, u64, u64p]
        lib.oracle_toeplitz_rows.argtypes = [u64p, u64, u64p, u64, ctypes.c_int, u64, u64, u64p]
        lib.oracle_dodis_rows.argtypes = [u64p, u64p, u64, u64, u64, u64p]
        lib.oracle_circulant_rows.argtypes = [u64p, u64, u64p, u64, u64, u64p]
        lib.oracle_von_neumann_bits.argtypes = [u64p, u64, u64p]
        lib.oracle_von_neumann_bits.restype = ctypes.c_uint64
        sz = ctypes.c_size_t
        lib.gf2_force_software.argtypes = [ctypes.c_int]
        lib.gf2_force_software.restype = ctypes.c_int
        lib.gf2_clmul64.argtypes = [u64, u64, u64p, u64p]
        lib.gf2_clmul64.restype = None
        lib.gf2_set_threads_depth.argtypes = [ctypes.c_int]
        lib.gf2_set_threads_depth.restype = None
        lib.gf2_mul.argtypes = [u64p, sz, u64p, sz, u64p]
        lib.gf2_toeplitz_linear.argtypes = [u64p, u64, u64p, u64, u64p]
        lib.gf2_toeplitz_block.argtypes = [u64p, u64, u64p, u64, u64, u64, u64p]
        lib.gf2_paper_to_linear.argtypes = [u64p, u64, u64, u64p]
        lib.gf2_circulant_rows.argtypes = [u64p, u64, u64p, u64, u64p]
        for f in (lib.gf2_mul, lib.gf2_toeplitz_linear, lib.gf2_toeplitz_block, lib.gf2_paper_to_linear,
                  lib.gf2_circulant_rows):
            f.restype = ctypes.c_int
        for f in (lib.oracle_toeplitz_bits, lib.oracle_dodis_bits, lib.oracle_circulant_bits,
                  lib.oracle_toeplitz_rows, lib.oracle_dodis_rows, lib.oracle_circulant_rows):
            f.restype = None
        _lib = lib
    return _lib


def _nw(nbits: int) -> int:
    return (int(nbits) + 63) >> 6


def _masked(words, nbits: int) -> np.ndarray:
    """Copy of the first ceil(nbits/64) words with bits >= nbits cleared (inputs'
    tail bits are ignored), plus one spare zero word."""
    w = np.zeros(_nw(nbits) + 1, dtype=np.uint64)
    src = np.asarray(words, dtype=np.uint64)[: _nw(nbits)]
    w[: src.size] = src
    r = int(nbits) & 63
    if r:
        w[_nw(nbits) - 1] &= np.uint64((1 << r) - 1)
    return w


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


# ------------------------------------------------------------------ primes with primitive root 2

def is_prime(v: int) -> bool:
    """Trial division by 2, 3 and 6k +- 1 up to sqrt(v)."""
    v = int(v)
    if v < 2:
        return False
    if v < 4:
        return True
    if v % 2 == 0 or v % 3 == 0:
        return False
    d = 5
    while d * d <= v:
        if v % d == 0 or v % (d + 2) == 0:
            return False
        d += 6
    return True


def prime_factors(v: int):
    """Distinct prime factors of v by trial division."""
    v = int(v)
    out = []
    d = 2
    while d * d <= v:
        if v % d == 0:
            out.append(d)
            while v % d == 0:
                v //= d
        d += 1 if d == 2 else 2
    if v > 1:
        out.append(v)
    return out


def is_na_prime(n: int) -> bool:
    """n is prime and 2 generates the multiplicative group mod n, i.e. the order of
    2 mod n is n - 1: 2^((n-1)/q) != 1 mod n for every prime q dividing n - 1."""
    n = int(n)
    if n == 2:
        return False  # the group mod 2 is trivial; 2 is not a unit
    if not is_prime(n):
        return False
    return all(pow(2, (n - 1) // q, n) != 1 for q in prime_factors(n - 1))


def next_na(v: int) -> int:
    """Smallest prime >= v with primitive root 2."""
    c = max(int(v), 3)
    while not is_na_prime(c):
        c += 1
    return c


def prev_na(v: int) -> int:
    """Largest prime <= v with primitive root 2 (0 if none)."""
    c = int(v)
    while c >= 3 and not is_na_prime(c):
        c -= 1
    return c if c >= 3 else 0


def closest_na(v: int) -> int:
    """Prime with primitive root 2 nearest to v; on a tie the smaller one."""
    up, lo = next_na(v), prev_na(v)
    if lo == 0:
        return up
    return lo if (int(v) - lo) <= (up - int(v)) else up


# ------------------------------------------------------------------ preconditions

def check(kind: str, n: int, m: int, x=None) -> int:
    n, m = int(n), int(m)
    if kind == "toeplitz":
        return OK if (n >= 1 and 1 <= m <= n) else EINVAL
    if kind == "circulant":
        if n < 1 or m < 1 or m > n:  # m <= (n+1) - 1
            return EINVAL
        return OK if is_na_prime(n + 1) else ENOTNA
    if kind == "dodis":
        if n < 1 or m < 1 or m > n:
            return EINVAL
        if not is_na_prime(n):
            return ENOTNA
        if x is not None:
            w = _masked(x, n)[: _nw(n)]
            ones = sum(int(v).bit_count() for v in w)
            if ones == 0 or ones == n:
                return EDEGENERATE
        return OK
    return EINVAL


# ------------------------------------------------------------------ extractors (whole output)

def toeplitz(x, y, n: int, m: int, seed_order: str = "paper"):
    """(code, z): z packed m bits, from the bit-by-bit definition."""
    code = check("toeplitz", n, m)
    if code:
        return code, None
    z = np.zeros(_nw(m) + 1, np.uint64)
    xx, yy = _masked(x, n), _masked(y, n + m - 1)
    _load().oracle_toeplitz_bits(_p(xx), n, _p(yy), m, int(seed_order == "linear"), _p(z))
    return OK, z[: _nw(m)]


def circulant(x, y, n_in: int, m: int):
    code = check("circulant", n_in, m)
    if code:
        return code, None
    z = np.zeros(_nw(m) + 1, np.uint64)
    xx, yy = _masked(x, n_in), _masked(y, n_in + 1)
    _load().oracle_circulant_bits(_p(xx), n_in, _p(yy), m, _p(z))
    return OK, z[: _nw(m)]


def dodis(x, y, n: int, m: int):
    code = check("dodis", n, m, x)
    if code:
        return code, None
    z = np.zeros(_nw(m) + 1, np.uint64)
    xx, yy = _masked(x, n), _masked(y, n)
    _load().oracle_dodis_bits(_p(xx), _p(yy), n, m, _p(z))
    return OK, z[: _nw(m)]


# ------------------------------------------------------------------ selected rows, 64 terms per step

def toeplitz_rows(x, y, n: int, m: int, i0: int, cnt: int, seed_order: str = "paper") -> np.ndarray:
    """Packed z_{i0} .. z_{i0+cnt-1} (bit r of the result is z_{i0+r})."""
    assert check("toeplitz", n, m) == OK and 0 <= i0 and i0 + cnt <= m
    out = np.zeros(_nw(cnt) + 1, np.uint64)
    xx, yy = _masked(x, n), _masked(y, n + m - 1)
    _load().oracle_toeplitz_rows(_p(xx), n, _p(yy), m, int(seed_order == "linear"), i0, cnt, _p(out))
    return out[: _nw(cnt)]


def circulant_rows(x, y, n_in: int, m: int, i0: int, cnt: int) -> np.ndarray:
    assert check("circulant", n_in, m) == OK and 0 <= i0 and i0 + cnt <= m
    out = np.zeros(_nw(cnt) + 1, np.uint64)
    xx, yy = _masked(x, n_in), _masked(y, n_in + 1)
    _load().oracle_circulant_rows(_p(xx), n_in, _p(yy), i0, cnt, _p(out))
    return out[: _nw(cnt)]


def dodis_rows(x, y, n: int, m: int, i0: int, cnt: int) -> np.ndarray:
    assert check("dodis", n, m, x) == OK and 0 <= i0 and i0 + cnt <= m
    out = np.zeros(_nw(cnt) + 1, np.uint64)
    xx, yy = _masked(x, n), _masked(y, n)
    _load().oracle_dodis_rows(_p(xx), _p(yy), n, i0, cnt, _p(out))
    return out[: _nw(cnt)]


def extract(kind: str, x, y, n: int, m: int, seed_order: str = "paper", packed: bool = True):
    """Whole output via the packed row routine (fast enough up to n ~ 2^22).
    Returns (code, z)."""
    code = check(kind, n, m, x if kind == "dodis" else None)
    if code:
        return code, None
    if kind == "toeplitz":
        return OK, toeplitz_rows(x, y, n, m, 0, m, seed_order)
    if kind == "circulant":
        return OK, circulant_rows(x, y, n, m, 0, m)
    return OK, dodis_rows(x, y, n, m, 0, m)


# ------------------------------------------------------------------ Von Neumann

def von_neumann(x, n: int):
    """(code, z, m): the Von Neumann output (section "Von Neumann", Alg. 3) as
    ceil(m/64) packed words and its length m. code EINVAL for n < 2;
    EDEGENERATE (with z empty and m = 0) when no pair of bits differs."""
    n = int(n)
    if n < 2:
        return EINVAL, None, 0
    out = np.zeros(_nw(n // 2) + 1, np.uint64)
    xx = _masked(x, n)
    m = int(_load().oracle_von_neumann_bits(_p(xx), n, _p(out)))
    if m == 0:
        return EDEGENERATE, out[:0], 0
    return OK, out[: _nw(m)], m


# ------------------------------------------------------------------ whole outputs as GF(2)[t] products

def gf2_force_software(on: bool) -> bool:
    """Use the shift-and-XOR carry-less product instead of the CPU instruction (a
    testing aid); returns whether the instruction is available."""
    return bool(_load().gf2_force_software(int(bool(on))))


def gf2_set_threads_depth(depth: int) -> None:
    """Top levels of the Karatsuba recursion that run on threads (3^depth leaves)."""
    _load().gf2_set_threads_depth(int(depth))


def clmul64(a: int, b: int) -> int:
    """Carry-less product of two 64-bit words as a 128-bit int."""
    lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
    _load().gf2_clmul64(int(a), int(b), ctypes.byref(lo), ctypes.byref(hi))
    return lo.value | (hi.value << 64)


def gf2_mul(a, b) -> np.ndarray:
    """Product of two GF(2)[t] polynomials given as packed words (bit k = coefficient
    of t^k); len(a) + len(b) words."""
    aa = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
    bb = np.ascontiguousarray(np.asarray(b, dtype=np.uint64))
    r = np.zeros(aa.size + bb.size + 1, np.uint64)
    if _load().gf2_mul(_p(aa), aa.size, _p(bb), bb.size, _p(r)) != 0:
        raise MemoryError("gf2_mul")
    return r[: aa.size + bb.size]


def _linear_seed(y, N: int, m: int, seed_order: str) -> np.ndarray:
    yy = _masked(y, N)
    if seed_order == "linear":
        return yy
    s = np.zeros(_nw(N) + 1, np.uint64)
    if _load().gf2_paper_to_linear(_p(yy), N, m, _p(s)) != 0:
        raise MemoryError("gf2_paper_to_linear")
    return s


def toeplitz_product(x, y, n: int, m: int, seed_order: str = "paper", block_bits: int = 0, progress=None):
    """(code, z): the whole Toeplitz output as the coefficients t^(n-1) .. t^(n+m-2)
    of X(t) S(t) over GF(2) (S the seed in the linear order), by Karatsuba.
    block_bits > 0 splits the sum over input positions into shares of that many
    positions (a multiple of 64), XORed together; progress(done, total) is called
    after each share."""
    code = check("toeplitz", n, m)
    if code:
        return code, None
    n, m = int(n), int(m)
    N = n + m - 1
    s = _linear_seed(y, N, m, seed_order)
    xx = _masked(x, n)
    z = np.zeros(_nw(m) + 1, np.uint64)
    w = n if block_bits <= 0 else max(64, (int(block_bits) // 64) * 64)
    for j0 in range(0, n, w):
        k = min(w, n - j0)
        if _load().gf2_toeplitz_block(_p(xx), n, _p(s), m, j0, k, _p(z)) != 0:
            raise MemoryError("gf2_toeplitz_block")
        if progress is not None:
            progress(j0 + k, n)
    return OK, z[: _nw(m)]


def _circulant_product(a, n: int, y, m: int) -> np.ndarray:
    aa, yy = _masked(a, n), _masked(y, n)
    z = np.zeros(_nw(m) + 1, np.uint64)
    if _load().gf2_circulant_rows(_p(aa), int(n), _p(yy), int(m), _p(z)) != 0:
        raise MemoryError("gf2_circulant_rows")
    return z[: _nw(m)]


def dodis_product(x, y, n: int, m: int):
    """(code, z): Dodis et al. as the cyclic convolution (length n) of the reflected
    input b_k = x_(-k mod n) with y over GF(2), by Karatsuba."""
    code = check("dodis", n, m, x)
    if code:
        return code, None
    return OK, _circulant_product(x, n, y, m)


def circulant_product(x, y, n_in: int, m: int):
    """(code, z): Circulant as the cyclic convolution of length n_in + 1 with the
    generator x' = [x, 0] (the input's bits beyond n_in read as zero)."""
    code = check("circulant", n_in, m)
    if code:
        return code, None
    return OK, _circulant_product(_masked(x, n_in), int(n_in) + 1, y, m)


def extract_product(kind: str, x, y, n: int, m: int, seed_order: str = "paper"):
    """Whole output of any convolution extractor through the GF(2)[t] products."""
    if kind == "toeplitz":
        return toeplitz_product(x, y, n, m, seed_order)
    if kind == "circulant":
        return circulant_product(x, y, n, m)
    return dodis_product(x, y, n, m)
