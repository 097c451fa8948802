"""The kernels' field arithmetic (csrc/field.h), compiled for the CPU, against
exact integer arithmetic: Goldilocks product, sum, difference, canonical form,
every power-of-two multiplier 2^s (s < 192, the roots of the in-register DFTs
among them) and the 128-bit reduction on arbitrary limbs; Montgomery product,
sum and difference of the two 32-bit fields; the lazy field 7*2^26+1 (values
anywhere in [0, 4P)): Montgomery product, the butterfly's sum and difference with
their operand preparation, canonical form, Shoup products by in-pass twiddle
pairs and by the in-register roots, each with its output range. Random operands plus the edge
values of each field (0, 1, P - 1, P and the non-canonical 64-bit values above P,
products whose upper limbs are zero). The GPU parity tests check the same
routines inside the kernels; these pin each routine on its own."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "field_host", "field_host.cpp")
PG = (1 << 64) - (1 << 32) + 1
P32 = {0: 15 * (1 << 27) + 1, 1: 3 * (1 << 30) + 1}
CLANG = shutil.which("clang++") or "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ not available (the field code uses clang's add/sub-with-carry builtins)")
    out = str(tmp_path_factory.mktemp("field") / "field_host.so")
    subprocess.check_call([CLANG, "-O2", "-std=c++17", "-shared", "-fPIC", "-I", os.path.join(HERE, "field_host"),
                           "-o", out, SRC])
    L = ctypes.CDLL(out)
    u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
    u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
    L.fgl_op.argtypes = [ctypes.c_int, u64p, u64p, u64p, ctypes.c_size_t]
    L.f32_op.argtypes = [ctypes.c_int, ctypes.c_int, u32p, u32p, u32p, ctypes.c_size_t]
    L.flz_op.argtypes = [ctypes.c_int, u32p, u32p, u32p, ctypes.c_size_t]
    return L


def gl(L, op, a, b):
    a = np.ascontiguousarray(a, np.uint64)
    b = np.ascontiguousarray(b, np.uint64)
    out = np.empty_like(a)
    L.fgl_op(op, a, b, out, len(a))
    return [int(v) for v in out]


def operands64(n, seed):
    g = np.random.default_rng(seed)
    edge = [0, 1, 2, (1 << 32) - 1, 1 << 32, PG - 2, PG - 1, PG, PG + 1, (1 << 64) - 1, (1 << 64) - 2,
            (1 << 63), 0xFFFFFFFF00000000, 0xFFFFFFFEFFFFFFFF, 5980198667562970375]
    a = [int(v) for v in g.integers(0, 1 << 64, size=n, dtype=np.uint64)]
    b = [int(v) for v in g.integers(0, 1 << 64, size=n, dtype=np.uint64)]
    # small operands (products with zero upper limbs), values just above P, shifted values
    a[: n // 8] = [v >> (i % 64) for i, v in enumerate(a[: n // 8])]
    b[n // 8: n // 4] = [PG + (v & 0xFFFFFFFF) if PG + (v & 0xFFFFFFFF) < (1 << 64) else v for v in b[n // 8: n // 4]]
    A = [x for x in edge for _ in edge] + a
    B = [y for _ in edge for y in edge] + b
    return A, B


def test_goldilocks_mul_add_sub_canon(lib):
    A, B = operands64(40000, 1)
    for op, ref in ((0, lambda x, y: x * y % PG), (1, lambda x, y: (x + y) % PG), (2, lambda x, y: (x - y) % PG)):
        got = gl(lib, op, A, B)
        bad = [(x, y) for x, y, r in zip(A, B, got) if r % PG != ref(x % PG, y % PG)]
        assert not bad, (op, bad[:3])
        assert all(r < (1 << 64) for r in got)
    got = gl(lib, 3, A, B)
    assert all(r == x % PG for x, r in zip(A, got))


def test_goldilocks_reduce_limbs(lib):
    g = np.random.default_rng(2)
    n = 30000
    hi = [int(v) for v in g.integers(0, 1 << 64, size=n, dtype=np.uint64)]
    lo = [int(v) for v in g.integers(0, 1 << 64, size=n, dtype=np.uint64)]
    hi[:3000] = [v & 0xFFFFFFFF00000000 for v in hi[:3000]]      # x2 = 0 (the borrow case)
    hi[3000:4000] = [0] * 1000                                     # x3 = x2 = 0
    hi[4000:5000] = [v & 0xFFFFFFFF for v in hi[4000:5000]]        # x3 = 0
    lo[5000:6000] = [(1 << 64) - 1 - (v & 0xFF) for v in lo[5000:6000]]  # lo near 2^64
    got = gl(lib, 5, hi, lo)
    assert all(r % PG == ((h << 64) | l) % PG for h, l, r in zip(hi, lo, got))


def test_goldilocks_powers_of_two(lib):
    A, _ = operands64(2000, 3)
    for s in range(192):
        got = gl(lib, 4, A, [s] * len(A))
        w = pow(2, s, PG)
        assert all(r % PG == x % PG * w % PG for x, r in zip(A, got)), s
    # the roots of unity they implement: 2^(192/RAD) has order RAD
    for rad in (2, 4, 8, 16, 32, 64):
        w = pow(2, 192 // rad, PG)
        assert pow(w, rad, PG) == 1 and pow(w, rad // 2, PG) == PG - 1


@pytest.mark.parametrize("field", [0, 1])
def test_32bit_montgomery_add_sub(lib, field):
    P = P32[field]
    g = np.random.default_rng(10 + field)
    edge = [0, 1, 2, P - 2, P - 1, P // 2, (1 << 31) - 1 if (1 << 31) - 1 < P else 3]
    a = [x for x in edge for _ in edge] + [int(v) for v in g.integers(0, P, size=60000)]
    b = [y for _ in edge for y in edge] + [int(v) for v in g.integers(0, P, size=60000)]
    A = np.array(a, np.uint32)
    Bv = np.array(b, np.uint32)
    rinv = pow(1 << 32, -1, P)
    for op, ref in ((0, lambda x, y: x * y * rinv % P), (1, lambda x, y: (x + y) % P), (2, lambda x, y: (x - y) % P)):
        out = np.empty_like(A)
        lib.f32_op(field, op, A, Bv, out, len(A))
        got = [int(v) for v in out]
        bad = [(x, y, r) for x, y, r in zip(a, b, got) if r != ref(x, y)]  # canonical results
        assert not bad, (field, op, bad[:3])


PLZ = 7 * (1 << 26) + 1


def lz(L, op, a, b):
    A = np.ascontiguousarray(a, np.uint32)
    B = np.ascontiguousarray(b, np.uint32)
    out = np.empty_like(A)
    L.flz_op(op, A, B, out, len(A))
    return [int(v) for v in out]


def lazy_operands(n, seed, hi=4 * PLZ):
    g = np.random.default_rng(seed)
    edge = [0, 1, 2, PLZ - 1, PLZ, PLZ + 1, 2 * PLZ - 1, 2 * PLZ, 2 * PLZ + 1, 3 * PLZ, 4 * PLZ - 2, hi - 1]
    a = [x for x in edge for _ in edge] + [int(v) for v in g.integers(0, hi, size=n)]
    b = [y for _ in edge for y in edge] + [int(v) for v in g.integers(0, hi, size=n)]
    return a, b


def test_lazy_field_mont_add_sub_canon(lib):
    a, b = lazy_operands(60000, 20)
    rinv = pow(1 << 32, -1, PLZ)
    got = lz(lib, 0, a, b)
    assert all(r % PLZ == x * y * rinv % PLZ and r < 3 * PLZ for x, y, r in zip(a, b, got))
    got = lz(lib, 1, a, b)
    assert all(r % PLZ == (x + y) % PLZ and r < 4 * PLZ for x, y, r in zip(a, b, got))
    got = lz(lib, 2, a, b)
    assert all(r % PLZ == (x - y) % PLZ and r < 4 * PLZ for x, y, r in zip(a, b, got))
    got = lz(lib, 3, a, b)
    assert all(r == x % PLZ for x, r in zip(a, got))


def test_lazy_field_shoup_products(lib):
    g = np.random.default_rng(21)
    # any 32-bit x (the Shoup bound holds for x < 2^32), twiddles w < P
    x = [0, 1, 4 * PLZ - 1, (1 << 32) - 1] * 4 + [int(v) for v in g.integers(0, 1 << 32, size=60000, dtype=np.uint64)]
    w = [0, 1, PLZ - 1, PLZ // 2] * 4 + [int(v) for v in g.integers(0, PLZ, size=60000)]
    got = lz(lib, 4, x, w)
    assert all(r % PLZ == xi * wi % PLZ and r < 2 * PLZ for xi, wi, r in zip(x, w, got))
    # the in-register roots: w_RAD^k = WMAX^(2^26 k / RAD), WMAX = 3^7 of order 2^26
    wmax = pow(3, 7, PLZ)
    assert pow(wmax, 1 << 25, PLZ) == PLZ - 1
    xs = x[:5000]
    for op, rad in ((5, 2), (6, 4), (7, 8), (8, 16)):
        for k in range(rad):
            w = pow(wmax, (1 << 26) // rad * k, PLZ)
            got = lz(lib, op, xs, [k] * len(xs))
            assert all(r % PLZ == xi * w % PLZ and r < 2 * PLZ for xi, r in zip(xs, got)), (rad, k)


def test_lazy_field_butterfly_on_unreduced_constant_products(lib):
    """The lazy field's DFT layers feed the results of products by constants
    (in-register roots, Stockham twiddles) to the butterfly without reducing them
    again: those results lie in [0, 2P) for any 32-bit input, so the sum and the
    difference plus 2P stay in [0, 4P)."""
    g = np.random.default_rng(23)
    edge = [0, 1, PLZ - 1, 2 * PLZ - 1, 4 * PLZ - 1, (1 << 32) - 1]
    a = [x for x in edge for _ in edge] + [int(v) for v in g.integers(0, 4 * PLZ, size=40000)]
    b = [y for _ in edge for y in edge] + [int(v) for v in g.integers(0, 1 << 32, size=40000, dtype=np.uint64)]
    w = pow(3, 7, PLZ)
    a_ok = [x if x < 4 * PLZ else x % (4 * PLZ) for x in a]  # butterfly inputs are lazy values (< 4P)
    got = lz(lib, 9, a_ok, b)
    assert all(r % PLZ == (x + y * w) % PLZ and r < 4 * PLZ for x, y, r in zip(a_ok, b, got))
    got = lz(lib, 10, a_ok, b)
    assert all(r % PLZ == (x - y * w) % PLZ and r < 4 * PLZ for x, y, r in zip(a_ok, b, got))
    got = lz(lib, 11, b, a_ok)
    assert all(r % PLZ == (x * w + y) % PLZ and r < 4 * PLZ for x, y, r in zip(b, a_ok, got))
    got = lz(lib, 12, b, a_ok)
    assert all(r % PLZ == (x * w - y) % PLZ and r < 4 * PLZ for x, y, r in zip(b, a_ok, got))
