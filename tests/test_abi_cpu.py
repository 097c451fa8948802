"""The C-ABI library on the CPU: exported symbols match the header, host-only
entry points (prime utilities, plan and workspace sizes, error strings) and the
context-creation error path. No GPU compute is called."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2402_09481_amd import _lib
    return _lib.load()


def declared():
    h = open(os.path.join(ROOT, "include", "extractor.h")).read()
    h = re.sub(r"/\*.*?\*/", "", h, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(ext_[a-z_]+|extract_[a-z_]+)\s*\(", h,
                                 flags=re.M)))


def test_every_declared_symbol_is_exported(lib):
    from paper_2402_09481_amd import _lib
    names = declared()
    assert len(names) >= 20
    assert sorted(_lib.SYMBOLS) == names
    for n in names:
        assert hasattr(lib, n), n


def test_na_utilities_match_oracle(lib):
    for v in range(0, 4000):
        assert bool(lib.ext_is_na_prime(v)) == oracle.is_na_prime(v), v
    for v in [1 << 20, 10**6, 10**7 + 19, 1 << 30, 6_500_000_001, 1_738_000_001]:
        assert lib.ext_next_na(v) == oracle.next_na(v)
        assert lib.ext_closest_na(v) == oracle.closest_na(v)
    assert lib.ext_closest_na(6_500_000_001) == 6_500_000_069


def test_plan_lengths_and_workspace(lib):
    wb = ctypes.c_int32()
    # Toeplitz n = 2^30, m = 2^29 runs as two pieces of 2^29 input bits, each a
    # transform of 2^30 over 3*2^30+1, and so do Dodis/Circulant shapes whose halves
    # fit 2^30; shapes whose halves do not keep one transform over the 64-bit field.
    # Likewise a transform of 2^27 (15*2^27+1) becomes two pieces of 2^26 over
    # 7*2^26+1 where the halves fit (n = 2^26, m = 2^25), and stays one transform
    # where they do not (m = n = 2^26). From 2^25 up, any single transform whose
    # halves fit half its length runs as two pieces of that half (Toeplitz
    # n = 2^24, m = 2^23: 2^24 instead of 2^25); below, one transform (Dodis
    # n = m = 1,048,589 keeps 2^22)
    big_na = lib.ext_next_na(1 << 31)
    cases = [(0, 4096, 2048, 8192, 32), (2, 1048589, 1 << 19, 1 << 21, 32), (0, 1 << 30, 1 << 29, 1 << 30, 32),
             (1, 1048588, 1000, 1 << 21, 32), (2, 1048589, 1048589, 1 << 22, 32), (0, 1 << 24, 1 << 23, 1 << 24, 32), (0, 1, 1, 64, 32),
             (0, (1 << 26), (1 << 25), 1 << 26, 32), (0, 1 << 26, 1 << 26, 1 << 27, 32),
             (0, 1 << 28, 1 << 28, 1 << 29, 32),
             (2, 1073741827, 1 << 20, 1 << 30, 32), (1, 1738000138, 23998262, 1 << 30, 32),
             (0, (1 << 31) - 64, 1 << 20, 1 << 32, 64), (2, big_na, 1000, 1 << 32, 64)]
    for kind, n, m, L, bits in cases:
        assert lib.ext_plan_length(kind, n, m, ctypes.byref(wb)) == L
        assert wb.value == bits
    assert lib.ext_workspace_bytes(0, 4096, 2048) == 0  # one workgroup, no workspace
    big = lib.ext_workspace_bytes(0, 1 << 30, 1 << 29)  # four arrays of 2^30 32-bit words
    assert 4 * (1 << 30) * 4 <= big < 4 * (1 << 30) * 4 + (1 << 30)
    big = lib.ext_workspace_bytes(2, 1073741827, 1 << 20)  # two pieces: four arrays of 2^30 32-bit words
    assert 4 * (1 << 30) * 4 <= big < 4 * (1 << 30) * 4 + (1 << 30)
    big = lib.ext_workspace_bytes(2, big_na, 1000)  # one transform: two arrays of 2^32 64-bit words
    assert 2 * (1 << 32) * 8 <= big < 2 * (1 << 32) * 8 + (1 << 31)
    # beyond one transform of 2^32: the piece schedule over the 64-bit field
    assert lib.ext_plan_length(0, 1 << 33, 1 << 31, ctypes.byref(wb)) == 1 << 32 and wb.value == 64
    # invalid shapes
    for kind, n, m in [(0, 10, 0), (0, 10, 11), (1, 10, 11), (2, 5, 6), (7, 10, 5), (0, (1 << 41), 10)]:
        assert lib.ext_plan_length(kind, n, m, None) == 0
        assert lib.ext_workspace_bytes(kind, n, m) == 0


def test_error_strings(lib):
    for code in range(0, -8, -1):
        s = lib.ext_strerror(code).decode()
        assert s and "unknown" not in s
    assert "unknown" in lib.ext_strerror(-99).decode()
    assert lib.ext_version().decode().startswith("paper_2402_09481_amd")


def test_create_rejects_bad_device(lib):
    h = ctypes.c_void_p()
    rc = lib.ext_create(ctypes.byref(h), 1 << 20, 0, None)
    assert rc == -6 and not h.value  # EXT_EDEVICE, no context
    assert lib.ext_create(None, 0, 0, None) == -1
    lib.ext_destroy(None)  # no-op


def test_null_context_calls(lib):
    assert lib.extract_toeplitz(None, None, 10, None, 5, None, 0, None, None) == -1
    assert lib.extract_batch(None, None, 0, 0, None) == -1
    assert lib.ext_mem_stats(None, None, None, None) == -1
    assert lib.ext_profile(None, 1) == -1
    assert lib.ext_tune_set(None, 32, 20, 2, None) == -1
    assert lib.ext_tune_set_single(None, 32, 20, 2, None) == -1
    assert lib.ext_tune_get_single(None, 32, 20, None, None) == -1


def test_paper_qrng_shapes_run_as_pieces_of_the_64bit_field(lib):
    """The QRNG example (n = 6.5e9) is longer than one transform of 2^32: it runs as
    the piece schedule over the 64-bit field, pieces of transforms of 2^31 (four
    arrays of 2^31 words); the QKD Toeplitz and Circulant shapes run as two pieces
    of 2^30 each over 3*2^30+1."""
    import workloads as W
    wb = ctypes.c_int32()
    assert lib.ext_plan_length(0, W.QRNG_N, W.QRNG_M, ctypes.byref(wb)) == 1 << 31 and wb.value == 64
    n_in, m = W.qrng_circulant_shape(oracle.closest_na)
    assert n_in + 1 == 6_500_000_069 and m == 516_294_932
    assert lib.ext_plan_length(1, n_in, m, ctypes.byref(wb)) == 1 << 31 and wb.value == 64
    ws = lib.ext_workspace_bytes(0, W.QRNG_N, W.QRNG_M)
    assert 4 * (1 << 31) * 8 <= ws < 4 * (1 << 31) * 8 + (1 << 30)
    assert lib.ext_plan_length(0, W.QKD_N, W.QKD_M, None) == 1 << 30
    n_in, m = W.qkd_circulant_shape(oracle.next_na)
    assert lib.ext_plan_length(1, n_in, m, None) == 1 << 30
    # the output alone must leave room in a transform of 2^32
    assert lib.ext_plan_length(0, 1 << 40, (1 << 32) - 63, None) == 0


def test_von_neumann_host_surface(lib):
    # workspace: look-back state, first and last partial word per tile of 2^19 input bits
    assert lib.ext_workspace_bytes(3, 1, 0) == 0
    assert lib.ext_workspace_bytes(3, (1 << 40) + 2, 0) == 0
    tiles = lambda n: -(-((n & ~1) // 64 + (1 if (n & ~1) % 64 else 0)) // 8192)  # noqa: E731
    for n in (2, 1000, 1 << 19, (1 << 19) + 1, 5 * 10 ** 8, 1 << 33):
        want = (3 * 8 * tiles(n) + 256 + 255) // 256 * 256
        assert lib.ext_workspace_bytes(3, n, 0) == want, n
    # the convolution kinds reject nothing they did before; Von Neumann is not a plan
    assert lib.ext_plan_length(3, 1000, 10, None) == 0
    assert lib.extract_von_neumann(None, None, 1000, None, 100, None, 0, None, None) == -1
