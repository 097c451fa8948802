"""GPU parity: the HIP path against the oracle, bit for bit, through the C-ABI.
Default contexts run transforms up to 2^26 over the lazy field 7*2^26+1 (one
workgroup per job up to 2^14); the forced-field contexts cover 15*2^27+1,
3*2^30+1 and the 64-bit field at small sizes."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import gpu_extract, show_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2402_09481_amd as P
    c = P.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_gl():
    """A context that runs every shape on the 64-bit field (checks that path at small sizes)."""
    import paper_2402_09481_amd as P
    os.environ["EXT_FORCE_FIELD"] = "gl"
    try:
        c = P.Context(0)
    finally:
        del os.environ["EXT_FORCE_FIELD"]
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_p0():
    """A context that runs every shape on 3*2^30+1 (the 32-bit field of transforms
    from 2^28 to 2^30), multi-pass, at small sizes."""
    import paper_2402_09481_amd as P
    os.environ["EXT_FORCE_FIELD"] = "p0"
    try:
        c = P.Context(0)
    finally:
        del os.environ["EXT_FORCE_FIELD"]
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_bb():
    """A context that runs every shape on 15*2^27+1 (the 32-bit field of transforms of
    2^27; below that the lazy field 7*2^26+1 runs by default), multi-pass, at small
    sizes."""
    import paper_2402_09481_amd as P
    os.environ["EXT_FORCE_FIELD"] = "bb"
    try:
        c = P.Context(0)
    finally:
        del os.environ["EXT_FORCE_FIELD"]
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_2p():
    """A context that runs every Toeplitz shape with n >= 128 as the two-piece
    schedule (input split in two word-aligned halves, products added in the
    transform domain of 3*2^30+1), at small sizes."""
    import paper_2402_09481_amd as P
    os.environ["EXT_FORCE_FIELD"] = "p0x2"
    try:
        c = P.Context(0)
    finally:
        del os.environ["EXT_FORCE_FIELD"]
    yield c
    c.close()


def seed_len(kind, n, m):
    return {"toeplitz": n + m - 1, "circulant": n + 1, "dodis": n}[kind]


def run_case(ctx, kind, n, m, order="paper", seed=0, px=0.5):
    g = W.rng(seed)
    x = W.bernoulli_bits(g, n, px)
    y = W.bernoulli_bits(g, seed_len(kind, n, m), 0.5)
    if kind == "dodis":
        x[0] = (int(x[0]) | 1) & ~2  # x_0 = 1, x_1 = 0: never degenerate
    show_case(kind, n, m, order, seed)
    code, z = gpu_extract(ctx, kind, x, y, n, m, order)
    assert code == 0, (kind, n, m, code)
    rc, want = oracle.extract(kind, x, y, n, m, order)
    assert rc == 0
    assert z.shape == want.shape
    bad = np.nonzero(z != want)[0]
    assert bad.size == 0, "first bad word %d of %d (%s n=%d m=%d)" % (bad[0], z.size, kind, n, m)


def test_toeplitz_small_workload(ctx):
    j = W.toeplitz_small()
    show_case("toeplitz_small")
    code, z = gpu_extract(ctx, "toeplitz", j.x, j.y, j.n, j.m, "linear")
    rc, want = oracle.extract("toeplitz", j.x, j.y, j.n, j.m, "linear")
    assert code == 0 and rc == 0 and (z == want).all()


@pytest.mark.parametrize("order", ["paper", "linear"])
def test_toeplitz_tiny_all_shapes(ctx, order):
    for n in list(range(1, 20)) + [63, 64, 65, 127, 128, 129]:
        for m in sorted({v for v in (1, 2, n // 2, n - 1, n) if 1 <= v <= n}):
            run_case(ctx, "toeplitz", n, m, order, seed=n * 1000 + m)


@pytest.mark.parametrize("n,m", [(2000, 1000), (4096, 4096), (5000, 3191), (8192, 1), (8191, 8191),
                                 (9000, 4500), (12345, 4000)])
def test_toeplitz_single_workgroup_sizes(ctx, n, m):
    run_case(ctx, "toeplitz", n, m, "paper", seed=n + m)
    run_case(ctx, "toeplitz", n, m, "linear", seed=n + m + 1)


@pytest.mark.parametrize("n,m", [(8193, 8193), (20000, 7777), (40000, 20000), (65536, 65536), (100003, 50001),
                                 (300000, 1000), (1 << 19, 1 << 18)])
def test_toeplitz_multipass_32bit(ctx, n, m):
    run_case(ctx, "toeplitz", n, m, "paper", seed=7 * n + m, px=0.4)


@pytest.mark.parametrize("field", ["default", "gl"])
@pytest.mark.parametrize("n,m", [(65536, 8192), (65536, 32768), (65536, 32769), (65537, 65536)])
def test_last_pass_row_bounds(ctx, ctx_gl, field, n, m):
    """The last inverse pass computes only the rows of its column transform that
    hold output coefficients (the first ceil(m/S) of R rows: a quarter, a half or
    all of its last step's outputs). Transform 2^17 here, with m = L/16, exactly
    L/4, one past L/4 and L/2: on and across those bounds, on both fields."""
    run_case(ctx if field == "default" else ctx_gl, "toeplitz", n, m, "paper", seed=19 * n + m, px=0.4)


def test_64bit_1024_row_columns(ctx, ctx_gl):
    """A transform of 2^23 on the 64-bit field splits as a strided level of 2^10
    rows (the column tile exchanged through LDS in 32-bit halves) and a row level
    of 2^13: sampled output words against the oracle, one row at a time, and the
    whole output against the 32-bit field's plan for the same length (the same
    integers, so the same bits)."""
    n, m = (1 << 22) - 5, (1 << 21) + 3  # n + m - 1 > 2^22: transform length 2^23
    g = W.rng(23)
    x, y = W.bernoulli_bits(g, n, 0.4), W.bernoulli_bits(g, n + m - 1, 0.5)
    show_case("toeplitz 64-bit 2^23", n, m)
    code, z = gpu_extract(ctx_gl, "toeplitz", x, y, n, m)
    assert code == 0
    nw = z.size
    for w in sorted({0, 1, nw // 2, nw - 2, nw - 1} | {int(v) for v in g.integers(0, nw - 1, 3)}):
        cnt = min(64, m - 64 * w)
        want = oracle.toeplitz_rows(x, y, n, m, 64 * w, cnt)
        assert int(z[w]) == int(want[0]), "word %d" % w
    code32, z32 = gpu_extract(ctx, "toeplitz", x, y, n, m)
    assert code32 == 0 and np.array_equal(z, z32)


@pytest.mark.parametrize("n,m", [(11, 5), (13, 13), (61, 60), (1019, 500), (4099, 4099), (8219, 8000),
                                 (16421, 9000), (65587, 32768)])
def test_dodis(ctx, n, m):
    assert oracle.is_na_prime(n)
    run_case(ctx, "dodis", n, m, seed=n, px=0.3)


@pytest.mark.parametrize("n_in,m", [(10, 10), (12, 6), (100, 99), (1018, 1018), (4098, 2049), (8218, 8218),
                                    (16420, 100), (65586, 65586)])
def test_circulant(ctx, n_in, m):
    assert oracle.is_na_prime(n_in + 1)
    run_case(ctx, "circulant", n_in, m, seed=n_in)


def test_dodis_workload(ctx):
    j = W.dodis_2p20()
    show_case("dodis_2p20")
    code, z = gpu_extract(ctx, "dodis", j.x, j.y, j.n, j.m)
    assert code == 0
    rc, want = oracle.extract("dodis", j.x, j.y, j.n, j.m)
    assert rc == 0 and (z == want).all()


@pytest.mark.parametrize("kind,n,m", [("toeplitz", 9000, 7000), ("toeplitz", 100000, 50000),
                                      ("dodis", 8219, 8219), ("circulant", 16420, 8000)])
def test_64bit_field_path(ctx_gl, kind, n, m):
    run_case(ctx_gl, kind, n, m, "paper", seed=3 * n + m)


@pytest.mark.parametrize("kind,n,m", [("toeplitz", 9000, 7000), ("toeplitz", 100000, 50000), ("toeplitz", 129, 64),
                                      ("toeplitz", 1 << 20, 1 << 19), ("dodis", 8219, 8219),
                                      ("circulant", 16420, 8000)])
def test_p0_field_path(ctx_p0, kind, n, m):
    run_case(ctx_p0, kind, n, m, "paper", seed=5 * n + m)
    if kind == "toeplitz":
        run_case(ctx_p0, kind, n, m, "linear", seed=7 * n + m)


@pytest.mark.parametrize("kind,n,m", [("toeplitz", 9000, 7000), ("toeplitz", 100000, 50000), ("toeplitz", 129, 64),
                                      ("toeplitz", 1 << 20, 1 << 19), ("toeplitz", (1 << 22) + 5, 1 << 21),
                                      ("dodis", 8219, 8219), ("circulant", 16420, 8000)])
def test_bb_field_path(ctx_bb, kind, n, m):
    run_case(ctx_bb, kind, n, m, "paper", seed=17 * n + m)
    if kind == "toeplitz":
        run_case(ctx_bb, kind, n, m, "linear", seed=19 * n + m)


@pytest.mark.parametrize("n,m", [(128, 1), (129, 64), (200, 199), (1000, 1), (4097, 2048), (9000, 7000),
                                 (65539, 65539), (100000, 50000), (1 << 20, 1 << 19), ((1 << 21) + 77, 300)])
def test_two_piece_schedule(ctx_2p, n, m):
    run_case(ctx_2p, "toeplitz", n, m, "paper", seed=11 * n + m)
    run_case(ctx_2p, "toeplitz", n, m, "linear", seed=13 * n + m, px=0.3)


@pytest.mark.parametrize("kind,n,m", [("dodis", 131, 1), ("dodis", 131, 131), ("dodis", 4099, 2048),
                                      ("dodis", 65539, 65539), ("dodis", 1048589, 1 << 19), ("circulant", 130, 1),
                                      ("circulant", 130, 129), ("circulant", 4132, 4000), ("circulant", 65580, 30000)])
def test_two_piece_dodis_circulant(ctx_2p, kind, n, m):
    """Dodis and Circulant in their Toeplitz form over the reversed input, split in
    two pieces (first piece: the reversed input's first a positions with the
    periodic seed's window from s_(n-a); second: the rest with the window from s_0)."""
    run_case(ctx_2p, kind, n, m, seed=17 * n + m)


def test_two_piece_dodis_degenerate(ctx_2p):
    n, m = 4099, 100
    y = W.bernoulli_bits(W.rng(3), n, 0.5)
    for x in (np.zeros(W.nwords(n), np.uint64), W.mask_tail(np.full(W.nwords(n), ~np.uint64(0)), n)):
        show_case("two-piece degenerate", int(x[0] & np.uint64(1)))
        code, z = gpu_extract(ctx_2p, "dodis", x, y, n, m)
        assert code == oracle.EDEGENERATE
        assert not z.any()


def test_dodis_degenerate_inputs(ctx):
    n, m = 1019, 300
    y = W.bernoulli_bits(W.rng(1), n, 0.5)
    for x in (np.zeros(W.nwords(n), np.uint64), W.mask_tail(np.full(W.nwords(n), ~np.uint64(0)), n)):
        show_case("degenerate", int(x[0] & np.uint64(1)))
        code, z = gpu_extract(ctx, "dodis", x, y, n, m)
        assert code == oracle.EDEGENERATE
        assert not z.any()
    # the same on the multi-pass path
    n = 65587
    y = W.bernoulli_bits(W.rng(2), n, 0.5)
    x = W.mask_tail(np.full(W.nwords(n), ~np.uint64(0)), n)
    code, z = gpu_extract(ctx, "dodis", x, y, n, 1000)
    assert code == oracle.EDEGENERATE and not z.any()


def test_host_side_errors(ctx):
    import torch
    x = torch.zeros(4, dtype=torch.int64, device="cuda")
    y = torch.zeros(8, dtype=torch.int64, device="cuda")
    z = torch.zeros(4, dtype=torch.int64, device="cuda")
    assert ctx.extract("toeplitz", x, y, 100, 0, z=z, check=False)[0] == oracle.EINVAL
    assert ctx.extract("toeplitz", x, y, 100, 101, z=z, check=False)[0] == oracle.EINVAL
    assert ctx.extract("dodis", x, y, 100, 10, z=z, check=False)[0] == oracle.ENOTNA
    assert ctx.extract("circulant", x, y, 11, 5, z=z, check=False)[0] == oracle.ENOTNA
    assert ctx.extract("toeplitz", x, y, 100, 50, z=x, check=False)[0] == oracle.EINVAL  # z overlaps x


def test_sync_flag_returns_status(ctx):
    import torch
    n, m = 1019, 64
    x = torch.zeros(W.nwords(n), dtype=torch.int64, device="cuda")
    y = torch.ones(W.nwords(n), dtype=torch.int64, device="cuda")
    rc, _ = ctx.extract("dodis", x, y, n, m, sync=True, check=False)
    assert rc == oracle.EDEGENERATE


def test_binding_rejects_short_buffers(ctx):
    """The binding checks buffer lengths before the library sees the raw pointers."""
    import torch
    n, m = 1000, 300
    x = torch.zeros(W.nwords(n), dtype=torch.int64, device="cuda")
    y = torch.zeros(W.nwords(n + m - 1), dtype=torch.int64, device="cuda")
    z = torch.zeros(W.nwords(m), dtype=torch.int64, device="cuda")
    with pytest.raises(ValueError):
        ctx.extract("toeplitz", x[:-1], y, n, m, z=z)
    with pytest.raises(ValueError):
        ctx.extract("toeplitz", x, y[:-1], n, m, z=z)
    with pytest.raises(ValueError):
        ctx.extract("toeplitz", x, y, n, m, z=z[:-1])
    with pytest.raises(TypeError):
        ctx.extract("toeplitz", x, y, n, m, z=z, status=torch.zeros(1, dtype=torch.int64, device="cuda"))
    with pytest.raises(TypeError):
        ctx.extract("toeplitz", x, y, n, m, z=z, status=torch.zeros(1, dtype=torch.int32))
    with pytest.raises(ValueError):
        ctx.batch([{"kind": "toeplitz", "n": n, "m": m, "x": x, "y": y[:-2], "z": z}])
    ctx.extract("toeplitz", x, y, n, m, z=z, sync=True)  # the full-length buffers pass
