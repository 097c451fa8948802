"""GPU parity of the Von Neumann extractor (section "Von Neumann", Alg. 3): the
HIP compaction against the oracle, bit for bit, through the C-ABI — output
length, every output word, untouched words past the output, error cases."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import show_case, to_dev, to_host

pytestmark = pytest.mark.gpu

TILE_BITS = 1 << 19  # input bits of one workgroup tile (1024 threads x 8 words)
SENTINEL = -0x123456789ABCDEF


@pytest.fixture(scope="module")
def ctx():
    import paper_2402_09481_amd as P
    c = P.Context(0)
    yield c
    c.close()


def run_vn(ctx, x, n, extra_words=3):
    """(code, m, z words [0, ceil(m/64)), the words after them) through the C-ABI."""
    import torch
    cap = W.nwords(n // 2) + extra_words
    z = torch.full((cap,), SENTINEL, dtype=torch.int64, device="cuda")
    m_out = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    st = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    rc, z, m_out = ctx.von_neumann(to_dev(x), n, z=z, m_out=m_out, status=st, check=False)
    assert rc == 0
    torch.cuda.synchronize()
    m = int(m_out.item())
    zh = to_host(z)
    return int(st.item()), m, zh[: W.nwords(m)], zh[W.nwords(m):]


def check_against_oracle(ctx, x, n, label):
    show_case("von_neumann", label, n)
    code, m, z, rest = run_vn(ctx, x, n)
    ocode, oz, om = oracle.von_neumann(x, n)
    assert code == ocode, (label, n, code, ocode)
    assert m == om, (label, n, m, om)
    assert np.array_equal(z, oz), (label, n)
    assert np.all(rest == np.uint64(SENTINEL & ((1 << 64) - 1))), (label, n)
    return m


def pattern(kind, n, g):
    if kind == "iid":
        return W.bernoulli_bits(g, n, W.VN_P)
    if kind == "half":
        return W.bernoulli_bits(g, n, 0.5)
    if kind == "biased":
        return W.bernoulli_bits(g, n, 0.03)
    if kind == "alternating":  # every pair differs: m = floor(n/2)
        return W.pack_bits(np.tile(np.array([1, 0], np.uint8), n // 2 + 1)[:n])
    if kind == "sparse":  # a few differing pairs, most tiles empty
        bits = np.zeros(n, np.uint8)
        bits[g.choice(n, size=max(1, n // 100_000), replace=False)] = 1
        return W.pack_bits(bits)
    if kind == "bursts":  # short random bursts between long constant runs
        bits = np.zeros(n, np.uint8)
        for s in range(0, n, 70_001):
            k = int(g.integers(0, 90))
            bits[s:s + k] = g.integers(0, 2, size=len(bits[s:s + k]))
        return W.pack_bits(bits)
    raise ValueError(kind)


SIZES = [2, 3, 63, 64, 65, 127, 128, 129, 1000, 4097, 65_535, TILE_BITS // 2 + 1,
         TILE_BITS - 1, TILE_BITS, TILE_BITS + 1, TILE_BITS + 64, 3 * TILE_BITS + 77, 1_000_003, 4_194_319]


@pytest.mark.parametrize("kind", ["iid", "half", "biased", "alternating", "sparse", "bursts"])
def test_parity_sizes(ctx, kind):
    g = W.rng(sum(map(ord, kind)))
    for n in SIZES:
        check_against_oracle(ctx, pattern(kind, n, g), n, kind)


def test_many_tiles_paper_shape(ctx):
    # the paper's largest input length of its throughput figure, i.i.d. with input
    # min-entropy n/2 (1908 tiles)
    n = W.VN_PAPER_N
    x = W.von_neumann_input(n)
    m = check_against_oracle(ctx, x, n, "paper")
    assert abs(m - n * W.VN_P * (1 - W.VN_P)) < 6 * np.sqrt(n)


def test_degenerate_and_tails(ctx):
    # no pair differs: status EXT_EDEGENERATE, m = 0, z untouched
    for bits in ([0, 0], [1, 1, 1], [0, 0, 1, 1] * 1000, [1] * 300_001):
        n = len(bits)
        code, m, z, rest = run_vn(ctx, W.pack_bits(np.array(bits, np.uint8)), n)
        assert code == oracle.EDEGENERATE and m == 0
        assert np.all(rest == np.uint64(SENTINEL & ((1 << 64) - 1)))
    # input bits past n are ignored; an odd last bit belongs to no pair
    g = W.rng(77)
    for n in (301, 262_145, 1_000_001):
        x = W.bernoulli_bits(g, n, 0.5)
        dirty = x.copy()
        r = n & 63
        dirty[-1] |= np.uint64(((1 << 64) - 1) ^ ((1 << r) - 1))
        a = run_vn(ctx, x, n)
        b = run_vn(ctx, dirty, n)
        c = run_vn(ctx, x, n - 1)
        assert a[1] == b[1] == c[1] and np.array_equal(a[2], b[2]) and np.array_equal(a[2], c[2])
        assert np.array_equal(a[2], oracle.von_neumann(x, n)[1])


def test_sync_and_errors(ctx):
    import torch

    import paper_2402_09481_amd as P
    g = W.rng(8)
    n = 100_000
    x = to_dev(W.bernoulli_bits(g, n, 0.4))
    z, m = ctx.von_neumann(x, n, sync=True)
    code, oz, om = oracle.von_neumann(to_host(x), n)
    assert m == om and np.array_equal(to_host(z)[: W.nwords(m)], oz)
    z2, m2 = P.VonNeumann(n, context=ctx).extract(x)
    assert m2 == m and np.array_equal(to_host(z2)[: W.nwords(m)], oz)
    # degenerate with EXT_SYNC: returned
    zero = torch.zeros(W.nwords(n), dtype=torch.int64, device="cuda")
    rc, _, _ = ctx.von_neumann(zero, n, sync=True, check=False)
    assert rc == oracle.EDEGENERATE
    # host-side errors: nothing enqueued
    small = torch.zeros(W.nwords(n // 2) - 1, dtype=torch.int64, device="cuda")
    assert ctx.von_neumann(x, n, z=small, check=False)[0] == oracle.EINVAL
    assert ctx.von_neumann(x, 1, check=False)[0] == oracle.EINVAL
    assert ctx.von_neumann(x, (1 << 40) + 2, z=small, check=False)[0] == P.EXT_ETOOLARGE
    assert ctx.von_neumann(x, n, z=x, check=False)[0] == oracle.EINVAL  # z overlaps x
    lib = ctx._lib
    mo = torch.zeros(1, dtype=torch.int64, device="cuda")
    zz = torch.zeros(W.nwords(n // 2), dtype=torch.int64, device="cuda")
    assert lib.extract_von_neumann(ctx.handle, x.data_ptr(), n, zz.data_ptr(), zz.numel(), mo.data_ptr(), 8, None,
                                   None) == oracle.EINVAL  # flags other than EXT_SYNC
    assert lib.extract_von_neumann(ctx.handle, x.data_ptr(), n, zz.data_ptr(), zz.numel(), None, 0, None,
                                   None) == oracle.EINVAL  # m_out is required
    assert ctx.workspace_bytes("von_neumann", n, 0) > 0


def test_large_sampled(ctx):
    """One HBM-scale call (2^33 bits, 1 GiB): the output length against the count of
    differing pairs, the first 2^30 input bits' output against the whole oracle (the
    output of an even-length prefix is a prefix of the output), and windows further
    in against the oracle run on the window's input words."""
    import torch
    n = W.VN_LARGE_N
    show_case("von_neumann large", n)
    xd = W.bernoulli_bits_device(n, W.VN_P, W.BASE_SEED + 9)
    z = torch.empty(W.nwords(n // 2), dtype=torch.int64, device="cuda")
    z, m = ctx.von_neumann(xd, n, z=z, sync=True)
    xh = to_host(xd)
    # the number of differing pairs per word, and where each word's output starts
    d = (xh ^ (xh >> np.uint64(1))) & np.uint64(0x5555555555555555)
    per = np.bitwise_count(d).astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(per)])
    assert m == int(starts[-1])
    zh = to_host(z)
    zbits_at = lambda off, cnt: W.unpack_bits(window(zh, off, cnt), cnt)  # noqa: E731
    head = 1 << 30
    code, oz, om = oracle.von_neumann(xh[: head >> 6], head)
    assert om == int(starts[head >> 6])
    assert np.array_equal(zh[: om >> 6], oz[: om >> 6])
    assert np.array_equal(zbits_at(0, om), W.unpack_bits(oz, om))
    g = W.rng(123)
    for w0 in g.integers(0, len(xh) - 4096, size=24):
        w0 = int(w0)
        cnt_w = int(g.integers(1, 4096))
        code, oz, om = oracle.von_neumann(xh[w0: w0 + cnt_w], 64 * cnt_w)
        assert om == int(starts[w0 + cnt_w] - starts[w0])
        if om:
            assert np.array_equal(zbits_at(int(starts[w0]), om), W.unpack_bits(oz, om)), w0
    tail = zh[W.nwords(m) - 1]
    if m & 63:
        assert int(tail) >> (m & 63) == 0


def window(words, off, cnt):
    """Packed bits off .. off+cnt-1 of a packed string."""
    w0, b = off >> 6, off & 63
    nw = (cnt + 63) >> 6
    seg = np.zeros(nw + 1, np.uint64)
    src = words[w0: w0 + nw + 1]
    seg[: len(src)] = src
    if b:
        out = (seg[:-1] >> np.uint64(b)) | (seg[1:] << np.uint64(64 - b))
    else:
        out = seg[:-1].copy()
    return W.mask_tail(out, cnt)
