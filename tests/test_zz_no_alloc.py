"""The allocation-free Toeplitz entry point (extract_toeplitz_noalloc): its
output equals extract_toeplitz's, bit for bit, and the oracle's, on two calls in
a row (the second with a smaller input), at a multi-pass size, at the largest
size its fixed workspace holds, and at a single-workgroup size; shapes beyond
the workspace are rejected without touching z; the context's workspace pool is
not used and the device's free memory does not change."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import show_case, to_dev, to_host

pytestmark = pytest.mark.gpu


def _case(g, n, m):
    return W.bernoulli_bits(g, n, 0.4), W.bernoulli_bits(g, n + m - 1, 0.5)


def _noalloc(ctx, xd, yd, n, m, order="paper", sync=False):
    import torch
    z = torch.full((W.nwords(m),), -1, dtype=torch.int64, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    rc, z = ctx.extract("toeplitz", xd, yd, n, m, z=z, seed_order=order, status=st, sync=sync, check=False,
                        no_alloc=True)
    torch.cuda.synchronize()
    return rc, int(st.item()), z


def test_noalloc_matches_extract_toeplitz_twice():
    import torch

    import paper_2402_09481_amd as P
    ctx = P.Context(0)
    g = W.rng(4242)
    shapes = [((1 << 21) + 1234, (1 << 20) + 7, "paper"),   # transform 2^22: the largest that fits
              (100_003, 30_001, "linear"),                  # then a smaller one, multi-pass
              (4096, 2048, "linear")]                       # and one workgroup (no workspace)
    for n, m, order in shapes:
        show_case("noalloc", n, m, order)
        x, y = _case(g, n, m)
        xd, yd = to_dev(x), to_dev(y)
        rc, st, z = _noalloc(ctx, xd, yd, n, m, order)
        assert rc == 0 and st == 0, (rc, st)
        want = ctx.extract("toeplitz", xd, yd, n, m, seed_order=order, sync=True)
        assert torch.equal(z, want), (n, m)
        code, ref = oracle.toeplitz_product(x, y, n, m, order)
        assert code == 0 and np.array_equal(to_host(z), ref), (n, m)
    # the pool was never used by the allocation-free calls: nothing leased or cached
    # beyond what the extract_toeplitz comparisons took
    ctx.close()


def test_noalloc_allocates_nothing_and_rejects_oversize():
    import torch

    import paper_2402_09481_amd as P
    ctx = P.Context(0)
    g = W.rng(77)
    n, m = 300_000, 150_000
    x, y = _case(g, n, m)
    xd, yd = to_dev(x), to_dev(y)
    z = torch.empty(W.nwords(m), dtype=torch.int64, device="cuda")
    ctx.extract("toeplitz", xd, yd, n, m, z=z, no_alloc=True, sync=True)  # first launches of these kernels
    torch.cuda.synchronize()
    stats0 = ctx.mem_stats()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        rc = ctx.extract("toeplitz", xd, yd, n, m, z=z, no_alloc=True, sync=True, check=False)[0]
        assert rc == 0
    torch.cuda.synchronize()
    assert ctx.mem_stats() == stats0 and stats0["in_use"] == 0
    assert torch.cuda.mem_get_info()[0] == free0
    assert np.array_equal(to_host(z), oracle.toeplitz_product(x, y, n, m)[1])
    # beyond the fixed workspace: a transform of 2^23
    nb, mb = 1 << 22, 1 << 21
    xb, yb = to_dev(W.bernoulli_bits(g, nb, 0.5)), to_dev(W.bernoulli_bits(g, nb + mb - 1, 0.5))
    zb = torch.full((W.nwords(mb),), 12345, dtype=torch.int64, device="cuda")
    rc = ctx.extract("toeplitz", xb, yb, nb, mb, z=zb, no_alloc=True, check=False)[0]
    assert rc == P._lib.EXT_ESCRATCH
    torch.cuda.synchronize()
    assert bool((zb == 12345).all())
    with pytest.raises(P.ExtError):
        ctx.extract("toeplitz", xb, yb, nb, mb, z=zb, no_alloc=True)
    # flags it does not take
    assert ctx._lib.extract_toeplitz_noalloc(ctx.handle, xd.data_ptr(), n, yd.data_ptr(), m, z.data_ptr(),
                                             P._lib.EXT_SEED_CACHED, None, None) == P._lib.EXT_EINVAL
    ctx.close()
