"""Serving on the GPU: requests served in overlapping rounds on several streams
give exactly the bits of the same request run alone, and of the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import show_case, to_host

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone_and_oracle():
    import torch

    import paper_2402_09481_amd as P
    from paper_2402_09481_amd.serve import GpuExecutor, Server, make_requests, resident, summarize

    pool, seeds = resident()
    ctx = P.Context(0)
    # offered far above capacity so that rounds overlap on the streams
    reqs = make_requests(20000.0, 160, pool, seeds, seed=11, log_hi=20.0)
    srv = Server(GpuExecutor(ctx, nstreams=4), budget_bytes=2 << 30, max_batch=24)
    show_case("serve 160 requests")
    out = srv.run(reqs, idle=lambda dt: None)
    torch.cuda.synchronize()
    s = summarize(out, srv)
    assert s["completed"] == 160 and srv.rounds > 1
    ph = pool.cpu().numpy().view(np.uint64)
    for r in out:
        alone = ctx.extract("toeplitz", r.x, r.y, r.n, r.m, sync=True)
        assert torch.equal(alone, r.z), r.rid
        if r.n <= (1 << 15):
            x = to_host(r.x)
            y = to_host(r.y)
            assert np.array_equal(to_host(r.z), oracle.extract("toeplitz", x, y, r.n, r.m)[1]), r.rid
    ctx.close()


def test_serving_workload_at_its_sizes():
    """Requests of the serving workload's full size range (n log-uniform in
    [2^12, 2^26], m uniform in [n/4, n/2]) offered far above capacity, so that they
    are served in overlapping rounds on several streams: every result equals the
    same request alone and the oracle's GF(2)[t] product route."""
    import time

    import torch

    import paper_2402_09481_amd as P
    from paper_2402_09481_amd.serve import GpuExecutor, Server, make_requests, resident, summarize

    pool, seeds = resident()
    ctx = P.Context(0)
    reqs = make_requests(50000.0, 96, pool, seeds, seed=23)
    assert max(r.n for r in reqs) > (1 << 25)
    srv = Server(GpuExecutor(ctx, nstreams=4), budget_bytes=8 << 30, max_batch=16)
    show_case("serve 96 requests up to 2^26")
    out = srv.run(reqs, idle=lambda dt: None)
    torch.cuda.synchronize()
    s = summarize(out, srv)
    assert s["completed"] == 96 and srv.rounds > 1
    t0 = time.time()
    for r in out:
        alone = ctx.extract("toeplitz", r.x, r.y, r.n, r.m, sync=True)
        assert torch.equal(alone, r.z), r.rid
        code, want = oracle.toeplitz_product(to_host(r.x), to_host(r.y), r.n, r.m, "paper")
        assert code == 0 and np.array_equal(to_host(r.z), want), r.rid
    show_case("serve: oracle checks %.0f s" % (time.time() - t0))
    ctx.close()
