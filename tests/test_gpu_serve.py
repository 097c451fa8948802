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
