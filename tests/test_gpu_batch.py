"""Batched extraction: every job of a mixed batch equals the oracle and the same
job run alone, bit for bit; invalid jobs are reported and skipped; replays of a
cached batch signature with new inputs stay correct; jobs that run as piece
schedules (two pieces over the lazy field at 2^27, two pieces over 3*2^30+1 in a
context that forces them) are batched with the others."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import show_case, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2402_09481_amd as P
    c = P.Context(0)
    yield c
    c.close()


def make_batch(count, seed, lo=6.0, hi=17.0):
    params = W.batch_params(count, seed=seed, next_na=oracle.next_na, log_lo=lo, log_hi=hi)
    jobs = []
    g = W.rng(seed + 1)
    for i, (kind, n, m, px, sub) in enumerate(params):
        if i % 7 == 3:  # some Dodis jobs as well
            n = oracle.next_na(n)
            kind, m = "dodis", max(1, n // 2)
        j = W.make_job(kind, n, m, px, sub, seed_order="linear" if (kind == "toeplitz" and i % 2) else "paper")
        if kind == "dodis":
            j.x[0] = (int(j.x[0]) | 1) & ~2
        jobs.append(j)
    return jobs


def run_batch(ctx, jobs, unbatched=False, graph=False, single_transform=False):
    import torch
    dev = []
    for j in jobs:
        z = torch.full((W.nwords(j.m),), -1, dtype=torch.int64, device="cuda")
        st = torch.full((1,), 777, dtype=torch.int32, device="cuda")
        dev.append({"kind": j.kind, "n": j.n, "m": j.m, "x": to_dev(j.x), "y": to_dev(j.y), "z": z, "status": st,
                    "seed_order": j.seed_order, "single_transform": single_transform})
    rc, errs = ctx.batch(dev, sync=True, unbatched=unbatched, graph=graph)
    torch.cuda.synchronize()
    return rc, errs, [to_host(d["z"]) for d in dev], [int(d["status"].item()) for d in dev]


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_oracle_and_single(ctx, graph):
    jobs = make_batch(160, seed=5)
    show_case("batch 160 jobs", graph)
    rc, errs, zs, sts = run_batch(ctx, jobs, graph=graph)
    assert rc == 0 and all(e == 0 for e in errs)
    rc2, errs2, zs2, sts2 = run_batch(ctx, jobs, unbatched=True)
    assert rc2 == 0
    for j, z, z2, st in zip(jobs, zs, zs2, sts):
        assert st == 0
        code, want = oracle.extract(j.kind, j.x, j.y, j.n, j.m, j.seed_order)
        assert code == 0
        assert np.array_equal(z, want), (j.kind, j.n, j.m)
        assert np.array_equal(z, z2)


def test_batch_replay_with_new_inputs(ctx):
    # same shapes (same batch signature, so the cached graph is replayed), new bits
    a = make_batch(40, seed=9, lo=8, hi=16)
    show_case("batch replay")
    run_batch(ctx, a, graph=True)
    b = []
    for j in a:
        g = W.rng(j.n * 31 + j.m)
        x = W.bernoulli_bits(g, j.n, 0.4)
        if j.kind == "dodis":
            x[0] = (int(x[0]) | 1) & ~2
        b.append(W.Job(j.kind, j.n, j.m, x, W.bernoulli_bits(g, j.seed_bits, 0.5), j.seed_order))
    for _ in range(2):
        rc, errs, zs, sts = run_batch(ctx, b, graph=True)
        assert rc == 0
        for j, z in zip(b, zs):
            assert np.array_equal(z, oracle.extract(j.kind, j.x, j.y, j.n, j.m, j.seed_order)[1])


def test_batch_reports_invalid_jobs(ctx):
    jobs = make_batch(12, seed=13, lo=8, hi=12)
    bad = W.Job("circulant", 11, 5, W.bernoulli_bits(W.rng(1), 11, 0.5), W.bernoulli_bits(W.rng(2), 12, 0.5))
    degen = W.Job("dodis", 1019, 100, np.zeros(W.nwords(1019), np.uint64), W.bernoulli_bits(W.rng(3), 1019, 0.5))
    jobs = jobs[:5] + [bad, degen] + jobs[5:]
    show_case("batch invalid")
    rc, errs, zs, sts = run_batch(ctx, jobs)
    assert errs[5] == oracle.ENOTNA and rc == oracle.ENOTNA
    assert errs[6] == 0 and sts[6] == oracle.EDEGENERATE and not zs[6].any()
    for i, j in enumerate(jobs):
        if i in (5, 6):
            continue
        assert errs[i] == 0 and sts[i] == 0
        assert np.array_equal(zs[i], oracle.extract(j.kind, j.x, j.y, j.n, j.m, j.seed_order)[1])


@pytest.mark.parametrize("unbatched", [False, True])
def test_linear_seed_order_is_a_toeplitz_option(ctx, unbatched):
    """A Circulant or Dodis job that asks for the linear seed order is rejected
    (EXT_EINVAL, as by extract_circulant / extract_dodis) in the batch and in the
    per-job comparison alike; the other jobs run."""
    jobs = make_batch(6, seed=31, lo=8, hi=12)
    na = oracle.next_na(200)
    circ = W.make_job("circulant", na - 1, 50, 0.4, 4, seed_order="linear")
    dod = W.make_job("dodis", na, 60, 0.4, 5, seed_order="linear")
    jobs = jobs[:3] + [circ, dod] + jobs[3:]
    show_case("batch linear order", unbatched)
    rc, errs, zs, sts = run_batch(ctx, jobs, unbatched=unbatched)
    assert errs[3] == oracle.EINVAL and errs[4] == oracle.EINVAL and rc == oracle.EINVAL
    for i, j in enumerate(jobs):
        if i in (3, 4):
            continue
        assert errs[i] == 0 and sts[i] == 0
        assert np.array_equal(zs[i], oracle.extract(j.kind, j.x, j.y, j.n, j.m, j.seed_order)[1])


def test_batched_workload_at_its_sizes():
    """The batched workload exactly as the benchmark runs it: 4096 Toeplitz/Circulant
    blocks, n log-uniform in [2^10, 2^22], m = n/2, one extract_batch replayed from a
    HIP graph (twice, the second a replay). Every block's whole output against the
    oracle: the GF(2)[t] product route for all blocks, the schoolbook rows as well
    for n <= 2^14."""
    import time

    import torch

    import paper_2402_09481_amd as P
    show_case("batched workload: generating 4096 blocks")
    jobs = W.batch_jobs(4096, next_na=oracle.next_na)
    assert len(jobs) == 4096 and max(j.n for j in jobs) > (1 << 21) and min(j.n for j in jobs) < (1 << 11)
    c = P.Context(0)
    dev = []
    for j in jobs:
        dev.append({"kind": j.kind, "n": j.n, "m": j.m, "x": to_dev(j.x), "y": to_dev(j.y),
                    "z": torch.full((W.nwords(j.m),), -1, dtype=torch.int64, device="cuda")})
    show_case("batched workload: graph capture + replay")
    for rep in range(2):
        for d in dev:
            d["z"].fill_(-1)
        rc, errs = c.batch(dev, sync=True, graph=True)
        assert rc == 0 and not any(errs)
    torch.cuda.synchronize()
    zs = [to_host(d["z"]) for d in dev]
    t0 = time.time()
    for i, (j, z) in enumerate(zip(jobs, zs)):
        if i % 512 == 0:
            show_case("batched workload: oracle block %d (%.0f s)" % (i, time.time() - t0))
        code, want = oracle.extract_product(j.kind, j.x, j.y, j.n, j.m, j.seed_order)
        assert code == 0
        assert np.array_equal(z, want), (i, j.kind, j.n, j.m)
        if j.n <= (1 << 14):
            assert np.array_equal(z, oracle.extract(j.kind, j.x, j.y, j.n, j.m, j.seed_order)[1])
    c.close()
    del dev
    torch.cuda.empty_cache()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_with_lazy_two_piece_jobs(ctx, graph):
    """Jobs whose one transform would be 2^27 run as two pieces over 7*2^26+1 in the
    batch too (both orders, Dodis with a degenerate input, Circulant), beside
    single-transform and single-workgroup jobs."""
    import os
    big = (1 << 26) - (1 << 20)
    p = oracle.next_na(big)
    shapes = [("toeplitz", 1 << 26, 1 << 25, "paper"), ("toeplitz", (1 << 26) - 4097, (1 << 25) - 3, "linear"),
              ("dodis", p, 1 << 24, "paper"), ("circulant", p - 1, (1 << 24) + 9, "paper"),
              ("toeplitz", 5000, 2000, "paper"), ("toeplitz", 300000, 150000, "linear"), ("dodis", 65587, 30000, "paper")]
    jobs = []
    for i, (kind, n, m, order) in enumerate(shapes):
        g = W.rng(1000 + i)
        x = W.bernoulli_bits(g, n, 0.4)
        if kind == "dodis":
            x[0] = (int(x[0]) | 1) & ~2
        y = W.bernoulli_bits(g, {"toeplitz": n + m - 1, "circulant": n + 1, "dodis": n}[kind], 0.5)
        jobs.append(W.Job(kind, n, m, x, y, order))
    # a degenerate Dodis input of the two-piece size
    jobs.append(W.Job("dodis", p, 1 << 24, np.zeros(W.nwords(p), np.uint64), jobs[2].y, "paper"))
    show_case("batch with lazy two-piece jobs", graph)
    rc, errs, zs, sts = run_batch(ctx, jobs, graph=graph)
    assert errs[:-1] == [0] * (len(jobs) - 1)
    assert sts[-1] == oracle.EDEGENERATE and not zs[-1].any()
    for j, z, st in zip(jobs[:-1], zs, sts):
        assert st == 0
        code, want = oracle.extract_product(j.kind, j.x, j.y, j.n, j.m, j.seed_order)
        assert code == 0 and np.array_equal(z, want), (j.kind, j.n, j.m)
    # the same batch with one transform per job (EXT_SINGLE_TRANSFORM per job)
    rc, errs, zs1, sts1 = run_batch(ctx, jobs, graph=graph, single_transform=True)
    assert rc == 0 and sts1 == sts
    assert all(np.array_equal(a, b) for a, b in zip(zs, zs1))


def test_batch_with_forced_two_piece_jobs():
    """A context that runs every multi-pass shape as two pieces over 3*2^30+1: the
    batch path's piece descriptors and launch phases at small sizes."""
    import os

    import paper_2402_09481_amd as P
    os.environ["EXT_FORCE_FIELD"] = "p0x2"
    try:
        c = P.Context(0)
    finally:
        del os.environ["EXT_FORCE_FIELD"]
    jobs = make_batch(48, seed=21, lo=8, hi=16)
    for graph in (False, True):
        show_case("forced two-piece batch", graph)
        rc, errs, zs, sts = run_batch(c, jobs, graph=graph)
        assert rc == 0 and not any(errs)
        for j, z, st in zip(jobs, zs, sts):
            assert st == 0
            assert np.array_equal(z, oracle.extract(j.kind, j.x, j.y, j.n, j.m, j.seed_order)[1]), (j.kind, j.n, j.m)
    c.close()

