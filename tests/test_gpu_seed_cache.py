"""Cached seed transforms: calls that reuse a seed's cached spectrum give the same
bits as cold calls and as the oracle; clearing the cache and changing the seed
gives the new seed's result."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import show_case, to_dev, to_host

pytestmark = pytest.mark.gpu


def seed_len(kind, n, m):
    return {"toeplitz": n + m - 1, "circulant": n + 1, "dodis": n}[kind]


def check(ctx, kind, n, m, order="paper", blocks=3, seed=0):
    g = W.rng(seed)
    y = W.bernoulli_bits(g, seed_len(kind, n, m), 0.5)
    yd = to_dev(y)
    for b in range(blocks):
        x = W.bernoulli_bits(g, n, 0.4)
        if kind == "dodis":
            x[0] = (int(x[0]) | 1) & ~2
        show_case("seed cache", kind, n, m, order, b)
        z = ctx.extract(kind, to_dev(x), yd, n, m, seed_order=order, sync=True, cache_seed=True)
        want = oracle.extract(kind, x, y, n, m, order)[1]
        assert np.array_equal(to_host(z), want), (kind, n, m, b)
    return yd


@pytest.fixture(scope="module")
def ctx():
    import paper_2402_09481_amd as P
    c = P.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("kind,n,m,order", [("toeplitz", 100003, 50001, "paper"), ("toeplitz", 100003, 50001, "linear"),
                                            ("toeplitz", 1 << 19, 1 << 18, "paper"), ("dodis", 65587, 30000, "paper"),
                                            ("circulant", 65586, 65586, "paper")])
def test_cached_seed_matches_oracle(ctx, kind, n, m, order):
    check(ctx, kind, n, m, order, seed=n + m)


def test_cache_clear_and_new_seed_bits(ctx):
    n, m = 70001, 30000
    g = W.rng(3)
    y1 = W.bernoulli_bits(g, n + m - 1, 0.5)
    x = W.bernoulli_bits(g, n, 0.5)
    yd = to_dev(y1)
    z1 = ctx.extract("toeplitz", to_dev(x), yd, n, m, sync=True, cache_seed=True)
    assert np.array_equal(to_host(z1), oracle.extract("toeplitz", x, y1, n, m)[1])
    y2 = W.bernoulli_bits(g, n + m - 1, 0.5)
    yd.copy_(to_dev(y2))  # same address, new bits: the cache must be cleared
    b, e = ctx.seed_cache_clear()
    assert e >= 1 and b > 0
    z2 = ctx.extract("toeplitz", to_dev(x), yd, n, m, sync=True, cache_seed=True)
    assert np.array_equal(to_host(z2), oracle.extract("toeplitz", x, y2, n, m)[1])


def test_cached_seed_64bit_field():
    import paper_2402_09481_amd as P
    os.environ["EXT_FORCE_FIELD"] = "gl"
    try:
        c = P.Context(0)
    finally:
        del os.environ["EXT_FORCE_FIELD"]
    check(c, "toeplitz", 50000, 20000, seed=5)
    check(c, "dodis", 8219, 8219, seed=6)
    c.close()


def test_plan_change_between_cached_calls():
    """A seed spectrum cached under one plan of its size class is not reused after
    the class's plan changes (the spectrum's order in memory follows the plan)."""
    import paper_2402_09481_amd as P
    c = P.Context(0, tune=False)
    n, m = 70001, 30000  # transform 2^17
    g = W.rng(11)
    y = W.bernoulli_bits(g, n + m - 1, 0.5)
    yd = to_dev(y)
    for plan in ([8, 9], [7, 10], [9, 8], [8, 9]):
        c.tune_set(32, 17, plan, single=True)
        x = W.bernoulli_bits(g, n, 0.4)
        show_case("seed cache under plan", plan)
        z = c.extract("toeplitz", to_dev(x), yd, n, m, sync=True, cache_seed=True)
        assert np.array_equal(to_host(z), oracle.extract("toeplitz", x, y, n, m)[1]), plan
    c.close()


def test_cached_seed_from_several_threads():
    """Calls from four host threads, each on its own stream, that share one cached
    seed (and, from the second repetition on, a fifth thread clearing the cache
    all the while): a call that finds the entry while another is still
    enqueueing its transform, or while a clear is under way, runs without the
    cache; a clear waits for calls that hold an entry; every result equals the
    oracle."""
    import threading

    import torch

    import paper_2402_09481_amd as P
    c = P.Context(0)
    n, m = 300007, 100003
    g = W.rng(21)
    y = W.bernoulli_bits(g, n + m - 1, 0.5)
    xs = [[W.bernoulli_bits(g, n, 0.4) for _ in range(6)] for _ in range(4)]
    wants = [[oracle.extract("toeplitz", x, y, n, m)[1] for x in row] for row in xs]
    yd = to_dev(y)
    for rep in range(3):
        c.seed_cache_clear()
        errors = []

        def worker(t):
            try:
                s = torch.cuda.Stream()
                xd = [to_dev(x) for x in xs[t]]
                torch.cuda.synchronize()
                for k, x in enumerate(xd):
                    z = c.extract("toeplitz", x, yd, n, m, sync=True, stream=s, cache_seed=True)
                    if not np.array_equal(to_host(z), wants[t][k]):
                        errors.append((rep, t, k))
            except Exception as e:  # reported by the main thread
                errors.append((rep, t, repr(e)))

        stop = threading.Event()

        def clearer():  # from the second repetition on, the cache is cleared while calls use it
            while rep > 0 and not stop.is_set():
                c.seed_cache_clear()

        show_case("seed cache threads", rep)
        th = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
        cl = threading.Thread(target=clearer)
        cl.start()
        for t in th:
            t.start()
        for t in th:
            t.join()
        stop.set()
        cl.join()
        torch.cuda.synchronize()
        assert not errors, errors[:4]
    c.close()
