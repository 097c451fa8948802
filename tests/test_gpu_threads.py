"""Calls on one context from several host threads at once, each on its own
stream: graph-mode batches that share one cached graph (same batch signature,
different inputs), and single extractions. Every result must equal the
oracle's, bit for bit, whatever the interleaving of the host-side steps."""
import threading

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import show_case, to_dev, to_host

pytestmark = pytest.mark.gpu

THREADS = 3
ITERS = 12


def _jobs(seed):
    """The same shapes for every thread (so one graph signature), seeded bits."""
    g = W.rng(seed)
    shapes = [("toeplitz", 4096, 2048), ("toeplitz", 70000, 30001), ("circulant", 16420, 9000),
              ("toeplitz", 300000, 100000), ("dodis", 65587, 30000), ("toeplitz", 1000, 999)]
    out = []
    for kind, n, m in shapes:
        seed_bits = {"toeplitz": n + m - 1, "circulant": n + 1, "dodis": n}[kind]
        x = W.bernoulli_bits(g, n, 0.4)
        if kind == "dodis":
            x[0] = (int(x[0]) | 1) & ~2
        y = W.bernoulli_bits(g, seed_bits, 0.5)
        want = oracle.extract(kind, x, y, n, m)[1]
        out.append((kind, n, m, x, y, want))
    return out


def test_concurrent_graph_batches_and_extractions():
    import torch

    import paper_2402_09481_amd as P
    ctx = P.Context(0)
    per_thread = [_jobs(1000 + t) for t in range(THREADS)]
    errors = []

    def worker(t):
        try:
            stream = torch.cuda.Stream()  # default priority
            jobs = per_thread[t]
            dev = [{"kind": k, "n": n, "m": m, "x": to_dev(x), "y": to_dev(y),
                    "z": torch.full((W.nwords(m),), -1, dtype=torch.int64, device="cuda")}
                   for k, n, m, x, y, _ in jobs]
            torch.cuda.synchronize()
            for it in range(ITERS):
                for d in dev:
                    d["z"].fill_(-1)
                torch.cuda.synchronize()
                rc, errs = ctx.batch(dev, stream=stream, graph=True, sync=True)
                if rc != 0 or any(errs):
                    errors.append((t, it, "batch rc", rc, errs))
                    return
                for d, (_, _, _, _, _, want) in zip(dev, jobs):
                    if not np.array_equal(to_host(d["z"]), want):
                        errors.append((t, it, "batch output", d["kind"], d["n"]))
                        return
                # a single extraction between the replays
                k, n, m, x, y, want = jobs[it % len(jobs)]
                with torch.cuda.stream(stream):
                    z = ctx.extract(k, dev[it % len(jobs)]["x"], dev[it % len(jobs)]["y"], n, m, sync=True,
                                    stream=stream)
                if not np.array_equal(to_host(z), want):
                    errors.append((t, it, "extract output", k, n))
                    return
        except Exception as e:  # reported by the main thread
            errors.append((t, "exception", repr(e)))

    show_case("threads: %d threads x %d graph-mode batches" % (THREADS, ITERS))
    th = [threading.Thread(target=worker, args=(t,)) for t in range(THREADS)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    ctx.close()
    assert not errors, errors[:5]
