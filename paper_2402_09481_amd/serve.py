"""Continuous-batching extraction server.

Requests (kind, n, m, input, seed) arrive on an open-loop schedule. The server
keeps a FIFO of arrived requests and admits them, in order, whenever (a) a
stream slot is free and (b) the device memory the request needs — the
library's workspace for its shape plus its output — fits in what the HBM
budget has left after the requests already in flight. Each admission round
launches the admitted requests as one ``extract_batch`` on a free HIP stream,
so requests that arrive while others are on the GPU join the next round and
their work overlaps on the device with the rounds still running; memory and
slots return as rounds complete. Latency is measured from each request's
scheduled arrival time (no coordinated omission) to the moment the host
observes its round complete.

The scheduling logic is plain Python over an executor interface, so it runs
on the CPU against a simulated executor in the tests; ``GpuExecutor`` is the
real one (C-ABI calls on torch streams, completion by HIP events).

This serves many privacy-amplification blocks at once (section "Cryptomite for
privacy amplification in QKD"), with seeds and twiddle tables kept resident.
"""
from __future__ import annotations

import collections
import dataclasses
import time


@dataclasses.dataclass
class Request:
    rid: int
    t_arrival: float          # seconds from the start of the run
    kind: str
    n: int
    m: int
    x: object = None          # device tensor of packed input words (a view into a resident pool)
    y: object = None          # device tensor of packed seed words (a resident seed)
    seed_order: str = "paper"
    footprint: int = 0        # device bytes while in flight
    z: object = None          # output (allocated at admission)
    t_admit: float | None = None
    t_done: float | None = None
    rejected: bool = False


class GpuExecutor:
    """Runs admission rounds as extract_batch calls on a fixed set of HIP streams."""

    def __init__(self, ctx, nstreams: int = 4):
        import torch
        self.ctx = ctx
        self.torch = torch
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]  # default priority
        self.free = list(range(nstreams))

    def footprint(self, r: Request) -> int:
        return self.ctx.workspace_bytes(r.kind, r.n, r.m) + 8 * ((r.m + 63) >> 6) + 512

    def slots(self) -> int:
        return len(self.free)

    def submit(self, reqs):
        torch = self.torch
        s = self.free.pop()
        stream = self.streams[s]
        jobs = []
        with torch.cuda.stream(stream):
            for r in reqs:
                r.z = torch.empty((r.m + 63) >> 6, dtype=torch.int64, device="cuda")
                jobs.append({"kind": r.kind, "n": r.n, "m": r.m, "x": r.x, "y": r.y, "z": r.z,
                             "seed_order": r.seed_order})
        rc, errs = self.ctx.batch(jobs, stream=stream)
        if rc != 0:
            raise RuntimeError("extract_batch failed: %d %s" % (rc, errs))
        ev = torch.cuda.Event()
        ev.record(stream)
        return (s, ev)

    def done(self, handle) -> bool:
        return handle[1].query()

    def release(self, handle):
        self.free.append(handle[0])


class SimExecutor:
    """CPU stand-in: a round completes `latency(reqs)` seconds after submission."""

    def __init__(self, nslots: int, footprint, latency, clock):
        self.nslots, self._fp, self._lat, self.clock = nslots, footprint, latency, clock
        self.busy = 0
        self.log = []  # (t_submit, t_done, [rid])

    def footprint(self, r):
        return self._fp(r)

    def slots(self):
        return self.nslots - self.busy

    def submit(self, reqs):
        self.busy += 1
        t = self.clock()
        h = (t, t + self._lat(reqs), [r.rid for r in reqs])
        self.log.append(h)
        return h

    def done(self, h):
        return self.clock() >= h[1]

    def release(self, h):
        self.busy -= 1


class Server:
    def __init__(self, executor, budget_bytes: int, max_batch: int = 256):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.in_use = 0
        self.peak_in_use = 0
        self.rounds = 0
        self.round_sizes = []

    def run(self, requests, clock=time.perf_counter, idle=lambda dt: None, until_drained: bool = True):
        """Serve `requests` (sorted by t_arrival, seconds relative to the start).
        Returns the requests with t_admit / t_done filled (relative seconds)."""
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        for r in reqs:
            r.footprint = self.ex.footprint(r)
            r.rejected = r.footprint > self.budget
        t0 = clock()
        now = lambda: clock() - t0
        pending = collections.deque()
        inflight = []  # (handle, [requests], bytes)
        i = 0
        max_pending = 0
        while i < len(reqs) or pending or inflight:
            t = now()
            while i < len(reqs) and reqs[i].t_arrival <= t:
                if not reqs[i].rejected:
                    pending.append(reqs[i])
                i += 1
            max_pending = max(max_pending, len(pending))
            # completions give back memory and a slot
            still = []
            for h, rs, nbytes in inflight:
                if self.ex.done(h):
                    td = now()
                    for r in rs:
                        r.t_done = td
                    self.in_use -= nbytes
                    self.ex.release(h)
                else:
                    still.append((h, rs, nbytes))
            inflight = still
            # admission: FIFO while memory and a slot allow
            if pending and self.ex.slots() > 0:
                batch, nbytes = [], 0
                while pending and len(batch) < self.max_batch and \
                        self.in_use + nbytes + pending[0].footprint <= self.budget:
                    r = pending.popleft()
                    batch.append(r)
                    nbytes += r.footprint
                if batch:
                    ta = now()
                    for r in batch:
                        r.t_admit = ta
                    h = self.ex.submit(batch)
                    self.in_use += nbytes
                    self.peak_in_use = max(self.peak_in_use, self.in_use)
                    inflight.append((h, batch, nbytes))
                    self.rounds += 1
                    self.round_sizes.append(len(batch))
                    continue
            if not until_drained and i >= len(reqs) and not pending:
                break
            # nothing to do right now: wait a little (next arrival or a completion)
            nxt = reqs[i].t_arrival - now() if i < len(reqs) else 1e-4
            idle(max(0.0, min(nxt, 1e-4)))
        self.max_pending = max_pending
        return reqs


def percentile(vals, q):
    if not vals:
        return float("nan")
    v = sorted(vals)
    k = min(len(v) - 1, max(0, int(round(q / 100.0 * (len(v) - 1)))))
    return v[k]


def summarize(reqs, server=None):
    done = [r for r in reqs if r.t_done is not None]
    lat = [(r.t_done - r.t_arrival) * 1e3 for r in done]
    if not done:
        return {"completed": 0}
    span = max(r.t_done for r in done) - min(r.t_arrival for r in done)
    out = {
        "completed": len(done),
        "rejected": sum(1 for r in reqs if r.rejected),
        "span_s": round(span, 4),
        "throughput_req_s": round(len(done) / span, 1) if span > 0 else None,
        "output_Mbit_s": round(sum(r.m for r in done) / span / 1e6, 1) if span > 0 else None,
        "p50_ms": round(percentile(lat, 50), 3),
        "p99_ms": round(percentile(lat, 99), 3),
        "max_ms": round(max(lat), 3),
    }
    if server is not None:
        out["rounds"] = server.rounds
        out["mean_round_size"] = round(sum(server.round_sizes) / max(1, len(server.round_sizes)), 2)
        out["peak_bytes_in_flight"] = server.peak_in_use
        out["max_pending"] = getattr(server, "max_pending", None)
    return out


def make_requests(rate: float, count: int, pool, seeds, seed: int = None, **kw):
    """Requests of the serving workload (Toeplitz, n log-uniform in [2^12, 2^26],
    m uniform in [n/4, n/2], x a slice of the resident pool, y a resident seed)."""
    import workloads as W
    if seed is not None:
        kw["seed"] = seed
    out = []
    for k, q in enumerate(W.serving_requests(rate, count, **kw)):
        nw = (q.n + 63) >> 6
        x = pool[q.x_offset >> 6: (q.x_offset >> 6) + nw]
        y = seeds[q.seed_id][: ((q.n + q.m - 1) + 63) >> 6]
        out.append(Request(k, q.t_arrival, "toeplitz", q.n, q.m, x, y))
    return out


def resident(device="cuda"):
    """The resident input pool and seeds on the GPU."""
    import numpy as np
    import torch

    import workloads as W
    pool, seeds = W.serving_pool()
    return (torch.from_numpy(pool.view(np.int64)).to(device),
            [torch.from_numpy(s.view(np.int64)).to(device) for s in seeds])


def bench(log=print, rates=(1000, 5000, 20000, 50000), count=800, budget_gib=24.0, nstreams=4):
    """Open-loop Poisson sweep of the serving workload on one GPU."""
    import torch

    import paper_2402_09481_amd as P
    log("serving: uploading resident pool and seeds")
    pool, seeds = resident()
    ctx = P.Context(0, hbm_budget_bytes=int((budget_gib + 4) * (1 << 30)))
    out = {"budget_gib": budget_gib, "streams": nstreams, "requests_per_rate": count, "rates": []}
    # warm the pool and the kernels
    Server(GpuExecutor(ctx, nstreams), int(budget_gib * (1 << 30))).run(
        make_requests(1000.0, 32, pool, seeds, seed=7), idle=time.sleep)
    torch.cuda.synchronize()
    for rate in rates:
        log("serving: rate %d req/s" % rate)
        srv = Server(GpuExecutor(ctx, nstreams), int(budget_gib * (1 << 30)))
        reqs = srv.run(make_requests(float(rate), count, pool, seeds), idle=time.sleep)
        torch.cuda.synchronize()
        s = summarize(reqs, srv)
        s["offered_req_s"] = rate
        out["rates"].append(s)
    ctx.close()
    del pool, seeds
    torch.cuda.empty_cache()
    return out
