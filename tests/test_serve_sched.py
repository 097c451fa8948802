"""Serving scheduler on the CPU with a simulated executor: memory budget never
exceeded, FIFO admission, continuous batching (arrivals join while earlier rounds
are in flight), over-budget requests rejected, every admitted request completes."""
import random

from paper_2402_09481_amd.serve import Request, Server, SimExecutor, summarize


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


def make(n, rate, seed=0, big=None):
    g = random.Random(seed)
    t, out = 0.0, []
    for k in range(n):
        t += g.expovariate(rate)
        size = g.choice([1, 2, 4, 8]) if big is None or k != big else 10_000
        out.append(Request(k, t, "toeplitz", size * 1000, size * 400))
    return out


def run(reqs, budget, slots, per_item=2e-4, max_batch=256):
    clk = FakeClock()
    ex = SimExecutor(slots, footprint=lambda r: r.n, latency=lambda rs: 1e-3 + per_item * len(rs), clock=clk)
    srv = Server(ex, budget, max_batch=max_batch)
    # track the budget at every submission
    seen = []
    orig = ex.submit

    def submit(rs):
        seen.append(srv.in_use + sum(r.footprint for r in rs))
        return orig(rs)
    ex.submit = submit
    out = srv.run(reqs, clock=clk, idle=clk.sleep)
    return srv, ex, out, seen


def test_budget_never_exceeded_and_all_complete():
    reqs = make(500, rate=5000.0, seed=1)
    srv, ex, out, seen = run(reqs, budget=20_000, slots=3)
    assert max(seen) <= 20_000
    assert srv.peak_in_use <= 20_000
    assert all(r.t_done is not None and r.t_done >= r.t_admit >= r.t_arrival for r in out)


def test_fifo_admission():
    reqs = make(300, rate=20000.0, seed=2)
    srv, ex, out, _ = run(reqs, budget=16_000, slots=2)
    admits = [r.t_admit for r in sorted(out, key=lambda r: r.rid)]
    assert admits == sorted(admits)


def test_continuous_batching_overlaps_rounds():
    # arrivals keep coming while rounds run: later rounds start before earlier ones end
    reqs = make(400, rate=10000.0, seed=3)
    srv, ex, out, _ = run(reqs, budget=10**9, slots=4, per_item=1e-3)
    overlaps = sum(1 for a, b in zip(ex.log, ex.log[1:]) if b[0] < a[1])
    assert overlaps > 0 and srv.rounds > 1
    s = summarize(out, srv)
    assert s["completed"] == 400 and s["p99_ms"] >= s["p50_ms"] > 0


def test_over_budget_request_rejected_not_blocking():
    reqs = make(50, rate=1000.0, seed=4, big=10)
    srv, ex, out, _ = run(reqs, budget=50_000, slots=2)
    assert out[10].rejected and out[10].t_done is None
    assert all(r.t_done is not None for r in out if r.rid != 10)


def test_one_slot_serialises_rounds():
    reqs = make(100, rate=20000.0, seed=5)
    srv, ex, out, _ = run(reqs, budget=10**9, slots=1)
    for a, b in zip(ex.log, ex.log[1:]):
        assert b[0] >= a[1]
