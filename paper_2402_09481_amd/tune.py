"""Autotuner for the per-size launch plans.

For every transform size class 2^lg it times each plan the library supports
(one workgroup per job where possible, and every split of the transform into
passes whose tile sizes are compiled in) on this GPU, keeps the fastest, and
writes the table that Context() loads by default (tune_gfx950.txt next to this
file). Timing uses batches of Toeplitz jobs of that class holding at least 2^26
coefficients, through extract_batch with graph replay, median of a few runs.
Any plan gives the same bits; only the speed differs.

With --single it also times one job per call (back-to-back single extraction
calls of the class) for every plan, and keeps a single-call plan where one is
faster than the batch plan by more than SINGLE_MARGIN: one job leaves most of
the GPU idle, and fewer, larger workgroups can finish it sooner.

    python -m paper_2402_09481_amd.tune [--lg 11-27] [--gl] [--single] [--out PATH]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tune_gfx950.txt")

CAPS = {32: {"strided": (7, 10), "contig": (7, 14), "small": 14}, 64: {"strided": (7, 10), "contig": (7, 13)}}


def candidates(word_bits: int, lg: int):
    caps = CAPS[word_bits]
    out = []
    if word_bits == 32 and lg <= caps["small"]:
        out.append([])
    s_lo, s_hi = caps["strided"]
    c_lo, c_hi = caps["contig"]
    for s in range(s_lo, s_hi + 1):
        c = lg - s
        if c_lo <= c <= c_hi:
            out.append([s, c])
    if lg >= 21:
        for s0 in range(s_lo, s_hi + 1):
            for s1 in range(s_lo, s_hi + 1):
                c = lg - s0 - s1
                if c_lo <= c <= c_hi:
                    out.append([s0, s1, c])
    return out


def _jobs_for(lg: int, count: int):
    import torch
    n = 1 << (lg - 1)
    m = (1 << (lg - 2)) + 1  # n + m - 1 = 3 * 2^(lg-2): transform length 2^lg
    g = torch.Generator(device="cuda")
    g.manual_seed(lg)
    jobs = []
    for _ in range(count):
        x = torch.randint(-(1 << 62), 1 << 62, ((n + 63) >> 6,), dtype=torch.int64, device="cuda", generator=g)
        y = torch.randint(-(1 << 62), 1 << 62, ((n + m - 1 + 63) >> 6,), dtype=torch.int64, device="cuda",
                          generator=g)
        z = torch.empty((m + 63) >> 6, dtype=torch.int64, device="cuda")
        # one transform of the class being tuned (no piece schedule)
        jobs.append({"kind": "toeplitz", "n": n, "m": m, "x": x, "y": y, "z": z, "single_transform": True})
    return jobs


def time_plan(ctx, word_bits, lg, levels, jobs, reps=5):
    import torch
    ctx.tune_set(word_bits, lg, levels)
    ctx.batch(jobs, sync=True, graph=True)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rc, _ = ctx.batch(jobs, graph=True)
        e1.record()
        torch.cuda.synchronize()
        assert rc == 0
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


SINGLE_MARGIN = 0.03


def time_single(ctx, word_bits, lg, levels, reps=None):
    """Milliseconds per call of back-to-back single extractions of the class 2^lg
    (the shape of _jobs_for), best of three runs."""
    import torch
    n = 1 << (lg - 1)
    m = (1 << (lg - 2)) + 1
    g = torch.Generator(device="cuda")
    g.manual_seed(lg)
    x = torch.randint(-(1 << 62), 1 << 62, ((n + 63) >> 6,), dtype=torch.int64, device="cuda", generator=g)
    y = torch.randint(-(1 << 62), 1 << 62, ((n + m - 1 + 63) >> 6,), dtype=torch.int64, device="cuda", generator=g)
    z = torch.empty((m + 63) >> 6, dtype=torch.int64, device="cuda")
    ctx.tune_set(word_bits, lg, levels, single=True)
    reps = reps or max(10, min(200, (1 << 27) >> lg))
    for _ in range(3):
        ctx.extract("toeplitz", x, y, n, m, z=z, single_transform=True)
    s = torch.cuda.current_stream()
    best = None
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            ctx.extract("toeplitz", x, y, n, m, z=z, single_transform=True)
        e1.record(s)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / reps
        best = t if best is None else min(best, t)
    return best


def tune(lgs=range(11, 28), gl=False, out=DEFAULT_TABLE, log=print, single=False):
    import torch

    import paper_2402_09481_amd as P
    ctx = P.Context(0, tune=False)
    results = []
    plan_sets = [(32, lg) for lg in lgs] + ([(64, 31)] if gl else [])
    for wb, lg in plan_sets:
        cands = candidates(wb, lg)
        if len(cands) < 2 and wb == 32:
            ctx.tune_set(wb, lg, cands[0]) if cands else None
            continue
        count = max(1, min(512, (1 << 26) >> lg))
        jobs = _jobs_for(lg, count)
        best = None
        for lv in cands:
            t = time_plan(ctx, wb, lg, lv, jobs)
            log("u%d lg=%d plan=%s  %.3f ms (%d jobs)" % (wb, lg, lv or "one-workgroup", t, count))
            if best is None or t < best[0]:
                best = (t, lv)
        ctx.tune_set(wb, lg, best[1])
        results.append((wb, lg, best[1], best[0]))
        del jobs
        torch.cuda.empty_cache()
        if single:
            times = {}
            for lv in cands:
                times[tuple(lv)] = time_single(ctx, wb, lg, lv)
                log("u%d lg=%d plan=%s  %.1f us per single call" % (wb, lg, lv or "one-workgroup",
                                                                      times[tuple(lv)] * 1e3))
            fast = min(times, key=times.get)
            if list(fast) != best[1] and times[fast] < (1 - SINGLE_MARGIN) * times[tuple(best[1])]:
                ctx.tune_set(wb, lg, list(fast), single=True)
                log("single u%d lg=%d %s" % (wb, lg, list(fast)))
            else:
                ctx.tune_set(wb, lg, None, single=True)
            torch.cuda.empty_cache()
    ctx.tune_save(out)
    ctx.close()
    return results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--lg", default="11-27")
    ap.add_argument("--gl", action="store_true", help="also tune the 2^31 64-bit plan")
    ap.add_argument("--single", action="store_true", help="also tune the plans of single calls")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    a = ap.parse_args()
    lo, hi = (int(v) for v in a.lg.split("-"))
    t0 = time.time()
    for wb, lg, lv, t in tune(range(lo, hi + 1), a.gl, a.out, log=lambda *x: print(*x, flush=True),
                              single=a.single):
        print("best u%d lg=%d %s %.3f ms" % (wb, lg, lv, t), flush=True)
    print("wrote %s in %.1f s" % (a.out, time.time() - t0), file=sys.stderr)


if __name__ == "__main__":
    main()
