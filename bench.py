#!/usr/bin/env python3
"""Benchmark of the convolution-extractor hot path on one MI355X.

Headline: output Mbit/s of one Toeplitz extraction with n = 2^30 input bits
(x ~ Bernoulli(0.4)), m = 2^29 output bits and an n+m-1 bit seed ~ Bernoulli(0.5)
— a cyclic convolution of length 2^31 over the prime 2^64 - 2^32 + 1 — with
inputs resident in HBM. A step is one full extraction (all passes, from packed
input bits to packed output bits).

Printed as one JSON line (rank 0). Besides the headline it reports:
  roofline      the dominant kernel's algorithmic bytes / its average duration
                (HIP events around every launch, on the launch stream, during
                the timed steps) against the 8 TB/s HBM peak, with measured
                traffic, its VALU view and the binding one of the two;
  path          the whole step's algorithmic bytes (the two-pass lower bound of
                10 L w + packed I/O) / step time;
  cpu_baseline  the oracle (plain schoolbook GF(2) rows, one thread) timed on a
                bounded sample of the same workload, scaled to Mbit/s;
  cpu_ntt       a single-threaded CPU NTT convolution, scaled to the headline;
  small_configs the small Toeplitz workload's call latency (p50/p99) and the
                Dodis workload's time per call (skip with --no-small);
  oracle_check  the timed extraction's first output bits against the oracle
                rows of the CPU leg (the run exits with status 3 on a mismatch);
  batched       the 4096-block batched workload: extract_batch vs one call
                sequence per block on the same GPU, outputs compared, and the
                oracle's rows on sampled blocks (skip with --no-batched);
  serving       open-loop Poisson serving at two offered rates, p50/p99 latency
                and output Mbit/s (--serving: the full sweep; --no-serving).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CHECK_WORDS = 64  # leading output words kept for the check against the oracle rows
METRIC = "output Mbit/s at Toeplitz n=2^30; batched-vs-per-block speedup; p99 latency"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_bytes(label: str, L: int, w: int, n: int, N: int, m: int) -> int:
    """Algorithmic HBM bytes of one launch of a pass kernel (label from the library's tracer).
    strided mode 0 (embed bits): writes L words, reads the packed input (n or N bits);
    strided mode 1/2 and contiguous mode 0: read + write L words; contiguous mode 1
    (fused seed transform, product, inverse): reads 2L, writes L; two-piece schedule:
    contiguous mode 3 (second piece's seed level times its input spectrum) reads 2L, writes
    L, contiguous mode 2 (first piece's fused pass plus that product) reads 3L, writes L;
    strided mode 3
    (last inverse pass): reads L words, writes m parity bits; pack: m bits in, m bits out;
    embed: both packed inputs in, both L-bit coefficient strings out; ptrans(_pack): the
    parity bits of the m output coefficients in, packed out. Forward strided levels
    run both operands in one launch (arr=2): twice the bytes."""
    if label.startswith("pack"):
        return 2 * (m // 8)
    if label.startswith("embed"):  # both packed inputs in, two L-bit coefficient strings out
        return (n + N) // 8 + 2 * (L // 8)
    if label.startswith("ptrans"):  # the parity bits of the m output coefficients in, z out
        return 2 * (m // 8)
    kind = label.split("[")[0]
    fields = dict(kv.split("=") for kv in label.split("[")[1].rstrip("]").split(",")[1:])
    mode, arr = int(fields["mode"]), int(fields.get("arr", 0))
    Lw = L * w
    if kind == "strided":
        # arr=2: both operands in one launch (the forward levels)
        if mode == 0:
            return {0: Lw + n // 8, 1: Lw + N // 8, 2: 2 * Lw + (n + N) // 8}[arr]
        if mode == 3:
            return Lw + m // 8
        return 2 * Lw * (2 if arr == 2 else 1)
    if kind == "contig":  # mode 2: the two-piece fused pass (3 arrays in, 1 out)
        return 4 * Lw if mode == 2 else 3 * Lw if mode in (1, 3) else 2 * Lw
    return 0


PROFILE_BYTES = os.path.join(ROOT, "profiles", "toeplitz_n2p30_hbm_bytes.md")
KERNEL_SOURCES = ["paper_2402_09481_amd/csrc/ntt.hip", "paper_2402_09481_amd/csrc/field.h",
                  "paper_2402_09481_amd/csrc/kernels.h"]
PROFILE_VN = os.path.join(ROOT, "profiles", "von_neumann_kernel_trace_and_bytes.md")
PROFILE_VALU = os.path.join(ROOT, "profiles", "toeplitz_n2p30_valu_lds.md")
VALU_PEAK_T = 256 * 64 * 2.4e9 / 1e12  # lane operations per second, 32-bit VALU, 10^12
VN_SOURCES = ["paper_2402_09481_amd/csrc/vonneumann.hip", "paper_2402_09481_amd/csrc/kernels.h"]


def _profile_blob(path: str, sources):
    """The machine-readable block of a committed rocprofv3 summary, or None if the
    summary does not exist or was taken on kernel sources other than these."""
    import hashlib
    try:
        text = open(path).read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    h = hashlib.sha256()
    for fn in sources:
        h.update(open(os.path.join(ROOT, fn), "rb").read())
    return blob if h.hexdigest() == blob.get("kernel_sources_sha256") else None


def _kernel_name(label: str) -> str:
    kind = label.split("[")[0]
    f = dict(kv.split("=") for kv in label.split("[")[1].rstrip("]").split(",")[1:])
    field = "FGL" if "[u64" in label else "FP0" if "[p0" in label else "FLZ" if "[lz" in label else "FBB"
    return "k_%s<%s, %s, %s>" % (kind, field, f["lgr"], f["mode"])


def profiled_traffic(label: str):
    """HBM bytes (read + write, calibrated) of one launch of the kernel behind a trace
    label, from the committed rocprofv3 summary — None if that summary does not exist or
    was taken on different kernel sources."""
    blob = _profile_blob(PROFILE_BYTES, KERNEL_SOURCES)
    e = None if blob is None else blob.get("per_launch", {}).get(_kernel_name(label))
    return None if e is None else e["read_bytes"] + e["write_bytes"]


def valu_view(label: str, avg_ms: float):
    """The ALU view of one launch: the wave instructions rocprofv3 counted for that
    kernel (SQ_INSTS_VALU, committed summary of the same kernel sources) as lane
    operations, over the launch's measured duration, against 256 CUs x 64 lanes x
    2.4 GHz. None without a matching summary."""
    blob = _profile_blob(PROFILE_VALU, KERNEL_SOURCES)
    e = None if blob is None else blob.get("per_launch", {}).get(_kernel_name(label))
    if e is None:
        return None
    lane_ops = e["valu_insts"] * 64
    achieved = lane_ops / (avg_ms * 1e-3) / 1e12
    out = {"lane_ops_per_launch": int(lane_ops), "achieved": round(achieved, 2), "peak": round(VALU_PEAK_T, 2),
           "unit": "T lane-op/s", "frac": round(achieved / VALU_PEAK_T, 4),
           "note": "peak = one wave64 instruction per 4 cycles per SIMD at 2.4 GHz (32-bit multiplies, carries, "
                   "64-bit adds); plain 32-bit adds, logic and moves issue faster, so frac can pass 1"}
    if e.get("gpu_cycles"):
        # the profile's own cycle count (GRBM_GUI_ACTIVE / 8 XCDs): the clock the kernel ran at
        # and its VALU issue rate against one wave64 instruction per 4 cycles per SIMD
        out["profiled_clock_ghz"] = round(e["gpu_cycles"] / (e["duration_ms"] * 1e-3) / 1e9, 3)
        out["profiled_issue_rate"] = round(e["valu_insts"] * 4 / (1024 * e["gpu_cycles"]), 3)
    return out


def profiled_vn_traffic(n: int):
    """Calibrated HBM bytes (read + write) of one Von Neumann main-kernel launch at
    input length n, from the committed summary; None if absent or taken on other
    kernel sources."""
    import hashlib
    try:
        text = open(PROFILE_VN).read()
        blob = json.loads(text.rsplit("```json", 1)[1].split("```", 1)[0])  # the last block
    except (OSError, IndexError, ValueError):
        return None
    h = hashlib.sha256()
    for fn in VN_SOURCES:
        h.update(open(os.path.join(ROOT, fn), "rb").read())
    if h.hexdigest() != blob.get("kernel_sources_sha256"):
        return None
    e = blob.get("per_launch", {}).get(str(n))
    return None if e is None else e["read_bytes"] + e["write_bytes"]


def cpu_ntt_baseline(lg: int = 22, batch_sample: int = 48):
    """The single-threaded CPU NTT (`baseline/`, the 64-bit prime of the headline
    configuration) timed on: a Toeplitz extraction whose transform is 2^lg
    (n = 2^(lg-1), m = 2^(lg-2)), scaled to the headline's 2^31 transform by
    L log L; the small Toeplitz workload (n = 4096) and the Dodis workload's shape
    (n = 1,048,589, m = 2^19, run as the Toeplitz extraction of the same lengths:
    the same transform and work) in full; and a seeded sample of the batched
    workload's blocks, scaled to all 4096 blocks by their sum of L log L."""
    import math

    import baseline
    import workloads as W
    n, m = 1 << (lg - 1), 1 << (lg - 2)
    g = W.rng(W.BASE_SEED + 12)
    x, y = W.bernoulli_bits(g, n, 0.4), W.bernoulli_bits(g, n + m - 1, 0.5)
    baseline.toeplitz(x[:1], y[:1], 1, 1)  # build and load outside the timing

    def timed(xx, yy, nn, mm, order="paper"):
        t0 = time.perf_counter()
        baseline.toeplitz(xx, yy, nn, mm, order)
        return time.perf_counter() - t0

    dt = timed(x, y, n, m)
    L, LH = 1 << lg, 1 << 31
    t_head = dt * (LH * 31) / (L * lg)
    out = {"value": round(m / dt / 1e6, 3), "unit": "Mbit/s", "cores": 1, "kind": "cpu_ntt",
           "sample": "Toeplitz n=2^%d, m=2^%d, transform 2^%d over 2^64-2^32+1, %.2f s" % (lg - 1, lg - 2, lg, dt),
           "headline_extrapolated": {"value": round((1 << 29) / t_head / 1e6, 3), "unit": "Mbit/s",
                                     "seconds": round(t_head, 1), "scaling": "L log2 L to L = 2^31"}}
    sm = W.toeplitz_small()
    t = min(timed(sm.x, sm.y, sm.n, sm.m, "linear") for _ in range(20))
    out["toeplitz_4096"] = {"us_per_call": round(t * 1e6, 1), "output_Mbit_s": round(sm.m / t / 1e6, 2)}
    d = W.dodis_2p20()
    t = timed(d.x, d.y, d.n, d.m)
    out["dodis_1048589_shape"] = {"ms_per_call": round(t * 1e3, 2), "output_Mbit_s": round(d.m / t / 1e6, 3)}
    params = W.batch_params(4096, next_na=lambda v: v)  # lengths only (no primality needed for timing)
    lgs = [max(6, math.ceil(math.log2(n_ + m_ - 1))) for (_, n_, m_, _, _) in params]
    cost = lambda k: (1 << k) * k  # noqa: E731
    pick = sorted(int(i) for i in W.rng(W.BASE_SEED + 13).choice(len(params), size=batch_sample, replace=False))
    t_s, m_s = 0.0, 0
    for i in pick:
        _, n_, m_, px, sub = params[i]
        j = W.make_job("toeplitz", n_, m_, px, sub)
        t_s += timed(j.x, j.y, n_, m_)
        m_s += m_
    scale = sum(cost(k) for k in lgs) / sum(cost(lgs[i]) for i in pick)
    t_all = t_s * scale
    sum_m = sum(p_[2] for p_ in params)
    out["batched_4096_extrapolated"] = {"value": round(sum_m / t_all / 1e6, 3), "unit": "Mbit/s",
                                        "seconds": round(t_all, 1),
                                        "sample": "%d seeded blocks in %.1f s, scaled by sum of L log2 L"
                                                  % (len(pick), t_s)}
    return out


def cpu_baseline(job, seconds: float):
    """Oracle rows of the same workload for about `seconds` of one core."""
    import oracle
    # the row routine pays a setup (seed reversal) per call: fit setup + rows * per_row
    t0 = time.perf_counter()
    oracle.toeplitz_rows(job.x, job.y, job.n, job.m, 0, 2, job.seed_order)
    t1 = time.perf_counter()
    oracle.toeplitz_rows(job.x, job.y, job.n, job.m, 0, 34, job.seed_order)
    t2 = time.perf_counter()
    per_row = max(((t2 - t1) - (t1 - t0)) / 32, 1e-4)
    setup = max((t1 - t0) - 2 * per_row, 0.0)
    rows = int(max(8, min(64 * CHECK_WORDS, (seconds - setup) / per_row)))
    t0 = time.perf_counter()
    got = oracle.toeplitz_rows(job.x, job.y, job.n, job.m, 0, rows, job.seed_order)
    dt = time.perf_counter() - t0
    return {"value": rows / dt / 1e6, "unit": "Mbit/s", "cores": 1, "kind": "oracle",
            "sample": "output bits z_0..z_%d of the n=2^30, m=2^29 Toeplitz extraction computed row by row by the "
                      "schoolbook GF(2) oracle in %.1f s (one call, setup included); rate scaled to Mbit/s"
                      % (rows - 1, dt)}, rows, got


def check_rows(z_head, rows: int, want) -> dict:
    """The GPU's first `rows` output bits of the timed extraction against the oracle
    rows the CPU leg computed (bit for bit)."""
    import numpy as np
    nw = (rows + 63) // 64
    got = np.array(z_head[:nw], dtype=np.uint64)
    if rows % 64:
        got[-1] &= np.uint64((1 << (rows % 64)) - 1)
    same = bool(np.array_equal(got, np.asarray(want, dtype=np.uint64)[:nw]))
    return {"rows": rows, "bits_equal": same}


def run_headline(args):
    import numpy as np
    import torch

    import paper_2402_09481_amd as P
    import workloads as W

    log("generating inputs (n=2^30, seed 1.5*2^30 bits)")
    job = W.toeplitz_large()
    x = torch.from_numpy(job.x.view(np.int64)).cuda()
    y = torch.from_numpy(job.y.view(np.int64)).cuda()
    z = torch.empty(P.words(job.m), dtype=torch.int64, device="cuda")
    ctx = P.Context(0)
    stream = torch.cuda.current_stream()
    log("warmup x%d" % args.warmup)
    # the configuration's transform: one of length 2^31 over the 64-bit prime
    for _ in range(args.warmup):
        ctx.extract("toeplitz", x, y, job.n, job.m, z=z, stream=stream, single_transform=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    log("timed x%d (tracing off)" % args.steps)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.extract("toeplitz", x, y, job.n, job.m, z=z, stream=stream, single_transform=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # per-kernel durations: the same steps again with every launch bracketed by HIP
    # events on the launch stream (a separate run, so that the events do not sit in
    # the timed steps)
    log("traced x%d (per-kernel durations)" % args.steps)
    ctx.profile(True)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(args.steps):
        ctx.extract("toeplitz", x, y, job.n, job.m, z=z, stream=stream, single_transform=True)
    t1.record(stream)
    torch.cuda.synchronize()
    ctx.profile(False)
    traced_ms = t0.elapsed_time(t1) / args.steps
    marks = ctx.profile_read()
    # the first output words, for the check against the oracle rows of the CPU leg
    z_head = z[:CHECK_WORDS].cpu().numpy().view(np.uint64).copy()

    L = 1 << 31
    w = 8
    N = job.n + job.m - 1
    agg = {}
    for label, t in marks:
        a = agg.setdefault(label, [0.0, 0])
        a[0] += t
        a[1] += 1
    kernels = []
    for label, (tot, cnt) in agg.items():
        b = kernel_bytes(label, L, w, job.n, N, job.m)
        avg = tot / cnt
        kernels.append({"kernel": label, "launches": cnt, "avg_ms": round(avg, 4),
                        "algo_bytes": b, "achieved_GBs": round(b / (avg * 1e-3) / 1e9, 1)})
    kernels.sort(key=lambda k: -k["avg_ms"] * k["launches"])
    dom = kernels[0]
    path_bytes = 10 * L * w + (job.n + N + job.m) // 8
    value = job.m / (ms * 1e-3) / 1e6
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded PCG64 Bernoulli bits)",
        "config": {"workload": "Toeplitz n=2^30 (x~B(0.4)), m=2^29, seed n+m-1 bits ~B(0.5); cyclic convolution of "
                               "length 2^31 mod 2^64-2^32+1, 3-level multi-pass NTT",
                   "n": job.n, "m": job.m, "transform_length": L, "word_bytes": w},
        "roofline": {"bound": "hbm", "kernel": dom["kernel"], "achieved": dom["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(dom["achieved_GBs"] / HBM_PEAK_GBS, 4),
                     "traffic": profiled_traffic(dom["kernel"]), "algo_bytes_per_launch": dom["algo_bytes"],
                     "valu": valu_view(dom["kernel"], dom["avg_ms"])},
        "path": {"algo_bytes": path_bytes, "achieved_GBs": round(path_bytes / (ms * 1e-3) / 1e9, 1),
                 "frac_of_hbm_roofline": round(path_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "roofline_Mbit_s": round(job.m / (path_bytes / (HBM_PEAK_GBS * 1e9)) / 1e6, 1)},
        "kernels": kernels,
        "traced_ms_per_step": round(traced_ms, 3),
        "paper_context": "paper: ~1 Mbit/s below n=2^29 and 3-4x lower above (64-bit-class prime), Apple M2 Max CPU",
    }
    # both fractions, and the one that binds (the higher)
    rv = out["roofline"]["valu"]
    out["roofline"]["binding"] = "valu" if rv is not None and rv["frac"] > out["roofline"]["frac"] else "hbm"
    if args.warm:
        # NEXT row f1: the same extraction with the seed's transform cached (a hit
        # skips one of the three transforms; 7 L w algorithmic bytes)
        ctx.extract("toeplitz", x, y, job.n, job.m, z=z, stream=stream, cache_seed=True, single_transform=True)
        torch.cuda.synchronize()
        w0, w1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0.record(stream)
        for _ in range(args.steps):
            ctx.extract("toeplitz", x, y, job.n, job.m, z=z, stream=stream, cache_seed=True,
                        single_transform=True)
        w1.record(stream)
        torch.cuda.synchronize()
        wms = w0.elapsed_time(w1) / args.steps
        wbytes = 7 * L * w + (job.n + job.m) // 8
        out["warm_seed_cached"] = {"ms_per_step": round(wms, 3), "value": round(job.m / (wms * 1e-3) / 1e6, 2),
                                   "unit": "Mbit/s", "algo_bytes": wbytes,
                                   "achieved_GBs": round(wbytes / (wms * 1e-3) / 1e9, 1)}
        ctx.seed_cache_clear()
    if args.two_piece:
        out["two_piece"] = run_two_piece(ctx, job, x, y, z, stream, args, ms)
    ctx.close()
    del x, y, z
    torch.cuda.empty_cache()
    return out, job, z_head


def run_two_piece(ctx, job, x, y, z, stream, args, single_ms):
    """NEXT row f2: the same extraction with the library's default plan for this
    shape, the two-piece schedule (input halves of 2^29 bits, transforms of 2^30 over
    3*2^30+1 in 32-bit words, products added before one inverse). Same output bits
    (checked here against the single transform); a different arithmetic path, so it is
    reported beside the headline, not as it."""
    import torch
    z1 = z.clone()
    ctx.extract("toeplitz", x, y, job.n, job.m, z=z, stream=stream)
    torch.cuda.synchronize()
    same = bool(torch.equal(z, z1))
    ctx.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        ctx.extract("toeplitz", x, y, job.n, job.m, z=z, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ctx.profile(False)
    ms = e0.elapsed_time(e1) / args.steps
    L, w = 1 << 30, 4
    a = job.n // 2
    agg = {}
    for label, t in ctx.profile_read():
        e = agg.setdefault(label, [0.0, 0])
        e[0] += t
        e[1] += 1
    kernels, total_bytes = [], 0
    for label, (tot, cnt) in agg.items():
        b = kernel_bytes(label, L, w, a, a + job.m - 1, job.m)
        total_bytes += b * cnt // args.steps
        kernels.append({"kernel": label, "launches_per_step": cnt // args.steps, "avg_ms": round(tot / cnt, 4),
                        "algo_bytes": b, "achieved_GBs": round(b / (tot / cnt * 1e-3) / 1e9, 1)})
    kernels.sort(key=lambda k: -k["avg_ms"] * k["launches_per_step"])
    return {"ms_per_step": round(ms, 3), "value": round(job.m / (ms * 1e-3) / 1e6, 2), "unit": "Mbit/s",
            "speedup_vs_single_transform": round(single_ms / ms, 2), "same_bits_as_single_transform": same,
            "transform_length": L, "word_bytes": w, "algo_bytes_per_step": total_bytes,
            "achieved_GBs": round(total_bytes / (ms * 1e-3) / 1e9, 1), "kernels": kernels}


def run_batched(log, count=4096, reps=10, per_block=True):
    """The batched workload (4096 Toeplitz/Circulant blocks, n log-uniform in
    [2^10, 2^22], m = n/2): extract_batch (one persistent launch for the
    single-workgroup sizes plus grouped multi-pass launches, replayed from a HIP
    graph) against one extraction call sequence per block, same jobs, same GPU.
    Returns the summary, the jobs and the batched outputs (host copies)."""
    import numpy as np
    import torch

    import paper_2402_09481_amd as P
    import workloads as W

    log("batched: generating %d blocks" % count)
    jobs = W.batch_jobs(count, next_na=P.next_na_set)
    ctx = P.Context(0)
    dev = []
    for j in jobs:
        dev.append({"kind": j.kind, "n": j.n, "m": j.m,
                    "x": torch.from_numpy(j.x.view(np.int64)).cuda(), "y": torch.from_numpy(j.y.view(np.int64)).cuda(),
                    "z": torch.empty(P.words(j.m), dtype=torch.int64, device="cuda")})
    dev_u = [dict(d, z=torch.empty_like(d["z"])) for d in dev]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def timed(fn, n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(n):
            rc, errs = fn()
            assert rc == 0, rc
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    log("batched: warmup")
    for _ in range(2):
        ctx.batch(dev, sync=True, graph=True)
    if per_block:
        ctx.batch(dev_u, sync=True, unbatched=True)
    log("batched: timed x%d each" % reps)
    t_b = timed(lambda: ctx.batch(dev, stream=stream, graph=True), reps)
    t_u = timed(lambda: ctx.batch(dev_u, stream=stream, unbatched=True), reps) if per_block else float("nan")
    same = all(torch.equal(a["z"], b["z"]) for a, b in zip(dev, dev_u)) if per_block else None
    zs = [d["z"].cpu().numpy().view(np.uint64).copy() for d in dev]
    sum_m = sum(j.m for j in jobs)
    sum_n = sum(j.n for j in jobs)
    kinds = {k: sum(1 for j in jobs if j.kind == k) for k in ("toeplitz", "circulant")}
    ctx.close()
    del dev, dev_u
    torch.cuda.empty_cache()
    return {"blocks": count, "kinds": kinds, "sum_n_bits": sum_n, "sum_m_bits": sum_m,
            "batched_ms": round(t_b, 3), "per_block_ms": round(t_u, 3), "speedup": round(t_u / t_b, 2),
            "batched_Mbit_s": round(sum_m / (t_b * 1e-3) / 1e6, 1),
            "per_block_Mbit_s": round(sum_m / (t_u * 1e-3) / 1e6, 1),
            "outputs_identical": same}, jobs, zs


def cpu_baseline_batched(jobs, zs, blocks=128, seed=5):
    """The CPU leg for the batched workload: the oracle's schoolbook rows (one
    thread) on a seeded sample of blocks — the first and one random output word of
    each — timed (rate scaled to Mbit/s), and compared with the GPU's batched
    outputs of those words."""
    import numpy as np

    import oracle
    import workloads as W
    g = W.rng(seed)
    pick = sorted(int(i) for i in g.choice(len(jobs), size=min(blocks, len(jobs)), replace=False))
    rows = 0
    bad = []
    t0 = time.perf_counter()
    for i in pick:
        j, z = jobs[i], zs[i]
        nw = (j.m + 63) // 64
        for w in sorted({0, int(g.integers(0, nw))}):
            cnt = min(64, j.m - 64 * w)
            if j.kind == "toeplitz":
                want = oracle.toeplitz_rows(j.x, j.y, j.n, j.m, 64 * w, cnt, j.seed_order)
            else:
                want = oracle.circulant_rows(j.x, j.y, j.n, j.m, 64 * w, cnt)
            got = int(z[w]) & ((1 << cnt) - 1)
            rows += cnt
            if got != int(want[0]):
                bad.append((i, w))
    dt = time.perf_counter() - t0
    return {"value": round(rows / dt / 1e6, 4), "unit": "Mbit/s", "cores": 1, "kind": "oracle",
            "sample": "%d output bits (the first and one random word of %d seeded blocks of all sizes) by the "
                      "schoolbook rows in %.1f s" % (rows, len(pick), dt)}, \
        {"blocks": len(pick), "bits": rows, "bits_equal": not bad, "mismatches": bad[:8]}


def run_paper_shapes(log, reps=2):
    """The paper's QKD privacy-amplification shapes and QRNG randomness-extraction
    shapes (NEXT row f3): QKD as two pieces of 2^30 over 3*2^30+1, QRNG (n = 6.5e9)
    as the piece schedule over the 64-bit field with transforms of 2^31."""
    import ctypes

    import numpy as np
    import torch

    import paper_2402_09481_amd as P
    import workloads as W
    out = {}
    ctx = P.Context(0)

    def host_job(make):
        def f():
            job = make()
            return (job.kind, job.n, job.m, torch.from_numpy(job.x.view(np.int64)).cuda(),
                    torch.from_numpy(job.y.view(np.int64)).cuda())
        return f

    def qrng_t():
        n, m, x, y = W.qrng_toeplitz_device()
        return "toeplitz", n, m, x, y

    def qrng_c():
        n, m, x, y = W.qrng_circulant_device(P.closest_na_set)
        return "circulant", n, m, x, y

    shapes = (("qkd_toeplitz", host_job(W.qkd_toeplitz)),
              ("qkd_circulant", host_job(lambda: W.qkd_circulant(P.next_na_set))),
              ("qrng_toeplitz", qrng_t), ("qrng_circulant", qrng_c))
    for name, make in shapes:
        log("paper shapes: %s" % name)
        kind, n, m, x, y = make()
        z = torch.empty(P.words(m), dtype=torch.int64, device="cuda")
        ctx.extract(kind, x, y, n, m, z=z, sync=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ctx.extract(kind, x, y, n, m, z=z)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        wb = ctypes.c_int32()
        L = int(ctx._lib.ext_plan_length(P.KINDS[kind], n, m, ctypes.byref(wb)))
        out[name] = {"kind": kind, "n": n, "m": m, "ms": round(ms, 3),
                     "output_Mbit_s": round(m / (ms * 1e-3) / 1e6, 2),
                     "input_Mbit_s": round(n / (ms * 1e-3) / 1e6, 2),
                     "transform_length": L, "word_bits": wb.value}
        del x, y, z
        ctx.trim()
        torch.cuda.empty_cache()
    ctx.close()
    torch.cuda.empty_cache()
    return out


def run_von_neumann(log, reps=10, oracle_bits=1 << 27):
    """The Von Neumann extractor (NEXT row f4(b)): i.i.d. input with min-entropy half
    its length (the paper's throughput-figure setting), at the figure's largest input
    length and at 2^33 bits. Input and output bytes against the HBM roofline; the
    oracle timed on a sample for context."""
    import time

    import numpy as np
    import torch

    import paper_2402_09481_amd as P
    import workloads as W
    ctx = P.Context(0)
    out = {"p_one": round(W.VN_P, 6), "shapes": []}
    for n in (W.VN_PAPER_N, W.VN_LARGE_N):
        log("von neumann: n=%d" % n)
        x = W.bernoulli_bits_device(n, W.VN_P, W.BASE_SEED + 10)
        z = torch.empty(P.words(n // 2), dtype=torch.int64, device="cuda")
        mo = torch.zeros(1, dtype=torch.int64, device="cuda")
        for _ in range(3):
            ctx.von_neumann(x, n, z=z, m_out=mo)
        torch.cuda.synchronize()
        ctx.profile(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ctx.von_neumann(x, n, z=z, m_out=mo)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        per = {}
        for name, t in ctx.profile_read():
            per.setdefault(name, []).append(t)
        ctx.profile(False)
        m = int(mo.item())
        main_ms = sum(per["vn_main"]) / len(per["vn_main"])
        algo = n // 8 + m // 8  # input read once, output written once
        out["shapes"].append({
            "n": n, "m": m, "ms_per_call": round(ms, 4),
            "input_Gbit_s": round(n / (ms * 1e-3) / 1e9, 2),
            "output_Mbit_s": round(m / (ms * 1e-3) / 1e6, 1),
            "kernels_ms": {k: round(sum(v) / len(v), 4) for k, v in per.items()},
            "roofline": {"bound": "hbm", "kernel": "vn_main", "achieved": round(algo / (main_ms * 1e-3) / 1e9, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(algo / (main_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "algo_bytes": algo,
                         "traffic": profiled_vn_traffic(n)},
        })
        del x, z
    ctx.close()
    torch.cuda.empty_cache()
    import oracle
    xs = W.von_neumann_input(oracle_bits, seed=W.BASE_SEED + 11)
    t0 = time.perf_counter()
    code, oz, om = oracle.von_neumann(xs, oracle_bits)
    dt = time.perf_counter() - t0
    out["cpu_baseline"] = {"value": round(om / dt / 1e6, 2), "unit": "Mbit/s (output)", "cores": 1, "kind": "oracle",
                           "sample": "%d i.i.d. input bits, p = %.4f" % (oracle_bits, W.VN_P)}
    return out


def run_small_configs(log, calls=10000):
    """The two small workloads: Toeplitz n = 4096, m = 2048 (linear seed order; one
    workgroup, latency-bound) as the host-measured latency of one synchronous call,
    p50/p99 over `calls` calls, plus the device time per call back to back; and the
    Dodis workload (n = 1,048,589, m = 2^19) as milliseconds per call from HIP
    events over 20 calls."""
    import numpy as np
    import torch

    import paper_2402_09481_amd as P
    import workloads as W

    ctx = P.Context(0)
    stream = torch.cuda.current_stream()
    out = {}
    j = W.toeplitz_small()
    x = torch.from_numpy(j.x.view(np.int64)).cuda()
    y = torch.from_numpy(j.y.view(np.int64)).cuda()
    z = torch.empty(P.words(j.m), dtype=torch.int64, device="cuda")
    for _ in range(200):
        ctx.extract("toeplitz", x, y, j.n, j.m, z=z, seed_order="linear", sync=True)
    log("small configs: %d synchronous calls" % calls)
    lat = np.empty(calls)
    for i in range(calls):
        t0 = time.perf_counter()
        ctx.extract("toeplitz", x, y, j.n, j.m, z=z, seed_order="linear", sync=True)
        lat[i] = time.perf_counter() - t0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(1000):
        ctx.extract("toeplitz", x, y, j.n, j.m, z=z, seed_order="linear", stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    dev_us = e0.elapsed_time(e1) * 1e3 / 1000
    out["toeplitz_4096"] = {"n": j.n, "m": j.m, "calls": calls,
                            "sync_call_us": {"p50": round(float(np.percentile(lat, 50)) * 1e6, 2),
                                             "p99": round(float(np.percentile(lat, 99)) * 1e6, 2),
                                             "mean": round(float(lat.mean()) * 1e6, 2)},
                            "back_to_back_us_per_call": round(dev_us, 2),
                            "output_Mbit_s_back_to_back": round(j.m / (dev_us * 1e-6) / 1e6, 1)}
    d = W.dodis_2p20()
    x = torch.from_numpy(d.x.view(np.int64)).cuda()
    y = torch.from_numpy(d.y.view(np.int64)).cuda()
    z = torch.empty(P.words(d.m), dtype=torch.int64, device="cuda")
    for _ in range(3):
        ctx.extract("dodis", x, y, d.n, d.m, z=z, sync=True)
    e0.record(stream)
    for _ in range(20):
        ctx.extract("dodis", x, y, d.n, d.m, z=z, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 20
    out["dodis_1048589"] = {"n": d.n, "m": d.m, "ms_per_call": round(ms, 4),
                            "output_Mbit_s": round(d.m / (ms * 1e-3) / 1e6, 1),
                            "transform_length": int(ctx._lib.ext_plan_length(P.EXT_KIND_DODIS, d.n, d.m, None))}
    ctx.close()
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample budget (0 = skip)")
    ap.add_argument("--batched", action="store_true", help="(default) the 4096-block batched comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched comparison")
    ap.add_argument("--batched-reps", type=int, default=10,
                    help="timed back-to-back repetitions of each batched form (the host marshalling of the\n"
                         "first call is not overlapped with GPU work, so few repetitions overstate the time)")
    ap.add_argument("--no-per-block", action="store_true",
                    help="batched: skip the one-call-per-block comparison (for profiling the batched launches)")
    ap.add_argument("--no-headline", action="store_true",
                    help="skip the headline and its CPU legs (for profiling the other legs alone)")
    ap.add_argument("--serving", action="store_true",
                    help="the full serving sweep (1k-50k req/s) instead of the default two offered rates")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--warm", action="store_true", help="also time the headline with the seed transform cached")
    ap.add_argument("--paper-shapes", action="store_true", help="also time the paper's QKD extraction shapes")
    ap.add_argument("--von-neumann", action="store_true", help="also time the Von Neumann extractor")
    ap.add_argument("--two-piece", action="store_true",
                    help="also time the headline shape with the default two-piece plan")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the small Toeplitz latency and Dodis timing (run by default, about a second)")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="run a plain device copy of this many GiB first (reference for byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported (use --gpus 1)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.copy_calibration_gib > 0:
        import torch
        nb = int(args.copy_calibration_gib * (1 << 30))
        src = torch.ones(nb // 8, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read + %d bytes written per copy kernel" % (nb, nb))
        del src, dst
        torch.cuda.empty_cache()
    if args.no_headline:
        out = {"metric": METRIC, "note": "headline skipped (--no-headline)"}
    else:
        out, job, z_head = run_headline(args)
        # the CPU leg: the oracle on a bounded sample of the same workload; its rows
        # also check the timed extraction's first output bits
        log("cpu baseline (oracle, %.0f s budget)" % max(args.cpu_seconds, 1.0))
        cb, rows, want = cpu_baseline(job, max(args.cpu_seconds, 1.0))
        if args.cpu_seconds > 0:
            out["cpu_baseline"] = cb
            log("cpu NTT baseline (one thread)")
            out["cpu_ntt"] = cpu_ntt_baseline()
        out["oracle_check"] = check_rows(z_head, rows, want)
        if not out["oracle_check"]["bits_equal"]:
            print(json.dumps(out), flush=True)
            log("MISMATCH: the timed extraction's first %d output bits differ from the oracle's rows" % rows)
            sys.exit(3)
    if not args.no_small:
        out["small_configs"] = run_small_configs(log)
    if not args.no_batched:
        b, bjobs, bzs = run_batched(log, reps=args.batched_reps, per_block=not args.no_per_block)
        log("batched: cpu leg (oracle rows on sampled blocks)")
        b["cpu_baseline"], b["oracle_check"] = cpu_baseline_batched(bjobs, bzs)
        out["batched"] = b
        del bjobs, bzs
        if not b["oracle_check"]["bits_equal"] or b["outputs_identical"] is False:
            print(json.dumps(out), flush=True)
            log("MISMATCH in the batched workload")
            sys.exit(3)
    if args.paper_shapes:
        out["paper_shapes"] = run_paper_shapes(log)
    if args.von_neumann:
        out["von_neumann"] = run_von_neumann(log)
    if not args.no_serving:
        from paper_2402_09481_amd import serve
        if args.serving:  # the full sweep
            out["serving"] = serve.bench(log=log)
        else:
            out["serving"] = serve.bench(log=log, rates=(2000, 20000), count=400)
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
