"""Every launch plan the tuner may pick gives the oracle's bits."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import gpu_extract, show_case

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lg", [14, 15, 18, 20, 22])
def test_all_u32_plans(lg):
    import paper_2402_09481_amd as P
    from paper_2402_09481_amd.tune import candidates
    ctx = P.Context(0, tune=False)
    n = (1 << (lg - 1)) - 37
    m = (1 << (lg - 2)) + 101  # n + m - 1 > 2^(lg-1): transform length 2^lg
    g = W.rng(lg)
    x, y = W.bernoulli_bits(g, n, 0.4), W.bernoulli_bits(g, n + m - 1, 0.5)
    want = oracle.extract("toeplitz", x, y, n, m)[1]
    for lv in candidates(32, lg):
        ctx.tune_set(32, lg, lv)
        assert ctx.tune_get(32, lg) == lv
        show_case("u32 plan", lg, lv)
        code, z = gpu_extract(ctx, "toeplitz", x, y, n, m)
        assert code == 0 and np.array_equal(z, want), lv
    ctx.close()


@pytest.mark.parametrize("lg", [16, 21, 22, 23, 24])
def test_all_u64_plans(lg):
    """Every 64-bit plan the tuner may pick (2 and 3 levels; at 2^24 the middle
    strided levels of 2^10 rows that the 2^31 plan uses), each against the whole
    output of the oracle, for two shapes: m = L/4 as in the large workload
    (the last inverse pass computes a quarter of its rows) and m just above L/4."""
    import paper_2402_09481_amd as P
    from paper_2402_09481_amd.tune import candidates
    os.environ["EXT_FORCE_FIELD"] = "gl"
    try:
        ctx = P.Context(0, tune=False)
    finally:
        del os.environ["EXT_FORCE_FIELD"]
    cands = candidates(64, lg)
    assert cands, lg
    g = W.rng(lg + 100)
    for n, m in ((1 << (lg - 1), 1 << (lg - 2)), ((1 << (lg - 1)) - 5, (1 << (lg - 2)) + 3)):
        x, y = W.bernoulli_bits(g, n, 0.4), W.bernoulli_bits(g, n + m - 1, 0.5)
        want = oracle.toeplitz_product(x, y, n, m, "paper")[1]
        if lg <= 16:
            assert np.array_equal(want, oracle.extract("toeplitz", x, y, n, m)[1])
        for lv in cands:
            ctx.tune_set(64, lg, lv)
            assert ctx.tune_get(64, lg) == lv
            show_case("u64 plan", lg, lv, n, m)
            code, z = gpu_extract(ctx, "toeplitz", x, y, n, m)
            assert code == 0 and np.array_equal(z, want), (lv, n, m)
    ctx.close()


def test_tune_set_rejects_unsupported():
    import paper_2402_09481_amd as P
    ctx = P.Context(0, tune=False)
    for wb, lg, lv in [(32, 20, [5, 15]), (32, 20, [10, 11]), (32, 15, []), (64, 20, []), (32, 22, [11, 11])]:
        with pytest.raises(P.ExtError):
            ctx.tune_set(wb, lg, lv)
    ctx.close()


def _labels(ctx, fn):
    ctx.profile(True)
    fn()
    import torch
    torch.cuda.synchronize()
    labels = [lab for lab, _ in ctx.profile_read()]
    ctx.profile(False)
    return labels


@pytest.mark.parametrize("lg,batch_plan,single_plan", [(17, [8, 9], [7, 10]), (21, [9, 12], [8, 13])])
def test_single_call_plans(lg, batch_plan, single_plan, tmp_path):
    """A single call takes its size class's single-call plan, a batch the batch plan
    (seen in the launched kernels' tile sizes), both give the oracle's bits, removing
    the single-call plan falls back to the batch one, and a saved table restores both."""
    import torch

    import paper_2402_09481_amd as P
    ctx = P.Context(0, tune=False)
    n = (1 << (lg - 1)) - 37
    m = (1 << (lg - 2)) + 101  # transform length 2^lg
    g = W.rng(lg + 7)
    x, y = W.bernoulli_bits(g, n, 0.4), W.bernoulli_bits(g, n + m - 1, 0.5)
    want = oracle.extract("toeplitz", x, y, n, m)[1]
    ctx.tune_set(32, lg, batch_plan)
    ctx.tune_set(32, lg, single_plan, single=True)
    assert ctx.tune_get(32, lg) == batch_plan and ctx.tune_get(32, lg, single=True) == single_plan
    contig = lambda labels: sorted({lab for lab in labels if lab.startswith("contig")})

    show_case("single-call plan", lg, single_plan)
    out = {}
    labels = _labels(ctx, lambda: out.setdefault("z", gpu_extract(ctx, "toeplitz", x, y, n, m)))
    code, z = out["z"]
    assert code == 0 and np.array_equal(z, want)
    assert contig(labels) and all(("lgr=%d," % single_plan[-1]) in lab for lab in contig(labels)), labels

    show_case("batch plan", lg, batch_plan)
    from gpu_helpers import to_dev, to_host
    jobs = [{"kind": "toeplitz", "n": n, "m": m, "x": to_dev(x), "y": to_dev(y), "single_transform": True,
             "z": torch.full((W.nwords(m),), -1, dtype=torch.int64, device="cuda")} for _ in range(2)]
    labels = _labels(ctx, lambda: ctx.batch(jobs, sync=True))
    assert contig(labels) and all(("lgr=%d," % batch_plan[-1]) in lab for lab in contig(labels)), labels
    for j in jobs:
        assert np.array_equal(to_host(j["z"]), want)

    path = str(tmp_path / "tune.txt")
    ctx.tune_save(path)
    assert any(line.startswith("single 32 %d " % lg) for line in open(path))
    ctx.tune_set(32, lg, None, single=True)
    assert ctx.tune_get(32, lg, single=True) == batch_plan
    ctx.close()
    ctx2 = P.Context(0, tune=path)
    assert ctx2.tune_get(32, lg) == batch_plan and ctx2.tune_get(32, lg, single=True) == single_plan
    ctx2.close()


def test_packaged_single_call_plans():
    """The packaged table's single-call plan for the Dodis workload's transform
    (2^21) differs from its batch plan."""
    import paper_2402_09481_amd as P
    ctx = P.Context(0)
    assert ctx.tune_get(32, 21) == [9, 12]
    assert ctx.tune_get(32, 21, single=True) == [8, 13]
    assert ctx.tune_get(32, 22, single=True) == ctx.tune_get(32, 22)  # no single-call plan of its own
    ctx.close()


def test_tuner_single_mode(tmp_path):
    """The tuner's --single mode on one size class: it writes the batch plan, and a
    single-call plan only if that plan is one of the candidates and differs from the
    batch plan; the written table loads into a context."""
    import paper_2402_09481_amd as P
    from paper_2402_09481_amd.tune import candidates, tune
    out = str(tmp_path / "t.txt")
    res = tune(range(17, 18), out=out, log=lambda *a: None, single=True)
    assert len(res) == 1 and res[0][:2] == (32, 17)
    lines = [ln.split() for ln in open(out) if not ln.startswith("#")]
    batch = [list(map(int, ln[3:])) for ln in lines if ln[0] == "32" and ln[1] == "17"]
    single = [list(map(int, ln[4:])) for ln in lines if ln[0] == "single" and ln[2] == "17"]
    assert batch == [res[0][2]]
    cands = candidates(32, 17)
    assert all(s in cands and s != batch[0] for s in single)
    ctx = P.Context(0, tune=out)
    assert ctx.tune_get(32, 17) == batch[0]
    assert ctx.tune_get(32, 17, single=True) == (single[0] if single else batch[0])
    ctx.close()
