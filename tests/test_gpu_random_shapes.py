"""Seeded random shapes through every plan family, each whole output against the
oracle's GF(2)[t] product: kinds, seed orders, input and output lengths drawn
log-uniformly (m from 1 to its bound, ragged tails, biased inputs), run in the
default context (single workgroup, lazy field, the lazy two-piece schedule where
a shape reaches it) and in contexts that force the other fields and schedules
(15*2^27+1, 3*2^30+1, the 64-bit field, two pieces over 3*2^30+1, the 64-bit
piece schedule with small pieces, two pieces of half length from transforms of
2^15 up). One batch of all the shapes runs as well."""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import gpu_extract, show_case, to_dev, to_host

pytestmark = pytest.mark.gpu

CONTEXTS = [("default", None, None), ("bb", "bb", None), ("p0", "p0", None), ("gl", "gl", None),
            ("p0x2", "p0x2", None), ("pieces", None, 2048), ("halving", None, None)]
SEEDS = {name: 1000 + i for i, (name, _, _) in enumerate(CONTEXTS)}


def _ctx(field, piece_bits, halving=False):
    import paper_2402_09481_amd as P
    keys = ("EXT_FORCE_FIELD", "EXT_PIECE_BITS", "EXT_SPLIT_MIN_LG", "EXT_BATCH_SPLIT_MIN_LG")
    old = {k: os.environ.get(k) for k in keys}
    if field:
        os.environ["EXT_FORCE_FIELD"] = field
    if piece_bits:
        os.environ["EXT_PIECE_BITS"] = str(piece_bits)
    if halving:  # two pieces of half length wherever the halves fit (single calls and batches)
        os.environ["EXT_SPLIT_MIN_LG"] = "15"
        os.environ["EXT_BATCH_SPLIT_MIN_LG"] = "15"
    try:
        return P.Context(0)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _shapes(seed, count, lo, hi):
    g = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = ("toeplitz", "toeplitz", "circulant", "dodis")[int(g.integers(0, 4))]
        n = int(2 ** g.uniform(lo, hi))
        if kind == "circulant":
            n = oracle.next_na(n + 1) - 1      # input length: n + 1 prime with primitive root 2
        elif kind == "dodis":
            n = oracle.next_na(max(n, 3))
        bound = n if kind != "circulant" else n  # m <= n (Circulant: m <= n_in)
        r = g.uniform()
        m = 1 if r < 0.08 else bound if r < 0.16 else max(1, int(2 ** g.uniform(0, math.log2(bound))))
        order = "linear" if (kind == "toeplitz" and g.uniform() < 0.5) else "paper"
        px = float(g.uniform(0.05, 0.6))
        out.append((kind, n, m, order, px, int(g.integers(0, 1 << 30))))
    return out


def _inputs(kind, n, m, px, s):
    g = W.rng(s)
    x = W.bernoulli_bits(g, n, px)
    if kind == "dodis":
        x[0] = (int(x[0]) | 1) & ~2
    y = W.bernoulli_bits(g, {"toeplitz": n + m - 1, "circulant": n + 1, "dodis": n}[kind], 0.5)
    return x, y


@pytest.mark.parametrize("name,field,piece_bits", CONTEXTS)
def test_random_shapes(name, field, piece_bits):
    c = _ctx(field, piece_bits, halving=name == "halving")
    lo, hi = (6, 21) if name == "default" else (6, 17)
    count = 40 if name == "default" else 20
    for kind, n, m, order, px, s in _shapes(SEEDS[name], count, lo, hi):
        x, y = _inputs(kind, n, m, px, s)
        show_case("random", name, kind, n, m, order)
        code, z = gpu_extract(c, kind, x, y, n, m, order)
        assert code == 0, (name, kind, n, m, code)
        rc, want = oracle.extract_product(kind, x, y, n, m, order)
        assert rc == 0 and np.array_equal(z, want), (name, kind, n, m, order)
    c.close()


def test_random_shapes_as_one_batch():
    import torch

    import paper_2402_09481_amd as P
    c = P.Context(0)
    shapes = _shapes(77, 60, 6, 20)
    dev, want = [], []
    for kind, n, m, order, px, s in shapes:
        x, y = _inputs(kind, n, m, px, s)
        dev.append({"kind": kind, "n": n, "m": m, "x": to_dev(x), "y": to_dev(y), "seed_order": order,
                    "z": torch.full((W.nwords(m),), -1, dtype=torch.int64, device="cuda")})
        want.append(oracle.extract_product(kind, x, y, n, m, order)[1])
    for graph in (False, True):
        show_case("random batch", graph)
        rc, errs = c.batch(dev, sync=True, graph=graph)
        assert rc == 0 and not any(errs)
        for d, w in zip(dev, want):
            assert np.array_equal(to_host(d["z"]), w), (d["kind"], d["n"], d["m"])
            d["z"].fill_(-1)
    c.close()
