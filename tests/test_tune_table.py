"""The packaged plan table (tune_gfx950.txt) on the CPU: every line parses, every
plan is one the tuner may pick for its size class (the library would reject the
others), batch plans cover each size class at most once, and single-call plans
only name classes whose plan they change."""
import os

import paper_2402_09481_amd as P
from paper_2402_09481_amd.tune import candidates

TABLE = os.path.join(os.path.dirname(P.__file__), "tune_gfx950.txt")


def _lines():
    for ln in open(TABLE):
        ln = ln.split("#", 1)[0].strip()
        if ln:
            yield ln.split()


def test_every_plan_is_a_candidate():
    batch, single = {}, {}
    for f in _lines():
        scope = single if f[0] == "single" else batch
        if f[0] == "single":
            f = f[1:]
        wb, lg, nlev = int(f[0]), int(f[1]), int(f[2])
        levels = [int(v) for v in f[3:]]
        assert len(levels) == nlev, f
        assert levels in candidates(wb, lg), (wb, lg, levels)
        assert (wb, lg) not in scope, ("twice", wb, lg)
        scope[(wb, lg)] = levels
    assert (64, 31) in batch  # the headline's plan
    for key, levels in single.items():
        assert key in batch and batch[key] != levels, key
