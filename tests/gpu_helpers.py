"""Shared helpers for the GPU tests: move packed words to the device, run one
extraction through the C-ABI, compare with the oracle."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def to_dev(words: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(words).view(np.int64)).to("cuda")


def to_host(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def gpu_extract(ctx, kind, x, y, n, m, seed_order="paper"):
    """Returns (code, z as numpy uint64 words or None)."""
    import torch
    xd, yd = to_dev(x), to_dev(y)
    z = torch.full(((m + 63) >> 6,), -1, dtype=torch.int64, device="cuda")  # garbage-filled: tail must be cleared
    st = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    rc, z = ctx.extract(kind, xd, yd, n, m, z=z, seed_order=seed_order, sync=False, status=st, check=False)
    if rc != 0:
        return rc, None
    torch.cuda.synchronize()
    code = int(st.item())
    return code, to_host(z)


def show_case(*a):
    print("CASE", *a, flush=True)
