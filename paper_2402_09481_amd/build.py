"""Build libextractor.so (gfx950) in-tree with hipcc.

The transform kernel file is compiled as several parts in parallel (one per
group of template instantiations), the Von Neumann kernels and the C-ABI as
one object each, then linked with the C-ABI into one shared
library next to this file. Always rebuilds when called."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libextractor.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("EXT_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are never wanted in this integer code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-value", "-Wno-unused-result",
]
NTT_PARTS = 10
# The Von Neumann kernel takes its next tile's ticket with one lane and reads it
# a whole tile later; LLVM's atomic optimizer would broadcast the result right
# away and so wait for the atomic's round trip on every tile.
VN_FLAGS = ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for part in range(NTT_PARTS):
        obj = os.path.join(BUILD, "ntt_part%d.o" % part)
        jobs.append(([HIPCC] + FLAGS + ["-DNTT_PART=%d" % part, "-c", os.path.join(CSRC, "ntt.hip"), "-o", obj], obj))
    for src, extra in (("vonneumann.hip", VN_FLAGS), ("abi.cpp", [])):
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        jobs.append(([HIPCC] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj], obj))
    workers = min(len(jobs), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(workers) as ex:
        for out in ex.map(lambda j: _run(j[0]), jobs):
            if verbose and out.strip():
                print(out)
    tmp = OUT + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-o", tmp] + [j[1] for j in jobs])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
