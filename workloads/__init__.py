"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module only draws random bits and lays them out in memory. It holds none
of the extraction arithmetic: no convolution, no field maths, no primality
test. Where a workload needs a prime length (Circulant and Dodis), the caller
passes the search function in, so that each side uses its own.

Bit layout (used everywhere): a bit string b_0 … b_{n-1} is stored as
little-endian uint64 words, bit i at ``(w[i >> 6] >> (i & 63)) & 1``. Bits of the
last word beyond n are zero.

Generator: NumPy ``Generator(PCG64(seed))``. Bernoulli(p) bits are drawn as
``random() < p`` in chunks of 2^24; p = 0.5 uses raw 64-bit words instead.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 2402_09481
CHUNK_BITS = 1 << 24


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def nwords(nbits: int) -> int:
    return (int(nbits) + 63) >> 6


def pack_bits(bits) -> np.ndarray:
    """uint8 0/1 array → packed LSB-first uint64 words (tail zero)."""
    bits = np.asarray(bits, dtype=np.uint8)
    n = bits.size
    pad = nwords(n) * 64 - n
    if pad:
        bits = np.concatenate([bits, np.zeros(pad, np.uint8)])
    return np.packbits(bits, bitorder="little").view("<u8").copy()


def unpack_bits(words, nbits: int) -> np.ndarray:
    """packed uint64 words → uint8 0/1 array of length nbits."""
    w = np.ascontiguousarray(np.asarray(words, dtype="<u8"))
    return np.unpackbits(w.view(np.uint8), bitorder="little")[: int(nbits)].copy()


def mask_tail(words: np.ndarray, nbits: int) -> np.ndarray:
    """Zero the bits of the last word beyond nbits (in place) and return words."""
    r = int(nbits) & 63
    if r and words.size:
        words[-1] &= np.uint64((1 << r) - 1)
    return words


def bernoulli_bits(g: np.random.Generator, nbits: int, p: float) -> np.ndarray:
    """nbits iid Bernoulli(p) bits, packed."""
    nbits = int(nbits)
    nw = nwords(nbits)
    out = np.empty(nw, dtype="<u8")
    if p == 0.5:
        out[:] = g.integers(0, 1 << 64, size=nw, dtype=np.uint64, endpoint=False)
        return mask_tail(out, nbits)
    done = 0
    while done < nbits:
        c = min(CHUNK_BITS, nbits - done)
        bits = (g.random(c) < p).astype(np.uint8)
        w = pack_bits(bits)
        # chunks are multiples of 64 bits except possibly the last one
        out[done >> 6: (done >> 6) + w.size] = w
        done += c
    return mask_tail(out, nbits)


@dataclasses.dataclass
class Job:
    """One extraction: kind in {"toeplitz", "circulant", "dodis"}.

    n is the input length in bits as the extractor's caller passes it (for
    Circulant the input x has n bits and the seed n + 1). seed_order is
    "paper" or "linear" (Toeplitz only)."""
    kind: str
    n: int
    m: int
    x: np.ndarray
    y: np.ndarray
    seed_order: str = "paper"

    @property
    def seed_bits(self) -> int:
        if self.kind == "toeplitz":
            return self.n + self.m - 1
        if self.kind == "circulant":
            return self.n + 1
        return self.n


# ---------------------------------------------------------------- the five workloads

def toeplitz_small(seed: int = BASE_SEED + 0) -> Job:
    """Toeplitz, n = 4096, m = 2048, x and seed iid Bernoulli(0.5), linear seed order."""
    g = rng(seed)
    n, m = 4096, 2048
    x = bernoulli_bits(g, n, 0.5)
    s = bernoulli_bits(g, n + m - 1, 0.5)
    return Job("toeplitz", n, m, x, s, "linear")


DODIS_N = 1048589  # smallest prime >= 2^20 with 2 as a primitive root (pinned in tests)


def dodis_2p20(seed: int = BASE_SEED + 1) -> Job:
    """Dodis et al., n = 1,048,589, x ~ B(0.3), y ~ B(0.5), m = 2^19."""
    g = rng(seed)
    n, m = DODIS_N, 1 << 19
    x = bernoulli_bits(g, n, 0.3)
    y = bernoulli_bits(g, n, 0.5)
    return Job("dodis", n, m, x, y)


def toeplitz_large(seed: int = BASE_SEED + 2, n: int = 1 << 30, m: int = 1 << 29) -> Job:
    """Toeplitz, n = 2^30, x ~ B(0.4), m = 2^29, seed n+m-1 bits ~ B(0.5)."""
    g = rng(seed)
    x = bernoulli_bits(g, n, 0.4)
    y = bernoulli_bits(g, n + m - 1, 0.5)
    return Job("toeplitz", n, m, x, y, "paper")


# The paper's QKD privacy-amplification example (section "Cryptomite for privacy
# amplification in QKD"): n = 1.738e9 raw-key bits, m = 41,378,264 output bits with
# the Toeplitz extractor; the improved variant uses Circulant with the input padded
# to n_adj - 1 bits, n_adj the next prime >= n + 1 with primitive root 2, a weak seed
# of min-entropy rate r = 0.99 and error 1e-10, and m = floor(k1 + k2 - n_adj +
# 2 log2(eps)) with k1 = m_toeplitz - 2 log2(eps) and k2 = r n_adj.
QKD_N = 1_738_000_000
QKD_M = 41_378_264
QKD_EPS = 1e-10
QKD_RATE = 0.99

# The QRNG example (section "Cryptomite for randomness extraction in (Q)RNG"):
# n = 6.5e9 raw bits of min-entropy k1 = floor(0.08943 n) = 581,295,000, error
# 1e-10, Toeplitz output m = floor(k1 + 2 log2(eps)) = 581,294,933; the improved
# variant uses Circulant with the input length adjusted to the prime with
# primitive root 2 closest to n + 1 (padding with zeros, or cutting and lowering
# k1) and a weak seed of min-entropy rate 0.99.
QRNG_N = 6_500_000_000
QRNG_M = 581_294_933
QRNG_K1 = 581_295_000
QRNG_EPS = 1e-10
QRNG_RATE = 0.99
# Bias of i.i.d. stand-in bits with the certified min-entropy rate 0.08943:
# -log2(max(p, 1 - p)) = 0.08943.
QRNG_P_ONE = 1.0 - 2.0 ** -0.08943


def qkd_toeplitz(seed: int = BASE_SEED + 6) -> Job:
    g = rng(seed)
    x = bernoulli_bits(g, QKD_N, 0.5)
    y = bernoulli_bits(g, QKD_N + QKD_M - 1, 0.5)
    return Job("toeplitz", QKD_N, QKD_M, x, y, "paper")


def qkd_circulant_shape(next_na):
    """(n_in, m) of the improved QKD extraction; next_na comes from the caller."""
    n_adj = int(next_na(QKD_N + 1))
    k1 = QKD_M - 2 * math.log2(QKD_EPS)
    k2 = QKD_RATE * n_adj
    m = int(math.floor(k1 + k2 - n_adj + 2 * math.log2(QKD_EPS)))
    return n_adj - 1, m


def qkd_circulant(next_na, seed: int = BASE_SEED + 7) -> Job:
    n_in, m = qkd_circulant_shape(next_na)
    g = rng(seed)
    x = np.zeros(nwords(n_in), dtype="<u8")
    x[: nwords(QKD_N)] = bernoulli_bits(g, QKD_N, 0.5)  # raw key padded with zeros to n_in bits
    y = bernoulli_bits(g, n_in + 1, 0.5)
    return Job("circulant", n_in, m, x, y)


def qrng_circulant_shape(closest_na):
    """(n_in, m) of the improved QRNG extraction; closest_na comes from the caller."""
    n_adj = int(closest_na(QRNG_N + 1))
    k1 = QRNG_K1 - max(0, QRNG_N + 1 - n_adj)
    k2 = QRNG_RATE * n_adj
    m = int(math.floor(k1 + k2 - n_adj + 2 * math.log2(QRNG_EPS)))
    return n_adj - 1, m


def qrng_toeplitz_device(seed: int = BASE_SEED + 14):
    """The QRNG Toeplitz shape as device tensors (x: n i.i.d. bits of the certified
    min-entropy rate, seed: n + m - 1 bits ~ B(1/2)), drawn with torch's seeded
    generator on the GPU (1.7 GB of bits). Returns (n, m, x, y)."""
    x = bernoulli_bits_device(QRNG_N, QRNG_P_ONE, seed)
    y = bernoulli_bits_device(QRNG_N + QRNG_M - 1, 0.5, seed + 1)
    return QRNG_N, QRNG_M, x, y


def qrng_circulant_device(closest_na, seed: int = BASE_SEED + 15):
    """The improved QRNG Circulant shape as device tensors: x is the raw bits padded
    with zeros to n_in bits, y the n_in + 1 seed bits. Returns (n_in, m, x, y)."""
    import torch
    n_in, m = qrng_circulant_shape(closest_na)
    raw = bernoulli_bits_device(QRNG_N, QRNG_P_ONE, seed)
    x = torch.zeros(nwords(n_in), dtype=torch.int64, device=raw.device)
    x[: raw.numel()] = raw
    y = bernoulli_bits_device(n_in + 1, 0.5, seed + 1)
    return n_in, m, x, y


def batch_params(count: int = 4096, seed: int = BASE_SEED + 3, next_na=None,
                 log_lo: float = 10.0, log_hi: float = 22.0):
    """Block parameters for the batched workload, drawn from one master stream.

    Returns a list of (kind, n, m, p_x, subseed). n = floor(2^u), u ~ U[lo, hi];
    kind is Toeplitz or Circulant with probability 1/2; a Circulant block's prime
    length is next_na(n + 1) and its input length that prime minus one; m = n // 2
    (capped at the Circulant bound); p_x ~ U[0.2, 0.5]."""
    if next_na is None:
        raise ValueError("batch_params needs the caller's next_na function")
    g = rng(seed)
    out = []
    for _ in range(count):
        u = g.uniform(log_lo, log_hi)
        n = int(math.floor(2.0 ** u))
        circ = bool(g.integers(0, 2))
        px = float(g.uniform(0.2, 0.5))
        sub = int(g.integers(0, 1 << 63))
        if circ:
            prime = int(next_na(n + 1))
            n_in = prime - 1
            m = min(n_in // 2, prime - 1)
            out.append(("circulant", n_in, m, px, sub))
        else:
            out.append(("toeplitz", n, n // 2, px, sub))
    return out


def make_job(kind: str, n: int, m: int, px: float, subseed: int, seed_order: str = "paper") -> Job:
    g = rng(subseed)
    x = bernoulli_bits(g, n, px)
    nseed = {"toeplitz": n + m - 1, "circulant": n + 1, "dodis": n}[kind]
    y = bernoulli_bits(g, nseed, 0.5)
    return Job(kind, n, m, x, y, seed_order)


def batch_jobs(count: int = 4096, seed: int = BASE_SEED + 3, next_na=None, **kw):
    return [make_job(k, n, m, px, sub) for (k, n, m, px, sub) in batch_params(count, seed, next_na, **kw)]


@dataclasses.dataclass
class Request:
    t_arrival: float  # seconds from the start of the run
    n: int
    m: int
    x_offset: int     # bit offset of x inside the resident input pool
    seed_id: int      # which resident seed; the request uses its first n+m-1 bits


SERVE_POOL_BITS = 1 << 27
SERVE_SEEDS = 16
SERVE_SEED_BITS = (1 << 26) + (1 << 25)


def serving_requests(rate: float, count: int, seed: int = BASE_SEED + 4,
                     log_lo: float = 12.0, log_hi: float = 26.0):
    """Open-loop Poisson arrivals of Toeplitz requests: n = floor(2^u), u ~ U[lo, hi],
    m ~ U{ceil(n/4) .. floor(n/2)}; x is a 64-bit aligned slice of the resident pool."""
    g = rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += float(g.exponential(1.0 / rate))
        u = g.uniform(log_lo, log_hi)
        n = int(math.floor(2.0 ** u))
        m = int(g.integers(-(-n // 4), n // 2 + 1))
        off = int(g.integers(0, (SERVE_POOL_BITS - n) // 64 + 1)) * 64
        sid = int(g.integers(0, SERVE_SEEDS))
        out.append(Request(t, n, m, off, sid))
    return out


def serving_pool(seed: int = BASE_SEED + 5):
    """The resident input pool (B(0.5)) and the resident seeds."""
    g = rng(seed)
    pool = bernoulli_bits(g, SERVE_POOL_BITS, 0.5)
    seeds = [bernoulli_bits(g, SERVE_SEED_BITS, 0.5) for _ in range(SERVE_SEEDS)]
    return pool, seeds


# ------------------------------------------------------------------ Von Neumann inputs

# The Von Neumann input of the paper's throughput figure: input min-entropy fixed to
# half the length, which for i.i.d. bits means max(p, 1 - p) = 2^(-1/2).
VN_P = 1.0 - 2.0 ** -0.5
VN_PAPER_N = 500_000_000    # the largest input length of the throughput figure
VN_LARGE_N = 1 << 33        # 1 GiB of input bits: one HBM-scale call


def von_neumann_input(n: int, p: float = VN_P, seed: int = BASE_SEED + 8) -> np.ndarray:
    """n i.i.d. bits with P(bit = 1) = p (host, PCG64)."""
    return bernoulli_bits(rng(seed), n, p)


def bernoulli_bits_device(n: int, p: float, seed: int, device="cuda", chunk_words: int = 1 << 21):
    """n i.i.d. bits with P(bit = 1) = p, packed as above, drawn on the device by
    torch's generator seeded with `seed` (for inputs too large to draw on the host
    in reasonable time). Returns an int64 tensor of nwords(n) words."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    W = nwords(n)
    out = torch.empty(W, dtype=torch.int64, device=device)
    weights = (2 ** torch.arange(8, device=device)).to(torch.uint8)
    for w0 in range(0, W, chunk_words):
        w1 = min(W, w0 + chunk_words)
        bits = torch.rand((w1 - w0, 8, 8), generator=gen, device=device) < p
        by = (bits.to(torch.uint8) * weights).sum(dim=2, dtype=torch.uint8)  # (words, 8) bytes
        out[w0:w1] = by.contiguous().view(torch.int64).view(-1)
        del bits, by
    r = n & 63
    if r:
        out[W - 1] &= (1 << r) - 1
    return out
