"""MI355X (gfx950) randomness extractors: Toeplitz, Circulant, Dodis et al.
(convolution extractors) and Von Neumann.

Python binding of libextractor.so (``include/extractor.h``). It only
marshals arguments: every step of an extraction runs in the library's HIP
kernels. PyTorch is used for device memory and streams.

Bit strings are packed little-endian uint64 words (bit i at
``(w[i >> 6] >> (i & 63)) & 1``), held in torch int64/uint64 tensors on the GPU.
The classes follow the paper's interface, ``Toeplitz(n_1, m).extract(x, y)``
(section "Cryptomite for privacy amplification in QKD"), with
``Circulant(n_1, m)`` taking the input length n_1 (n_1 + 1 must be a prime with
2 as a primitive root), ``Dodis(n, m)`` and ``VonNeumann(n)``, whose output
length depends on the data.
"""
from __future__ import annotations

import ctypes
import threading

from . import _lib
from ._lib import (EXT_EDEGENERATE, EXT_EINVAL, EXT_ENOMEM, EXT_ENOTNA, EXT_ETOOLARGE, EXT_OK,  # noqa: F401
                   EXT_KIND_CIRCULANT, EXT_KIND_DODIS, EXT_KIND_TOEPLITZ, EXT_SEED_LINEAR, EXT_SEED_PAPER,
                   EXT_SYNC, ExtError, ExtJob, KINDS)

__all__ = ["Context", "Toeplitz", "Circulant", "Dodis", "VonNeumann", "extract", "extract_batch", "is_na_prime", "next_na_set",
           "closest_na_set", "words", "ExtError", "ExtJob", "default_context"]


def words(nbits: int) -> int:
    return (int(nbits) + 63) >> 6


def is_na_prime(n: int) -> bool:
    return bool(_lib.load().ext_is_na_prime(int(n)))


def next_na_set(v: int) -> int:
    """Smallest prime >= v with 2 as a primitive root."""
    return int(_lib.load().ext_next_na(int(v)))


def closest_na_set(v: int) -> int:
    """Prime with 2 as a primitive root nearest to v (the smaller on a tie)."""
    return int(_lib.load().ext_closest_na(int(v)))


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a GPU tensor of packed uint64 words")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if t.element_size() != 8:
        raise TypeError("packed words must be 64-bit (torch.int64 or torch.uint64)")
    return t.data_ptr()


def _seed_bits(kind: str, n: int, m: int) -> int:
    return {"toeplitz": n + m - 1, "circulant": n + 1, "dodis": n}[kind]


def _check_len(t, nbits: int, what: str):
    """t must hold at least ceil(nbits/64) packed words: the library takes raw device
    pointers, so a short buffer would be read or written past its end."""
    if t.numel() < words(nbits):
        raise ValueError("%s holds %d words; %d bits need %d" % (what, t.numel(), nbits, words(nbits)))


def _status_ptr(status):
    """Device pointer of an int32 status word on the GPU (or None)."""
    import torch
    if status is None:
        return None
    if not isinstance(status, torch.Tensor) or not status.is_cuda or status.dtype != torch.int32 \
            or status.numel() < 1:
        raise TypeError("status must be an int32 GPU tensor with at least one element")
    return ctypes.c_void_p(status.data_ptr())


def _stream_handle(stream, device=None):
    """The HIP stream handle: of `stream` (a torch stream or a raw handle), or torch's
    current stream on `device` (read without building a stream object)."""
    import torch
    if stream is None:
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None and device is not None:
            return ctypes.c_void_p(raw(device))
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Context:
    """An extractor context on one device (twiddle tables, workspace pool)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, tune=True):
        """tune: True loads the packaged tuning table (tune_gfx950.txt) when present,
        False keeps the built-in plans, a str is the path of a table."""
        lib = _lib.load()
        h = ctypes.c_void_p()
        if tune is True:
            import os
            path = os.path.join(_lib.HERE, "tune_gfx950.txt")
            tune = path if os.path.exists(path) else None
        elif tune is False:
            tune = None
        rc = lib.ext_create(ctypes.byref(h), int(device), int(hbm_budget_bytes), tune.encode() if tune else None)
        if rc != EXT_OK:
            raise ExtError(rc, "ext_create")
        self.handle = h
        self.device = int(device)
        self._lib = lib

    def close(self):
        if getattr(self, "handle", None):
            self._lib.ext_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mem_stats(self):
        b, u, r = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        self._lib.ext_mem_stats(self.handle, ctypes.byref(b), ctypes.byref(u), ctypes.byref(r))
        return {"budget": b.value, "in_use": u.value, "reserved": r.value}

    def trim(self):
        self._lib.ext_trim(self.handle)

    def seed_cache_clear(self):
        """Drop every cached seed transform; returns (bytes, entries) held before."""
        b, e = ctypes.c_size_t(), ctypes.c_size_t()
        self._lib.ext_seed_cache_clear(self.handle, ctypes.byref(b), ctypes.byref(e))
        return b.value, e.value

    def profile(self, enable: bool = True):
        """Bracket every kernel launch of later extraction calls with HIP events."""
        self._lib.ext_profile(self.handle, 1 if enable else 0)

    def profile_read(self):
        """[(kernel label, milliseconds)] for the launches traced since the last read."""
        cap = 1 << 22
        buf = ctypes.create_string_buffer(cap)
        n = self._lib.ext_profile_read(self.handle, buf, cap)
        if n < 0:
            raise ExtError(n, "ext_profile_read")
        out = []
        for line in buf.value.decode().splitlines():
            name, ms = line.rsplit(" ", 1)
            out.append((name, float(ms)))
        return out

    # -- raw calls (device tensors in, device tensor out) --------------------------------
    def extract(self, kind: str, x, y, n: int, m: int, z=None, seed_order: str = "paper", sync: bool = False,
                status=None, stream=None, check: bool = True, cache_seed: bool = False,
                single_transform: bool = False, no_alloc: bool = False) -> "object":
        """cache_seed: keep / reuse the seed's transform (the seed bits at y must not
        change while cached; see seed_cache_clear). single_transform: no two-piece
        split (one transform: over the 64-bit field beyond 2^30, over 15*2^27+1 at 2^27).
        no_alloc: Toeplitz through extract_toeplitz_noalloc (the library's fixed
        per-GPU workspace; calls on one GPU must not overlap)."""
        import torch
        if kind not in ("toeplitz", "circulant", "dodis"):
            raise ValueError("unknown extractor kind %r" % kind)
        n, m = int(n), int(m)
        if z is None:
            z = torch.empty(words(m), dtype=torch.int64, device=x.device)
        px, py, pz = _ptr(x), _ptr(y), _ptr(z)
        if 1 <= m <= n <= (1 << 40):  # sizes the library accepts (it rejects the others itself)
            _check_len(x, n, "x")
            _check_len(y, _seed_bits(kind, n, m), "y")
            _check_len(z, m, "z")
        flags = (EXT_SEED_LINEAR if seed_order == "linear" else 0) | (EXT_SYNC if sync else 0) | \
            (_lib.EXT_SEED_CACHED if cache_seed else 0) | (_lib.EXT_SINGLE_TRANSFORM if single_transform else 0)
        st = _status_ptr(status)
        s = _stream_handle(stream, self.device)
        if no_alloc:
            if kind != "toeplitz" or cache_seed or single_transform:
                raise ValueError("no_alloc: Toeplitz only, without cache_seed / single_transform")
            rc = self._lib.extract_toeplitz_noalloc(self.handle, px, n, py, m, pz, flags, st, s)
        elif kind == "toeplitz":
            rc = self._lib.extract_toeplitz(self.handle, px, n, py, m, pz, flags, st, s)
        elif kind == "circulant":
            rc = self._lib.extract_circulant(self.handle, px, n, py, m, pz, flags, st, s)
        elif kind == "dodis":
            rc = self._lib.extract_dodis(self.handle, px, py, n, m, pz, flags, st, s)
        else:
            raise ValueError("unknown extractor kind %r" % kind)
        if check and rc != EXT_OK:
            raise ExtError(rc, "extract_" + kind)
        return z if check else (rc, z)

    def von_neumann(self, x, n: int, z=None, m_out=None, sync: bool = False, status=None, stream=None,
                    check: bool = True):
        """Von Neumann extractor (section "Von Neumann", Alg. 3) on the n bits of x.
        z: words(n // 2) words or more (allocated if None); m_out: one-element int64
        device tensor for the output length (allocated if None). Returns (z, m_out), with
        m_out read back as an int when sync=True; the first words(m) words of z carry
        the output. No differing pair: EXT_EDEGENERATE (raised when check and sync)."""
        import torch
        if z is None:
            z = torch.empty(max(1, words(int(n) // 2)), dtype=torch.int64, device=x.device)
        if m_out is None:
            m_out = torch.zeros(1, dtype=torch.int64, device=x.device)
        if m_out.element_size() != 8 or not m_out.is_cuda or m_out.numel() < 1:
            raise TypeError("m_out must be a 64-bit GPU tensor")
        _ptr(x), _ptr(z)
        if 2 <= int(n) <= _lib.EXT_VN_MAX_BITS:  # sizes the library accepts
            _check_len(x, int(n), "x")
        st = _status_ptr(status)
        rc = self._lib.extract_von_neumann(self.handle, _ptr(x), int(n), _ptr(z), int(z.numel()),
                                           ctypes.c_void_p(m_out.data_ptr()), EXT_SYNC if sync else 0, st,
                                           _stream_handle(stream, self.device))
        if check and rc != EXT_OK:
            raise ExtError(rc, "extract_von_neumann")
        if sync:
            m_out = int(m_out.item())
        return (z, m_out) if check else (rc, z, m_out)

    def tune_set(self, word_bits: int, lg: int, levels, single: bool = False):
        """Override the plan for transform length 2^lg: levels = [] for one workgroup per
        job, a list of pass sizes (log2) otherwise, None to drop the override. single:
        the plan of single extraction calls of that size (ext_tune_set_single) instead of
        the plan of batches (and of single calls without one of their own)."""
        fn = self._lib.ext_tune_set_single if single else self._lib.ext_tune_set
        if levels is None:
            rc = fn(self.handle, word_bits, lg, -1, None)
        else:
            arr = (ctypes.c_int * 4)(*(list(levels) + [0] * (4 - len(levels))))
            rc = fn(self.handle, word_bits, lg, len(levels), arr)
        if rc != EXT_OK:
            raise ExtError(rc, "ext_tune_set_single" if single else "ext_tune_set")

    def tune_get(self, word_bits: int, lg: int, single: bool = False):
        """The plan in use for transform length 2^lg (single: the one single calls use)."""
        nlev = ctypes.c_int()
        arr = (ctypes.c_int * 4)()
        fn = self._lib.ext_tune_get_single if single else self._lib.ext_tune_get
        rc = fn(self.handle, word_bits, lg, ctypes.byref(nlev), arr)
        if rc != EXT_OK:
            raise ExtError(rc, "ext_tune_get_single" if single else "ext_tune_get")
        return list(arr[: nlev.value])

    def tune_save(self, path: str):
        rc = self._lib.ext_tune_save(self.handle, path.encode())
        if rc != EXT_OK:
            raise ExtError(rc, "ext_tune_save")

    def workspace_bytes(self, kind: str, n: int, m: int) -> int:
        return int(self._lib.ext_workspace_bytes(KINDS[kind], int(n), int(m)))

    def batch(self, jobs, sync: bool = False, stream=None, unbatched: bool = False, graph: bool = False):
        """jobs: list of dicts with kind, n, m, x, y, z[, seed_order, status, single_transform]. Returns the
        library's return code and the per-job host validation codes. graph=True records
        the launch sequence of this batch signature into a HIP graph and replays it."""
        arr = (ExtJob * len(jobs))()
        for i, j in enumerate(jobs):
            kind = j["kind"]
            if kind not in ("toeplitz", "circulant", "dodis"):
                raise ValueError("job %d: unknown extractor kind %r" % (i, kind))
            n, m = int(j["n"]), int(j["m"])
            arr[i].kind = KINDS[kind]
            arr[i].flags = (EXT_SEED_LINEAR if j.get("seed_order") == "linear" else 0) | \
                (_lib.EXT_SINGLE_TRANSFORM if j.get("single_transform") else 0)
            arr[i].n = n
            arr[i].m = m
            arr[i].x = _ptr(j["x"])
            arr[i].y = _ptr(j["y"])
            arr[i].z = _ptr(j["z"])
            if 1 <= m <= n <= (1 << 40):
                _check_len(j["x"], n, "job %d: x" % i)
                _check_len(j["y"], _seed_bits(kind, n, m), "job %d: y" % i)
                _check_len(j["z"], m, "job %d: z" % i)
            st = _status_ptr(j.get("status"))
            arr[i].status = st.value if st is not None else None
        fn = self._lib.extract_batch_unbatched if unbatched else self._lib.extract_batch
        flags = (EXT_SYNC if sync else 0) | (_lib.EXT_GRAPH if (graph and not unbatched) else 0)
        rc = fn(self.handle, arr, len(jobs), flags, _stream_handle(stream, self.device))
        return rc, [arr[i].err for i in range(len(jobs))]


_default = {}
_default_lock = threading.Lock()


def default_context(device: int = 0) -> Context:
    with _default_lock:
        if device not in _default:
            _default[device] = Context(device)
        return _default[device]


def extract(kind: str, x, y, n: int, m: int, **kw):
    return default_context(x.device.index or 0).extract(kind, x, y, n, m, **kw)


def extract_batch(jobs, **kw):
    dev = jobs[0]["x"].device.index or 0 if jobs else 0
    return default_context(dev).batch(jobs, **kw)


class _Extractor:
    kind = ""

    def __init__(self, n: int, m: int, seed_order: str = "paper", context: Context | None = None):
        self.n, self.m, self.seed_order, self.context = int(n), int(m), seed_order, context

    def extract(self, x, y, z=None, stream=None, sync: bool = True):
        ctx = self.context or default_context(x.device.index or 0)
        return ctx.extract(self.kind, x, y, self.n, self.m, z=z, seed_order=self.seed_order, sync=sync,
                           stream=stream)


class Toeplitz(_Extractor):
    """Toeplitz(n_1, m): x has n_1 bits, the seed n_1 + m - 1 bits."""
    kind = "toeplitz"


class Circulant(_Extractor):
    """Circulant(n_1, m): x has n_1 bits, the seed n_1 + 1 bits (n_1 + 1 prime, primitive root 2)."""
    kind = "circulant"


class Dodis(_Extractor):
    """Dodis(n, m): x and y have n bits (n prime with primitive root 2)."""
    kind = "dodis"


class VonNeumann:
    """VonNeumann(n): x has n bits; extract returns (z, m) with m output bits."""

    def __init__(self, n: int, context: Context | None = None):
        self.n, self.context = int(n), context

    def extract(self, x, z=None, stream=None):
        ctx = self.context or default_context(x.device.index or 0)
        return ctx.von_neumann(x, self.n, z=z, sync=True, stream=stream)
