"""ctypes loader for libextractor.so (argument marshalling only).

The library must be built first (``python -m paper_2402_09481_amd.build`` or
``__graft_entry__.build()``); loading fails loudly otherwise — there is no
fallback implementation."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libextractor.so")

EXT_OK = 0
EXT_EINVAL = -1
EXT_ENOTNA = -2
EXT_EDEGENERATE = -3
EXT_ENOMEM = -4
EXT_ETOOLARGE = -5
EXT_EDEVICE = -6
EXT_ESCRATCH = -7
EXT_NOALLOC_SCRATCH_BYTES = 40 << 20

EXT_SEED_PAPER = 0
EXT_SEED_LINEAR = 1
EXT_SYNC = 2
EXT_GRAPH = 4
EXT_SEED_CACHED = 8
EXT_SINGLE_TRANSFORM = 16

EXT_KIND_TOEPLITZ = 0
EXT_KIND_CIRCULANT = 1
EXT_KIND_DODIS = 2
EXT_KIND_VON_NEUMANN = 3
EXT_VN_MAX_BITS = 1 << 40

KINDS = {"toeplitz": EXT_KIND_TOEPLITZ, "circulant": EXT_KIND_CIRCULANT, "dodis": EXT_KIND_DODIS,
         "von_neumann": EXT_KIND_VON_NEUMANN}

# every symbol declared in include/extractor.h
SYMBOLS = [
    "ext_create", "ext_destroy", "extract_toeplitz", "extract_circulant", "extract_dodis",
    "extract_batch", "extract_batch_unbatched", "ext_workspace_bytes", "ext_plan_length",
    "ext_mem_stats", "ext_trim", "ext_is_na_prime", "ext_next_na", "ext_closest_na",
    "ext_strerror", "ext_version", "ext_profile", "ext_profile_read",
    "ext_tune_set", "ext_tune_get", "ext_tune_set_single", "ext_tune_get_single", "ext_tune_save",
    "ext_seed_cache_clear", "extract_von_neumann",
    "extract_toeplitz_noalloc",
]


class ExtJob(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("n", ctypes.c_uint64), ("m", ctypes.c_uint64),
        ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
        ("status", ctypes.c_void_p), ("err", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class ExtError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__("%s: %s (%d)" % (what or "extractor", strerror(code), code))


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        raise ImportError(
            "libextractor.so is not built (%s). Build it with `python -m paper_2402_09481_amd.build`." % SO_PATH)
    # PyTorch ships its own HIP runtime with the same soname (libamdhip64.so.7) as
    # /opt/rocm's. Loading torch first makes the library bind to that already-loaded
    # runtime; the other order puts two HIP runtimes in one process, and the second
    # one to initialise finds no GPU.
    import torch  # noqa: F401
    lib = ctypes.CDLL(SO_PATH)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
    sz = ctypes.c_size_t
    lib.ext_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, sz, ctypes.c_char_p]
    lib.ext_create.restype = ctypes.c_int
    lib.ext_destroy.argtypes = [vp]
    lib.ext_destroy.restype = None
    lib.extract_toeplitz.argtypes = [vp, vp, u64, vp, u64, vp, u32, vp, vp]
    lib.extract_circulant.argtypes = [vp, vp, u64, vp, u64, vp, u32, vp, vp]
    lib.extract_dodis.argtypes = [vp, vp, vp, u64, u64, vp, u32, vp, vp]
    lib.extract_toeplitz_noalloc.argtypes = [vp, vp, u64, vp, u64, vp, u32, vp, vp]
    for f in (lib.extract_toeplitz, lib.extract_circulant, lib.extract_dodis, lib.extract_toeplitz_noalloc):
        f.restype = ctypes.c_int
    lib.extract_von_neumann.argtypes = [vp, vp, u64, vp, u64, vp, u32, vp, vp]
    lib.extract_von_neumann.restype = ctypes.c_int
    lib.extract_batch.argtypes = [vp, ctypes.POINTER(ExtJob), sz, u32, vp]
    lib.extract_batch.restype = ctypes.c_int
    lib.extract_batch_unbatched.argtypes = [vp, ctypes.POINTER(ExtJob), sz, u32, vp]
    lib.extract_batch_unbatched.restype = ctypes.c_int
    lib.ext_workspace_bytes.argtypes = [i32, u64, u64]
    lib.ext_workspace_bytes.restype = sz
    lib.ext_plan_length.argtypes = [i32, u64, u64, ctypes.POINTER(i32)]
    lib.ext_plan_length.restype = u64
    lib.ext_mem_stats.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.ext_mem_stats.restype = ctypes.c_int
    lib.ext_trim.argtypes = [vp]
    lib.ext_trim.restype = ctypes.c_int
    lib.ext_is_na_prime.argtypes = [u64]
    lib.ext_is_na_prime.restype = ctypes.c_int
    lib.ext_next_na.argtypes = [u64]
    lib.ext_next_na.restype = u64
    lib.ext_closest_na.argtypes = [u64]
    lib.ext_closest_na.restype = u64
    lib.ext_strerror.argtypes = [ctypes.c_int]
    lib.ext_strerror.restype = ctypes.c_char_p
    lib.ext_profile.argtypes = [vp, ctypes.c_int]
    lib.ext_profile.restype = ctypes.c_int
    lib.ext_profile_read.argtypes = [vp, ctypes.c_char_p, sz]
    lib.ext_profile_read.restype = ctypes.c_int
    lib.ext_tune_set.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.ext_tune_set.restype = ctypes.c_int
    lib.ext_tune_get.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.ext_tune_get.restype = ctypes.c_int
    lib.ext_tune_set_single.argtypes = lib.ext_tune_set.argtypes
    lib.ext_tune_set_single.restype = ctypes.c_int
    lib.ext_tune_get_single.argtypes = lib.ext_tune_get.argtypes
    lib.ext_tune_get_single.restype = ctypes.c_int
    lib.ext_tune_save.argtypes = [vp, ctypes.c_char_p]
    lib.ext_tune_save.restype = ctypes.c_int
    lib.ext_seed_cache_clear.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.ext_seed_cache_clear.restype = ctypes.c_int
    lib.ext_version.argtypes = []
    lib.ext_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(code: int) -> str:
    try:
        return load().ext_strerror(int(code)).decode()
    except ImportError:
        return "error %d" % code
