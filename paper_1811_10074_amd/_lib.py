"""ctypes declarations of libsws.so (the C ABI in include/sws.h).

Loading never falls back to anything: if the built library is missing the
import-time call raises, naming the build command."""
from __future__ import annotations

import ctypes
import os
import re
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsws.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sws.h")

SWS_OK = 0
SWS_ERR_INVALID = -1
SWS_ERR_CAPACITY = -2
SWS_ERR_WORKSPACE = -3
SWS_ERR_DEVICE = -4
SWS_ERR_UNSUPPORTED = -5
NOALLOC_SCRATCH_BYTES = 4 << 20  # SWS_NOALLOC_SCRATCH_BYTES

OPS = {"add": 0, "min": 1, "max": 2, "affine": 3}
PATHS = {"auto": 0, "generic": 1, "log": 2, "prefix": 3, "scalar": 4}
KMER_FORWARD = 1
HASH_IDENTITY = 2
SPLIT_AT_INVALID = 4
WORKSPACE_KEPT = 8

_lock = threading.Lock()
_lib = None

c_u32, c_u64, c_int, c_vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p

_SIGNATURES = {
    "sws_abi_version": (c_u32, []),
    "sws_status_str": (ctypes.c_char_p, [c_int]),
    "sws_sliding_sum": (c_int, [c_int, c_u64, c_vp, c_u64, c_vp, c_vp]),
    "sws_sliding_sum_ex": (c_int, [c_int, c_u64, c_vp, c_u64, c_vp, c_int, c_vp]),
    "sws_sliding_sum_workspace": (c_int, [c_int, c_u64, c_u64, c_int, ctypes.POINTER(c_u64)]),
    "sws_sliding_sum_ws": (c_int, [c_int, c_u64, c_vp, c_u64, c_vp, c_int, c_vp, c_u64, c_vp]),
    "sws_pack2bit": (c_int, [c_vp, c_u64, c_vp, c_vp, c_vp]),
    "sws_kmers": (c_int, [c_vp, c_u64, c_u32, c_u32, c_vp, c_vp]),
    "sws_minimizers_workspace": (c_int, [c_u64, c_u32, c_u32, ctypes.POINTER(c_u64)]),
    "sws_minimizers": (c_int, [c_vp, c_u64, c_u32, c_u32, c_u32, c_vp, c_vp, c_u64, c_vp, c_vp,
                               c_u64, c_vp]),
    "sws_minimizers_2bit": (c_int, [c_vp, c_vp, c_u64, c_u32, c_u32, c_u32, c_vp, c_vp, c_u64,
                                    c_vp, c_vp, c_u64, c_vp]),
    "sws_minimizers_noalloc": (c_int, [c_vp, c_u64, c_u32, c_u32, c_u32, c_vp, c_vp, c_u64, c_vp,
                                       c_vp]),
    "sws_minimizers_batch_workspace": (c_int, [c_u64, c_u32, c_u32, c_u32, ctypes.POINTER(c_u64)]),
    "sws_minimizers_batch": (c_int, [c_vp, c_vp, c_u32, c_u64, c_u32, c_u32, c_u32, c_vp, c_vp,
                                     c_vp, c_u64, c_vp, c_vp, c_u64, c_vp]),
    "sws_minimizers_batch_ex": (c_int, [c_vp, c_vp, c_u32, c_u64, c_u32, c_u32, c_u32, c_vp, c_vp,
                                        c_vp, c_u64, c_vp, c_vp, c_u64, c_u32, c_vp]),
    "sws_set_sliding_waves": (c_int, [c_u64]),
    "sws_seed_table_workspace": (c_int, [c_u64, c_u32, c_vp]),
    "sws_seed_table": (c_int, [c_vp, c_vp, c_u64, c_u32, c_u32, c_vp, c_vp, c_vp, c_vp, c_u64,
                               c_vp]),
}


class SwsError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__("%s: %s" % (what, status_str(status)))


def header_functions(path: str = HEADER):
    """Names of the functions the public header declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sws_[a-z0-9_]+)\s*\(", text)))


def load():
    """The loaded library.  Raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("libsws.so is not built (%s); run "
                                  "`python paper_1811_10074_amd/build.py`" % LIB_PATH)
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGNATURES.items():
                f = getattr(lib, name)
                f.restype = res
                f.argtypes = args
            _lib = lib
    return _lib


def status_str(status: int) -> str:
    try:
        return load().sws_status_str(status).decode()
    except ImportError:
        return "status %d" % status


def check(status: int, what: str) -> None:
    if status == SWS_OK:
        return
    if status in (SWS_ERR_INVALID, SWS_ERR_CAPACITY, SWS_ERR_WORKSPACE, SWS_ERR_UNSUPPORTED):
        raise ValueError("%s: %s" % (what, status_str(status)))
    raise SwsError(status, what)
