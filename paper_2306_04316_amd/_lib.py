"""ctypes view of libpip.so (argument marshalling only; all work runs in the HIP library)."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpip.so")

PIP_OK, PIP_EINVAL, PIP_ERANGE, PIP_EDOM, PIP_ENOMEM, PIP_EHIP, PIP_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
PIP_NOALLOC_MAX_POINTS = 4194304   # include/pip.h
STATUS_NAMES = {0: "PIP_OK", -1: "PIP_EINVAL", -2: "PIP_ERANGE", -3: "PIP_EDOM", -4: "PIP_ENOMEM",
                -5: "PIP_EHIP", -6: "PIP_ENOTSUP"}

MODES = {"exact": 0, "fp64": 0, "filtered": 1, "fp32": 1}
KERNELS = {"auto": 0, "per_pair": 1, "segmented": 2, "staged": 3, "runs": 4, "batched": 5}
PREDICATES = {"side": 0, "c1": 0, "intersection": 1, "c2": 1}


class PipError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class pip_options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("mode", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("pairs_per_lane", ctypes.c_int32), ("block", ctypes.c_int32),
                ("lds_slots", ctypes.c_int32), ("persistent", ctypes.c_int32), ("order", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("tune", ctypes.c_int32), ("force_recheck", ctypes.c_int32),
                ("bound_scale", ctypes.c_float), ("tune_cache", ctypes.c_char_p), ("timing", ctypes.c_int32),
                ("predicate", ctypes.c_int32), ("index", ctypes.c_int32), ("stats", ctypes.c_int32),
                ("wave_k", ctypes.c_int32)]


class pip_plan_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("mode", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("pairs_per_lane", ctypes.c_int32), ("lds_slots", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("order", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("n_items", ctypes.c_int32), ("tuned", ctypes.c_int32), ("tune_ms", ctypes.c_float),
                ("index", ctypes.c_int32), ("wave_k", ctypes.c_int32)]


class pip_stats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_uint64), ("tests", ctypes.c_uint64), ("ambiguous_tests", ctypes.c_uint64),
                ("rechecked_pairs", ctypes.c_uint64), ("ms_prep", ctypes.c_float),
                ("ms_main", ctypes.c_float), ("ms_recheck", ctypes.c_float)]


_VP = ctypes.c_void_p
_I64 = ctypes.c_int64

_SIGS = {
    "pip_options_init": (None, [ctypes.POINTER(pip_options)]),
    "pip_abi_version": (ctypes.c_int, []),
    "pip_last_error": (ctypes.c_char_p, []),
    "pip_classify": (ctypes.c_int, [_VP, _VP, _I64, _VP, _I64, _VP, _VP, _I64, _VP, _VP,
                                    ctypes.POINTER(pip_options), _VP]),
    "pip_classify_noalloc": (ctypes.c_int, [_VP, _VP, _I64, _VP, _I64, _VP, _VP, _I64, _VP, _VP,
                                            ctypes.POINTER(pip_options), _VP]),
    "pip_probe_copy": (ctypes.c_int, [_VP, _VP, _I64, _VP]),
    "pip_probe_read": (ctypes.c_int, [_VP, _I64, _VP, _VP]),
    "pip_probe_valu": (ctypes.c_int, [_I64, _VP, ctypes.POINTER(ctypes.c_int64), _VP]),
    "pip_plan_create": (ctypes.c_int, [ctypes.POINTER(_VP), _VP, _VP, _I64, _VP, _I64, _VP, _VP, _I64, _VP, _VP,
                                       ctypes.POINTER(pip_options), _VP]),
    "pip_classify_rings": (ctypes.c_int, [_VP, _VP, _I64, _VP, _I64, _VP, _I64, _VP, _VP, _I64, _VP, _VP,
                                          ctypes.POINTER(pip_options), _VP]),
    "pip_plan_create_rings": (ctypes.c_int, [ctypes.POINTER(_VP), _VP, _VP, _I64, _VP, _I64, _VP, _I64, _VP, _VP,
                                             _I64, _VP, _VP, ctypes.POINTER(pip_options), _VP]),
    "pip_join_create": (ctypes.c_int, [ctypes.POINTER(_VP), _VP, _VP, _I64, _VP, _I64, _VP, _I64, _VP, _VP, _I64,
                                       ctypes.POINTER(ctypes.c_int64), _VP]),
    "pip_join_fill": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "pip_join_destroy": (ctypes.c_int, [_VP]),
    "pip_join_timing": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "pip_plan_execute": (ctypes.c_int, [_VP, ctypes.POINTER(pip_stats), _VP]),
    "pip_plan_stats": (ctypes.c_int, [_VP, ctypes.POINTER(pip_stats)]),
    "pip_plan_timing": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                       ctypes.POINTER(ctypes.c_float)]),
    "pip_plan_get_config": (ctypes.c_int, [_VP, ctypes.POINTER(pip_plan_config)]),
    "pip_plan_destroy": (ctypes.c_int, [_VP]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree libpip.so; fails loudly when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2306_04316_amd.build` "
                          "(there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != PIP_OK:
        raise PipError(rc, load().pip_last_error().decode(errors="replace"))


def declared_symbols() -> list:
    return list(_SIGS)
