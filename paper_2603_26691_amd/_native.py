"""ctypes binding of libscaletrack.so (argument marshalling only).

torch is imported before the library is loaded: torch ships its own HIP
runtime under the same soname, and loading it first makes the library bind
to that one runtime, so device pointers and streams from torch are valid in
the library.  There is no fallback: if the library is missing, loading
fails with an error that says how to build it.
"""
import ctypes
import os

import torch  # noqa: F401  (must precede the CDLL below)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscaletrack.so")

ST_OK, ST_ERR_INVALID, ST_ERR_OOM, ST_ERR_DEVICE, ST_ERR_STATE, ST_ERR_CAPACITY = range(6)
STATUS_NAMES = {0: "ST_OK", 1: "ST_ERR_INVALID", 2: "ST_ERR_OOM", 3: "ST_ERR_DEVICE",
                4: "ST_ERR_STATE", 5: "ST_ERR_CAPACITY"}
FORMS = {"fp64": 0, "fp32_local": 1, "fp32": 2}
INTERPS = {"trilinear": 0, "ngp": 1}
DRAGS = {"stokes": 0, "schiller_naumann": 1}


class MeshDesc(ctypes.Structure):
    """Mirror of st_mesh_desc (include/st.h)."""
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("chunk_edge", ctypes.c_int32),
        ("L", ctypes.c_double * 3),
        ("rho_f", ctypes.c_double),
        ("mu_f", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("rho_p", ctypes.c_double),
        ("parcel_weight", ctypes.c_double),
        ("form", ctypes.c_int32),
        ("interp", ctypes.c_int32),
        ("drag", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("capacity", ctypes.c_int64),
    ]


# name -> (restype, argtypes); the exported symbols of include/st.h
_P = ctypes.c_void_p
_I = ctypes.c_int
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double
SIGNATURES = {
    "st_create_mesh": (_I, [ctypes.POINTER(MeshDesc), _I, ctypes.POINTER(_P)]),
    "st_destroy": (_I, [_P]),
    "st_last_error": (ctypes.c_char_p, [_P]),
    "st_inject": (_I, [_P, _I64, _P, _P, _P, _I, _P]),
    "st_count": (_I, [_P, ctypes.POINTER(_I64)]),
    "st_step": (_I, [_P, _P, _D, _I32, _I32, _P]),
    "st_get_sources": (_I, [_P, _P, _I32, _I, _P]),
    "st_get_particles": (_I, [_P, _P, _P, _P, _P, _P, _I, _P]),
    "st_backward": (_I, [_P, _P, _P, _P, _P]),
    "st_tape_clear": (_I, [_P]),
    "st_tape_reserve": (_I, [_P, _I32, _I64]),
    "st_run_coupled": (_I, [_P, _P, _P, _I32, _D, ctypes.POINTER(ctypes.c_float),
                            ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), _P]),
    "st_stats": (_I, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                      ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64), _P]),
    "st_timing": (_I, [_P, _I32, ctypes.POINTER(_D), ctypes.POINTER(_I64)]),
    "st_ec_estimate": (_I, [_P, _I32, _P, _P, _I, _P]),
    "st_ec_reset": (_I, [_P, _P]),
    "st_hilbert_positions": (_I, [_P, _I32, _I64, _I64, _I64, _I64, _P, _P, _I32, _P]),
    "st_inject_hilbert": (_I, [_P, _I32, _I64, _I64, _I64, _I64, _P, _P, _P, _I32, _P]),
    "st_bounding_boxes": (_I, [_P, _I64, _I64, _I64, _P, _I32, _P]),
    "st_bounding_boxes_noalloc": (_I, [_P, _I64, _I64, _I64, _P, _I32, _P]),
    "st_stream_copy": (_I, [_P, _P, _I64, _P]),
}
NOALLOC_MAX_PARTS = 65536
EXTRAPOLATORS = {"zero": 0, "const": 1, "linear": 2}

_lib = None


class STError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """The loaded library (loaded on first use)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                f"g.build()'` or `python paper_2603_26691_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status, ctx=None, what=""):
    if status != ST_OK:
        msg = lib().st_last_error(ctx).decode() if ctx else what
        raise STError(status, msg or what)
