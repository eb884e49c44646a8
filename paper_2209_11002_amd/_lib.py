"""ctypes declarations of the C ABI in include/edaa.h.

Loading fails loudly when libedaa.so has not been built: there is no fallback
implementation anywhere in this package.
"""
import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int, c_longlong, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libedaa.so")

EDAA_OK, EDAA_EINVAL, EDAA_ENOMEM, EDAA_EDEVICE, EDAA_ENUMERIC, EDAA_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "EDAA_OK", -1: "EDAA_EINVAL", -2: "EDAA_ENOMEM", -3: "EDAA_EDEVICE",
                -4: "EDAA_ENUMERIC", -5: "EDAA_EUNSUPPORTED"}
EDAA_X_F32, EDAA_X_BF16 = 0, 1
EDAA_COHERENCE_COSINE, EDAA_COHERENCE_RAW = 0, 1
EDAA_FLAG_GRAPH = 1
EDAA_FLAG_TIME_PASSES = 2
EDAA_FLAG_RAGGED_GROUPED = 4
EDAA_FLAG_BF16_WIDEN = 8
EDAA_FLAG_F32_MFMA = 16


class EdaaParams(ctypes.Structure):
    _fields_ = [("T", c_int), ("K1", c_int), ("K2", c_int),
                ("gamma", c_double), ("eta1", c_double), ("eta2", c_double),
                ("init_scale", c_double), ("select_threshold", c_double),
                ("x_dtype", c_int), ("coherence_mode", c_int), ("flags", c_int),
                ("runs_per_chunk", c_int), ("pixel_groups", c_int), ("tiles_per_item", c_int)]


class EdaaImageDesc(ctypes.Structure):
    _fields_ = [("X", c_void_p), ("L", c_int), ("N", c_int), ("p", c_int),
                ("seed", c_uint64), ("gamma", c_double),
                ("A", c_void_p), ("B", c_void_p), ("E", c_void_p),
                ("loss_trace", POINTER(c_double)), ("pixel_groups", c_int)]


class EdaaLaunchPlan(ctypes.Structure):
    _fields_ = [("runs_per_chunk", c_int), ("chunks", c_int), ("pixel_groups", c_int),
                ("double_buffer", c_int), ("source", c_int), ("bf16_passes", c_int)]


EDAA_PLAN_DEFAULT, EDAA_PLAN_TUNED, EDAA_PLAN_REQUESTED = 0, 1, 2

# name -> (restype, argtypes)
SIGNATURES = {
    "edaa_default_params": (None, [POINTER(EdaaParams)]),
    "edaa_create": (c_int, [POINTER(c_void_p), c_int, c_void_p]),
    "edaa_destroy": (None, [c_void_p]),
    "edaa_last_error": (ctypes.c_char_p, []),
    "edaa_last_launch_count": (c_longlong, [c_void_p]),
    "edaa_pass_times": (c_int, [c_void_p, c_int, POINTER(c_int), POINTER(c_double)]),
    "edaa_normalize_pixels": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, POINTER(c_int)]),
    "edaa_fit": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, POINTER(EdaaParams), c_uint64,
                         c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                         POINTER(c_double), POINTER(c_double)]),
    "edaa_fit_noalloc": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, POINTER(EdaaParams), c_uint64,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "edaa_abundances": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, POINTER(EdaaParams),
                                c_void_p, c_void_p, c_void_p, POINTER(c_double), POINTER(c_double)]),
    "edaa_ensemble": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, POINTER(EdaaParams), c_int,
                              POINTER(c_uint64), POINTER(c_double), c_void_p, c_void_p, c_void_p,
                              POINTER(c_double), POINTER(c_double), POINTER(c_double),
                              POINTER(c_int), POINTER(c_int)]),
    "edaa_fit_ragged": (c_int, [c_void_p, c_int, POINTER(EdaaImageDesc), POINTER(EdaaParams)]),
    "edaa_loss_fwd": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
    "edaa_loss_bwd": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p,
                              c_void_p, c_void_p]),
    "edaa_mirror_step_A": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_float]),
    "edaa_mirror_step_B": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_float]),
    "edaa_select": (c_int, [POINTER(c_double), POINTER(c_double), c_int, c_double]),
    "edaa_plan": (c_int, [c_int, c_int, c_int, c_int, POINTER(EdaaParams), POINTER(EdaaLaunchPlan)]),
    "edaa_set_graph_cache": (c_int, [c_void_p, c_int]),
    "edaa_autotune": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_int, POINTER(EdaaParams),
                              POINTER(EdaaLaunchPlan), POINTER(c_double)]),
    "edaa_autotune_ragged": (c_int, [c_void_p, c_int, POINTER(EdaaImageDesc), POINTER(EdaaParams), POINTER(c_int),
                                     POINTER(c_double)]),
}

_lib = None


def load():
    """Load libedaa.so (built by paper_2209_11002_amd/build.py) once."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'` "
                           "or `python paper_2209_11002_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class EdaaError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


def check(status):
    if status != EDAA_OK:
        raise EdaaError(status, load().edaa_last_error().decode(errors="replace"))
    return status


def default_params():
    p = EdaaParams()
    load().edaa_default_params(ctypes.byref(p))
    return p
