"""ctypes view of include/plv.h.  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os
import threading

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libplv.so")

PLV_OK = 0
STATUS = {0: "PLV_OK", 1: "PLV_ERR_INVALID_ARG", 2: "PLV_ERR_WORKSPACE", 3: "PLV_ERR_DEVICE",
          4: "PLV_ERR_UNSUPPORTED"}
PREC = {"f64": 0, "f32": 1, "split_bf16": 2, "bf16": 3, "f16": 4}
INPUT_ANALYTIC, INPUT_REAL = 0, 1
OP_FROM_ANALYTIC, OP_FROM_REAL, OP_BACKWARD_ANALYTIC, OP_BACKWARD_REAL, OP_COHERENCE = 0, 1, 2, 3, 4
NOALLOC_MAX_BYTES = 64 << 20  # PLV_NOALLOC_MAX_BYTES


class Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("t", C.c_int64), ("ld", C.c_int64), ("t0", C.c_int64), ("t1", C.c_int64),
                ("in_", C.c_void_p), ("plv", C.c_void_p), ("iplv", C.c_void_p), ("ciplv", C.c_void_p),
                ("g", C.c_void_p)]


class Trials(C.Structure):
    _fields_ = [("n", C.c_int64), ("ntr", C.c_int64), ("t", C.c_int64), ("ld", C.c_int64),
                ("tstride", C.c_int64), ("sstride", C.c_int64), ("t0", C.c_int64), ("t1", C.c_int64),
                ("in_", C.c_void_p), ("plv", C.c_void_p), ("iplv", C.c_void_p), ("ciplv", C.c_void_p),
                ("g", C.c_void_p)]


class Band(C.Structure):
    _fields_ = [("f_lo", C.c_double), ("f_hi", C.c_double), ("fir_order", C.c_int32), ("reserved", C.c_int32)]


class Stft(C.Structure):
    _fields_ = [("seg", C.c_int32), ("hop", C.c_int32), ("k_lo", C.c_int32), ("k_hi", C.c_int32),
                ("window", C.c_int32), ("reserved", C.c_int32)]


WINDOW = {"hamming": 0, "hann": 1, "rect": 2}


class Grad(C.Structure):
    _fields_ = [("dplv", C.c_void_p), ("diplv", C.c_void_p), ("dciplv", C.c_void_p), ("din", C.c_void_p)]


# every symbol include/plv.h declares
EXPORTS = ("plv_create", "plv_destroy", "plv_status_str", "plv_last_error", "plv_version",
           "plv_timing_enable", "plv_timing_read", "plv_timing_list",
           "plv_workspace_size", "plv_from_analytic", "plv_from_analytic_noalloc", "plv_from_real", "plv_coherence",
           "plv_trials_workspace_size", "plv_over_trials", "plv_backward", "plv_autotune",
           "plv_tile_edge", "plv_set_tile_edge", "plv_coherence_stft_workspace_size", "plv_coherence_stft")

STAGES = ("hilbert", "normalise", "gram", "epilogue", "backward", "stft")
NSTAGES = 8


class Timing(C.Structure):
    _fields_ = [("ms", C.c_double * NSTAGES), ("calls", C.c_int64 * NSTAGES), ("launches", C.c_int64 * NSTAGES)]

_LIB = None
_LOCK = threading.Lock()


class LibraryMissing(ImportError):
    pass


def lib():
    """The loaded libplv.so.  Raises LibraryMissing when it has not been built:
    there is no fallback path."""
    global _LIB
    with _LOCK:
        if _LIB is None:
            if not os.path.exists(LIB_PATH):
                raise LibraryMissing("libplv.so is not built (%s); run `python -m paper_1710_08037_amd.build`"
                                     % LIB_PATH)
            L = C.CDLL(LIB_PATH)
            P = C.c_void_p
            L.plv_create.argtypes = [C.POINTER(P), C.c_int]
            L.plv_create.restype = C.c_int
            L.plv_destroy.argtypes = [P]
            L.plv_destroy.restype = C.c_int
            L.plv_status_str.argtypes = [C.c_int]
            L.plv_status_str.restype = C.c_char_p
            L.plv_last_error.argtypes = [P]
            L.plv_last_error.restype = C.c_char_p
            L.plv_version.argtypes = []
            L.plv_version.restype = C.c_int32
            L.plv_timing_enable.argtypes = [P, C.c_int32]
            L.plv_timing_enable.restype = C.c_int
            L.plv_timing_read.argtypes = [P, C.POINTER(Timing), C.c_int32]
            L.plv_timing_read.restype = C.c_int
            L.plv_timing_list.argtypes = [P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int64,
                                          C.POINTER(C.c_int64)]
            L.plv_timing_list.restype = C.c_int
            L.plv_workspace_size.argtypes = [P, C.c_int, C.c_int, C.POINTER(Problem), C.c_int64, C.POINTER(Band),
                                             C.c_int32, C.POINTER(C.c_size_t)]
            L.plv_workspace_size.restype = C.c_int
            L.plv_from_analytic.argtypes = [P, C.c_int, C.POINTER(Problem), C.c_int64, P, C.c_size_t, P]
            L.plv_from_analytic.restype = C.c_int
            L.plv_from_analytic_noalloc.argtypes = [P, C.c_int, C.POINTER(Problem), C.c_int64, P]
            L.plv_from_analytic_noalloc.restype = C.c_int
            L.plv_coherence.argtypes = [P, C.c_int, C.POINTER(Problem), C.c_int64, P, C.c_size_t, P]
            L.plv_coherence.restype = C.c_int
            L.plv_trials_workspace_size.argtypes = [P, C.c_int, C.POINTER(Trials), C.POINTER(C.c_size_t)]
            L.plv_trials_workspace_size.restype = C.c_int
            L.plv_over_trials.argtypes = [P, C.c_int, C.POINTER(Trials), P, C.c_size_t, P]
            L.plv_over_trials.restype = C.c_int
            L.plv_from_real.argtypes = [P, C.c_int, C.POINTER(Problem), C.c_int64, C.POINTER(Band), C.c_int32,
                                        C.c_double, P, C.c_size_t, P]
            L.plv_from_real.restype = C.c_int
            L.plv_backward.argtypes = [P, C.c_int, C.c_int, C.POINTER(Problem), C.POINTER(Grad), C.c_int64,
                                       C.POINTER(Band), C.c_int32, C.c_double, P, C.c_size_t, P]
            L.plv_backward.restype = C.c_int
            L.plv_autotune.argtypes = [P, C.c_int, C.c_int, C.POINTER(Problem), C.c_int64, C.POINTER(Band), C.c_int32,
                                       C.c_double, P, C.c_size_t, P, C.POINTER(C.c_int32)]
            L.plv_autotune.restype = C.c_int
            L.plv_coherence_stft_workspace_size.argtypes = [P, C.c_int, C.POINTER(Problem), C.c_int64,
                                                            C.POINTER(Stft), C.POINTER(C.c_size_t)]
            L.plv_coherence_stft_workspace_size.restype = C.c_int
            L.plv_coherence_stft.argtypes = [P, C.c_int, C.POINTER(Problem), C.c_int64, C.POINTER(Stft), P,
                                             C.c_size_t, P]
            L.plv_coherence_stft.restype = C.c_int
            L.plv_tile_edge.argtypes = [P, C.c_int, C.c_int64, C.POINTER(C.c_int32)]
            L.plv_tile_edge.restype = C.c_int
            L.plv_set_tile_edge.argtypes = [P, C.c_int, C.c_int64, C.c_int32]
            L.plv_set_tile_edge.restype = C.c_int
            _LIB = L
    return _LIB


class PLVError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


def check(status: int, ctx=None):
    if status != PLV_OK:
        msg = lib().plv_last_error(ctx).decode() if ctx else ""
        if not msg:
            msg = lib().plv_status_str(status).decode()
        raise PLVError(status, msg)


def problems(items) -> C.Array:
    arr = (Problem * len(items))()
    for k, p in enumerate(items):
        arr[k] = p
    return arr


def bands(pairs):
    if pairs is None:
        return None, 1
    arr = (Band * len(pairs))()
    for k, band in enumerate(pairs):
        lo, hi = band[0], band[1]
        order = int(band[2]) if len(band) > 2 and band[2] else 0
        arr[k] = Band(float(lo), float(hi), order, 0)
    return arr, len(pairs)
