"""ctypes binding of libmtp.so (argument marshalling only; every step runs in the library)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmtp.so")

MTP_OK = 0
MTP_ERR_ARG = 1
MTP_ERR_CELL = 2
MTP_ERR_CAPACITY = 3
MTP_ERR_NONFINITE = 4
MTP_ERR_HIP = 5
MTP_ERR_OOM = 6
MTP_ERR_LEVEL = 7
MTP_GRADE_BREAK = 8
MTP_GRADE_SELECT = 9

MTP_FP64 = 0
MTP_FP32_MOMENTS = 1
MTP_GRADE_FP64 = 0
MTP_GRADE_FP32SPLIT = 1

EXPORTS = ("mtp_batch_create", "mtp_batch_run", "mtp_batch_vjp", "mtp_batch_tune", "mtp_batch_schedule", "mtp_batch_sizes",
           "mtp_batch_neighbors", "mtp_batch_destroy", "mtp_levels", "mtp_level_info", "mtp_profile", "mtp_profile_read", "mtp_profile_reset", "mtp_create", "mtp_destroy", "mtp_last_error", "mtp_sizes", "mtp_set_params",
           "mtp_neighbors", "mtp_compute", "mtp_compute_static", "mtp_grade", "mtp_grade_config", "mtp_param_grad", "mtp_maxvol")

c_double_p = ctypes.POINTER(ctypes.c_double)


class MtpParams(ctypes.Structure):
    _fields_ = [
        ("level", ctypes.c_int),
        ("n_species", ctypes.c_int),
        ("n_cheb", ctypes.c_int),
        ("r_min", ctypes.c_double),
        ("r_cut", ctypes.c_double),
        ("radial", c_double_p),
        ("linear", c_double_p),
        ("shift", c_double_p),
        ("precision", ctypes.c_int),
        ("chunk_atoms", ctypes.c_int),
        ("grade_select", ctypes.c_double),
        ("grade_break", ctypes.c_double),
        ("lanes_per_atom", ctypes.c_int),
    ]


class MtpSystem(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int),
        ("pos", ctypes.c_void_p),
        ("species", ctypes.c_void_p),
        ("cell", ctypes.c_double * 9),
    ]


class MtpNlist(ctypes.Structure):
    _fields_ = [
        ("off", ctypes.c_void_p),
        ("j", ctypes.c_void_p),
        ("shift", ctypes.c_void_p),
        ("rev", ctypes.c_void_p),
        ("n_pairs", ctypes.c_longlong),
        ("checked", ctypes.c_int),
    ]


class MtpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmtp error {code}: {msg}")
        self.code = code


_LIB = None


def load():
    """The process-wide libmtp.so handle; raises if the library has not been built."""
    global _LIB
    if _LIB is None:
        _LIB = open_library(LIB_PATH)
    return _LIB


def open_library(path: str):
    """Open and type one copy of the library (there is no fallback when it is missing)."""
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2510_00193_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i, ll, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_double
    lib.mtp_levels.argtypes = [ctypes.POINTER(i), ctypes.POINTER(i)]
    lib.mtp_level_info.argtypes = [i, ctypes.POINTER(i), i]
    lib.mtp_profile.argtypes = [vp, i]
    lib.mtp_profile_reset.argtypes = [vp]
    lib.mtp_profile_read.argtypes = [vp, i, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(d), ctypes.POINTER(ll)]
    lib.mtp_create.argtypes = [ctypes.POINTER(MtpParams), ctypes.POINTER(vp)]
    lib.mtp_destroy.argtypes = [vp]
    lib.mtp_destroy.restype = None
    lib.mtp_last_error.restype = ctypes.c_char_p
    lib.mtp_sizes.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]
    lib.mtp_set_params.argtypes = [vp, vp, vp, vp, i, vp]
    lib.mtp_neighbors.argtypes = [vp, ctypes.POINTER(MtpSystem), vp, vp, vp, vp, ll, ctypes.POINTER(ll), vp]
    lib.mtp_compute.argtypes = [vp, ctypes.POINTER(MtpSystem), ctypes.POINTER(MtpNlist), vp, vp, vp, vp, vp]
    lib.mtp_compute_static.argtypes = [vp, ctypes.POINTER(MtpSystem), ctypes.POINTER(MtpNlist), vp, vp, vp, vp,
                                       vp]
    if hasattr(lib, "mtp_grade"):
        lib.mtp_grade.argtypes = [vp, ctypes.POINTER(MtpSystem), ctypes.POINTER(MtpNlist), vp, i, vp, vp, vp]
    if hasattr(lib, "mtp_grade_config"):
        lib.mtp_grade_config.argtypes = [vp, ctypes.POINTER(MtpSystem), ctypes.POINTER(MtpNlist), vp, vp, vp, vp]
    if hasattr(lib, "mtp_param_grad"):
        lib.mtp_param_grad.argtypes = [vp, ctypes.POINTER(MtpSystem), ctypes.POINTER(MtpNlist), d, vp, vp, vp,
                                       vp, vp]
    lib.mtp_maxvol.argtypes = [vp, vp, i, i, vp, vp, d, i, ctypes.POINTER(i), c_double_p, ctypes.POINTER(i), vp]
    lib.mtp_maxvol.restype = ctypes.c_int
    lib.mtp_batch_create.argtypes = [vp, i, ctypes.POINTER(i), vp, vp, c_double_p, ctypes.POINTER(vp), vp]
    lib.mtp_batch_run.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i, vp]
    lib.mtp_batch_vjp.argtypes = [vp, vp, vp, vp, vp, vp, i, vp]
    lib.mtp_batch_tune.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(i), vp]
    lib.mtp_batch_schedule.argtypes = [vp, i, i, i]
    lib.mtp_batch_sizes.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(ll), ctypes.POINTER(i), ctypes.POINTER(i),
                                    ctypes.POINTER(i)]
    lib.mtp_batch_neighbors.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                        ctypes.POINTER(vp)]
    lib.mtp_batch_destroy.argtypes = [vp]
    lib.mtp_batch_destroy.restype = None
    for name in ("mtp_batch_create", "mtp_batch_run", "mtp_batch_vjp", "mtp_batch_tune", "mtp_batch_schedule", "mtp_batch_sizes",
                 "mtp_batch_neighbors"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("mtp_levels", "mtp_level_info", "mtp_profile", "mtp_profile_read", "mtp_profile_reset",
                 "mtp_create", "mtp_sizes", "mtp_set_params", "mtp_neighbors", "mtp_compute",
                 "mtp_compute_static", "mtp_grade", "mtp_grade_config", "mtp_param_grad"):
        if hasattr(lib, name):
            getattr(lib, name).restype = ctypes.c_int
    return lib


def check(code, allowed=(MTP_OK,)):
    if code not in allowed:
        msg = load().mtp_last_error()
        raise MtpError(code, msg.decode() if msg else "")
    return code
