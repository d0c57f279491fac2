"""ctypes declarations of the C ABI in include/nbody.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnbody.so")

NB_OK = 0
NB_E_INVAL = -1
NB_E_HIP = -2
NB_E_NOMEM = -3
NB_E_NONFINITE = -4
NB_E_MISMATCH = -5
NB_E_LIMIT = -6
NB_STATIC_MAX_SYS = 256

NB_FP32_PLAIN = 0
NB_FP32_KAHAN = 1
NB_FP64 = 2
NB_L1_LOG_CAP = 4096

MODES = {"plain": NB_FP32_PLAIN, "kahan": NB_FP32_KAHAN, "fp64": NB_FP64}
NB_LAW_CONTACT = 0
NB_LAW_PAPER = 1
LAWS = {"contact": NB_LAW_CONTACT, "paper": NB_LAW_PAPER}

EXPORTED = (
    "nb_scratch_bytes",
    "nb_create",
    "nb_forces",
    "nb_step",
    "nb_step_static",
    "nb_diagnostics",
    "nb_l1_log",
    "nb_nonfinite_async",
    "nb_retention",
    "nb_sorted_order",
    "nb_resort",
    "nb_timing_enable",
    "nb_timing_read",
    "nb_timing_reset",
    "nb_tile_config",
    "nb_tile_override",
    "nb_set_force_grid",
    "nb_set_workspace_budget",
    "nb_valu_probe",
    "nb_graph_create",
    "nb_graph_launch",
    "nb_graph_destroy",
    "nb_destroy",
    "nb_strerror",
    "nb_version",
)


class NbParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("n1", ctypes.c_int64),
        ("G", ctypes.c_double),
        ("m", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("D1", ctypes.c_double),
        ("D2", ctypes.c_double),
        ("q", ctypes.c_double),
        ("a", ctypes.c_double),
        ("R2_0", ctypes.c_double),
        ("growth_rate", ctypes.c_double),
        ("growth_on", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("law", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("eps", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("beta", ctypes.c_double),
    ]


class NbBuffers(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az", "side", "scratch")] + [
        ("scratch_bytes", ctypes.c_size_t)
    ]


class NbDiag(ctypes.Structure):
    _fields_ = [
        ("com", ctypes.c_double * 3),
        ("P", ctypes.c_double * 3),
        ("L", ctypes.c_double * 3),
        ("KE", ctypes.c_double),
        ("PE", ctypes.c_double),
        ("E", ctypes.c_double),
        ("D2", ctypes.c_double),
        ("R2", ctypes.c_double),
        ("step", ctypes.c_int64),
        ("n_past_L1", ctypes.c_int32),
        ("cross_fwd", ctypes.c_int32),
        ("cross_bwd", ctypes.c_int32),
        ("growth_stopped", ctypes.c_int32),
        ("nonfinite", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


def declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    P = ctypes.POINTER
    lib.nb_scratch_bytes.argtypes = [P(NbParams), P(ctypes.c_size_t)]
    lib.nb_create.argtypes = [P(NbParams), P(NbBuffers), _vp, P(_vp)]
    lib.nb_forces.argtypes = [_vp, _vp]
    lib.nb_step.argtypes = [P(_vp), _i32, _i32, _vp]
    lib.nb_step_static.argtypes = [P(_vp), _i32, _i32, _vp]
    lib.nb_diagnostics.argtypes = [_vp, _i32, P(NbDiag), _vp]
    lib.nb_l1_log.argtypes = [_vp, P(_i32), _i32, P(_i32), _vp]
    lib.nb_nonfinite_async.argtypes = [P(_vp), _i32, P(_i32), _vp]
    lib.nb_retention.argtypes = [_vp, P(_i32), P(_i32), _vp]
    lib.nb_sorted_order.argtypes = [_vp, P(_i32), _i64, P(_i64), _vp]
    lib.nb_resort.argtypes = [_vp, _vp]
    lib.nb_timing_enable.argtypes = [_i32]
    lib.nb_timing_read.argtypes = [P(ctypes.c_double), P(_i64)]
    lib.nb_timing_reset.argtypes = []
    lib.nb_tile_config.argtypes = [_i64, _i64, _i32, _i32, P(_i32), P(_i32), P(_i32), P(_i32),
                                   P(_i32)]
    lib.nb_tile_override.argtypes = [_i64, _i64, _i32, _i32, _i32, _i32]
    lib.nb_set_force_grid.argtypes = [_i32]
    lib.nb_set_workspace_budget.argtypes = [ctypes.c_size_t]
    lib.nb_valu_probe.argtypes = [_i32, _i32, _i32, _vp, _vp, P(ctypes.c_double), P(_i64),
                                  P(ctypes.c_double)]
    lib.nb_graph_create.argtypes = [P(_vp), _i32, _i32, _vp, P(_vp)]
    lib.nb_graph_launch.argtypes = [_vp, _vp]
    lib.nb_graph_destroy.argtypes = [_vp]
    lib.nb_graph_destroy.restype = None
    lib.nb_destroy.argtypes = [_vp]
    lib.nb_destroy.restype = None
    lib.nb_strerror.argtypes = [ctypes.c_int]
    lib.nb_strerror.restype = ctypes.c_char_p
    lib.nb_version.argtypes = []
    for name in EXPORTED:
        fn = getattr(lib, name)
        if name not in ("nb_destroy", "nb_strerror", "nb_graph_destroy"):
            fn.restype = ctypes.c_int
    return lib
