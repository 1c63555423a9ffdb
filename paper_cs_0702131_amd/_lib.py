"""ctypes binding of libaica.so (argument marshalling only; every step runs in the HIP library)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libaica.so")

AICA_OK = 0
AICA_E_INVAL = -1
AICA_E_MESH = -2
AICA_E_RCUT = -3
AICA_E_UNLOCATED = -4
AICA_E_NOMEM = -5
AICA_E_HIP = -6
AICA_FP32 = 1
AICA_FP64 = 2

ERROR_NAMES = {AICA_E_INVAL: "AICA_E_INVAL", AICA_E_MESH: "AICA_E_MESH", AICA_E_RCUT: "AICA_E_RCUT",
               AICA_E_UNLOCATED: "AICA_E_UNLOCATED", AICA_E_NOMEM: "AICA_E_NOMEM", AICA_E_HIP: "AICA_E_HIP"}

AICA_DIL_CLOSEST = 0
AICA_DIL_VERTEX = 1

EXPORTED = ["aica_build_dil", "aica_build_dil_ex", "aica_bin", "aica_forces", "aica_forces_noalloc",
            "aica_forces_adjoint", "aica_dil_export", "aica_pairs_export", "aica_pair_counts", "aica_bin_export",
            "aica_dil_info", "aica_work_stats", "aica_profile", "aica_profile_read", "aica_last_error",
            "aica_dil_free"]


class AicaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class aica_mesh(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("points", C.c_void_p), ("n_faces", C.c_int64),
                ("face_off", C.c_void_p), ("face_pts", C.c_void_p), ("owner", C.c_void_p),
                ("neighbour", C.c_void_p), ("n_cells", C.c_int64), ("n_periodic", C.c_int32),
                ("periodic_vec", (C.c_double * 3) * 3), ("periodic_rot", C.c_void_p)]


class aica_params(C.Structure):
    _fields_ = [("rcut", C.c_double), ("n_species", C.c_int32), ("eps", C.c_void_p), ("sigma", C.c_void_p),
                ("precision", C.c_int32), ("compensated", C.c_int32)]


class aica_info(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_dil", C.c_int64), ("n_groups", C.c_int64),
                ("n_group_pairs", C.c_int64), ("n_molecules", C.c_int64), ("n_jslots", C.c_int64),
                ("mesh_volume", C.c_double), ("build_seconds", C.c_double), ("group_seconds", C.c_double),
                ("lane_steps", C.c_int64), ("located_ball", C.c_int64), ("located_record", C.c_int64),
                ("located_search", C.c_int64)]


_lib = None


def lib():
    """Load libaica.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the HIP library is required; there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        p, i64, i32, f64 = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.aica_build_dil.argtypes = [C.POINTER(aica_mesh), f64, f64, C.POINTER(p)]
        L.aica_build_dil_ex.argtypes = [C.POINTER(aica_mesh), f64, f64, i32, C.POINTER(p)]
        L.aica_bin.argtypes = [p, p, i32, i64, p]
        L.aica_forces.argtypes = [p, p, p, C.POINTER(aica_params), p, p, p, p]
        L.aica_forces_noalloc.argtypes = [p, p, p, C.POINTER(aica_params), p, p, p, p]
        L.aica_forces_adjoint.argtypes = [p, p, p, C.POINTER(aica_params), p, f64, p, p, p, p]
        L.aica_dil_export.argtypes = [p, p, p, p, p]
        L.aica_pairs_export.argtypes = [p, p, C.POINTER(aica_params), i64, p, p, p, p, p]
        L.aica_pair_counts.argtypes = [p, p, C.POINTER(aica_params), p, p]
        L.aica_bin_export.argtypes = [p, p, p, p]
        L.aica_dil_info.argtypes = [p, C.POINTER(aica_info)]
        L.aica_work_stats.argtypes = [p, p, p]
        L.aica_profile.argtypes = [p, i32]
        L.aica_profile_read.argtypes = [p, C.c_char_p, p, p, i32]
        L.aica_last_error.restype = C.c_char_p
        L.aica_dil_free.argtypes = [p]
        L.aica_dil_free.restype = None
        for name in EXPORTED:
            if name not in ("aica_last_error", "aica_dil_free"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(rc):
    if rc != AICA_OK:
        raise AicaError(rc, lib().aica_last_error().decode())
    return rc


def ptr(a):
    return C.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else C.c_void_p(a)
