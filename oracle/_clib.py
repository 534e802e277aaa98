"""Loads (building on first use) the oracle's plain-C FP64 code (geom.c, refine.c).

TEST INFRASTRUCTURE ONLY: imported by the oracle package, which only the
tests, the smoke check and the benchmark's CPU-baseline leg may use.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "geom.c"), os.path.join(_HERE, "refine.c")]
_LIB = os.path.join(_HERE, "_build", "liboracle_geom.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle's C files with gcc (no fast-math: IEEE double semantics;
    OpenMP only splits independent probe poses across threads)."""
    newest = max(os.path.getmtime(f) for f in _SRCS)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        os.makedirs(os.path.dirname(_LIB), exist_ok=True)
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared",
                               "-fPIC", "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        d, i, p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        L.orc_probe_sdf.restype = d
        L.orc_probe_sdf.argtypes = [d, d, d, d, d]
        L.orc_point_tri_dist2.restype = d
        L.orc_point_tri_dist2.argtypes = [p, p, p, p]
        L.orc_solid_angle.restype = d
        L.orc_solid_angle.argtypes = [p, p, p, p]
        L.orc_object_points.restype = None
        L.orc_object_points.argtypes = [p, i, p, i, p, p, i, d, d, d, p, p, p]
        L.orc_object_grid.restype = None
        L.orc_object_grid.argtypes = [p, i, p, i, p, i, d, p, d, d, d, d, p, p, p]
        L.orc_swept_points.restype = None
        L.orc_swept_points.argtypes = [p, i, d, d, p, i, p]
        L.orc_swept_lattice.restype = None
        L.orc_swept_lattice.argtypes = [p, i, d, d, i, d, p, d, p]
        L.orc_face_min.restype = d
        L.orc_face_min.argtypes = [p, p, p, d, d, d, p, p]
        L.orc_distance_query.restype = None
        L.orc_distance_query.argtypes = [p, p, i, p, p, p, p, p, i, d, d, d, d, p, p, p, p]
        _lib = L
    return _lib


def ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None
