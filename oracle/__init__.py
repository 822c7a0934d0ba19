"""Test oracle for EC / perimeter / area / volume curves (TEST INFRASTRUCTURE ONLY).

Two implementations of the same definition, written from the paper and
independent of the HIP library (they share no code with it, and the product
never imports this package):

* ``o1_curves`` (:mod:`oracle.ec_oracle`): binarise the field at each level
  and count cells, Eq. (1)-(2); slow, O(N * levels).
* ``o2_curves`` (``ec_oracle_o2.c``): the level at which every cubical cell
  enters the closure of the active cells, histogrammed by dimension and
  summed over levels; O(N + levels).

* ``vertex_classes_2d`` / ``vertex_classes_per_level`` and the 3D pair
  ``vertex_classes_3d`` / ``vertex_classes_3d_per_level``
  (:mod:`oracle.vertex_classes`): counts of lattice vertices per class of
  Table 1 (2D) or Table 2 (3D) at every level (the vertex-contribution map).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline
leg may import this package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .ec_oracle import curves_per_level as o1_curves  # noqa: F401
from .vertex_classes import (class_counts, vertex_classes_2d, vertex_classes_3d,  # noqa: F401
                             vertex_classes_3d_per_level, vertex_classes_per_level)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ec_oracle_o2.c")
_LIB = os.path.join(_HERE, "libecc_oracle.so")
_lib = None

_DT = {np.dtype(np.uint8): 1, np.dtype(np.uint16): 2, np.dtype(np.float32): 3}


def build_o2(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP) into oracle/libecc_oracle.so."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-Wall", "-I", _HERE, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_o2(force=False)
        lib = ctypes.CDLL(_LIB)
        f = lib.ecc_oracle_o2
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_void_p,
                      ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_int]
        g = lib.ecc_oracle_compute
        g.restype = ctypes.c_int
        g.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
        _lib = lib
    return _lib


def o2_curves(field, n_levels: int, thresholds=None, connectivity=None,
              channels=("ec", "perimeter", "area", "volume"), n_threads: int = 1, superlevel: bool = False):
    """All-levels oracle.  Returns dict channel -> int64 curve of length n_levels.

    2D channels: ec, perimeter, area.  3D: ec, perimeter (crease), area
    (surface), volume.  ``superlevel``: sets {value >= t_l} over
    non-increasing thresholds (integer levels t_l = n_levels - 1 - l).
    """
    lib = _load()
    field = np.ascontiguousarray(field)
    if field.dtype not in _DT:
        raise TypeError(f"unsupported dtype {field.dtype}")
    nd = field.ndim
    if connectivity is None:
        connectivity = 8 if nd == 2 else 26
    shape = (ctypes.c_int64 * 3)(*field.shape)
    thr = None
    if thresholds is not None:
        thr = np.ascontiguousarray(thresholds, dtype=np.float32)
    want = [c for c in channels if not (nd == 2 and c == "volume")]
    out = {c: np.zeros(n_levels, dtype=np.int64) for c in want}

    def ptr(c):
        return out[c].ctypes.data if c in out else None

    rc = lib.ecc_oracle_o2(nd, shape, _DT[field.dtype], field.ctypes.data, int(n_levels),
                           thr.ctypes.data if thr is not None else None, int(connectivity),
                           1 if superlevel else 0, ptr("ec"), ptr("perimeter"), ptr("area"), ptr("volume"),
                           int(n_threads))
    if rc != 0:
        raise ValueError(f"ecc_oracle_o2 rejected the arguments (code {rc})")
    return out
