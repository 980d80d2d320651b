"""Plain CPU oracle for exact Density Peaks Clustering.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library and never imports it.

``dpc_oracle.c`` is the paper's Definitions 1-5 (Section 3) and the
single-linkage assignment of Algorithm 3 (Section 6.2) written out as O(n^2)
loops over exact 128-bit integer distances.  ``ref.py`` is a second, pure
Python version for tiny inputs.  This module wraps the C file through ctypes.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

OK, ERR_INVALID_ARG, ERR_RANGE, ERR_NOT_FOREST = 0, 1, 2, 3
INF = (1 << 63) - 1

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    P = ctypes.c_void_p
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.oracle_square_threshold.argtypes = [dbl, ctypes.c_int, P]
    lib.oracle_range_ok.argtypes = [P, i64, i32]
    lib.oracle_density.argtypes = [P, i64, i32, i64, P]
    lib.oracle_density.restype = None
    lib.oracle_density_at.argtypes = [P, i64, i32, i64, P, i64, P]
    lib.oracle_density_at.restype = None
    lib.oracle_dependent.argtypes = [P, i64, i32, P, i32, i32, P, P]
    lib.oracle_dependent.restype = None
    lib.oracle_dependent_at.argtypes = [P, i64, i32, P, P, i64, P, P]
    lib.oracle_dependent_at.restype = None
    lib.oracle_cluster.argtypes = [i64, P, P, P, i32, i64, P]
    lib.oracle_run.argtypes = [P, i64, i32, dbl, i32, dbl, i32, P, P, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _points(points) -> np.ndarray:
    p = np.ascontiguousarray(points, dtype=np.int32)
    if p.ndim != 2:
        raise ValueError("points must be [n, d]")
    return p


def square_threshold(r: float, round_up: bool = False) -> int:
    out = np.zeros(1, np.int64)
    st = _load().oracle_square_threshold(float(r), int(bool(round_up)), _ptr(out))
    if st != OK:
        raise ValueError(f"invalid radius {r!r}")
    return int(out[0])


def delta_threshold(delta_min: float) -> int:
    if delta_min != delta_min:
        raise ValueError("delta_min is NaN")
    if delta_min <= 0:
        return 0
    return square_threshold(delta_min, True)


def range_ok(points) -> bool:
    p = _points(points)
    return bool(_load().oracle_range_ok(_ptr(p), p.shape[0], p.shape[1]))


def density(points, T: int) -> np.ndarray:
    p = _points(points)
    rho = np.zeros(p.shape[0], np.int32)
    _load().oracle_density(_ptr(p), p.shape[0], p.shape[1], int(T), _ptr(rho))
    return rho


def density_at(points, T: int, queries) -> np.ndarray:
    p = _points(points)
    q = np.ascontiguousarray(queries, dtype=np.int64)
    out = np.zeros(q.shape[0], np.int32)
    _load().oracle_density_at(_ptr(p), p.shape[0], p.shape[1], int(T), _ptr(q), q.shape[0], _ptr(out))
    return out


def dependent(points, rho, rho_min: int = 0, skip_noise: bool = False):
    p = _points(points)
    r = np.ascontiguousarray(rho, dtype=np.int32)
    dep = np.zeros(p.shape[0], np.int32)
    d2 = np.zeros(p.shape[0], np.int64)
    _load().oracle_dependent(_ptr(p), p.shape[0], p.shape[1], _ptr(r), int(rho_min),
                             int(bool(skip_noise)), _ptr(dep), _ptr(d2))
    return dep, d2


def dependent_at(points, rho, queries):
    p = _points(points)
    r = np.ascontiguousarray(rho, dtype=np.int32)
    q = np.ascontiguousarray(queries, dtype=np.int64)
    dep = np.zeros(q.shape[0], np.int32)
    d2 = np.zeros(q.shape[0], np.int64)
    _load().oracle_dependent_at(_ptr(p), p.shape[0], p.shape[1], _ptr(r), _ptr(q), q.shape[0],
                                _ptr(dep), _ptr(d2))
    return dep, d2


def cluster(rho, dep, delta2, rho_min: int, Td: int) -> np.ndarray:
    r = np.ascontiguousarray(rho, dtype=np.int32)
    dp = np.ascontiguousarray(dep, dtype=np.int32)
    d2 = np.ascontiguousarray(delta2, dtype=np.int64)
    lab = np.zeros(r.shape[0], np.int32)
    st = _load().oracle_cluster(r.shape[0], _ptr(r), _ptr(dp), _ptr(d2), int(rho_min), int(Td), _ptr(lab))
    if st == ERR_NOT_FOREST:
        raise ValueError("not a dependent forest")
    return lab


def run(points, d_cut: float, rho_min: int, delta_min: float, skip_noise: bool = False):
    """(rho, dep, delta2, label) of the whole method, or ValueError on a bad input."""
    p = _points(points)
    n = p.shape[0]
    rho = np.zeros(n, np.int32)
    dep = np.zeros(n, np.int32)
    d2 = np.zeros(n, np.int64)
    lab = np.zeros(n, np.int32)
    st = _load().oracle_run(_ptr(p), n, p.shape[1], float(d_cut), int(rho_min), float(delta_min),
                            int(bool(skip_noise)), _ptr(rho), _ptr(dep), _ptr(d2), _ptr(lab))
    if st != OK:
        raise ValueError(f"oracle status {st}")
    return rho, dep, d2, lab
