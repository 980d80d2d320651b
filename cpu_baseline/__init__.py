"""Multithreaded CPU exact DPC (``dpc_cpu.cpp``): the speed baseline that
``bench.py`` times on the host cores beside the GPU library.

It is neither the oracle nor part of the GPU path and shares no code with
either; the CPU tests check it against the oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dpc_cpu.cpp")
LIB = os.path.join(HERE, "_build", "libdpc_cpu.so")

_lib = None


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O3", "-std=c++17", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread", SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is not built: run __graft_entry__.build() first")
        lib = ctypes.CDLL(LIB)
        P, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.dpc_cpu_run.argtypes = [P, i64, i32, dbl, i32, dbl, i32, P, P, P, P]
        lib.dpc_cpu_run.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads_available() -> int:
    """Host threads this process may use (affinity mask, capped by OMP_NUM_THREADS when set)."""
    n = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return n


def run(points, d_cut: float, rho_min: int, delta_min: float, threads: int = 0):
    """(rho, dep, delta2, label) as numpy arrays; threads 0 = threads_available()."""
    p = np.ascontiguousarray(points, dtype=np.int32)
    n, d = p.shape
    rho = np.empty(n, np.int32)
    dep = np.empty(n, np.int32)
    d2 = np.empty(n, np.int64)
    lab = np.empty(n, np.int32)
    t = threads if threads > 0 else threads_available()
    st = _load().dpc_cpu_run(p.ctypes.data, n, d, float(d_cut), int(rho_min), float(delta_min), t, rho.ctypes.data,
                             dep.ctypes.data, d2.ctypes.data, lab.ctypes.data)
    if st != 0:
        raise RuntimeError(f"dpc_cpu_run failed with status {st}")
    return rho, dep, d2, lab
