"""Vectorised, unrolled CPU code for the Lorenz RK4 ensemble (measurement
baseline for bench.py; not part of the GPU library and not the oracle).  See
lorenz_simd.c for what it does."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lorenz_simd.c")
LIB = os.path.join(HERE, "liblorenz_simd.so")
_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=gnu11", "-O3", "-Wno-psabi", "-ffp-contract=fast", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} not built: run __graft_entry__.build()")
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        L.cpu_lorenz_rk4.argtypes = [dp, dp, dp, C.c_int64, C.c_double, C.c_int64, C.c_double,
                                     C.c_double, C.c_int]
        _lib = L
    return _lib


def lorenz_rk4(P, y0, dt, nsteps, sigma, beta, nthreads=1):
    """Returns (Y [3][n], max x [n]) for rho = P[0], IC y0 [3][n]."""
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(-1)
    Y = np.array(y0, dtype=np.float64, order="C").reshape(3, P.size)
    M = np.empty(P.size)
    dp = C.POINTER(C.c_double)
    rc = lib().cpu_lorenz_rk4(P.ctypes.data_as(dp), Y.ctypes.data_as(dp), M.ctypes.data_as(dp),
                              P.size, float(dt), int(nsteps), float(sigma), float(beta),
                              int(nthreads))
    if rc:
        raise ValueError("cpu_lorenz_rk4 rejected its arguments")
    return Y, M
