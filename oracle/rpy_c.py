"""Compiled FP64 route of the oracle's blob mobility (Sec. 2.3, Eq. RPY):
ctypes binding of rpy_sum.c (plain C loops, OpenMP over targets).

TEST INFRASTRUCTURE ONLY.  Built by ``build()`` (gcc, -O2, no fast-math) into
oracle/librpy_oracle.so; ``__graft_entry__.build()`` calls it.  Loading fails
loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "librpy_oracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "rpy_sum.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=HERE)
    if r.returncode != 0:
        raise RuntimeError("gcc failed on the oracle:\n" + r.stderr[-4000:])
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: build it with oracle.rpy_c.build()")
        lib = C.CDLL(LIB)
        D = C.POINTER(C.c_double)
        I = C.POINTER(C.c_int)
        lib.oracle_rpy_apply.restype = C.c_int
        lib.oracle_rpy_apply.argtypes = [C.c_int, D, D, C.c_double, C.c_double, C.c_int,
                                         C.c_int, I, D, C.c_int]
        lib.oracle_rpy_matrix.restype = C.c_int
        lib.oracle_rpy_matrix.argtypes = [C.c_int, D, C.c_double, C.c_double, C.c_int, D,
                                          C.c_int]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def mobility_apply(pos, lam, a, eta, wall, targets=None, threads=0, return_threads=False):
    """u_i = sum_j M_ij lam_j over every source, for the target rows given (all by
    default); (len(targets), 3).  threads = 0: OpenMP's default (all cores)."""
    pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
    lam = np.ascontiguousarray(lam, np.float64).reshape(-1, 3)
    n = len(pos)
    if lam.shape != pos.shape:
        raise ValueError("lam must have one 3-vector per blob")
    if wall and np.any(pos[:, 2] <= a):
        raise ValueError("blob at or below z = a with a no-slip wall")
    tg = None if targets is None else np.ascontiguousarray(targets, np.int32)
    nt = n if tg is None else len(tg)
    if tg is not None and nt and (tg.min() < 0 or tg.max() >= n):
        raise ValueError("target index out of range")
    u = np.zeros((nt, 3))
    used = load().oracle_rpy_apply(
        n, _dp(pos), _dp(lam), float(a), float(eta), int(bool(wall)), nt,
        None if tg is None else tg.ctypes.data_as(C.POINTER(C.c_int)), _dp(u), int(threads))
    return (u, used) if return_threads else u


def mobility_matrix(pos, a, eta, wall, threads=0):
    """Dense 3N x 3N blob mobility, xyz interleaved per blob."""
    pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
    n = len(pos)
    if wall and np.any(pos[:, 2] <= a):
        raise ValueError("blob at or below z = a with a no-slip wall")
    Mm = np.empty((3 * n, 3 * n))
    load().oracle_rpy_matrix(n, _dp(pos), float(a), float(eta), int(bool(wall)), _dp(Mm),
                             int(threads))
    return Mm
