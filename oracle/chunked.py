"""ctypes front end and build step for oracle/chunked.c.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

`build()` compiles two shared objects from chunked.c with gcc: the plain
one (OpenMP over points; timed as the CPU baseline) and an operation-
counting one (-DCHESSFAD_COUNT_OPS; single-threaded).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "chunked.c")
LIB_PLAIN = os.path.join(HERE, "liboracle_chunked.so")
LIB_COUNT = os.path.join(HERE, "liboracle_chunked_count.so")

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)


def build(verbose: bool = False) -> None:
    common = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas"]
    cmds = [
        common + ["-fopenmp", SRC, "-o", LIB_PLAIN, "-lm"],
        common + ["-DCHESSFAD_COUNT_OPS", SRC, "-o", LIB_COUNT, "-lm"],
    ]
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)


_libs = {}


def _lib(path):
    if path not in _libs:
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(path)
        for name in ("oracle_hvp", "oracle_hessian", "oracle_hvp_sym", "oracle_hessian_sym"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
        lib.oracle_value_grad.restype = ctypes.c_int
        if path == LIB_COUNT:
            lib.oracle_count_hvp.restype = ctypes.c_int
            lib.oracle_count_op.restype = ctypes.c_int
        _libs[path] = lib
    return _libs[path]


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _params(func, A, B, E):
    if func != 2:
        return None, None, None
    return (np.ascontiguousarray(A, np.float64), np.ascontiguousarray(B, np.float64),
            np.ascontiguousarray(E, np.float64))


def hvp(func, x, v, csize, A=None, B=None, E=None, nthreads=1, sym=False):
    """CHESS-VEC, or SC-HESS-VEC with sym=True, at every point."""
    x = np.ascontiguousarray(np.atleast_2d(x), np.float64)
    v = np.ascontiguousarray(np.atleast_2d(v), np.float64)
    npts, n = x.shape
    out = np.empty_like(x)
    A, B, E = _params(func, A, B, E)
    name = "oracle_hvp_sym" if sym else "oracle_hvp"
    rc = getattr(_lib(LIB_PLAIN), name)(func, n, ctypes.c_long(npts), _ptr(x), _ptr(v), _ptr(out), csize,
                                        _ptr(A), _ptr(B), _ptr(E), nthreads)
    if rc:
        raise ValueError(f"{name} failed: {rc}")
    return out


def hessian(func, x, csize, A=None, B=None, E=None, nthreads=1, sym=False):
    """CHUNK-HESS, or SCHUNK-HESS with sym=True, at every point."""
    x = np.ascontiguousarray(np.atleast_2d(x), np.float64)
    npts, n = x.shape
    H = np.full((npts, n, n), np.nan)
    A, B, E = _params(func, A, B, E)
    name = "oracle_hessian_sym" if sym else "oracle_hessian"
    rc = getattr(_lib(LIB_PLAIN), name)(func, n, ctypes.c_long(npts), _ptr(x), _ptr(H), csize,
                                        _ptr(A), _ptr(B), _ptr(E), nthreads)
    if rc:
        raise ValueError(f"{name} failed: {rc}")
    return H


def value_grad(func, x, csize, A=None, B=None, E=None):
    x = np.ascontiguousarray(x, np.float64).ravel()
    n = x.size
    g = np.empty(n)
    fv = ctypes.c_double()
    A, B, E = _params(func, A, B, E)
    rc = _lib(LIB_PLAIN).oracle_value_grad(func, n, _ptr(x), ctypes.byref(fv), _ptr(g), csize,
                                           _ptr(A), _ptr(B), _ptr(E))
    if rc:
        raise ValueError(f"oracle_value_grad failed: {rc}")
    return fv.value, g


def count_hvp(func, x, v, csize, A=None, B=None, E=None, sym=False):
    """(adds, muls, calls) executed by one CHESS-VEC (or SC-HESS-VEC) on one point."""
    x = np.ascontiguousarray(x, np.float64).ravel()
    v = np.ascontiguousarray(v, np.float64).ravel()
    n = x.size
    out = np.empty(n)
    adds, muls, calls = ctypes.c_long(), ctypes.c_long(), ctypes.c_long()
    A, B, E = _params(func, A, B, E)
    rc = _lib(LIB_COUNT).oracle_count_hvp(func, n, _ptr(x), _ptr(v), _ptr(out), csize, _ptr(A), _ptr(B),
                                          _ptr(E), ctypes.byref(adds), ctypes.byref(muls),
                                          ctypes.byref(calls), int(sym))
    if rc:
        raise ValueError(f"oracle_count_hvp failed: {rc}")
    return adds.value, muls.value, calls.value


def count_op(op, csize):
    """(adds, muls) of one operator application: 0 = +, 1 = x, 2 = scalar x, 3 = unary."""
    adds, muls = ctypes.c_long(), ctypes.c_long()
    rc = _lib(LIB_COUNT).oracle_count_op(op, csize, ctypes.byref(adds), ctypes.byref(muls))
    if rc:
        raise ValueError("bad op")
    return adds.value, muls.value
