"""Build and load the oracle's plain-C pair-integral library (test infrastructure).

``build()`` compiles oracle/pairs.c with gcc (-O2, OpenMP, no fast-math) into oracle/_pairs.so.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pairs.c")
LIB = os.path.join(HERE, "_pairs.so")

_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                               "-std=c11", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        i64 = ctypes.c_int64
        ci = ctypes.c_int
        L.oracle_pair_integrals.argtypes = [dp, ip, dp, dp, ci, dp, dp, i64, ip, dp]
        L.oracle_I_rows.argtypes = [dp, ip, i64, dp, dp, ci, dp, dp, i64, i64, dp]
        L.oracle_W.argtypes = [dp, ip, i64, dp, dp, ci, dp, dp, i64, lp, lp, dp, lp, lp, dp, i64, dp]
        L.oracle_W_rows.argtypes = [dp, ip, i64, dp, dp, ci, dp, dp, i64, lp, lp, dp, lp, lp, dp, i64, lp, dp]
        L.oracle_W_accumulate.argtypes = [i64, i64, lp, lp, dp, lp, lp, dp, i64, i64, dp, i64, i64, dp]
        L.oracle_near_generic.argtypes = [ci, dp, dp, ci, dp, dp, ci]
        L.oracle_near_generic.restype = ctypes.c_double
        L.oracle_far_pair.argtypes = [dp, dp, dp, dp, dp, dp, dp, dp, ci]
        L.oracle_far_pair.restype = ctypes.c_double
        _lib = L
    return _lib


def dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def iptr(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def lptr(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
