"""Loader for the oracle's plain-C reaction sums (test infrastructure only).

The library is compiled with gcc from ``oracle/direct.c``; if the shared object
is missing it is compiled here on first use.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "direct.c")
LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile direct.c -> liboracle.so (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_dyadic.argtypes = [ctypes.c_double] * 4 + [dp]
        L.oracle_dyadic.restype = None
        L.oracle_reaction.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, dp,
                                      ctypes.c_int, dp, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, dp]
        L.oracle_reaction.restype = None
        L.oracle_reaction_grid.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                           ctypes.c_int, dp, ctypes.c_int, dp, dp,
                                           ctypes.c_double, dp]
        L.oracle_reaction_grid.restype = None
        _lib = L
    return _lib


def ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
