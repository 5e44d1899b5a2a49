"""ctypes loader for libharp.so (the gfx950 HIP library).

The library is built in-tree by ``paper_1702_03781_amd/build.py``.  There is
no fallback: if the shared object is missing, every entry point raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libharp.so")

_lib = None

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_dbl = ctypes.c_double
c_sz = ctypes.c_size_t
c_vp = ctypes.c_void_p
c_szp = ctypes.POINTER(ctypes.c_size_t)
c_i32p = ctypes.POINTER(ctypes.c_int32)
c_dblp = ctypes.POINTER(ctypes.c_double)
c_i64p = ctypes.POINTER(ctypes.c_int64)


class HarpElement(ctypes.Structure):
    _fields_ = [("n_mbf", c_i32), ("n_samp", c_i32), ("d_samples", c_vp), ("wire_radius", c_dbl)]


class HarpRefine(ctypes.Structure):
    _fields_ = [("d_Z", c_vp), ("ldz", c_i64), ("stride_z", c_i64), ("tol", c_dbl),
                ("max_iter", c_i32), ("d_report", c_vp), ("z_complex64", c_i32)]


class HarpTuningEntry(ctypes.Structure):
    _fields_ = [("max_order", c_i32), ("panel_width_c64", c_i32), ("panel_width_c128", c_i32),
                ("small_grid_wgs", c_i32)]


class HarpRefineReport(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("converged", c_i32), ("resid_rel", c_dbl)]


# name -> (restype, argtypes); mirrors include/harp.h
SIGNATURES = {
    "harp_status_str": (ctypes.c_char_p, [c_i32]),
    "harp_version": (c_i32, []),
    "harp_model_bytes": (c_sz, [c_i32, c_i32, c_i32, c_i32]),
    "harp_fit_ws": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_szp]),
    "harp_fit": (c_i32, [ctypes.POINTER(HarpElement), c_dbl, c_i32, c_i32, c_dbl, c_i32, c_i32,
                         c_vp, c_sz, c_vp, c_sz, c_vp]),
    "harp_fill": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_i32, c_i32, c_vp, c_vp, c_i32, c_dbl, c_i32,
                          c_vp, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp, c_vp]),
    "harp_batch_plan": (c_i32, [c_i32p, c_i32, c_i32, c_i32, c_i32, c_i32, c_dblp, c_i32p, c_i32p,
                                c_i32p, c_i32p]),
    "harp_fill_systems": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_i32, c_i32, c_vp, c_vp, c_i64, c_vp, c_i32,
                                  c_i32, c_dbl, c_i32, c_vp, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp, c_vp]),
    "harp_port_rhs_systems": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_vp, c_i32, c_i32, c_i32, c_vp, c_i64,
                                      c_i64, c_vp]),
    "harp_port_admittance_systems": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_vp, c_i32, c_i32, c_i32, c_vp,
                                             c_i64, c_i64, c_vp, c_i64, c_i64, c_vp]),
    "harp_tessellate": (c_i32, [c_dblp, c_dblp, c_i32, c_dbl, c_dbl, c_dbl, c_dbl, c_i32p, c_i64p, c_i64p,
                                c_i32p, c_i32p, c_dblp]),
    "harp_port_rhs": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_i32, c_vp, c_i64, c_i64, c_vp]),
    "harp_port_admittance": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_i32, c_vp, c_i64, c_i64, c_vp,
                                     c_i64, c_i64, c_vp]),
    "harp_set_tuning": (c_i32, [ctypes.POINTER(HarpTuningEntry), c_i32]),
    "harp_get_tuning": (c_i32, [ctypes.POINTER(HarpTuningEntry), c_i32, c_i32p]),
    "harp_default_tuning": (c_i32, [c_i32, ctypes.POINTER(HarpTuningEntry)]),
    "reduced_factor_ws": (c_i32, [c_i32, c_i32, c_i32, c_szp]),
    "reduced_factor": (c_i32, [c_i32, c_i32, c_i32, c_vp, c_i64, c_i64, c_vp, c_vp, c_vp, c_sz,
                               c_vp]),
    "reduced_solve_ws": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_i32, c_szp]),
    "reduced_solve": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_vp, c_i64, c_i64, c_vp, c_vp, c_sz, c_vp, c_i64,
                              c_i64, c_vp, c_i64, c_i64, ctypes.POINTER(HarpRefine),
                              ctypes.POINTER(HarpRefineReport), c_vp, c_sz, c_vp]),
    "reduced_solve_noalloc_max_bytes": (c_sz, []),
    "reduced_solve_noalloc": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_vp, c_i64, c_i64, c_vp, c_vp, c_sz, c_vp,
                                      c_i64, c_i64, c_vp, c_i64, c_i64, ctypes.POINTER(HarpRefine),
                                      ctypes.POINTER(HarpRefineReport), c_vp]),
    "embedded_patterns_ws": (c_i32, [c_i32, c_i32, c_i32, c_szp]),
    "embedded_patterns": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_i32, c_vp, c_i64, c_i32, c_vp, c_vp,
                                  c_i32, c_vp, c_vp, c_sz, c_vp]),
    "harp_cgemm": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_i32, c_dbl, c_vp, c_i64, c_i64, c_vp,
                           c_i64, c_i64, c_dbl, c_vp, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp]),
    "harp_cmatrix_copy": (c_i32, [c_i32, c_i32, c_i32, c_vp, c_i64, c_i64, c_vp, c_i64, c_i64, c_i32,
                                  c_i32, c_vp]),
    "harp_port_admittance_vjp": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_i32, c_vp, c_i64, c_i64, c_vp,
                                         c_i64, c_i64, c_vp]),
    "harp_fill_vjp_ws": (c_i32, [c_i32, c_szp]),
    "harp_fill_vjp": (c_i32, [c_vp, c_i32, c_i32, c_vp, c_vp, c_i32, c_dbl, c_vp, c_i64, c_vp, c_vp,
                              c_vp, c_vp, c_sz, c_vp]),
    "embedded_patterns_vjp_ws": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_szp]),
    "embedded_patterns_vjp": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_i32, c_vp, c_i64, c_i32, c_vp, c_vp,
                                      c_i32, c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_sz, c_vp]),
}


# test hook (include/harp_debug.h) and kernel-class timers
# (include/harp_prof.h); neither is part of the solver boundary
DEBUG_SIGNATURES = {
    "harp_prof_enable": (c_i32, [c_i32]),
    "harp_prof_release": (c_i32, []),
    "harp_prof_read_site": (c_i32, [c_i32, c_i32, ctypes.POINTER(c_i64), ctypes.POINTER(c_dbl),
                                    ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl)]),
    "harp_prof_read": (c_i32, [c_i32, ctypes.POINTER(c_i64), ctypes.POINTER(c_dbl),
                               ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl)]),
    "harp_debug_cgemm": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_i32, c_dbl, c_vp, c_i64, c_i64, c_vp,
                                 c_i64, c_i64, c_dbl, c_vp, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp]),
}


def lib():
    """Load libharp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libharp.so not found at {LIB_PATH}: run "
                               "`python -m paper_1702_03781_amd.build` (or "
                               "__graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in {**SIGNATURES, **DEBUG_SIGNATURES}.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        # pooled profiler events are destroyed while the HIP runtime is alive
        atexit.register(L.harp_prof_release)
    return _lib


class HarpError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().harp_status_str(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


def check(status: int, where: str) -> None:
    if status != 0:
        raise HarpError(status, where)
