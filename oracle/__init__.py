"""ORACLE -- test infrastructure, not product code.

Plain, slow CPU implementation of the FFT-free MOT-JVIE: direct evaluation of the
interaction kernels, the excitation, the direct history sum of eq:PnMOT and the
per-step solve of eq:MOTInversion.  Only tests/, __graft_entry__.smoke() and
bench.py's cpu_baseline leg may import it.  It shares no code with the HIP library
(paper_2407_03323_amd) and never imports it.

The C parts (kquad.c, direct.c) are compiled with gcc into oracle/_build/.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, f) for f in ("kquad.c", "direct.c", "pairs.c", "klist.c")]
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")
_lib = None


def compile_oracle(force: bool = False) -> str:
    """Compile the oracle's C sources with gcc (OpenMP)."""
    os.makedirs(_BUILD, exist_ok=True)
    stale = force or not os.path.exists(_LIB) or any(
        os.path.getmtime(s) > os.path.getmtime(_LIB) for s in _SRC)
    if stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp] + _SRC + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        path = compile_oracle()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.or_kernel_entry.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, dp]
        L.or_kernel_table.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, dp]
        L.or_kernel_entry_h.argtypes = [ctypes.c_double, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, dp]
        L.or_kernel_table_h.argtypes = [ctypes.c_double, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, dp]
        L.or_kernel_list_h.argtypes = [ctypes.c_double, dp, ctypes.c_long, ctypes.POINTER(ctypes.c_int), dp,
                                       ctypes.c_int, ctypes.c_int, dp]
        L.or_conv.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp,
                              ctypes.POINTER(ctypes.c_long), ctypes.c_long, dp]
        L.or_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        ip = ctypes.POINTER(ctypes.c_int)
        L.or_conv_pairs.argtypes = [ctypes.c_double, dp, ctypes.c_int, ip, ctypes.c_long, ip, ctypes.c_long, dp,
                                    ctypes.c_int, dp]
        L.or_probe_kernels.argtypes = [ctypes.c_double, dp, ctypes.c_int, dp, ctypes.c_long, ip, ctypes.c_long,
                                       ctypes.c_int, dp]
        L.or_box_integrals.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.or_plane_integral.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int]
        L.or_plane_integral.restype = ctypes.c_double
        L.or_bspline.argtypes = [ctypes.c_double]
        L.or_bspline.restype = ctypes.c_double
        _lib = L
    return _lib


def iptr(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
