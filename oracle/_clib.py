"""Build and load the oracle's plain C loops (gcc -O2 -fopenmp, no fast-math).

Test infrastructure only; see the package docstring.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dsbi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_dsbi.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle C file into ``liboracle_dsbi.so`` next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        d = ctypes.c_double
        i64 = ctypes.c_int64
        p = ctypes.c_void_p
        L.orc_green.argtypes = [p, p, p, p, d, p]
        L.orc_kernels.argtypes = [p, p, p, p, d, d, p]
        L.orc_matvec.argtypes = [i64, p, p, p, d, d, p, p, i64, p, p, p, p, p]
        L.orc_matvec_t.argtypes = [i64, p, p, p, d, d, p, p, i64, p, p, p, p, p]
        L.orc_assemble.argtypes = [i64, p, p, p, d, d, p]
        L.orc_assemble_subset.argtypes = [i64, p, p, p, d, d, i64, p, p]
        L.orc_source.argtypes = [i64, p, p, i64, p, p, d, i64, p, p, p]
        L.orc_reaction.argtypes = [i64, p, p, p, d, d, p, p, i64, p, p, p]
        L.orc_adjoint_rhs.argtypes = [i64, p, p, p, d, d, i64, p, p, p, p]
        L.orc_source_adjoint.argtypes = [i64, p, p, d, p, p, i64, p, p, p]
        L.orc_coulomb.argtypes = [i64, p, i64, p, p, d, ctypes.c_int, p]
        for f in (L.orc_green, L.orc_kernels, L.orc_matvec, L.orc_matvec_t, L.orc_assemble,
                  L.orc_assemble_subset,
                  L.orc_source, L.orc_reaction, L.orc_adjoint_rhs, L.orc_source_adjoint,
                  L.orc_coulomb):
            f.restype = None
        _lib = L
    return _lib


def ptr(a):
    """Pointer to a C-contiguous float64/int64 array (None -> NULL)."""
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return ctypes.c_void_p(a.ctypes.data)


def f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)
