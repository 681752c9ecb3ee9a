"""O-num: Python side of the Algorithm 1 oracle (Section 2.1.1).

Test infrastructure: see oracle/__init__.py. Values of the ordered matrix
P A P^T are formed here from the caller's lower CSC and permutation; the
column structures come from ``oracle.osym``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import osym

_lib = None


def _load():
    global _lib
    if _lib is None:
        from .build import LIB, build
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        lib.oracle_alg1.restype = ctypes.c_int64
        lib.oracle_alg1.argtypes = [ctypes.c_int64, p, p, p, p, p, p, ctypes.c_int64,
                                    ctypes.c_int32]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def pattern_csc(structs):
    """CSC pattern (colptr, rowidx) of L from per-column sorted structures."""
    cnt = np.array([len(s) for s in structs], np.int64)
    cp = np.zeros(len(structs) + 1, np.int64)
    np.cumsum(cnt, out=cp[1:])
    ri = np.concatenate(structs).astype(np.int64) if structs else np.zeros(0, np.int64)
    return cp, ri


def alg1(n, a_cp, a_ri, a_x, l_cp, l_ri, ncols=None, reverse=False):
    """Run Algorithm 1 on the ordered lower CSC. Returns (L values, info).

    info = 0 on success, else the 1-based column of the first non-positive
    pivot (the columns before it are complete).
    """
    ncols = n if ncols is None else int(ncols)
    a_cp = np.ascontiguousarray(a_cp, np.int64)
    a_ri = np.ascontiguousarray(a_ri, np.int64)
    a_x = np.ascontiguousarray(a_x, np.float64)
    l_cp = np.ascontiguousarray(l_cp, np.int64)
    l_ri = np.ascontiguousarray(l_ri, np.int64)
    l_x = np.zeros(int(l_cp[ncols]), np.float64)
    info = _load().oracle_alg1(n, _ptr(a_cp), _ptr(a_ri), _ptr(a_x), _ptr(l_cp), _ptr(l_ri),
                               _ptr(l_x), ncols, 1 if reverse else 0)
    if info < 0:
        raise RuntimeError("oracle_alg1: bad argument or out of memory")
    return l_x, int(info)


def factor(A, perm, structs=None, ncols=None, reverse=False):
    """Factor P A P^T (perm[new] = old) with Algorithm 1.

    Returns dict(colptr, rowidx, values, info, ncols) of L in the exact
    structure (the first `ncols` columns when a prefix is asked for).
    """
    n = A.n
    a_cp, a_ri, a_x = osym.permute_lower(n, A.colptr, A.rowidx, A.values, perm)
    if structs is None:
        upto = n if ncols is None else int(ncols)
        structs, _ = osym.column_structures(n, a_cp, a_ri, upto=upto)
    nc = len(structs) if ncols is None else int(ncols)
    l_cp, l_ri = pattern_csc(structs[:nc])
    l_x, info = alg1(n, a_cp, a_ri, a_x, l_cp, l_ri, ncols=nc, reverse=reverse)
    return {"colptr": l_cp, "rowidx": l_ri, "values": l_x, "info": info, "ncols": nc,
            "a": (a_cp, a_ri, a_x)}
