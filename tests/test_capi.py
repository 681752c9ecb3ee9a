"""The C-ABI library: loads without a GPU, exports every symbol include/rlb.h
declares, and turns malformed input into the documented error codes (host
side only; no compute call needs a device here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2409_13090_amd import rlb
from paper_2409_13090_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "rlb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rlb_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = rlb.lib()
    names = declared_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(rlb.EXPORTED)


def analyze_raw(n, cp, ri, opt=None):
    L = rlb.lib()
    h = ctypes.c_void_p()
    cp = np.ascontiguousarray(cp, np.int64)
    ri = np.ascontiguousarray(ri, np.int64)
    st = L.rlb_analyze(n, cp.ctypes.data, ri.ctypes.data, opt, ctypes.byref(h))
    if h.value:
        L.rlb_symbolic_free(h)
    return st


def test_malformed_patterns_rejected():
    ok = analyze_raw(3, [0, 2, 4, 5], [0, 1, 1, 2, 2])
    assert ok == 0
    assert analyze_raw(3, [0, 2, 4, 5], [1, 0, 1, 2, 2]) == -2      # unsorted / no diagonal first
    assert analyze_raw(3, [0, 2, 4, 5], [0, 0, 1, 2, 2]) == -2      # duplicate
    assert analyze_raw(3, [0, 1, 3, 4], [0, 0, 1, 2]) == -2         # upper-triangle entry
    assert analyze_raw(3, [0, 1, 1, 2], [0, 2]) == -2               # missing diagonal
    assert analyze_raw(3, [0, 2, 4, 5], [0, 1, 1, 3, 2]) == -2      # row out of range
    assert analyze_raw(0, [0], []) == 0                             # empty matrix
    L = rlb.lib()
    h = ctypes.c_void_p()
    assert L.rlb_analyze(3, None, None, None, ctypes.byref(h)) == -1  # null pointers


def test_bad_options_rejected():
    A = W.small_grid("5pt", (4, 4, 1))
    o = rlb.Options()
    rlb.lib().rlb_default_options(ctypes.byref(o))
    o.grid[0], o.grid[1], o.grid[2], o.grid[3] = 4, 4, 1, 1
    assert analyze_raw(A.n, A.colptr, A.rowidx, ctypes.byref(o)) == 0
    o.struct_size = 3
    assert analyze_raw(A.n, A.colptr, A.rowidx, ctypes.byref(o)) == -1
    rlb.lib().rlb_default_options(ctypes.byref(o))
    o.grid[0], o.grid[1], o.grid[2], o.grid[3] = 5, 4, 1, 1   # does not match n
    assert analyze_raw(A.n, A.colptr, A.rowidx, ctypes.byref(o)) == -1
    rlb.lib().rlb_default_options(ctypes.byref(o))
    o.ordering = 2                                            # user ordering, no permutation
    assert analyze_raw(A.n, A.colptr, A.rowidx, ctypes.byref(o)) == -1
    with pytest.raises(rlb.RlbError):
        rlb.Symbolic.from_matrix(A, ordering="user", user_perm=np.zeros(A.n, np.int64))


def test_info_and_plan_consistency():
    A = W.config1()
    s = rlb.Symbolic.from_matrix(A)
    i = s.info()
    assert i["n"] == 900 and i["nnz_a"] == A.nnz
    assert i["n_supernodes"] < i["n_fundamental"]
    assert i["nnz_exact"] <= i["nnz_stored"]
    assert i["merge_added"] <= 0.125 * i["merge_base"]
    assert i["factor_bytes"] >= 8 * i["nnz_stored"]
    assert i["n_launches"] >= 2 * i["n_levels"] - 1
    assert i["flops_exact"] == 316301.0
    assert rlb.lib().rlb_status_string(-2).decode().startswith("malformed")
    assert rlb.lib().rlb_status_string(5).decode().startswith("matrix not positive")
    with pytest.raises(rlb.RlbError):
        s.array("no_such_array")
