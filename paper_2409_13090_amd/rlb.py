"""Thin Python binding of the rlb C-ABI (include/rlb.h).

Argument marshalling only: every step of the factorization and the solves
runs in the library's HIP kernels. PyTorch provides device memory and the
current HIP stream. Importing this module fails loudly when the compiled
library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librlb.so")

RLB_ORDER_NATURAL = 0
RLB_ORDER_GRID_ND = 1
RLB_ORDER_USER = 2
RLB_ORDER_GRAPH_ND = 3
RLB_PREC_FP64 = 0
RLB_PREC_FP32_UPDATES = 1
RLB_PREC_BF16_UPDATES = 2
RLB_PREC_FP16_UPDATES = 3

_c_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p


class RlbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"rlb status {status}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("ordering", ctypes.c_int32),
                ("user_perm", _c_i64p), ("grid", ctypes.c_int64 * 4),
                ("merge_cap", ctypes.c_double), ("reorder", ctypes.c_int32),
                ("maximal_blocks", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("panel_spread", ctypes.c_int32), ("deterministic", ctypes.c_int32),
                ("outer_block", ctypes.c_int32), ("big_tile_min", ctypes.c_int32),
                ("method", ctypes.c_int32), ("tile_order", ctypes.c_int32),
                ("tall_tile_min", ctypes.c_int32), ("hybrid_step_us", ctypes.c_double),
                ("split_chunks", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("n", "nnz_a", "n_supernodes", "n_fundamental", "n_levels", "nnz_exact",
                 "nnz_stored")] + [
                ("flops_exact", ctypes.c_double), ("flops_padded", ctypes.c_double)] + [
                (k, ctypes.c_int64) for k in
                ("n_blocks", "n_pairs", "n_calls", "merge_added", "merge_base", "factor_bytes",
                 "n_panel_tiles", "n_update_tiles", "n_merged_tiles", "n_split_tiles",
                 "n_launches")] + [
                ("flops_tiles", ctypes.c_double), ("flops_upd_alg", ctypes.c_double),
                ("flops_panel", ctypes.c_double), ("flops_upd_launch", ctypes.c_double),
                ("u_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RefineReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("backward_error", ctypes.c_double * 16), ("history", ctypes.c_double * 64),
                ("pcg_from", ctypes.c_int32), ("reserved", ctypes.c_int32)]


EXPORTED = [
    "rlb_default_options", "rlb_analyze", "rlb_symbolic_info", "rlb_symbolic_array",
    "rlb_symbolic_free", "rlb_numeric_create", "rlb_factor", "rlb_factor_status", "rlb_solve",
    "rlb_refine", "rlb_backward_error", "rlb_factor_export", "rlb_numeric_free",
    "rlb_batch_create", "rlb_batch_factor", "rlb_batch_status", "rlb_batch_solve",
    "rlb_batch_free", "rlb_set_graph_mode", "rlb_batch_set_graph_mode", "rlb_set_profiling",
    "rlb_last_profile", "rlb_status_string", "rlb_last_error", "rlb_factor_pivots_patched",
    "rlb_batch_set_schedule", "rlb_batch_autotune", "rlb_solve_noalloc",
    "rlb_last_profile_launches", "rlb_batch_set_narrow_min", "rlb_batch_get_tuning",
]

_lib = None


def lib():
    """Load the compiled library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    i32 = ctypes.c_int32
    i64 = ctypes.c_int64
    sig = {
        "rlb_default_options": [ctypes.POINTER(Options)],
        "rlb_analyze": [i64, _vp, _vp, ctypes.POINTER(Options), ctypes.POINTER(_vp)],
        "rlb_symbolic_info": [_vp, ctypes.POINTER(Info)],
        "rlb_symbolic_array": [_vp, ctypes.c_char_p, _vp, ctypes.POINTER(i64)],
        "rlb_numeric_create": [_vp, i32, ctypes.POINTER(_vp)],
        "rlb_factor": [_vp, _vp, _vp, ctypes.c_size_t, _vp],
        "rlb_factor_status": [_vp, ctypes.POINTER(i64)],
        "rlb_solve": [_vp, i64, _vp, i64, _vp],
        "rlb_solve_noalloc": [_vp, i64, _vp, i64, _vp],
        "rlb_refine": [_vp, _vp, i64, _vp, _vp, i64, ctypes.c_double, i32, _vp,
                       ctypes.POINTER(RefineReport)],
        "rlb_backward_error": [_vp, _vp, i64, _vp, _vp, i64, _vp, _vp],
        "rlb_factor_export": [_vp, _vp, _vp, _vp],
        "rlb_batch_create": [i32, _vp, i32, ctypes.POINTER(_vp), ctypes.POINTER(i64)],
        "rlb_batch_factor": [_vp, _vp, _vp, ctypes.c_size_t, _vp],
        "rlb_batch_status": [_vp, _vp],
        "rlb_batch_solve": [_vp, i32, i64, _vp, i64, _vp],
        "rlb_set_graph_mode": [_vp, i32],
        "rlb_batch_set_graph_mode": [_vp, i32],
        "rlb_set_profiling": [_vp, i32],
        "rlb_last_profile": [_vp, _vp, _vp, _vp, _vp],
        "rlb_last_profile_launches": [_vp, _vp, ctypes.POINTER(i64)],
        "rlb_factor_pivots_patched": [_vp, ctypes.POINTER(i64)],
        "rlb_batch_set_schedule": [_vp, i32],
        "rlb_batch_set_narrow_min": [_vp, ctypes.c_int64],
        "rlb_batch_get_tuning": [_vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_int64)],
        "rlb_batch_autotune": [_vp, _vp, _vp, ctypes.c_size_t, _vp, i32, ctypes.POINTER(i32), _vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = i32
    for name in ("rlb_symbolic_free", "rlb_numeric_free", "rlb_batch_free"):
        f = getattr(L, name)
        f.argtypes = [_vp]
        f.restype = None
    L.rlb_status_string.argtypes = [i32]
    L.rlb_status_string.restype = ctypes.c_char_p
    L.rlb_last_error.argtypes = []
    L.rlb_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(st, allow_positive=False):
    if st < 0 or (st > 0 and not allow_positive):
        raise RlbError(st, lib().rlb_last_error().decode())
    return st


def _ptr(a):
    """Device or host address of a torch tensor or numpy array."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    if torch.cuda.is_available():
        return torch.cuda.current_stream().cuda_stream
    return None


# ---------------------------------------------------------------------------


class Symbolic:
    """rlb_analyze: host symbolic phase of a lower-triangle CSC pattern."""

    def __init__(self, n, colptr, rowidx, ordering="grid", grid=(0, 0, 0, 1), merge_cap=0.125,
                 reorder=True, maximal_blocks=True, user_perm=None, panel_spread=0,
                 deterministic=True, outer_block=0, big_tile_min=0, method="rlb",
                 tile_order="weight", hybrid_step_us=0.0, tall_tile_min=None, split_chunks=0):
        L = lib()
        self._cp = np.ascontiguousarray(colptr, np.int64)
        self._ri = np.ascontiguousarray(rowidx, np.int64)
        o = Options()
        _check(L.rlb_default_options(ctypes.byref(o)))
        o.ordering = {"natural": RLB_ORDER_NATURAL, "grid": RLB_ORDER_GRID_ND,
                      "user": RLB_ORDER_USER, "graph": RLB_ORDER_GRAPH_ND}[ordering]
        for k in range(4):
            o.grid[k] = int(grid[k])
        o.merge_cap = float(merge_cap)
        o.reorder = 1 if reorder else 0
        o.maximal_blocks = 1 if maximal_blocks else 0
        o.panel_spread = int(panel_spread)
        o.deterministic = 1 if deterministic else 0
        o.outer_block = int(outer_block)
        o.big_tile_min = int(big_tile_min)
        o.method = {"rlb": 0, "rl": 1, "hybrid": 2}[method]
        o.tile_order = {"weight": 0, "xcd": 1}[tile_order]
        o.hybrid_step_us = float(hybrid_step_us)
        if tall_tile_min is not None:
            o.tall_tile_min = int(tall_tile_min)
        o.split_chunks = int(split_chunks)
        if user_perm is not None:
            self._up = np.ascontiguousarray(user_perm, np.int64)
            o.user_perm = self._up.ctypes.data_as(_c_i64p)
        h = _vp()
        _check(L.rlb_analyze(int(n), self._cp.ctypes.data, self._ri.ctypes.data,
                             ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self.n = int(n)

    @classmethod
    def from_matrix(cls, A, **kw):
        kw.setdefault("grid", A.grid if A.grid[0] else (0, 0, 0, 1))
        if A.grid[0] == 0:
            kw.setdefault("ordering", "natural")
        return cls(A.n, A.colptr, A.rowidx, **kw)

    def info(self):
        i = Info()
        _check(lib().rlb_symbolic_info(self.h, ctypes.byref(i)))
        return i.as_dict()

    def array(self, name):
        n = ctypes.c_int64()
        _check(lib().rlb_symbolic_array(self.h, name.encode(), None, ctypes.byref(n)))
        out = np.zeros(n.value, np.int64)
        _check(lib().rlb_symbolic_array(self.h, name.encode(), out.ctypes.data, ctypes.byref(n)))
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().rlb_symbolic_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Numeric:
    """rlb_numeric_create + rlb_factor / rlb_solve / rlb_refine on one matrix."""

    def __init__(self, sym: Symbolic, precision=RLB_PREC_FP64):
        self.sym = sym  # keeps the symbolic handle alive
        h = _vp()
        _check(lib().rlb_numeric_create(sym.h, int(precision), ctypes.byref(h)))
        self.h = h
        self.workspace = None
        self.values = None

    def factor(self, values, workspace=None, stream=None, check=True):
        """values: device float64 tensor of the analysed CSC entries."""
        import torch
        info = self.sym.info()
        if workspace is None:
            if self.workspace is None or self.workspace.numel() * 8 < info["factor_bytes"]:
                self.workspace = torch.empty(max(1, info["factor_bytes"] // 8),
                                             dtype=torch.float64, device=values.device)
            workspace = self.workspace
        self.workspace = workspace
        self.values = values
        _check(lib().rlb_factor(self.h, _ptr(values), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream)))
        if check:
            return self.status()
        return None

    def status(self):
        info = ctypes.c_int64()
        st = lib().rlb_factor_status(self.h, ctypes.byref(info))
        _check(st, allow_positive=True)
        return int(info.value)

    def pivots_patched(self):
        c = ctypes.c_int64()
        _check(lib().rlb_factor_pivots_patched(self.h, ctypes.byref(c)))
        return int(c.value)

    def solve(self, B, stream=None):
        """In place; B is an (n, nrhs) or (n,) float64 device tensor, column-major
        storage expected (use B.T.contiguous().T for an (n, nrhs) tensor)."""
        nrhs, ldb = _cm(B)
        _check(lib().rlb_solve(self.h, nrhs, _ptr(B), ldb, _stream(stream)))
        return B

    def solve_noalloc(self, B, stream=None):
        """rlb_solve_noalloc: as solve(), with the library's fixed per-GPU work
        vectors (no device allocation); nrhs <= 16 and n * nrhs <= 2^21."""
        nrhs, ldb = _cm(B)
        _check(lib().rlb_solve_noalloc(self.h, nrhs, _ptr(B), ldb, _stream(stream)))
        return B

    def refine(self, B, X, tol=1e-14, max_iter=30, values=None, stream=None):
        nrhs, ld = _cm(B)
        rep = RefineReport()
        st = lib().rlb_refine(self.h, _ptr(values if values is not None else self.values), nrhs,
                              _ptr(B), _ptr(X), ld, float(tol), int(max_iter), _stream(stream),
                              ctypes.byref(rep))
        if st not in (0, -7):
            _check(st)
        return {"converged": bool(rep.converged), "iterations": rep.iterations,
                "backward_error": list(rep.backward_error)[:nrhs],
                "history": list(rep.history)[:rep.iterations + 1],
                "pcg_from": rep.pcg_from}

    def backward_error(self, B, X, values=None, stream=None):
        nrhs, ld = _cm(B)
        out = np.zeros(nrhs)
        _check(lib().rlb_backward_error(self.h, _ptr(values if values is not None else self.values),
                                        nrhs, _ptr(B), _ptr(X), ld, _stream(stream),
                                        out.ctypes.data))
        return out

    def export(self):
        """Factor in a host CSC with the stored supernodal structure (final order)."""
        info = self.sym.info()
        n = info["n"]
        cp = np.zeros(n + 1, np.int64)
        ri = np.zeros(info["nnz_stored"], np.int64)
        vx = np.zeros(info["nnz_stored"], np.float64)
        _check(lib().rlb_factor_export(self.h, cp.ctypes.data, ri.ctypes.data, vx.ctypes.data))
        return cp, ri, vx

    def set_graph_mode(self, on=True):
        _check(lib().rlb_set_graph_mode(self.h, 1 if on else 0))

    def set_profiling(self, on=True):
        _check(lib().rlb_set_profiling(self.h, 1 if on else 0))

    def last_profile(self):
        u = ctypes.c_double()
        p = ctypes.c_double()
        nu = ctypes.c_int64()
        npn = ctypes.c_int64()
        _check(lib().rlb_last_profile(self.h, ctypes.byref(u), ctypes.byref(p), ctypes.byref(nu),
                                      ctypes.byref(npn)))
        return {"update_ms": u.value, "panel_ms": p.value, "n_update": nu.value,
                "n_panel": npn.value}

    def last_profile_launches(self):
        """Milliseconds of every launch of the last profiled factorization."""
        n = ctypes.c_int64(0)
        _check(lib().rlb_last_profile_launches(self.h, None, ctypes.byref(n)))
        out = np.zeros(n.value)
        _check(lib().rlb_last_profile_launches(self.h, out.ctypes.data, ctypes.byref(n)))
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().rlb_numeric_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """rlb_batch_*: many independent matrices with one merged level schedule."""

    def __init__(self, syms, precision=RLB_PREC_FP64):
        self.syms = list(syms)
        arr = (_vp * len(self.syms))(*[s.h.value for s in self.syms])
        h = _vp()
        ws = ctypes.c_int64()
        _check(lib().rlb_batch_create(len(self.syms), ctypes.cast(arr, _vp), int(precision),
                                      ctypes.byref(h), ctypes.byref(ws)))
        self.h = h
        self.ws_bytes = ws.value
        self.workspace = None

    def factor(self, values_list, workspace=None, stream=None, check=True):
        import torch
        if workspace is None:
            if self.workspace is None:
                self.workspace = torch.empty(max(1, self.ws_bytes // 8), dtype=torch.float64,
                                             device=values_list[0].device)
            workspace = self.workspace
        self.workspace = workspace
        self._vals = list(values_list)
        arr = (_vp * len(self._vals))(*[_ptr(v) for v in self._vals])
        _check(lib().rlb_batch_factor(self.h, ctypes.cast(arr, _vp), _ptr(workspace),
                                      workspace.numel() * 8, _stream(stream)))
        if check:
            return self.status()
        return None

    SCHEDULES = ("leaves", "roots", "centered")

    def set_schedule(self, name):
        _check(lib().rlb_batch_set_schedule(self.h, self.SCHEDULES.index(name)))

    def set_narrow_min(self, min_items):
        """Narrow work items per merged launch from which they run one per
        wavefront (0: never)."""
        _check(lib().rlb_batch_set_narrow_min(self.h, int(min_items)))

    def tuning(self):
        """(schedule name, narrow-item threshold; 0 = never)."""
        sch, nm = ctypes.c_int32(), ctypes.c_int64()
        _check(lib().rlb_batch_get_tuning(self.h, ctypes.byref(sch), ctypes.byref(nm)))
        return self.SCHEDULES[sch.value], nm.value

    def autotune(self, values_list, workspace=None, stream=None, reps=2):
        """Time the level schedules, each with the narrow-item thresholds
        256, 1024, 4096 and never, on the device and keep the fastest pair;
        returns (chosen schedule name, {name: best ms of that schedule})."""
        import torch
        if workspace is None:
            if self.workspace is None:
                self.workspace = torch.empty(max(1, self.ws_bytes // 8), dtype=torch.float64,
                                             device=values_list[0].device)
            workspace = self.workspace
        self.workspace = workspace
        self._vals = list(values_list)
        arr = (_vp * len(self._vals))(*[_ptr(v) for v in self._vals])
        chosen = ctypes.c_int32()
        ms = np.zeros(3)
        _check(lib().rlb_batch_autotune(self.h, ctypes.cast(arr, _vp), _ptr(workspace),
                                        workspace.numel() * 8, _stream(stream), int(reps),
                                        ctypes.byref(chosen), ms.ctypes.data))
        return self.SCHEDULES[chosen.value], dict(zip(self.SCHEDULES, ms.tolist()))

    def status(self):
        out = np.zeros(len(self.syms), np.int64)
        st = lib().rlb_batch_status(self.h, out.ctypes.data)
        _check(st, allow_positive=True)
        return out

    def solve(self, i, B, stream=None):
        nrhs, ldb = _cm(B)
        _check(lib().rlb_batch_solve(self.h, int(i), nrhs, _ptr(B), ldb, _stream(stream)))
        return B

    def set_graph_mode(self, on=True):
        _check(lib().rlb_batch_set_graph_mode(self.h, 1 if on else 0))

    def close(self):
        if getattr(self, "h", None):
            lib().rlb_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _cm(B):
    """(nrhs, leading dimension) of a column-major device matrix or vector."""
    if B.dim() == 1:
        return 1, B.shape[0]
    n, nrhs = B.shape
    if nrhs == 1:
        return 1, n
    if B.stride(0) != 1:
        raise ValueError("B must be column-major (use B.T.contiguous().T)")
    return nrhs, B.stride(1)
