"""Helpers shared by the GPU parity tests: run the device path through the
C-ABI binding and compare with the CPU oracle."""
import numpy as np
import scipy.sparse as sp

from oracle import onum, osym
from paper_2409_13090_amd import rlb

FP64_TOL = 1e-10  # relative Frobenius error of L against the oracle, FP64


def oracle_factor(A, ncols=None, **kw):
    """Oracle's own analysis and Algorithm 1 factor (optionally a column prefix)."""
    o = osym.analyze(A, **kw)
    f = onum.factor(A, o["perm"], o["structs"], ncols=ncols)
    return o, f


def keys(cp, ri, n):
    cols = np.repeat(np.arange(len(cp) - 1, dtype=np.int64), np.diff(cp))
    return cols * n + np.asarray(ri, np.int64)


def compare_factor(gpu_csc, ora, n, ncols=None, tol=FP64_TOL):
    """Structure rule + values. gpu_csc: (colptr, rowidx, vals) of the stored
    structure; ora: oracle factor dict (exact structure). Only columns < ncols
    are compared when given. Returns the relative Frobenius error."""
    gcp, gri, gvx = gpu_csc
    ocp, ori, ovx = ora["colptr"], ora["rowidx"], ora["values"]
    nc = ora["ncols"] if ncols is None else ncols
    gend = gcp[nc]
    gk = keys(gcp[:nc + 1], gri[:gend], n)
    gv = gvx[:gend]
    ok = keys(ocp[:nc + 1], ori[:ocp[nc]], n)
    ov = ovx[:ocp[nc]]
    pos = np.searchsorted(gk, ok)
    assert np.all(pos < gk.size) and np.array_equal(gk[np.minimum(pos, gk.size - 1)], ok), \
        "oracle structure not contained in the stored structure"
    only = np.ones(gk.size, bool)
    only[pos] = False
    assert np.all(gv[only] == 0.0), "stored-only position holds a nonzero"
    err = np.linalg.norm(gv[pos] - ov) / np.linalg.norm(ov)
    assert err <= tol, f"relative Frobenius error {err:.3e} > {tol:.1e}"
    return err


def factor_elems(sym):
    """Elements of the factor storage at the start of the workspace (what
    follows it -- update matrices, the part blocks of split tiles -- is
    scratch whose unwritten entries keep whatever the buffer held)."""
    return int(sym.array("off")[-1])


def gpu_factor(A, precision=0, device="cuda", graph=False, **kw):
    import torch
    s = rlb.Symbolic.from_matrix(A, **kw)
    num = rlb.Numeric(s, precision)
    if graph:
        num.set_graph_mode(True)
    vals = torch.from_numpy(A.values).to(device)
    info = num.factor(vals)
    return s, num, vals, info


def probe_residual(A, perm, gpu_csc, nprobe=4, seed=0):
    """max over random v of ||P A P^T v - L (L^T v)|| / (||A||_F ||v||): a
    property of the whole factor, cheap at any size."""
    n = A.n
    gcp, gri, gvx = gpu_csc
    L = sp.csc_matrix((gvx, gri, gcp), shape=(n, n))
    Af = A.to_scipy_full()
    Ap = Af[perm][:, perm]
    an = sp.linalg.norm(Ap)
    rng = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(nprobe):
        v = rng.standard_normal(n)
        r = Ap @ v - L @ (L.T @ v)
        worst = max(worst, np.linalg.norm(r) / (an * np.linalg.norm(v)))
    return worst


def stored_lower_positions(sym):
    """Positions in factor storage of the stored factor entries (the lower
    trapezoid of every supernode's m x w block), in the column order of
    rlb_factor_export, with that CSC's colptr and row indices."""
    sn = sym.array("sn_ptr")
    off = sym.array("off")
    gp = sym.array("gl_ptr")
    gl = sym.array("gl")
    n = int(sn[-1])
    pos, rows = [], []
    cp = np.zeros(n + 1, np.int64)
    q = 0
    for J in range(len(sn) - 1):
        f, w, m = int(sn[J]), int(sn[J + 1] - sn[J]), int(gp[J + 1] - gp[J])
        g = gl[gp[J]:gp[J + 1]]
        for c in range(w):
            pos.append(off[J] + c * m + np.arange(c, m, dtype=np.int64))
            rows.append(g[c:])
            q += m - c
            cp[f + c + 1] = q
    return np.concatenate(pos), cp, np.concatenate(rows).astype(np.int64)


def export_from_storage(sym, storage):
    """rlb_factor_export's CSC, read from a host copy of factor storage (a
    batch member's slice of the batch workspace)."""
    pos, cp, ri = stored_lower_positions(sym)
    return cp, ri, np.asarray(storage)[pos]


def bits(a):
    return np.ascontiguousarray(a, np.float64).view(np.uint64)
