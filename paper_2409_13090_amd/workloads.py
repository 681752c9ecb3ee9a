"""Seeded synthetic SPD workloads (grid Laplacians and a 3-dof elasticity-like
block matrix) in the input convention of the analysis phase: CSC of the lower
triangle including the diagonal, 0-based int64 indices, rows strictly
ascending inside each column, float64 values.

This module only *generates inputs*. It holds none of the factorization's
arithmetic, and both the device path and the CPU oracle take its matrices as
plain arrays. The paper measures on SuiteSparse matrices (Section 3.1); these
PDE-like grids stand in for them.

Draw-order conventions (so that a seed fixes every value):
  * generator: numpy PCG64 ``default_rng(seed)``;
  * one draw per edge: the stencil offsets of the positive half-space are taken
    in lexicographic (dz, dy, dx) order, and the edges of one offset by
    ascending lower endpoint (node index x + nx*(y + ny*z));
  * the right-hand sides are drawn after all matrix values, n*nrhs standard
    normals in column-major order;
  * assembly: A_ij = -w for an edge (i, j), A_ii = sum of incident weights
    plus a diagonal shift.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# stencils


def _positive_offsets(kind: str):
    """Offsets (dz, dy, dx) of the positive half-space, lexicographic order."""
    if kind == "5pt":
        cand = [(0, 0, 1), (0, 1, 0)]
    elif kind == "9pt":
        cand = [(0, dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    elif kind == "7pt":
        cand = [(0, 0, 1), (0, 1, 0), (1, 0, 0)]
    elif kind == "27pt":
        cand = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    else:
        raise ValueError(f"unknown stencil {kind!r}")
    pos = [o for o in cand if o > (0, 0, 0)]
    return sorted(pos)


def grid_edges(dims, kind):
    """Yield (offset, lower endpoints, upper endpoints) per positive offset."""
    nx, ny, nz = dims
    x = np.arange(nx)
    y = np.arange(ny)
    z = np.arange(nz)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")  # C order = ascending node index
    X = X.ravel()
    Y = Y.ravel()
    Z = Z.ravel()
    node = X + nx * (Y + ny * Z)
    for (dz, dy, dx) in _positive_offsets(kind):
        ok = ((X + dx >= 0) & (X + dx < nx) & (Y + dy >= 0) & (Y + dy < ny)
              & (Z + dz >= 0) & (Z + dz < nz))
        lo = node[ok]
        hi = lo + dx + nx * (dy + ny * dz)
        yield (dz, dy, dx), lo.astype(np.int64), hi.astype(np.int64)


# ---------------------------------------------------------------------------
# container


@dataclass
class SparseSPD:
    """Lower-triangle CSC (incl. diagonal) of a symmetric positive definite A."""

    n: int
    colptr: np.ndarray
    rowidx: np.ndarray
    values: np.ndarray
    grid: tuple = (0, 0, 0, 1)  # nx, ny, nz, dofs per node (0 = no grid)
    name: str = ""
    rhs: np.ndarray | None = None  # n x nrhs, Fortran order
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    def to_scipy_full(self):
        """Full symmetric matrix as scipy CSR (test helper)."""
        import scipy.sparse as sp

        low = sp.csc_matrix((self.values, self.rowidx, self.colptr), shape=(self.n, self.n))
        d = sp.diags(low.diagonal())
        return (low + low.T - d).tocsr()


def _lower_csc(n, rows, cols, vals):
    """Assemble lower-triangle CSC from unique (row >= col) triplets."""
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    vals = np.asarray(vals, np.float64)
    assert np.all(rows >= cols)
    order = np.lexsort((rows, cols))
    rows = rows[order]
    cols = cols[order]
    vals = vals[order]
    key = cols * n + rows
    if key.size > 1 and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate entries in generator output")
    colptr = np.zeros(n + 1, np.int64)
    np.add.at(colptr, cols + 1, 1)
    colptr = np.cumsum(colptr)
    return colptr, rows, vals


def grid_laplacian(dims, kind, rng, weight_fn, shift_fn, name=""):
    """Weighted graph Laplacian of a grid stencil plus a diagonal shift.

    weight_fn(rng, count) draws the weights of one stencil offset;
    shift_fn(incident_sums) returns the scalar shift added to every diagonal.
    """
    nx, ny, nz = dims
    n = nx * ny * nz
    lo_all, hi_all, w_all = [], [], []
    for _, lo, hi in grid_edges(dims, kind):
        w = np.asarray(weight_fn(rng, lo.size), np.float64)
        lo_all.append(lo)
        hi_all.append(hi)
        w_all.append(w)
    lo = np.concatenate(lo_all) if lo_all else np.zeros(0, np.int64)
    hi = np.concatenate(hi_all) if hi_all else np.zeros(0, np.int64)
    w = np.concatenate(w_all) if w_all else np.zeros(0)
    inc = np.bincount(lo, weights=w, minlength=n) + np.bincount(hi, weights=w, minlength=n)
    shift = float(shift_fn(inc))
    diag = inc + shift
    rows = np.concatenate([np.arange(n, dtype=np.int64), hi])
    cols = np.concatenate([np.arange(n, dtype=np.int64), lo])
    vals = np.concatenate([diag, -w])
    colptr, rowidx, values = _lower_csc(n, rows, cols, vals)
    return SparseSPD(n, colptr, rowidx, values, (nx, ny, nz, 1), name,
                     meta={"shift": shift, "stencil": kind, "dims": tuple(dims)})


def _quat_rot(q):
    """Rotation matrices from quaternions q[..., 4] (normalised here)."""
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def elasticity_like(dims, rng, shift=1e-6, name=""):
    """3 dofs per node, 7-point node coupling, K_e = E R diag(1,1,1e-2) R^T.

    Per offset the draws are: E ~ U[1,100] for every edge, then one N(0,1)^4
    quaternion per edge. A_vv = sum of incident K_e + shift*I, A_uv = -K_e.
    """
    nx, ny, nz = dims
    nn = nx * ny * nz
    n = 3 * nn
    lo_all, hi_all, K_all = [], [], []
    D = np.diag([1.0, 1.0, 1e-2])
    for _, lo, hi in grid_edges(dims, "7pt"):
        E = rng.uniform(1.0, 100.0, lo.size)
        q = rng.standard_normal((lo.size, 4))
        R = _quat_rot(q)
        K = E[:, None, None] * (R @ D @ np.swapaxes(R, 1, 2))
        K = 0.5 * (K + np.swapaxes(K, 1, 2))  # exact symmetry
        lo_all.append(lo)
        hi_all.append(hi)
        K_all.append(K)
    lo = np.concatenate(lo_all)
    hi = np.concatenate(hi_all)
    K = np.concatenate(K_all)
    blk = np.zeros((nn, 3, 3))
    for a in range(3):
        for b in range(3):
            blk[:, a, b] = (np.bincount(lo, weights=K[:, a, b], minlength=nn)
                            + np.bincount(hi, weights=K[:, a, b], minlength=nn))
    blk += shift * np.eye(3)[None]
    rows, cols, vals = [], [], []
    node = np.arange(nn, dtype=np.int64)
    for a in range(3):
        for b in range(a + 1):
            rows.append(3 * node + a)
            cols.append(3 * node + b)
            vals.append(blk[:, a, b])
    for a in range(3):
        for b in range(3):
            rows.append(3 * hi + a)
            cols.append(3 * lo + b)
            vals.append(-K[:, a, b])
    colptr, rowidx, values = _lower_csc(n, np.concatenate(rows), np.concatenate(cols),
                                        np.concatenate(vals))
    return SparseSPD(n, colptr, rowidx, values, (nx, ny, nz, 3), name,
                     meta={"shift": shift, "stencil": "7pt-3dof", "dims": tuple(dims)})


def draw_rhs(rng, n, nrhs):
    """n x nrhs standard normals, drawn column by column (Fortran order)."""
    return np.asfortranarray(rng.standard_normal(n * nrhs).reshape(nrhs, n).T)


# ---------------------------------------------------------------------------
# the five workload recipes


def config1(seed=1):
    """2D 5-point Laplacian, 30x30 (n=900), weights U[0.5,1.5], shift +1e-2, 1 RHS."""
    rng = np.random.default_rng(seed)
    A = grid_laplacian((30, 30, 1), "5pt", rng, lambda r, c: r.uniform(0.5, 1.5, c),
                       lambda inc: 1e-2, name="lap2d5_30")
    A.rhs = draw_rhs(rng, A.n, 1)
    return A


def config2(seed=2, side=48):
    """3D 7-point Laplacian, side^3 (48^3: n=110592), weights 10^U(-2,2),
    shift 1e-6 * max diagonal, 4 RHS."""
    rng = np.random.default_rng(seed)
    A = grid_laplacian((side, side, side), "7pt", rng,
                       lambda r, c: 10.0 ** r.uniform(-2.0, 2.0, c),
                       lambda inc: 1e-6 * float(inc.max()), name=f"lap3d7_{side}")
    A.rhs = draw_rhs(rng, A.n, 4)
    return A


def batch_member(i, count=512, base_seed=3):
    """Matrix i of the batched workload: 2D 9-point Laplacian on a square grid
    with side ~ U{16..96}, weights U[0.5,1.5], shift +1e-3, 1 RHS."""
    child = np.random.SeedSequence(base_seed).spawn(count)[i]
    rng = np.random.default_rng(child)
    side = int(rng.integers(16, 97))
    A = grid_laplacian((side, side, 1), "9pt", rng, lambda r, c: r.uniform(0.5, 1.5, c),
                       lambda inc: 1e-3, name=f"lap2d9_{side}_b{i}")
    A.rhs = draw_rhs(rng, A.n, 1)
    return A


def config3(count=512):
    """The batched workload: `count` independent 9-point grid Laplacians."""
    return [batch_member(i, count) for i in range(count)]


def config4(seed=4, side=64):
    """3D 27-point stencil, side^3 (64^3: n=262144), weights U[0.1,1],
    shift +1e-4, 8 RHS."""
    rng = np.random.default_rng(seed)
    A = grid_laplacian((side, side, side), "27pt", rng, lambda r, c: r.uniform(0.1, 1.0, c),
                       lambda inc: 1e-4, name=f"lap3d27_{side}")
    A.rhs = draw_rhs(rng, A.n, 8)
    return A


def config5(seed=5, side=40):
    """3-dof elasticity-like block matrix on a side^3 node grid (40^3: n=192000),
    shift 1e-6 * I, 16 RHS."""
    rng = np.random.default_rng(seed)
    A = elasticity_like((side, side, side), rng, 1e-6, name=f"elast3_{side}")
    A.rhs = draw_rhs(rng, A.n, 16)
    return A


def small_grid(kind, dims, seed=0, shift=1e-2, lo=0.5, hi=1.5, nrhs=1):
    """A small generic grid Laplacian for tests."""
    rng = np.random.default_rng(seed)
    A = grid_laplacian(dims, kind, rng, lambda r, c: r.uniform(lo, hi, c),
                       lambda inc: shift, name=f"{kind}_{'x'.join(map(str, dims))}_s{seed}")
    A.rhs = draw_rhs(rng, A.n, nrhs)
    return A


def from_dense_lower(Ad, grid=(0, 0, 0, 1), name="dense"):
    """Lower-triangle CSC of the nonzeros of a dense symmetric matrix."""
    Ad = np.asarray(Ad, np.float64)
    n = Ad.shape[0]
    rows, cols = np.nonzero(np.tril(Ad))
    diag = np.arange(n)
    # the diagonal is always stored, even when it is zero
    mask = rows != cols
    rows = np.concatenate([rows[mask], diag])
    cols = np.concatenate([cols[mask], diag])
    vals = Ad[rows, cols]
    colptr, rowidx, values = _lower_csc(n, rows, cols, vals)
    return SparseSPD(n, colptr, rowidx, values, grid, name)


def irregular3d(n, k=10, seed=6, shift=1e-2, nrhs=4, name=None):
    """Irregular SPD workload (general sparse input, no grid): n points drawn
    uniform in the unit cube, each joined to its k nearest neighbours (the
    union of both directions), one weight U[0.5,1.5] per edge drawn in
    ascending (lower, upper) endpoint order, A_ij = -w, A_ii = sum of
    incident weights + shift; the points are numbered in the order drawn, so
    the natural order has no locality. nrhs right-hand sides N(0,1) last."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, (n, 3))
    _, nb = cKDTree(pts).query(pts, k=k + 1)
    a = np.repeat(np.arange(n, dtype=np.int64), k)
    b = nb[:, 1:].reshape(-1).astype(np.int64)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = np.unique(lo * n + hi)
    lo, hi = key // n, key % n
    w = rng.uniform(0.5, 1.5, lo.size)
    inc = np.bincount(lo, weights=w, minlength=n) + np.bincount(hi, weights=w, minlength=n)
    rows = np.concatenate([np.arange(n, dtype=np.int64), hi])
    cols = np.concatenate([np.arange(n, dtype=np.int64), lo])
    vals = np.concatenate([inc + shift, -w])
    colptr, rowidx, values = _lower_csc(n, rows, cols, vals)
    A = SparseSPD(n, colptr, rowidx, values, (0, 0, 0, 1), name or f"irr3d_{n}_k{k}",
                  meta={"shift": shift, "k": k})
    A.rhs = draw_rhs(rng, n, nrhs)
    return A
