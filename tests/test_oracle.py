"""Pins of the CPU oracle against things other than itself: the values the paper
prints for its worked example, dense LAPACK Cholesky, exact rational
arithmetic, closed forms, brute-force elimination, and invariants."""
import itertools
import json
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import onum, osym
from paper_2409_13090_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def fig1():
    g = json.load(open(os.path.join(GOLD, "fig1.json")))
    n = g["n"]
    Ad = np.zeros((n, n))
    for i, j in g["A_offdiag_lower"]["pairs"]:
        Ad[i - 1, j - 1] = Ad[j - 1, i - 1] = -1.0
    Ad += np.diag(-Ad.sum(1) + 1.0)
    return g, W.from_dense_lower(Ad), Ad


def dense_L(f, n):
    L = np.zeros((n, f["ncols"]))
    for j in range(f["ncols"]):
        s, e = f["colptr"][j], f["colptr"][j + 1]
        L[f["rowidx"][s:e], j] = f["values"][s:e]
    return L


def ordered_dense(A, perm):
    Ad = A.to_scipy_full().toarray()
    return Ad[np.ix_(perm, perm)]


# ---------------------------------------------------------------------------
# the paper's worked example


def test_fig1_symbolic():
    g, A, Ad = fig1()
    r = osym.analyze(A, ordering="natural", merge_cap=0, reorder=False)
    assert list(r["parent"] + 1) == [p if p else 0 for p in g["etree_parent"]["parent"]]
    fill = {(int(i) + 1, j + 1) for j, s in enumerate(r["structs"]) for i in s
            if i != j and Ad[i, j] == 0}
    assert fill == {tuple(p) for p in g["fill"]["pairs"]}
    sn = r["sn_ptr"]
    got = [list(range(sn[J] + 1, sn[J + 1] + 1)) for J in range(len(sn) - 1)]
    assert got == g["supernodes"]["J"]
    assert list(r["glbind"][0] + 1) == g["glbind"]["J1"]
    assert list(r["glbind"][1] + 1) == g["glbind"]["J2"]
    assert list(r["sn_parent"] + 1) == g["supernodal_parent"]["parent"]
    assert list(r["relind"][0]) == g["relind"]["J1_J3"]
    assert list(r["relind"][1]) == g["relind"]["J2_J3"]
    assert [len(b) for b in g["blocks"]["J1"]] == list(r["blocks"][0])
    assert [len(b) for b in g["blocks"]["J2"]] == list(r["blocks"][1])
    assert r["relindB"][0] == [(2, pytest.approx(g["relindB"]["J1_J3"]))]
    assert list(r["relindB"][0][0][1]) == g["relindB"]["J1_J3"]
    assert list(r["relindB"][1][0][1]) == g["relindB"]["J2_J3"]


def test_fig2_reordering():
    g, A, Ad = fig1()
    r = osym.analyze(A, ordering="natural", merge_cap=0, reorder=True)
    assert list(r["perm"][4:] + 1) == g["reordering"]["new_order_of_J3"]
    assert list(r["blocks"][0]) == [3] and list(r["blocks"][1]) == [3]
    assert list(r["glbind"][0][2:] + 1) == g["reordering"]["blocks_after"]["J1"][0]
    assert list(r["glbind"][1][2:] + 1) == g["reordering"]["blocks_after"]["J2"][0]
    # the supernodal storage stays the same; the exact structure may shrink
    for J in range(3):
        lo, hi = r["sn_ptr"][J], r["sn_ptr"][J + 1]
        for j in range(lo, hi):
            stored = set(int(i) for i in r["glbind"][J] if i >= j)
            assert set(int(i) for i in r["structs"][j]) <= stored
    # Fig. 2 draws J3 dense, but under the new order entry (9,5) is not filled
    assert 8 not in set(r["structs"][4])


def test_relind_composition_matches_direct():
    """relind(J,P) = relind(J,C) o relind(C,P) (Section 2.2.1), checked on the
    paper's example and on every chain J -> C -> P of a real analysis."""
    g, _, _ = fig1()
    ex = g["relind_composition"]
    cp = [None] * ex["C_P_len"]
    for k, v in ex["C_P_known"].items():
        cp[int(k)] = v
    # distance d in relind(J,C) selects the entry d from the bottom of relind(C,P)
    assert [cp[len(cp) - 1 - d] for d in ex["J_C"]] == ex["J_P"]

    A = W.small_grid("7pt", (7, 6, 5), seed=3)
    r = osym.analyze(A)
    glb, par, sn = r["glbind"], r["sn_parent"], r["sn_ptr"]
    for J in range(len(sn) - 1):
        C = par[J]
        if C < 0 or par[C] < 0:
            continue
        P = par[C]
        rows = glb[J][glb[J] >= sn[P]]
        rows_c = glb[C][glb[C] > sn[C + 1] - 1]
        rel_jc = osym.relind(rows, glb[C])
        rel_cp = osym.relind(rows_c, glb[P])
        comp = [rel_cp[len(rel_cp) - 1 - d] for d in rel_jc]
        assert list(comp) == list(osym.relind(rows, glb[P]))


# ---------------------------------------------------------------------------
# structure: brute force


def elimination_game(M):
    """Boolean symbolic elimination on a dense pattern (lower columns)."""
    M = M.copy()
    n = M.shape[0]
    for k in range(n):
        nz = [i for i in range(k + 1, n) if M[i, k]]
        for a in nz:
            for b in nz:
                M[a, b] = True
    return [sorted([k] + [i for i in range(k + 1, n) if M[i, k]]) for k in range(n)]


@pytest.mark.parametrize("seed", range(4))
def test_structure_vs_elimination_game_all_orderings(seed):
    rng = np.random.default_rng(seed)
    n = 6
    G = rng.random((n, n)) < 0.35
    G = np.triu(G, 1)
    G = G | G.T
    for perm in itertools.permutations(range(n)):
        P = np.array(perm)
        M = G[np.ix_(P, P)] | np.eye(n, dtype=bool)
        Ad = np.where(M, -0.1, 0.0) + np.eye(n) * 2.0
        A = W.from_dense_lower(Ad)
        structs, parent = osym.column_structures(n, A.colptr, A.rowidx)
        want = elimination_game(M)
        assert [list(s) for s in structs] == want
        for j in range(n):
            rest = [i for i in want[j] if i != j]
            assert parent[j] == (min(rest) if rest else -1)


# ---------------------------------------------------------------------------
# numeric: dense LAPACK, exact arithmetic, closed forms


@pytest.mark.parametrize("case", ["c1", "2d9", "3d7", "3d27", "elast"])
def test_alg1_vs_dense_cholesky(case):
    if case == "c1":
        A = W.config1()
    elif case == "2d9":
        A = W.small_grid("9pt", (23, 17, 1), seed=5)
    elif case == "3d7":
        A = W.small_grid("7pt", (9, 8, 7), seed=6)
    elif case == "3d27":
        A = W.small_grid("27pt", (7, 6, 6), seed=7, shift=1e-4)
    else:
        A = W.elasticity_like((4, 5, 4), np.random.default_rng(8), 1e-6)
    r = osym.analyze(A)
    f = onum.factor(A, r["perm"], r["structs"])
    assert f["info"] == 0
    L = dense_L(f, A.n)
    Ap = ordered_dense(A, r["perm"])
    Ld = np.linalg.cholesky(Ap)
    err = np.linalg.norm(L - Ld) / np.linalg.norm(Ld)
    assert err < 1e-12, err
    # exact structure: every entry of L outside the structure is zero in LAPACK's
    mask = np.zeros_like(L, bool)
    for j in range(A.n):
        mask[r["structs"][j], j] = True
    assert np.abs(Ld[~mask]).max() < 1e-12 * np.abs(Ld).max()


def rational_cholesky(Ad):
    """Exact LDL^T in fractions, then 50-digit square roots."""
    n = Ad.shape[0]
    Afr = [[Fraction(float(Ad[i, j])) for j in range(n)] for i in range(n)]
    Lu = [[Fraction(0)] * n for _ in range(n)]
    D = [Fraction(0)] * n
    for j in range(n):
        D[j] = Afr[j][j] - sum(Lu[j][k] ** 2 * D[k] for k in range(j))
        Lu[j][j] = Fraction(1)
        for i in range(j + 1, n):
            Lu[i][j] = (Afr[i][j] - sum(Lu[i][k] * Lu[j][k] * D[k] for k in range(j))) / D[j]
    getcontext().prec = 50
    out = np.zeros((n, n))
    for j in range(n):
        s = (Decimal(D[j].numerator) / Decimal(D[j].denominator)).sqrt()
        for i in range(j, n):
            v = Decimal(Lu[i][j].numerator) / Decimal(Lu[i][j].denominator) * s
            out[i, j] = float(v)
    return out


@pytest.mark.parametrize("seed", range(3))
def test_alg1_vs_exact_rational(seed):
    rng = np.random.default_rng(100 + seed)
    n = 8
    G = np.triu(rng.random((n, n)) < 0.4, 1)
    W_ = np.where(G, rng.uniform(0.2, 1.0, (n, n)), 0.0)
    W_ = W_ + W_.T
    Ad = -W_ + np.diag(W_.sum(1) + rng.uniform(0.01, 0.5, n))
    A = W.from_dense_lower(Ad)
    r = osym.analyze(A, ordering="natural", merge_cap=0, reorder=False)
    f = onum.factor(A, r["perm"], r["structs"])
    L = dense_L(f, n)
    P = r["perm"]  # the postorder may renumber even the natural order
    Lx = rational_cholesky(Ad[np.ix_(P, P)])
    assert np.abs(L - Lx).max() <= 8 * np.finfo(float).eps * np.abs(Lx).max()


def test_alg1_closed_form_tridiagonal():
    """tridiag(-1,2,-1): L_kk = sqrt((k+1)/k), L_{k+1,k} = -sqrt(k/(k+1)), 1-based."""
    n = 50
    Ad = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    A = W.from_dense_lower(Ad)
    r = osym.analyze(A, ordering="natural", merge_cap=0, reorder=False)
    f = onum.factor(A, r["perm"], r["structs"])
    L = dense_L(f, n)
    k = np.arange(1, n + 1, dtype=float)
    assert np.allclose(np.diag(L), np.sqrt((k + 1) / k), rtol=1e-14, atol=0)
    assert np.allclose(np.diag(L, -1), -np.sqrt(k[:-1] / (k[:-1] + 1)), rtol=1e-14, atol=0)


def test_alg1_diagonal_and_forest():
    rng = np.random.default_rng(9)
    d = rng.uniform(0.5, 4.0, 12)
    A = W.from_dense_lower(np.diag(d))
    r = osym.analyze(A, ordering="natural", merge_cap=0, reorder=False)
    f = onum.factor(A, r["perm"], r["structs"])
    assert np.array_equal(f["values"], np.sqrt(d))
    assert all(p == -1 for p in r["parent"])
    # two disjoint blocks give a forest whose factor is block diagonal
    B1 = 3 * np.eye(4) - 0.5 * (np.eye(4, k=1) + np.eye(4, k=-1))
    B2 = 4 * np.eye(3) - 1.0 * (np.eye(3, k=2) + np.eye(3, k=-2))
    Ad = np.zeros((7, 7))
    Ad[:4, :4] = B1
    Ad[4:, 4:] = B2
    A = W.from_dense_lower(Ad)
    r = osym.analyze(A, ordering="natural", merge_cap=0, reorder=False)
    f = onum.factor(A, r["perm"], r["structs"])
    P = r["perm"]
    assert sorted(P[:4]) == [0, 1, 2, 3]  # the postorder keeps the two trees apart
    L = dense_L(f, 7)
    assert np.allclose(L[:4, :4], np.linalg.cholesky(Ad[np.ix_(P[:4], P[:4])]), rtol=0, atol=1e-15)
    assert np.allclose(L[4:, 4:], np.linalg.cholesky(Ad[np.ix_(P[4:], P[4:])]), rtol=0, atol=1e-15)
    assert np.all(L[4:, :4] == 0)
    assert sum(1 for p in r["parent"] if p < 0) == 3  # B2 has an isolated middle node


def test_alg1_not_positive_definite_info():
    n = 12
    Ad = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    Ad[5, 5] = 0.2  # pivot of column 6 (1-based) is 0.2 - 5/6 < 0
    A = W.from_dense_lower(Ad)
    r = osym.analyze(A, ordering="natural", merge_cap=0, reorder=False)
    f = onum.factor(A, r["perm"], r["structs"])
    first_bad = next(k for k in range(1, n + 1) if np.linalg.eigvalsh(Ad[:k, :k]).min() <= 0)
    assert f["info"] == first_bad == 6


def test_alg1_residual_and_positive_diagonal():
    A = W.small_grid("7pt", (12, 11, 10), seed=11, shift=1e-3)
    r = osym.analyze(A)
    f = onum.factor(A, r["perm"], r["structs"])
    n = A.n
    L = sp.csc_matrix((f["values"], f["rowidx"], f["colptr"]), shape=(n, n))
    assert np.all(L.diagonal() > 0)
    Af = A.to_scipy_full()
    P = r["perm"]
    Ap = Af[P][:, P]
    res = sp.linalg.norm(L @ L.T - Ap) / sp.linalg.norm(Ap)
    assert res < 1e-13, res


def test_alg1_prefix_is_exact_and_reverse_order_noise():
    A = W.small_grid("7pt", (10, 9, 8), seed=12)
    r = osym.analyze(A)
    full = onum.factor(A, r["perm"], r["structs"])
    k = A.n // 3
    pre = onum.factor(A, r["perm"], r["structs"], ncols=k)
    assert np.array_equal(pre["values"], full["values"][:pre["colptr"][k]])
    rev = onum.factor(A, r["perm"], r["structs"], reverse=True)
    d = np.linalg.norm(rev["values"] - full["values"]) / np.linalg.norm(full["values"])
    assert 0 <= d < 1e-14


# ---------------------------------------------------------------------------
# ordering, merging, reordering


@pytest.mark.parametrize("dims,kind", [((30, 30, 1), "5pt"), ((11, 9, 7), "7pt"),
                                       ((8, 8, 8), "27pt"), ((17, 5, 1), "9pt")])
def test_nested_dissection_properties(dims, kind):
    A = W.small_grid(kind, dims, seed=1)
    nx, ny, nz, d = A.grid
    perm = osym.nested_dissection(nx, ny, nz, d)
    assert np.array_equal(np.sort(perm), np.arange(A.n))
    # top-level split: low box, high box, then the cut plane
    ext = [nx, ny, nz]
    ax = int(np.argmax(ext))
    m = ext[ax] // 2
    coords = np.stack(np.unravel_index(perm, (nz, ny, nx))[::-1], 1)  # x, y, z
    c = coords[:, ax]
    nlow = int(np.sum(c < m))
    nhigh = int(np.sum(c > m))
    assert np.all(c[:nlow] < m) and np.all(c[nlow:nlow + nhigh] > m) and np.all(c[nlow + nhigh:] == m)
    # no edge joins the two boxes
    inv = np.empty(A.n, np.int64)
    inv[perm] = np.arange(A.n)
    cols = np.repeat(np.arange(A.n), np.diff(A.colptr))
    a, b = inv[A.rowidx], inv[cols]
    low = lambda x: x < nlow
    high = lambda x: (x >= nlow) & (x < nlow + nhigh)
    assert not np.any((low(a) & high(b)) | (high(a) & low(b)))
    # and it reduces fill against the natural order
    r_nd = osym.analyze(A, merge_cap=0, reorder=False)
    r_nat = osym.analyze(A, ordering="natural", merge_cap=0, reorder=False)
    assert osym.exact_nnz(r_nd["structs"]) < osym.exact_nnz(r_nat["structs"])


@pytest.mark.parametrize("dims,kind", [((30, 30, 1), "5pt"), ((12, 11, 10), "7pt"),
                                       ((9, 9, 9), "27pt")])
def test_merge_invariants(dims, kind):
    A = W.small_grid(kind, dims, seed=2)
    r0 = osym.analyze(A, merge_cap=0, reorder=False)
    r = osym.analyze(A, merge_cap=0.125, reorder=False)
    base = osym.exact_nnz(r0["structs"])
    sn = r["sn_ptr"]
    stored = 0
    for J in range(len(sn) - 1):
        w = sn[J + 1] - sn[J]
        m = len(r["glbind"][J])
        stored += m * w - w * (w - 1) // 2
        for j in range(sn[J], sn[J + 1]):
            assert set(r["structs"][j]) <= set(int(i) for i in r["glbind"][J] if i >= j)
    assert stored - base == r["merge_added"]
    assert 0 < stored - base <= 0.125 * base
    assert len(sn) < len(r0["sn_ptr"])
    # fundamental supernodes: same structure below the diagonal block
    f = r0["sn_ptr"]
    for J in range(len(f) - 1):
        for j in range(f[J], f[J + 1] - 1):
            assert np.array_equal(r0["structs"][j][1:], r0["structs"][j + 1])


@pytest.mark.parametrize("dims,kind", [((16, 16, 16), "7pt"), ((12, 12, 12), "27pt"),
                                       ((40, 40, 1), "9pt")])
def test_partition_refinement_invariants(dims, kind):
    A = W.small_grid(kind, dims, seed=4)
    r0 = osym.analyze(A, reorder=False)
    r = osym.analyze(A, reorder=True)
    sn = r["sn_ptr"]
    assert np.array_equal(sn, r0["sn_ptr"])
    for J in range(len(sn) - 1):
        assert set(r["perm"][sn[J]:sn[J + 1]]) == set(r0["perm"][sn[J]:sn[J + 1]])
        assert len(r["glbind"][J]) == len(r0["glbind"][J])
        for j in range(sn[J], sn[J + 1]):
            assert set(r["structs"][j]) <= set(int(i) for i in r["glbind"][J] if i >= j)
    nb0 = sum(len(b) for b in r0["blocks"])
    nb = sum(len(b) for b in r["blocks"])
    assert nb <= nb0
    if kind != "9pt":
        assert nb < nb0


def _simulate_merges(fund_ptr, structs, cap):
    """Section 3.1's merging, simulated from the row sets alone: every
    supernode is (first column, last column, set of its rows = union of the
    exact structures of its columns); a candidate is a supernode whose
    supernodal parent starts right after it; the new fill of a merge is the
    stored entries of the merged trapezoid minus those of the two parts,
    counted from the sets (not from a closed-form cost). The candidate of
    least new fill goes first (ties: smaller first column); the loop ends at
    the first merge that would take the added entries past cap * base."""
    import bisect

    def stored(f, l, rows):
        return sum(len(rows) - bisect.bisect_left(rows, c) for c in range(f, l + 1))

    sns = {}
    for J in range(len(fund_ptr) - 1):
        f, l = int(fund_ptr[J]), int(fund_ptr[J + 1]) - 1
        U = set()
        for c in range(f, l + 1):
            U |= set(int(r) for r in structs[c])
        sns[f] = (f, l, sorted(U))
    base = sum(stored(*v) for v in sns.values())
    owner = {}
    for f, (_, l, _) in sns.items():
        for c in range(f, l + 1):
            owner[c] = f

    def parent(f):
        _, l, U = sns[f]
        i = bisect.bisect_right(U, l)
        return owner[U[i]] if i < len(U) else None

    fill_cache = {}

    def fill(fj, fq):
        key = (sns[fj][1], fj, sns[fq][1], fq)
        if key not in fill_cache:
            (_, lj, Uj), (_, lq, Uq) = sns[fj], sns[fq]
            Um = sorted(set(Uj) | set(Uq))
            fill_cache[key] = stored(fj, lq, Um) - stored(*sns[fj]) - stored(*sns[fq])
        return fill_cache[key]

    added = 0
    seq = []
    while True:
        cands = []
        for f, (_, l, _) in sns.items():
            q = parent(f)
            if q is not None and l + 1 == q:
                cands.append((fill(f, q), f, q))
        if not cands:
            seq.append(("exhausted",))
            break
        c, fj, fq = min(cands)
        if added + c > cap * base:
            seq.append(("stop", fj, c))
            break
        seq.append(("merge", fj, fq, c))
        added += c
        (_, _, Uj), (_, lq, Uq) = sns.pop(fj), sns.pop(fq)
        sns[fj] = (fj, lq, sorted(set(Uj) | set(Uq)))
        for col in range(fj, lq + 1):
            owner[col] = fj
    ptr = sorted(sns) + [int(fund_ptr[-1])]
    return seq, np.array(ptr, np.int64), added, base


@pytest.mark.parametrize("dims,kind", [((30, 30, 1), "5pt"), ((20, 17, 1), "9pt"),
                                       ((12, 11, 10), "7pt"), ((8, 8, 8), "7pt"),
                                       ((9, 9, 9), "27pt"), ((6, 7, 6), "27pt")])
def test_merge_selection_order_and_stop_rule(dims, kind):
    """Pins the order in which the oracle merges supernodes (Section 3.1:
    least new fill first) and the point where it stops, against a simulation
    that recomputes every candidate's new fill from the row sets."""
    A = W.small_grid(kind, dims, seed=2)
    r0 = osym.analyze(A, merge_cap=0, reorder=False)
    cp, ri, _ = osym.permute_lower(A.n, A.colptr, A.rowidx, None, r0["perm_post"])
    structs, _ = osym.column_structures(A.n, cp, ri)
    fund = r0["fund_ptr"]
    trace = []
    sn_ptr, _, added, base = osym.merge_supernodes(fund, structs, 0.125, trace=trace)
    seq, ptr, added_s, base_s = _simulate_merges(fund, structs, 0.125)
    assert base == base_s
    assert len(trace) == len(seq) and sum(1 for t in seq if t[0] == "merge") > 10
    for step, (got, want) in enumerate(zip(trace, seq)):
        assert tuple(int(v) if not isinstance(v, str) else v for v in got) == want, step
    assert seq[-1][0] == "stop" and added + seq[-1][2] > 0.125 * base
    assert added == added_s <= 0.125 * base
    assert np.array_equal(sn_ptr, ptr)
    # the merged partition is the one the analysis reports
    r = osym.analyze(A, merge_cap=0.125, reorder=False)
    assert np.array_equal(r["sn_ptr"], ptr)


def _pattern_from_edges(n, edges):
    A = np.eye(n) * 4.0
    for a, b in edges:
        A[a, b] = A[b, a] = -1.0
    return W.from_dense_lower(A)


def test_graph_nested_dissection_hand_cases():
    """Orderings worked out by hand from the rule (BFS levels from a
    pseudo-peripheral root, separator = first level reaching half the
    component, parts before/after dissected, separator last; leaves of at
    most 8 vertices and components of fewer than three levels ascending)."""
    path = _pattern_from_edges(20, [(i, i + 1) for i in range(19)])
    assert osym.graph_nested_dissection(path.n, path.colptr, path.rowidx).tolist() == \
        [0, 1, 2, 3, 5, 6, 7, 8, 4, 10, 11, 12, 13, 15, 16, 17, 18, 19, 14, 9]
    # components in the order of their smallest vertex, each on its own: a
    # path over the even vertices 0..18 (dissected at its fifth vertex), a
    # path 1-3-5 (a leaf) and the isolated vertices 7, 9, ..., 19, 20, 21
    two = _pattern_from_edges(22, [(i, i + 2) for i in range(0, 18, 2)] + [(1, 3), (3, 5)])
    assert osym.graph_nested_dissection(two.n, two.colptr, two.rowidx).tolist() == \
        [0, 2, 4, 6, 10, 12, 14, 16, 18, 8, 1, 3, 5, 7, 9, 11, 13, 15, 17, 19, 20, 21]
    # a clique of 12 has two levels from any root: emitted ascending
    clique = _pattern_from_edges(12, [(a, b) for a in range(12) for b in range(a)])
    assert osym.graph_nested_dissection(clique.n, clique.colptr, clique.rowidx).tolist() == \
        list(range(12))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_graph_nested_dissection_separates(seed):
    """Every split of the graph ordering: the separator removes every edge
    between the two parts, the three sets partition the component, and the
    final order is a permutation; and the product's ordering equals it."""
    from paper_2409_13090_amd import rlb
    A = W.irregular3d(1500 + 500 * seed, k=8, seed=seed)
    trace = []
    perm = osym.graph_nested_dissection(A.n, A.colptr, A.rowidx, trace=trace)
    assert np.array_equal(np.sort(perm), np.arange(A.n))
    assert len(trace) > 10
    adj = [set() for _ in range(A.n)]
    for j in range(A.n):
        for i in A.rowidx[A.colptr[j]:A.colptr[j + 1]]:
            if i != j:
                adj[i].add(j)
                adj[j].add(int(i))
    for before, after, sep in trace:
        b = set(before)
        assert not any(adj[v] & b for v in after)
        assert not (b & set(after)) and not (b & set(sep)) and not (set(after) & set(sep))
    s = rlb.Symbolic(A.n, A.colptr, A.rowidx, ordering="graph")
    assert np.array_equal(s.array("perm_nd"), perm)
