"""The product's host symbolic phase (C++, through the C-ABI) against the
oracle's naive analysis: every integer array bit for bit."""
import numpy as np
import pytest

from oracle import osym
from paper_2409_13090_amd import rlb
from paper_2409_13090_amd import workloads as W


def both(A, **kw):
    ordering = kw.pop("ordering", "grid")
    o = osym.analyze(A, ordering=ordering, merge_cap=kw.get("merge_cap", 0.125),
                     reorder=kw.get("reorder", True))
    s = rlb.Symbolic.from_matrix(A, ordering=ordering, **kw)
    return o, s


def flat(lists):
    return np.concatenate([np.asarray(x, np.int64) for x in lists]) if lists else np.zeros(0)


def assert_same(o, s):
    S = len(o["sn_ptr"]) - 1
    assert np.array_equal(s.array("perm_nd"), o["perm_nd"])
    assert np.array_equal(s.array("perm_post"), o["perm_post"])
    assert np.array_equal(s.array("etree_post"), o["parent_post"])
    assert np.array_equal(s.array("fund_ptr"), o["fund_ptr"])
    assert np.array_equal(s.array("sn_ptr"), o["sn_ptr"])
    assert np.array_equal(s.array("perm"), o["perm"])
    assert np.array_equal(s.array("etree"), o["parent"])
    assert np.array_equal(s.array("sn_parent"), o["sn_parent"])
    gp = s.array("gl_ptr")
    assert np.array_equal(np.diff(gp), [len(g) for g in o["glbind"]])
    assert np.array_equal(s.array("gl"), flat(o["glbind"]))
    assert np.array_equal(s.array("rel"), flat(o["relind"]))
    assert np.array_equal(np.diff(s.array("rel_ptr")), [len(r) for r in o["relind"]])
    assert np.array_equal(s.array("blk"), flat(o["blocks"]))
    assert np.array_equal(np.diff(s.array("blk_ptr")), [len(b) for b in o["blocks"]])
    # relindB(J, P) for every touched ancestor
    rbp, anc = s.array("rbp_ptr"), s.array("rbp_anc")
    rbv_ptr, rbv = s.array("rbv_ptr"), s.array("rbv")
    for J in range(S):
        pairs = o["relindB"][J]
        assert rbp[J + 1] - rbp[J] == len(pairs)
        for q, (P, vals) in zip(range(rbp[J], rbp[J + 1]), pairs):
            assert anc[q] == P
            assert np.array_equal(rbv[rbv_ptr[q]:rbv_ptr[q + 1]], vals)
    cc = s.array("colcount")
    assert np.array_equal(cc, [len(x) for x in o["structs"]])
    info = s.info()
    assert info["nnz_exact"] == osym.exact_nnz(o["structs"])
    assert info["flops_exact"] == osym.exact_flops(o["structs"])
    assert info["merge_added"] == o["merge_added"]


def fig1_matrix():
    pairs = [(2, 1), (5, 1), (6, 1), (9, 1), (5, 2), (9, 2), (4, 3), (5, 3), (7, 3), (8, 3),
             (5, 4), (8, 4), (6, 5), (8, 5), (7, 6), (9, 6), (8, 7), (9, 8)]
    Ad = np.zeros((9, 9))
    for i, j in pairs:
        Ad[i - 1, j - 1] = Ad[j - 1, i - 1] = -1.0
    Ad += np.diag(-Ad.sum(1) + 1.0)
    return W.from_dense_lower(Ad)


@pytest.mark.parametrize("reorder", [False, True])
def test_fig1_bit_exact(reorder):
    A = fig1_matrix()
    o, s = both(A, ordering="natural", merge_cap=0.0, reorder=reorder)
    assert_same(o, s)


CASES = [
    ("c1", lambda: W.config1()),
    ("2d9_37", lambda: W.small_grid("9pt", (37, 29, 1), seed=3)),
    ("3d7_16", lambda: W.small_grid("7pt", (16, 16, 16), seed=4)),
    ("3d7_13x11x9", lambda: W.small_grid("7pt", (13, 11, 9), seed=5)),
    ("3d27_10", lambda: W.small_grid("27pt", (10, 10, 10), seed=6)),
    ("elast_5", lambda: W.elasticity_like((5, 6, 5), np.random.default_rng(7), 1e-6)),
    ("batch_side16", lambda: W.batch_member(0)),
    ("thin_1d", lambda: W.small_grid("5pt", (40, 1, 1), seed=8)),
    ("tiny_2x2", lambda: W.small_grid("5pt", (2, 2, 1), seed=9)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_bit_exact_grids(name, make):
    A = make()
    o, s = both(A)
    assert_same(o, s)


@pytest.mark.parametrize("cap,reorder,maximal", [(0.0, True, True), (0.25, False, True),
                                                 (0.125, True, False)])
def test_bit_exact_options(cap, reorder, maximal):
    A = W.small_grid("7pt", (11, 10, 9), seed=10)
    o = osym.analyze(A, merge_cap=cap, reorder=reorder)
    s = rlb.Symbolic.from_matrix(A, merge_cap=cap, reorder=reorder, maximal_blocks=maximal)
    assert_same(o, s)


def test_bit_exact_user_and_natural_orderings():
    A = W.small_grid("9pt", (15, 14, 1), seed=11)
    rng = np.random.default_rng(12)
    up = rng.permutation(A.n)
    o = osym.analyze(A, ordering="user", user_perm=up)
    s = rlb.Symbolic.from_matrix(A, ordering="user", user_perm=up)
    assert_same(o, s)
    o = osym.analyze(A, ordering="natural")
    s = rlb.Symbolic.from_matrix(A, ordering="natural")
    assert_same(o, s)


def test_amap_places_every_entry_in_its_supernode():
    A = W.small_grid("7pt", (9, 8, 7), seed=13)
    s = rlb.Symbolic.from_matrix(A)
    amap = s.array("amap")
    off = s.array("off")
    sn = s.array("sn_ptr")
    gp, gl = s.array("gl_ptr"), s.array("gl")
    perm = s.array("perm")
    inv = np.empty(A.n, np.int64)
    inv[perm] = np.arange(A.n)
    assert len(np.unique(amap)) == A.nnz
    cols = np.repeat(np.arange(A.n), np.diff(A.colptr))
    for e in range(A.nnz):
        a, b = inv[A.rowidx[e]], inv[cols[e]]
        r, c = max(a, b), min(a, b)
        J = np.searchsorted(sn, c, side="right") - 1
        m = gp[J + 1] - gp[J]
        pos = amap[e] - off[J]
        assert pos // m == c - sn[J]
        assert gl[gp[J] + pos % m] == r
