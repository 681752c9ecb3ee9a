"""The device work lists (panel groups, update target tiles with their
contributions, diagonal-tile inverses, solve steps), replayed on the CPU with
numpy exactly as the kernels index factor storage, reproduce the oracle's
factor (Algorithm 1) and solve A x = b to backward error ~1e-16.

This pins the host lowering of Alg. 5 (storage offsets, ancestor rectangles
cut by the target tile grid, relind-based target positions, level and step
order, single-owner / split ownership of target tiles, the previous block's
update applied inside a panel launch and the update tiles that run beside its
workgroups) independently of the GPU. Each kernel's dense block arithmetic is
replaced by numpy here, so only the indexing and the ordering are under test."""
import numpy as np
import pytest

from parity_util import compare_factor, oracle_factor
from paper_2409_13090_amd import rlb
from paper_2409_13090_amd import workloads as W


def unfused(launches):
    """The launch list with every fused panel step expanded into the previous
    step's update launch (the tiles beside the panels and the ones the panels
    apply themselves) followed by plain panel launches, as the batch runs it."""
    out, done = [], set()
    for j, l in enumerate(launches):
        kind, lev, step, st, cnt, variant, pre, ust, ucnt, ncnt, ast, acnt = (int(v) for v in l)
        if kind == 0 and pre:
            if (lev, step) not in done:
                done.add((lev, step))
                for q in launches[j:]:
                    if int(q[0]) != 0 or int(q[1]) != lev or int(q[2]) != step:
                        break
                    if int(q[8]) + int(q[9]) > 0:
                        out.append((1, lev, step - 1, int(q[7]), int(q[8]) + int(q[9]), 1, 0, 0, 0,
                                    0, 0, 0))
            out.append((kind, lev, step, st, cnt, variant, 0, 0, 0, 0, 0, 0))
        else:
            out.append((kind, lev, step, st, cnt, variant, pre, ust, ucnt, ncnt, ast, acnt))
    return out


def with_alt(launches):
    """Launches of 128x128 or 128x64 target tiles replaced by the same work in
    64x64 tiles, as the reduced-precision update forms run them."""
    out = []
    for l in launches:
        l = [int(v) for v in l]
        if l[0] == 1 and l[5] in (2, 6):
            assert l[11] > 0
            l[3], l[4], l[5] = l[10], l[11], 0
        out.append(tuple(l))
    return out


def replay_factor(A, expand=False, alt=False, **kw):
    s = rlb.Symbolic.from_matrix(A, **kw)
    size = s.info()["factor_bytes"] // 8
    Lb = np.zeros(size)
    Lb[s.array("amap")] = A.values
    U = s.array("update_tiles").reshape(-1, 7)
    G = s.array("update_segs").reshape(-1, 9)
    P = s.array("panel_tiles").reshape(-1, 11)

    def updates(tiles):
        """Every target tile sums its contributions, then subtracts them once;
        returns the entries read (sources) and written (targets)."""
        owner, reads = {}, set()
        for c, ldc, m, n, flags, seg0, nseg in tiles:
            acc = np.zeros((m, n))
            for x, y, lds, k, ra, rb, ca, cb, src in G[seg0:seg0 + nseg]:
                assert 0 <= ra < rb <= m and 0 <= ca < cb <= n and k > 0
                assert x + (k - 1) * lds + (rb - ra) - 1 < size
                assert y + (k - 1) * lds + (cb - ca) - 1 < size
                X = np.array([Lb[x + q * lds: x + q * lds + (rb - ra)] for q in range(k)]).T
                Y = np.array([Lb[y + q * lds: y + q * lds + (cb - ca)] for q in range(k)]).T
                acc[ra:rb, ca:cb] += X @ Y.T
                for q in range(k):
                    reads.update(range(x + q * lds, x + q * lds + rb - ra))
                    reads.update(range(y + q * lds, y + q * lds + cb - ca))
            for j in range(n):
                for r in range(m):
                    prev = owner.get(c + j * ldc + r)
                    # one owner per entry, except the parts of a split tile
                    assert prev is None or (prev and (flags & 2)), "two owners"
                    owner[c + j * ldc + r] = bool(flags & 2)
                col = acc[:, j].copy()
                if flags & 4:  # RL's update matrix: written, not added (lower part)
                    lo = j if flags & 1 else 0
                    Lb[c + j * ldc + lo: c + j * ldc + m] = -col[lo:]
                    continue
                if flags & 1:
                    col[:j] = 0.0
                Lb[c + j * ldc: c + j * ldc + m] -= col
        return reads, set(owner)

    launches = s.array("launches").reshape(-1, 12)
    if expand:
        launches = unfused(launches)
    if alt:
        launches = with_alt(launches)
    AC = s.array("asm_cols").reshape(-1, 4)
    AR = s.array("asm_rows")
    PR = s.array("part_reduces").reshape(-1, 7)
    for kind, lev, step, st, cnt, variant, pre, ust, ucnt, ncnt, ast, acnt in launches:
        if kind == 3:
            # the parts of split tiles (64x64 blocks, -(their sums)) added into
            # their tiles in part order
            for c, pbase, ldc, m, n, flags, nparts in PR[st:st + cnt]:
                assert nparts >= 2 and pbase + 4096 * nparts <= size
                for j in range(n):
                    lo = j if flags & 1 else 0
                    acc = Lb[pbase + 64 * j + lo: pbase + 64 * j + m].copy()
                    for q in range(1, nparts):
                        acc += Lb[pbase + 4096 * q + 64 * j + lo: pbase + 4096 * q + 64 * j + m]
                    Lb[c + j * ldc + lo: c + j * ldc + m] += acc
            continue
        if kind == 2:
            # RL: every update-matrix column added into its ancestor column
            for src, dst, rp, ln in AC[st:st + cnt]:
                Lb[dst + AR[rp:rp + ln]] += Lb[src:src + ln]
            continue
        if kind == 0:
            groups = {}
            for t in P[st:st + cnt]:
                groups.setdefault(int(t[7]), []).append(t)
            touched = set()
            for mem in groups.values():
                assert len(mem) == mem[0][8], "group size"
                diag, ld, nb, nrows = (int(v) for v in mem[0][:4])
                assert nb <= 16 * variant
                D = np.array([Lb[diag + j * ld: diag + j * ld + nb] for j in range(nb)]).T
                if pre:
                    # the previous 64-column block's update of this column block
                    assert step >= 1 and diag - 64 * ld >= 0
                    Y = np.array([Lb[diag + (q - 64) * ld: diag + (q - 64) * ld + nb]
                                  for q in range(64)]).T
                    D = D - Y @ Y.T
                Lt = np.linalg.cholesky(np.tril(D) + np.tril(D, -1).T)
                covered = 0
                for t in mem:
                    for rt in range(int(t[10])):
                        row0 = int(t[4]) + 64 * rt
                        r1 = min(row0 + 64, nrows)
                        assert nb <= row0 < nrows and diag + (nb - 1) * ld + r1 - 1 < size
                        Arow = np.array([Lb[diag + j * ld + row0: diag + j * ld + r1]
                                         for j in range(nb)]).T
                        if pre:
                            X = np.array([Lb[diag + (q - 64) * ld + row0: diag + (q - 64) * ld + r1]
                                          for q in range(64)]).T
                            Arow = Arow - X @ Y.T
                        Xr = np.linalg.solve(Lt, Arow.T).T
                        for j in range(nb):
                            Lb[diag + j * ld + row0: diag + j * ld + r1] = Xr[:, j]
                        covered += r1 - row0
                assert covered == nrows - nb, "row tiles cover the panel once"
                for j in range(nb):
                    Lb[diag + j * ld + j: diag + j * ld + nb] = Lt[j:, j]
                for j in range(nb):
                    touched.update(range(diag + j * ld, diag + j * ld + nrows))

            if ucnt:
                # the previous step's remaining update tiles run in the same
                # launch: they may neither write nor read the column blocks
                # the panel workgroups write
                assert pre
                reads, writes = updates(U[ust:ust + ucnt])
                assert not (reads & touched) and not (writes & touched), "fused overlap"
                assert all(int(U[i][6]) == 1 and G[int(U[i][5])][3] <= 64
                           for i in range(ust, ust + ucnt))
        else:
            tiles = U[st:st + cnt]
            rows = 128 if variant in (2, 6) else 64
            cols = 128 if variant == 2 else 64
            assert all(m <= rows and n <= cols for _, _, m, n, _, _, _ in tiles)
            updates(tiles)
    for diag, ld, nb in s.array("diag_tiles").reshape(-1, 3):
        Lt = np.array([[Lb[diag + j * ld + i] if i >= j else 0.0 for j in range(nb)]
                       for i in range(nb)])
        Li = np.linalg.inv(Lt)
        for j in range(nb):
            Lb[diag + j * ld: diag + j * ld + j] = Li[j, :j]
    return s, Lb


def export(s, Lb):
    sn, gp, gl, off = s.array("sn_ptr"), s.array("gl_ptr"), s.array("gl"), s.array("off")
    cp, ri, vx = [0], [], []
    for J in range(len(sn) - 1):
        w, m = sn[J + 1] - sn[J], gp[J + 1] - gp[J]
        for c in range(w):
            for r in range(c, m):
                ri.append(gl[gp[J] + r])
                vx.append(Lb[off[J] + c * m + r])
            cp.append(len(ri))
    return np.array(cp), np.array(ri), np.array(vx)


def replay_solve(s, Lb, B):
    perm, gl = s.array("perm"), s.array("gl")
    T = s.array("solve_tiles").reshape(-1, 11)
    nrhs = B.shape[1]
    y = B[perm].copy()
    z = np.full_like(y, np.nan)
    x = np.full_like(y, np.nan)

    def inv_tile(off, ld, c0, nb):
        assert nb <= 64
        V = np.zeros((nb, nb))
        for i in range(nb):
            V[i, i] = 1.0 / Lb[off + (c0 + i) * ld + c0 + i]
            V[i, :i] = Lb[off + (c0 + i) * ld + c0: off + (c0 + i) * ld + c0 + i]
        return V

    def diag_solve(off, ld, c0, nb, rhs, transposed):
        """One or two 64-column chunks: the stored inverses of their diagonal
        tiles and the block between them, as the step kernels use them."""
        if nb <= 64:
            V = inv_tile(off, ld, c0, nb)
            return (V.T if transposed else V) @ rhs
        nbb = nb - 64
        VA, VB = inv_tile(off, ld, c0, 64), inv_tile(off, ld, c0 + 64, nbb)
        LBA = np.array([[Lb[off + (c0 + c) * ld + c0 + 64 + i] for c in range(64)]
                        for i in range(nbb)])
        if not transposed:
            xa = VA @ rhs[:64]
            xb = VB @ (rhs[64:] - LBA @ xa)
        else:
            xb = VB.T @ rhs[64:]
            xa = VA.T @ (rhs[:64] - LBA.T @ xb)
        return np.concatenate([xa, xb])

    need = s.array("solve_need")
    for kind, lev, st, cnt, chain in s.array("solve_launches").reshape(-1, 5):
        # a chained launch runs its tiles concurrently, each after the
        # earlier tiles of the launch that write into the columns it reads
        # have signalled its step counter: count those writers from the
        # write sets themselves and compare with the plan's signal counts
        writers = {}  # global column -> earlier tiles of the launch writing it
        for ti, (off, ld, f, w, g0, c0, nb, r0, r1, flags, cslot) in enumerate(T[st:st + cnt]):
            if chain >= 0 and kind != 1:
                reads = set()
                for col in range(f + c0, f + c0 + nb):
                    reads |= writers.get(col, set())
                if cslot >= 0:
                    assert len(reads) == need[cslot + c0 // 128], (kind, lev, ti)
                else:
                    assert not reads, "a tile without a counter reads what the launch writes"
                if kind == 0:
                    written = [gl[g0 + q] for q in range(r0, r1)]
                else:
                    written = list(range(f + r0, f + r1))
                for col in written:
                    writers.setdefault(col, set()).add(ti)
        for off, ld, f, w, g0, c0, nb, r0, r1, flags, _ in T[st:st + cnt]:
            assert 1 <= nb <= 128
            # kernels of the two-chunk steps split the work by chunk (flags bit 1)
            half = (flags >> 1) & 1
            assert half == 0 or nb > 64
            ca, cb = 64 * half, min(nb, 64 * (half + 1))
            if kind == 0:
                xk = diag_solve(off, ld, c0, nb, y[f + c0: f + c0 + nb], False)[ca:cb]
                if flags & 1:
                    z[f + c0 + ca: f + c0 + cb] = xk
                for q in range(r0, r1):
                    lrow = Lb[off + (c0 + ca) * ld + q: off + (c0 + cb) * ld + q: ld]
                    y[gl[g0 + q]] -= lrow @ xk
            elif kind == 1:
                assert w <= r0 < r1 <= ld and nb <= 64
                for q in range(r0, r1):
                    lrow = Lb[off + c0 * ld + q: off + (c0 + nb) * ld + q: ld]
                    assert not np.isnan(x[gl[g0 + q]]).any(), "ancestor solved first"
                    z[f + c0: f + c0 + nb] -= np.outer(lrow, x[gl[g0 + q]])
            else:
                zk = z[f + c0: f + c0 + nb]
                assert not np.isnan(zk).any(), "forward result present"
                xk = diag_solve(off, ld, c0, nb, zk, True)[ca:cb]
                if flags & 1:
                    x[f + c0 + ca: f + c0 + cb] = xk
                assert r1 == r0 or (r1 - r0 <= 64 and r1 <= c0), "push into earlier columns"
                if r1 > r0:
                    Lblk = np.array([[Lb[off + (r0 + c) * ld + c0 + ca + i] for c in range(r1 - r0)]
                                     for i in range(cb - ca)])
                    z[f + r0: f + r1] -= Lblk.T @ xk
    out = np.empty_like(x)
    out[perm] = x
    return out


CASES = [
    ("c1_lap2d5_30", lambda: W.config1(), {}),
    ("lap3d7_17", lambda: W.small_grid("7pt", (17, 17, 17), seed=3), {}),
    ("lap3d27_11x11x9_spread3", lambda: W.small_grid("27pt", (11, 11, 9), seed=26, shift=1e-3),
     {"panel_spread": 3}),
    ("elast_6x6x5", lambda: W.elasticity_like((6, 6, 5), np.random.default_rng(7), 1e-6), {}),
    ("batch_member_7", lambda: W.batch_member(7), {}),
    # outer blocks of 128 columns and 128x128 target tiles in every long part
    ("lap3d27_13_outer128_big", lambda: W.small_grid("27pt", (13, 13, 13), seed=24, lo=0.1,
                                                     hi=1.0, shift=1e-4),
     {"outer_block": 128, "big_tile_min": 1}),
    ("lap3d7_17_outer64_big", lambda: W.small_grid("7pt", (17, 17, 17), seed=3),
     {"outer_block": 64, "big_tile_min": 1}),
    ("lap3d27_11x11x9_atomic_big", lambda: W.small_grid("27pt", (11, 11, 9), seed=26, shift=1e-3),
     {"outer_block": 128, "big_tile_min": 1, "deterministic": False}),
    # RL (Algorithm 4): update matrices in working storage, then assembly
    ("rl_lap3d27_13", lambda: W.small_grid("27pt", (13, 13, 13), seed=24, lo=0.1, hi=1.0,
                                           shift=1e-4), {"method": "rl"}),
    ("rl_lap2d9_45x38", lambda: W.small_grid("9pt", (45, 38, 1), seed=21), {"method": "rl"}),
    # hybrid: RL's update matrices for some supernodes, in-place updates for the rest
    ("hybrid_lap3d27_13", lambda: W.small_grid("27pt", (13, 13, 13), seed=24, lo=0.1, hi=1.0,
                                               shift=1e-4),
     {"method": "hybrid", "hybrid_step_us": -1}),
    ("hybrid_irregular_3000", lambda: W.irregular3d(3000, k=10, seed=40),
     {"method": "hybrid", "hybrid_step_us": -1, "ordering": "graph"}),
    # 128x64 target tiles for the long updates (outer blocks and ancestors)
    ("lap3d27_13_outer128_tall", lambda: W.small_grid("27pt", (13, 13, 13), seed=24, lo=0.1,
                                                      hi=1.0, shift=1e-4),
     {"outer_block": 128, "tall_tile_min": 1}),
    ("lap3d7_17_tall", lambda: W.small_grid("7pt", (17, 17, 17), seed=22, shift=1e-4),
     {"tall_tile_min": 1}),
    ("irregular_3000_tall", lambda: W.irregular3d(3000, k=10, seed=40),
     {"tall_tile_min": 1, "ordering": "graph"}),
    # several wide supernodes in one level, outer blocks of 64 columns
    ("lap3d27_16_outer64", lambda: W.small_grid("27pt", (16, 16, 16), seed=27, lo=0.1, hi=1.0,
                                                shift=1e-4),
     {"outer_block": 64}),
    # several outer blocks of 64 columns
    ("lap3d27_14_outer64", lambda: W.small_grid("27pt", (14, 14, 14), seed=25, lo=0.1, hi=1.0,
                                                shift=1e-4),
     {"outer_block": 64}),
    # heavy target tiles cut into parts that a reduce launch sums in order
    ("lap3d27_13_split", lambda: W.small_grid("27pt", (13, 13, 13), seed=24, lo=0.1, hi=1.0,
                                              shift=1e-4),
     {"split_chunks": 2}),
    ("irregular_3000_split", lambda: W.irregular3d(3000, k=10, seed=40),
     {"split_chunks": 3, "ordering": "graph"}),
    # the automatic rule: tiles above the balanced share of launches with a long tail
    ("irregular_3000_split_auto", lambda: W.irregular3d(3000, k=10, seed=40),
     {"split_chunks": -1, "ordering": "graph"}),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_work_lists_replayed_match_oracle(name, make, kw):
    A = make()
    s, Lb = replay_factor(A, **kw)
    o, f = oracle_factor(A, **({"ordering": kw["ordering"]} if "ordering" in kw else {}))
    err = compare_factor(export(s, Lb), f, A.n)
    assert err <= 1e-12
    # the unfused form (the batch's) reaches the same factor
    s2, Lb2 = replay_factor(A, expand=True, **kw)
    assert compare_factor(export(s2, Lb2), f, A.n) <= 1e-12
    L12 = s.array("launches").reshape(-1, 12)
    if kw.get("split_chunks", 0) != 0:
        # heavy tiles were cut: every reduce follows the update launch of its parts
        red = np.flatnonzero(L12[:, 0] == 3)
        assert red.size and np.all(L12[red - 1, 0] == 1)
    if kw.get("tall_tile_min") == 1:
        # the long parts went to 128x64 tiles; their 64x64 form (FP32, 16-bit) too
        assert np.any((L12[:, 0] == 1) & (L12[:, 5] == 6))
        s5, Lb5 = replay_factor(A, alt=True, **kw)
        assert compare_factor(export(s5, Lb5), f, A.n) <= 1e-12
    if kw.get("big_tile_min") == 1:
        # the long parts went to 128x128 tiles; their 64x64 form (16-bit) too
        assert np.any((L12[:, 0] == 1) & (L12[:, 5] == 2))
        s3, Lb3 = replay_factor(A, alt=True, **kw)
        assert compare_factor(export(s3, Lb3), f, A.n) <= 1e-12
    # algorithmic flops of the tiles of update launches of their own, from the
    # exported lists (entries written, lower part only on diagonal tiles)
    U = s.array("update_tiles").reshape(-1, 7)
    G = s.array("update_segs").reshape(-1, 9)
    fl = 0.0
    for l in s.array("launches").reshape(-1, 12):
        if l[0] != 1:
            continue
        for c, ldc, m, n, flags, seg0, nseg in U[l[3]:l[3] + l[4]]:
            for x, y, lds, k, ra, rb, ca, cb, src in G[seg0:seg0 + nseg]:
                ent = sum(max(0, rb - max(ra, j)) for j in range(ca, cb)) if flags & 1 \
                    else (rb - ra) * (cb - ca)
                fl += 2.0 * k * ent
    info = s.info()
    assert fl == pytest.approx(info["flops_upd_launch"], rel=1e-12)
    assert info["flops_upd_launch"] <= info["flops_upd_alg"] * (1 + 1e-12)
    B = np.random.default_rng(0).standard_normal((A.n, 3))
    X = replay_solve(s, Lb, B)
    Af = A.to_scipy_full()
    be = np.abs(Af @ X - B).max(axis=0) / (abs(Af).sum(axis=1).max() * np.abs(X).max(axis=0))
    assert be.max() <= 1e-14, be


@pytest.mark.parametrize("name,make,kw", [
    ("lap2d9_45x38", lambda: W.small_grid("9pt", (45, 38, 1), seed=21), {}),
    ("batch_member_7", lambda: W.batch_member(7), {}),
    ("irregular_3000", lambda: W.irregular3d(3000, k=10, seed=40), {"ordering": "graph"}),
])
def test_update_variant_follows_chunk_rounds(name, make, kw):
    """Each update launch's kernel variant is the way of staging K with the
    fewest chunk rounds, taken only when it saves at least 30 %: KCH = 16 deep
    chunks of every contribution (dense), chunks shaped to the contribution's
    rectangle (16- and 32-row windows 4 and 2 times deeper), or the tile's
    contributions end to end, each padded to a multiple of 4 (packed). The
    2D lower levels take the packed form."""
    s = rlb.Symbolic.from_matrix(make(), **kw)
    L = s.array("launches").reshape(-1, 12)
    U = s.array("update_tiles").reshape(-1, 7)
    G = s.array("update_segs").reshape(-1, 9)
    seen = set()
    for l in L:
        kind, st, cnt, var = int(l[0]), int(l[3]), int(l[4]), int(l[5])
        if kind != 1 or var not in (0, 4, 5):
            continue
        rounds = win = pack = 0
        for t in U[st:st + cnt]:
            g = G[t[5]:t[5] + t[6]]
            k, ra, rb, ca, cb = g[:, 3], g[:, 4], g[:, 5], g[:, 6], g[:, 7]
            r16 = ((ra >> 4) == ((rb - 1) >> 4)) & ((ca >> 4) == ((cb - 1) >> 4))
            r32 = ((ra >> 5) == ((rb - 1) >> 5)) & ((ca >> 5) == ((cb - 1) >> 5))
            kc = np.where(r16, 64, np.where(r32, 32, 16))
            rounds += int(((k + 15) // 16).sum())
            win += int(((k + kc - 1) // kc).sum())
            pack += -(-int(((k + 3) & ~3).sum()) // 16)
        best = min(win, pack)
        want = 0 if 10 * best > 7 * rounds else (5 if pack < win else 4)
        assert var == want, (name, var, rounds, win, pack)
        seen.add(var)
    if name != "irregular_3000":
        assert 5 in seen, seen


def test_split_rule_cuts_only_long_tails():
    """The automatic cut (split_chunks < 0): in every update launch it cuts,
    the heaviest original tile held more than twice the launch's balanced
    share of K chunks; the parts of a cut tile are assign tiles into
    consecutive 64x64 workspace blocks past the factor storage, each part at
    most about half a share, and together they carry the tile's K chunks.
    Off by default (Algorithm 5 writes every update in place)."""
    A = W.irregular3d(3000, k=10, seed=40)
    assert rlb.Symbolic.from_matrix(A, ordering="graph").info()["n_split_tiles"] == 0
    s = rlb.Symbolic.from_matrix(A, ordering="graph", split_chunks=-1)
    L = s.array("launches").reshape(-1, 12)
    U = s.array("update_tiles").reshape(-1, 7)
    G = s.array("update_segs").reshape(-1, 9)
    PR = s.array("part_reduces").reshape(-1, 7)
    lel = int(s.array("off")[-1])
    red = np.flatnonzero(L[:, 0] == 3)
    assert red.size >= 1
    for j in red:
        up = L[j - 1]
        assert up[0] == 1 and up[1] == L[j, 1] and up[2] == L[j, 2]
        tiles = U[up[3]:up[3] + up[4]]
        chunks = np.array([int(((G[t[5]:t[5] + t[6], 3] + 15) // 16).sum()) for t in tiles])
        recs = PR[L[j, 3]:L[j, 3] + L[j, 4]]
        is_part = (tiles[:, 4] & 4) != 0
        assert is_part.sum() == recs[:, 6].sum()
        # the launch's tiles before the cut: parts regrouped into their tiles
        whole = list(chunks[~is_part])
        by_block = {int(t[0]): c for t, c in zip(tiles[is_part], chunks[is_part])}
        for c, pbase, ldc, m, n, flags, nparts in recs:
            assert pbase >= lel and nparts >= 2
            parts = [by_block[int(pbase) + 4096 * q] for q in range(nparts)]
            whole.append(sum(parts))
            assert max(parts) <= min(parts) + 1 + max(parts) // 2  # nearly even parts
        share = sum(whole) / min(len(whole), 1024)
        assert max(whole) > 2 * share
        for (c, pbase, ldc, m, n, flags, nparts) in recs:
            assert sum(by_block[int(pbase) + 4096 * q] for q in range(nparts)) > share
