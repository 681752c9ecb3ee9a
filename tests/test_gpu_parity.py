"""Device path (HIP kernels through the C-ABI) against the CPU oracle.

Small and medium matrices are compared element by element (structure rule:
the oracle's exact structure lies inside the stored structure and every
stored-only entry is exactly 0.0; values within relative Frobenius 1e-10).
The 48^3 workload is compared on the columns the oracle can afford (a prefix
of the factored order, which Algorithm 1 computes exactly on its own) and on
properties of the whole factor."""
import numpy as np
import pytest

from parity_util import (FP64_TOL, compare_factor, factor_elems, gpu_factor, oracle_factor,
                         probe_residual)
from paper_2409_13090_amd import rlb
from paper_2409_13090_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    return torch


def cpu_backward_error(A, B, X):
    """||b - A x||_inf / (||A||_inf ||x||_inf) per column, from A on the host
    (scipy), independent of the device's residual and norm kernels."""
    Af = A.to_scipy_full()
    b = np.asarray(B, dtype=np.float64).reshape(A.n, -1, order="F")
    x = np.asarray(X, dtype=np.float64).reshape(A.n, -1, order="F")
    r = b - Af @ x
    anorm = np.abs(Af).sum(axis=1).max()
    return np.abs(r).max(axis=0) / (anorm * np.abs(x).max(axis=0))


def solve_check(num, A, tol=1e-14):
    torch = _torch()
    B = torch.from_numpy(np.asfortranarray(A.rhs)).cuda()
    B = B.T.contiguous().T if B.dim() == 2 else B
    X = B.clone()
    X = X.T.contiguous().T
    num.solve(X)
    be = num.backward_error(B, X)
    assert np.all(be <= tol), be
    # the host's backward error of the device's x meets the same bound
    be_cpu = cpu_backward_error(A, A.rhs, X.cpu().numpy())
    assert np.all(be_cpu <= tol), be_cpu
    # at roundoff level both are noise; for an x perturbed by 1e-6 (relative)
    # the residual is A times the perturbation, and the device's residual
    # and norm kernels must give the host's value closely
    rng = np.random.default_rng(5)
    xp = X.cpu().numpy() * (1.0 + 1e-6 * rng.uniform(-1.0, 1.0, X.shape))
    Xp = torch.from_numpy(np.asfortranarray(xp)).cuda()
    Xp = Xp.T.contiguous().T if Xp.dim() == 2 else Xp
    bp = num.backward_error(B, Xp)
    bp_cpu = cpu_backward_error(A, A.rhs, xp)
    assert np.all(bp_cpu > 1e-9), bp_cpu
    assert np.allclose(bp, bp_cpu, rtol=1e-8, atol=0.0), (bp, bp_cpu)
    return be


CASES = [
    ("c1_lap2d5_30", lambda: W.config1()),
    ("lap2d9_45x38", lambda: W.small_grid("9pt", (45, 38, 1), seed=21)),
    ("lap3d7_17", lambda: W.small_grid("7pt", (17, 17, 17), seed=22, shift=1e-4)),
    ("lap3d7_23x19x15", lambda: W.small_grid("7pt", (23, 19, 15), seed=23)),
    ("lap3d27_13", lambda: W.small_grid("27pt", (13, 13, 13), seed=24, lo=0.1, hi=1.0,
                                        shift=1e-4)),
    ("elast_7x6x6", lambda: W.elasticity_like((7, 6, 6), np.random.default_rng(25), 1e-6)),
    ("batch_member_7", lambda: W.batch_member(7)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_factor_matches_oracle(name, make):
    A = make()
    print(f"[case] {name} n={A.n} nnz={A.nnz}", flush=True)
    o, f = oracle_factor(A)
    s, num, vals, info = gpu_factor(A)
    assert info == 0 and f["info"] == 0
    assert np.array_equal(s.array("perm"), o["perm"])
    if name in ("lap2d9_45x38", "batch_member_7"):
        # the 2D lower levels take the contributions end to end along K
        L = s.array("launches").reshape(-1, 12)
        assert ((L[:, 0] == 1) & (L[:, 5] == 5)).sum() >= 1
    err = compare_factor(num.export(), f, A.n)
    print(f"[case] {name} rel_err={err:.3e}", flush=True)
    if A.rhs is not None:
        solve_check(num, A)


def test_supernode_wider_than_many_panels():
    """A dense-ish 3D block whose top separator spans several 64-column panels
    and ragged tails (widths not multiples of 64)."""
    A = W.small_grid("27pt", (11, 11, 9), seed=26, shift=1e-3)
    s = rlb.Symbolic.from_matrix(A)
    sn = s.array("sn_ptr")
    assert np.max(np.diff(sn)) > 128 and np.max(np.diff(sn)) % 64 != 0
    o, f = oracle_factor(A)
    s2, num, vals, info = gpu_factor(A)
    compare_factor(num.export(), f, A.n)


def test_panel_workgroups_with_several_row_tiles():
    """Panel launches whose workgroups each take several consecutive 64-row
    tiles (the spread of busy launches, forced low here)."""
    A = W.small_grid("7pt", (17, 17, 17), seed=33, shift=1e-4)
    s = rlb.Symbolic.from_matrix(A, panel_spread=3)
    assert s.array("panel_tiles").reshape(-1, 11)[:, 10].max() > 1
    o, f = oracle_factor(A)
    s2, num, vals, info = gpu_factor(A, panel_spread=3)
    assert info == 0
    compare_factor(num.export(), f, A.n)
    solve_check(num, A)


def test_narrow_tiles_run_one_per_wavefront():
    """A 2D grid large enough that an update launch holds more than 1024 narrow
    target tiles (<= 16 columns) and a panel launch more than 1024 column
    blocks of at most 16 columns, which then run one per wavefront."""
    A = W.small_grid("9pt", (320, 300, 1), seed=41)
    s = rlb.Symbolic.from_matrix(A)
    T = s.array("update_tiles").reshape(-1, 7)
    L = s.array("launches").reshape(-1, 12)
    most = 0
    for l in L[L[:, 0] == 1]:
        c = 0
        for _, _, m, n, _, _, _ in T[l[3]:l[3] + l[4]]:
            if n <= 16:
                c += 1
        most = max(most, c)
    assert most >= 1024, most
    narrow_panels = [l[4] for l in L if l[0] == 0 and l[5] == 1 and l[6] == 0]
    assert max(narrow_panels) >= 1024, narrow_panels
    o, f = oracle_factor(A)
    s2, num, vals, info = gpu_factor(A)
    assert info == 0
    compare_factor(num.export(), f, A.n)
    solve_check(num, A)


def test_edge_cases_tiny_diagonal_chain():
    torch = _torch()
    # n = 1
    A = W.from_dense_lower(np.array([[4.0]]))
    s, num, vals, info = gpu_factor(A)
    cp, ri, vx = num.export()
    assert info == 0 and vx[0] == 2.0
    # diagonal: no updates at all
    d = np.arange(1.0, 40.0)
    A = W.from_dense_lower(np.diag(d))
    s, num, vals, info = gpu_factor(A)
    cp, ri, vx = num.export()
    assert np.array_equal(vx, np.sqrt(d))
    # tridiagonal chain (one supernode after merging), closed form
    n = 200
    Ad = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    A = W.from_dense_lower(Ad)
    o, f = oracle_factor(A, ordering="natural")
    s, num, vals, info = gpu_factor(A, ordering="natural")
    compare_factor(num.export(), f, n)
    k = np.arange(1, n + 1, dtype=float)
    L = np.zeros((n, n))
    cp, ri, vx = num.export()
    for j in range(n):
        L[ri[cp[j]:cp[j + 1]], j] = vx[cp[j]:cp[j + 1]]
    assert np.allclose(np.diag(L), np.sqrt((k + 1) / k), rtol=1e-13)
    # no merging, no reordering
    A = W.small_grid("7pt", (9, 9, 9), seed=27)
    o, f = oracle_factor(A, merge_cap=0.0, reorder=False)
    s, num, vals, info = gpu_factor(A, merge_cap=0.0, reorder=False)
    compare_factor(num.export(), f, A.n)


def test_empty_matrix_through_every_call():
    """Order 0: factor, status, export, both solves, backward error and
    refinement accept the empty buffers (null device pointers), and a batch
    with an empty member between two others gives those two the bits of
    their own single factorizations."""
    torch = _torch()
    E = W.from_dense_lower(np.zeros((0, 0)))
    s, num, vals, info = gpu_factor(E)
    assert info == 0
    cp, ri, vx = num.export()
    assert cp.tolist() == [0] and ri.size == 0 and vx.size == 0
    X = torch.zeros(0, dtype=torch.float64, device="cuda")
    num.solve(X)
    num.solve_noalloc(X)
    assert num.backward_error(X, X).tolist() == [0.0]
    rep = num.refine(X, X.clone())
    assert rep["converged"] and rep["iterations"] == 0
    mats = [W.batch_member(0), E, W.batch_member(1)]
    syms = [rlb.Symbolic.from_matrix(A) for A in mats]
    b = rlb.Batch(syms)
    bv = [torch.from_numpy(A.values).cuda() for A in mats]
    assert np.all(b.factor(bv) == 0)
    ws_b = b.workspace.cpu().numpy()
    elems = [sy.info()["factor_bytes"] // 8 for sy in syms]
    assert elems[1] == 0
    base = np.concatenate([[0], np.cumsum(elems)])
    for i in (0, 2):
        single = rlb.Numeric(syms[i])
        assert single.factor(bv[i]) == 0
        nf = factor_elems(syms[i])
        assert np.array_equal(ws_b[base[i]:base[i] + nf],
                              single.workspace[:nf].cpu().numpy()), i
    b.solve(1, torch.zeros(0, dtype=torch.float64, device="cuda"))
    B = torch.from_numpy(mats[2].rhs[:, 0].copy()).cuda()
    Xb = B.clone()
    b.solve(2, Xb)
    single = rlb.Numeric(syms[2])
    single.factor(bv[2])
    assert single.backward_error(B, Xb)[0] <= 1e-14


def test_not_positive_definite_reports_oracle_column():
    A = W.small_grid("7pt", (10, 10, 10), seed=28)
    # make it indefinite: a large negative shift on a set of late diagonals
    A.values = A.values.copy()
    diag_pos = A.colptr[:-1]
    A.values[diag_pos[700:]] -= 50.0
    o, f = oracle_factor(A)
    assert f["info"] > 0
    s, num, vals, info = gpu_factor(A)
    assert info == f["info"]
    with pytest.raises(rlb.RlbError):
        torch = _torch()
        num.solve(torch.zeros(A.n, dtype=torch.float64, device="cuda"))


def test_repeat_factor_is_stable_and_graph_replay_matches():
    torch = _torch()
    A = W.small_grid("7pt", (14, 13, 12), seed=29)
    o, f = oracle_factor(A)
    s, num, vals, info = gpu_factor(A)
    ref = num.export()[2].copy()
    compare_factor(num.export(), f, A.n)
    num2 = rlb.Numeric(s)
    num2.set_graph_mode(True)
    for rep in range(3):
        assert num2.factor(vals) == 0
        got = num2.export()[2]
        compare_factor(num2.export(), f, A.n)
        # eager work between replays
        num.factor(vals)
        torch.cuda.synchronize()
        d = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert d < 1e-13, d


def test_batched_matches_unbatched_and_oracle():
    torch = _torch()
    mats = [W.batch_member(i) for i in range(12)]
    syms = [rlb.Symbolic.from_matrix(A) for A in mats]
    b = rlb.Batch(syms)
    vals = [torch.from_numpy(A.values).cuda() for A in mats]
    info = b.factor(vals)
    assert np.all(info == 0)
    # the batch workspace holds each matrix's factor storage in turn; its
    # merged launches (with narrow tiles run one per wavefront) give each
    # matrix's factor of the unbatched path, element by element
    ws_b = b.workspace.cpu().numpy()
    elems = [s.info()["factor_bytes"] // 8 for s in syms]
    assert sum(elems) <= ws_b.size
    base = np.concatenate([[0], np.cumsum(elems)])
    for i, A in enumerate(mats):
        num = rlb.Numeric(syms[i])
        num.factor(vals[i])
        nf = factor_elems(syms[i])
        ws_s = num.workspace[:nf].cpu().numpy()
        part = ws_b[base[i]:base[i] + nf]
        err = np.linalg.norm(part - ws_s) / np.linalg.norm(ws_s)
        assert err <= 1e-12, (i, err)
        # the batch's factor of matrix i, solved through the batch handle
        B = torch.from_numpy(A.rhs[:, 0].copy()).cuda()
        X = B.clone()
        b.solve(i, X)
        be = num.backward_error(B, X)
        assert be[0] <= 1e-14, (i, be)
        if i < 3:
            o, f = oracle_factor(A)
            compare_factor(num.export(), f, A.n)


def test_batch_schedules_agree_and_autotune_picks_one():
    torch = _torch()
    mats = [W.batch_member(i) for i in range(10)]
    syms = [rlb.Symbolic.from_matrix(A) for A in mats]
    b = rlb.Batch(syms)
    vals = [torch.from_numpy(A.values).cuda() for A in mats]
    outs = {}
    for name in rlb.Batch.SCHEDULES:
        b.set_schedule(name)
        assert np.all(b.factor(vals) == 0)
        xs = []
        for i, A in enumerate(mats):
            B = torch.from_numpy(A.rhs[:, 0].copy()).cuda()
            X = B.clone()
            b.solve(i, X)
            num = rlb.Numeric(syms[i])
            num.values = vals[i]
            assert num.backward_error(B, X)[0] <= 1e-14, (name, i)
            xs.append(X.cpu().numpy())
        outs[name] = xs
    # the same factors up to the order of floating-point additions
    for name in rlb.Batch.SCHEDULES[1:]:
        for a, c in zip(outs["leaves"], outs[name]):
            assert np.linalg.norm(a - c) <= 1e-9 * np.linalg.norm(a), name
    chosen, ms = b.autotune(vals, reps=1)
    assert chosen in rlb.Batch.SCHEDULES and all(v > 0 for v in ms.values())
    assert np.all(b.status() == 0)
    sch, nmin = b.tuning()
    assert sch == chosen and nmin in (256, 1024, 4096, 0)


def test_batch_narrow_threshold_kernels_agree():
    """The one-per-wavefront kernels for narrow work items (forced with a
    threshold of 1) and the 256-thread kernels only (threshold 0: never) give
    the same factors up to rounding, both solving to <= 1e-14."""
    torch = _torch()
    mats = [W.batch_member(i) for i in range(12)]
    syms = [rlb.Symbolic.from_matrix(A) for A in mats]
    b = rlb.Batch(syms)
    vals = [torch.from_numpy(A.values).cuda() for A in mats]
    xs = {}
    for nmin in (1, 0):
        b.set_narrow_min(nmin)
        assert b.tuning()[1] == nmin
        assert np.all(b.factor(vals) == 0)
        out = []
        for i, A in enumerate(mats):
            B = torch.from_numpy(A.rhs[:, 0].copy()).cuda()
            X = B.clone()
            b.solve(i, X)
            num = rlb.Numeric(syms[i])
            num.values = vals[i]
            assert num.backward_error(B, X)[0] <= 1e-14, (nmin, i)
            out.append(X.cpu().numpy())
        xs[nmin] = out
    for a, c in zip(xs[1], xs[0]):
        assert np.linalg.norm(a - c) <= 1e-9 * np.linalg.norm(a)


def test_fp32_updates_with_refinement_reach_1e14():
    torch = _torch()
    A = W.small_grid("27pt", (14, 14, 14), seed=30, lo=0.1, hi=1.0, shift=1e-4, nrhs=4)
    s = rlb.Symbolic.from_matrix(A)
    num = rlb.Numeric(s, rlb.RLB_PREC_FP32_UPDATES)
    vals = torch.from_numpy(A.values).cuda()
    assert num.factor(vals) == 0
    # the FP32-update factor is close to the FP64 oracle, not equal
    o, f = oracle_factor(A)
    err = compare_factor(num.export(), f, A.n, tol=1e-3)
    assert err > 1e-12
    B = torch.from_numpy(np.asfortranarray(A.rhs)).cuda().T.contiguous().T
    X = torch.zeros_like(B).T.contiguous().T
    rep = num.refine(B, X, tol=1e-14, max_iter=30)
    assert rep["converged"], rep
    assert max(rep["backward_error"]) <= 1e-14


@pytest.mark.parametrize("prec,name", [(rlb.RLB_PREC_BF16_UPDATES, "bf16"),
                                       (rlb.RLB_PREC_FP16_UPDATES, "fp16")])
@pytest.mark.parametrize("case", ["lap3d7_15", "elast_8x8x8"])
def test_16bit_updates_with_refinement_reach_1e14(prec, name, case):
    """Scaled BF16/FP16 update operands with FP32 accumulation; the FP64
    refinement (IR, then factor-preconditioned CG if IR stalls) reaches 1e-14."""
    torch = _torch()
    if case == "lap3d7_15":
        A = W.small_grid("7pt", (15, 15, 15), seed=31, lo=0.1, hi=10.0, shift=1e-4, nrhs=4)
    else:
        rng = np.random.default_rng(32)
        A = W.elasticity_like((8, 8, 8), rng, 1e-6)
        A.rhs = W.draw_rhs(rng, A.n, 4)
    print(f"[case] {case} {name} n={A.n}", flush=True)
    s = rlb.Symbolic.from_matrix(A)
    num = rlb.Numeric(s, prec)
    vals = torch.from_numpy(A.values).cuda()
    assert num.factor(vals) == 0
    patched = num.pivots_patched()
    # close to the FP64 oracle at the operands' precision, not equal
    o, f = oracle_factor(A)
    err = compare_factor(num.export(), f, A.n, tol=0.5)
    print(f"[case] factor rel err {err:.2e}, patched pivots {patched}", flush=True)
    assert err > 1e-10
    B = torch.from_numpy(np.asfortranarray(A.rhs)).cuda().T.contiguous().T
    X = torch.zeros_like(B).T.contiguous().T
    rep = num.refine(B, X, tol=1e-14, max_iter=60)
    print(f"[case] iterations {rep['iterations']} pcg_from {rep['pcg_from']} "
          f"be {max(rep['backward_error']):.2e}", flush=True)
    assert rep["converged"], rep
    assert max(rep["backward_error"]) <= 1e-14


@pytest.mark.timeout(900)
def test_full_size_lap3d7_48_every_column_and_properties():
    """The 48^3 workload in the launch configuration the benchmark times
    (graph replay), compared with the oracle on every column, root included."""
    torch = _torch()
    A = W.config2()
    print(f"[case] lap3d7_48 n={A.n}", flush=True)
    s, num, vals, info = gpu_factor(A, graph=True)
    assert info == 0
    assert num.factor(vals) == 0  # a replay of the captured graph
    gpu = num.export()
    # whole-factor properties
    perm = s.array("perm")
    pr = probe_residual(A, perm, gpu, nprobe=3)
    print(f"[case] probe residual {pr:.3e}", flush=True)
    assert pr < 1e-14
    assert np.all(gpu[2][gpu[0][:-1]] > 0)  # positive diagonal
    be = solve_check(num, A, tol=1e-14)
    print(f"[case] backward errors {be}", flush=True)
    # every column: the oracle's own analysis, then Algorithm 1 on the whole
    # factor (about a minute on one core)
    from oracle import onum, osym
    o = osym.analyze(A)
    print("[case] oracle analysis done", flush=True)
    assert np.array_equal(o["perm"], perm)
    f = onum.factor(A, o["perm"], o["structs"])
    assert f["info"] == 0
    err = compare_factor(gpu, f, A.n)
    print(f"[case] all {A.n} columns rel_err={err:.3e}", flush=True)


RL_CASES = [
    ("lap3d27_13", lambda: W.small_grid("27pt", (13, 13, 13), seed=24, lo=0.1, hi=1.0,
                                        shift=1e-4)),
    ("lap2d9_45x38", lambda: W.small_grid("9pt", (45, 38, 1), seed=21)),
    ("elast_7x6x6", lambda: W.elasticity_like((7, 6, 6), np.random.default_rng(25), 1e-6)),
    ("lap3d7_23x19x15", lambda: W.small_grid("7pt", (23, 19, 15), seed=23)),
]


@pytest.mark.parametrize("method", ["rl", "hybrid"])
@pytest.mark.parametrize("name,make", RL_CASES, ids=[c[0] for c in RL_CASES])
def test_rl_method_matches_oracle(name, make, method):
    """RL (Algorithm 4): update matrices in working storage, assembled into the
    ancestors through relative indices; the hybrid method takes that route for
    the supernodes whose rectangles are small and writes the others' updates
    in place; the same factor as the oracle's."""
    A = make()
    o, f = oracle_factor(A)
    # hybrid: no least saving per step, so that these small matrices take both routes
    s, num, vals, info = gpu_factor(A, method=method,
                                    **({"hybrid_step_us": -1} if method == "hybrid" else {}))
    assert info == 0
    assert s.info()["u_bytes"] > 0
    L = s.array("launches").reshape(-1, 12)
    assert (L[:, 0] == 2).sum() >= 1
    err = compare_factor(num.export(), f, A.n)
    print(f"[case] {method} {name} rel_err={err:.3e} u_bytes={s.info()['u_bytes']}", flush=True)
    if A.rhs is not None:
        solve_check(num, A)


@pytest.mark.parametrize("n,method", [(3000, "rlb"), (6000, "rlb"), (3000, "rl"),
                                      (6000, "hybrid")])
def test_irregular_graph_ordering_matches_oracle(n, method):
    """General sparse input: a k-nearest-neighbour graph Laplacian of random
    points (no grid) ordered by graph nested dissection, the oracle deriving
    the same ordering on its own."""
    A = W.irregular3d(n, k=10, seed=40 + n % 7)
    o, f = oracle_factor(A, ordering="graph")
    s, num, vals, info = gpu_factor(A, ordering="graph", method=method,
                                    **({"hybrid_step_us": -1} if method == "hybrid" else {}))
    assert info == 0
    if method == "hybrid":
        L = s.array("launches").reshape(-1, 12)
        assert (L[:, 0] == 2).sum() >= 1
    if method == "rlb":
        # most update launches take the K chunks shaped to small rectangles
        L = s.array("launches").reshape(-1, 12)
        assert ((L[:, 0] == 1) & (L[:, 5] == 4)).sum() >= 4
    assert np.array_equal(s.array("perm"), o["perm"])
    err = compare_factor(num.export(), f, A.n)
    print(f"[case] irregular n={n} {method} rel_err={err:.3e}", flush=True)
    solve_check(num, A)


@pytest.mark.parametrize("name,make,kw", [
    ("lap3d27_13", lambda: W.small_grid("27pt", (13, 13, 13), seed=24, lo=0.1, hi=1.0,
                                        shift=1e-4), {"split_chunks": 2}),
    ("irregular_3000", lambda: W.irregular3d(3000, k=10, seed=40),
     {"split_chunks": 3, "ordering": "graph"}),
    ("irregular_3000_auto", lambda: W.irregular3d(3000, k=10, seed=40),
     {"split_chunks": -1, "ordering": "graph"}),
])
def test_split_tiles_match_oracle_and_repeat_bitwise(name, make, kw):
    """Heavy target tiles cut into parts (every part a workgroup writing its
    sum into a block of the workspace, a reduce launch adding the parts in
    part order): the factor meets the oracle, repeats bit for bit, eagerly
    and from the HIP graph, and the FP32 and 16-bit update forms (whose
    kernels write the parts the same way) refine to 1e-14."""
    torch = _torch()
    A = make()
    o, f = oracle_factor(A, **({"ordering": kw["ordering"]} if "ordering" in kw else {}))
    s, num, vals, info = gpu_factor(A, **kw)
    assert info == 0
    L = s.array("launches").reshape(-1, 12)
    assert (L[:, 0] == 3).sum() >= 1 and s.info()["n_split_tiles"] > 0
    err = compare_factor(num.export(), f, A.n)
    print(f"[case] split {name} reduces={(L[:, 0] == 3).sum()} rel_err={err:.3e}", flush=True)
    first = num.workspace.clone()
    num.set_graph_mode(True)
    for _ in range(3):
        assert num.factor(vals) == 0
        assert torch.equal(num.workspace, first)
    solve_check(num, A)
    B = torch.from_numpy(np.asfortranarray(A.rhs)).cuda().T.contiguous().T
    for prec in (rlb.RLB_PREC_FP32_UPDATES, rlb.RLB_PREC_BF16_UPDATES):
        red = rlb.Numeric(s, prec)
        assert red.factor(vals) == 0
        compare_factor(red.export(), f, A.n,
                       tol=1e-3 if prec == rlb.RLB_PREC_FP32_UPDATES else 0.5)
        X = torch.zeros_like(B).T.contiguous().T
        rep = red.refine(B, X, tol=1e-14, max_iter=100)
        assert rep["converged"] and max(rep["backward_error"]) <= 1e-14, (prec, rep)


def test_batch_of_split_plans_is_bitwise_single():
    """Members whose plans cut heavy tiles into parts: each member's factor
    storage in the batch workspace equals its own factorization's, bit for
    bit (the part blocks after it are scratch: only the entries a part writes
    are ever read)."""
    torch = _torch()
    mats = [W.batch_member(i) for i in (3, 5, 9)]
    syms = [rlb.Symbolic.from_matrix(A, split_chunks=2) for A in mats]
    assert all(sy.info()["n_split_tiles"] > 0 for sy in syms)
    b = rlb.Batch(syms)
    vals = [torch.from_numpy(A.values).cuda() for A in mats]
    assert np.all(b.factor(vals) == 0)
    ws_b = b.workspace.cpu().numpy()
    elems = [sy.info()["factor_bytes"] // 8 for sy in syms]
    base = np.concatenate([[0], np.cumsum(elems)])
    for i, A in enumerate(mats):
        sy = syms[i]
        lel = factor_elems(sy)
        assert lel < elems[i]
        single = rlb.Numeric(sy)
        assert single.factor(vals[i]) == 0
        assert np.array_equal(ws_b[base[i]:base[i] + lel],
                              single.workspace[:lel].cpu().numpy()), i
    o, f = oracle_factor(mats[0])
    single = rlb.Numeric(syms[0])
    single.factor(vals[0])
    compare_factor(single.export(), f, mats[0].n)


def test_xcd_tile_order_matches_oracle():
    """Update launches in 8x8 blocks of neighbouring tiles, a contiguous eighth
    per XCD (the kernel's workgroup-to-tile remapping): the same factor."""
    A = W.small_grid("7pt", (30, 30, 30), seed=22, shift=1e-4)
    s = rlb.Symbolic.from_matrix(A, tile_order="xcd")
    L = s.array("launches").reshape(-1, 12)
    assert (L[:, 5] == 3).sum() >= 1
    o, f = oracle_factor(A)
    s2, num, vals, info = gpu_factor(A, tile_order="xcd")
    assert info == 0
    err = compare_factor(num.export(), f, A.n)
    print(f"[case] lap3d7_30 xcd order rel_err={err:.3e}", flush=True)
    solve_check(num, A)


@pytest.mark.parametrize("name,make,kw", [
    ("lap3d27_13_outer128", lambda: W.small_grid("27pt", (13, 13, 13), seed=24, lo=0.1, hi=1.0,
                                                 shift=1e-4), {"outer_block": 128}),
    ("lap3d7_23x19x15", lambda: W.small_grid("7pt", (23, 19, 15), seed=23), {}),
    ("irregular_3000", lambda: W.irregular3d(3000, k=10, seed=40), {"ordering": "graph"}),
])
def test_tall_target_tiles_match_oracle(name, make, kw):
    """The long updates on 128x64 target tiles (eight wavefronts, 128 rows of X
    and 64 of Y staged per K chunk): the same factor as the oracle's; the FP32
    form runs the same work from its 64x64 tiling and refines to 1e-14."""
    A = make()
    o, f = oracle_factor(A, **({"ordering": kw["ordering"]} if "ordering" in kw else {}))
    s, num, vals, info = gpu_factor(A, tall_tile_min=1, **kw)
    assert info == 0
    L = s.array("launches").reshape(-1, 12)
    assert ((L[:, 0] == 1) & (L[:, 5] == 6)).sum() >= 1
    err = compare_factor(num.export(), f, A.n)
    print(f"[case] tall {name} rel_err={err:.3e}", flush=True)
    if A.rhs is not None:
        solve_check(num, A)
    s32, num32, vals32, info32 = gpu_factor(A, precision=rlb.RLB_PREC_FP32_UPDATES,
                                            tall_tile_min=1, **kw)
    assert info32 == 0
    torch = _torch()
    rhs = A.rhs if A.rhs is not None else np.ones((A.n, 1))
    B = torch.from_numpy(np.asfortranarray(rhs)).cuda().T.contiguous().T
    X = torch.zeros_like(B).T.contiguous().T
    rep = num32.refine(B, X, tol=1e-14, max_iter=30)
    assert rep["converged"], rep
    assert max(rep["backward_error"]) <= 1e-14
