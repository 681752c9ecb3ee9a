"""Deterministic factorization (rlb_options.deterministic, the default) and
the batched form against single factorizations and the oracle, through the
C-ABI.

With deterministic = 1 every target tile of an update launch has one owner
that sums its contributions in a fixed order (no floating-point atomics), so
repeated factorizations give the same bits and the batched form gives every
matrix the bits of its own factorization. deterministic = 0 (tiles cut into
parts added atomically) must still meet the oracle."""
import numpy as np
import pytest

from parity_util import (bits, compare_factor, export_from_storage, factor_elems, gpu_factor,
                         oracle_factor, stored_lower_positions)
from paper_2409_13090_amd import rlb
from paper_2409_13090_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_repeated_factorizations_are_bitwise_equal():
    import torch
    A = W.small_grid("27pt", (20, 20, 20), seed=61, lo=0.1, hi=1.0, shift=1e-4)
    s = rlb.Symbolic.from_matrix(A)
    # no tile is added atomically (heavy tiles may be cut into parts that a
    # reduce launch sums in a fixed order)
    assert not np.any(s.array("update_tiles").reshape(-1, 7)[:, 4] & 2)
    nf = factor_elems(s)
    num = rlb.Numeric(s)
    vals = torch.from_numpy(A.values).cuda()
    assert num.factor(vals) == 0
    ref = num.workspace[:nf].cpu().numpy().copy()
    g = rlb.Numeric(s)
    g.set_graph_mode(True)
    for rep in range(3):
        assert num.factor(vals) == 0
        assert np.array_equal(bits(num.workspace[:nf].cpu().numpy()), bits(ref)), rep
        assert g.factor(vals) == 0  # graph replays, eager work in between
        assert np.array_equal(bits(g.workspace[:nf].cpu().numpy()), bits(ref)), rep
    o, f = oracle_factor(A)
    compare_factor(num.export(), f, A.n)


def test_atomic_split_form_meets_oracle():
    A = W.small_grid("27pt", (20, 20, 20), seed=61, lo=0.1, hi=1.0, shift=1e-4)
    s, num, vals, info = gpu_factor(A, deterministic=False)
    assert info == 0
    assert s.info()["n_split_tiles"] > 0
    o, f = oracle_factor(A)
    err = compare_factor(num.export(), f, A.n)
    print(f"[case] atomic split form rel_err={err:.3e}", flush=True)


@pytest.mark.timeout(900)
def test_batch512_every_member_bitwise_single_and_oracle():
    """All 512 matrices of the batched workload: the batch's factor of each
    equals its single factorization bit for bit, and the oracle element by
    element (Algorithm 1 on every member, about a minute and a half)."""
    import torch
    from oracle import onum, osym
    mats = [W.batch_member(i) for i in range(512)]
    syms = [rlb.Symbolic.from_matrix(A) for A in mats]
    b = rlb.Batch(syms)
    b.set_graph_mode(True)
    vals = [torch.from_numpy(A.values).cuda() for A in mats]
    chosen, _ = b.autotune(vals, reps=1)
    print(f"[case] schedule {chosen}", flush=True)
    assert np.all(b.factor(vals) == 0)
    ws_b = b.workspace.cpu().numpy()
    elems = [s.info()["factor_bytes"] // 8 for s in syms]
    base = np.concatenate([[0], np.cumsum(elems)])
    worst = 0.0
    for i, A in enumerate(mats):
        part = ws_b[base[i]:base[i] + elems[i]]
        num = rlb.Numeric(syms[i])
        assert num.factor(vals[i]) == 0
        single = num.workspace[:elems[i]].cpu().numpy()
        pos, _, _ = stored_lower_positions(syms[i])
        assert np.array_equal(bits(part[pos]), bits(single[pos])), i
        o = osym.analyze(A)
        assert np.array_equal(o["perm"], syms[i].array("perm")), i
        f = onum.factor(A, o["perm"], o["structs"])
        worst = max(worst, compare_factor(export_from_storage(syms[i], part), f, A.n))
        if i % 64 == 63:
            print(f"[case] {i + 1} members checked, worst rel_err {worst:.3e}", flush=True)
    # a solve through the batch handle after the autotuner's last schedule
    B = torch.from_numpy(mats[5].rhs[:, 0].copy()).cuda()
    X = B.clone()
    b.solve(5, X)
    num = rlb.Numeric(syms[5])
    num.values = vals[5]
    assert num.backward_error(B, X)[0] <= 1e-14


def test_backward_error_after_values_changed_in_place():
    """Refactor new values written into the same device buffer: the backward
    error must use the new ||A||, as the host recomputes it."""
    import torch
    from test_gpu_parity import cpu_backward_error
    A = W.small_grid("7pt", (12, 11, 10), seed=62, nrhs=2)
    s, num, vals, info = gpu_factor(A)
    B = torch.from_numpy(np.asfortranarray(A.rhs)).cuda().T.contiguous().T
    X = B.clone().T.contiguous().T
    num.solve(X)
    num.backward_error(B, X)
    vals.mul_(10.0)
    assert num.factor(vals) == 0
    A10 = W.SparseSPD(A.n, A.colptr, A.rowidx, A.values * 10.0, A.grid, "x10")
    X = B.clone().T.contiguous().T
    num.solve(X)
    rng = np.random.default_rng(3)
    xp = X.cpu().numpy() * (1.0 + 1e-6 * rng.uniform(-1.0, 1.0, X.shape))
    Xp = torch.from_numpy(np.asfortranarray(xp)).cuda().T.contiguous().T
    got = num.backward_error(B, Xp)
    want = cpu_backward_error(A10, A.rhs, xp)
    assert np.allclose(got, want, rtol=1e-8, atol=0.0), (got, want)


def test_solve_after_failed_factor_is_refused_without_status_call():
    import torch
    A = W.small_grid("7pt", (10, 10, 10), seed=28)
    A.values = A.values.copy()
    A.values[A.colptr[:-1][700:]] -= 50.0
    s = rlb.Symbolic.from_matrix(A)
    num = rlb.Numeric(s)
    vals = torch.from_numpy(A.values).cuda()
    num.factor(vals, check=False)
    with pytest.raises(rlb.RlbError) as e:
        num.solve(torch.zeros(A.n, dtype=torch.float64, device="cuda"))
    assert e.value.status == -6


def test_batch_unfused_merged_launches_meet_oracle():
    """Matrices analysed with deterministic = 0: the batch unfuses their panel
    steps and merges every matrix's update launches of a step into one whose
    kernel (dense, windowed or packed K staging) is chosen from the merged
    tiles; each member's factor still meets the oracle."""
    import torch
    mats = [W.batch_member(i) for i in range(16)]
    syms = [rlb.Symbolic.from_matrix(A, deterministic=False) for A in mats]
    b = rlb.Batch(syms)
    vals = [torch.from_numpy(A.values).cuda() for A in mats]
    assert np.all(b.factor(vals) == 0)
    ws_b = b.workspace.cpu().numpy()
    elems = [s.info()["factor_bytes"] // 8 for s in syms]
    base = np.concatenate([[0], np.cumsum(elems)])
    worst = 0.0
    for i in (0, 3, 7, 15):
        part = ws_b[base[i]:base[i] + elems[i]]
        o, f = oracle_factor(mats[i])
        worst = max(worst, compare_factor(export_from_storage(syms[i], part), f, mats[i].n))
    print(f"[case] unfused batch of 16, worst rel_err {worst:.3e}", flush=True)


@pytest.mark.parametrize("method", ["rl", "hybrid"])
def test_update_matrix_assembly_is_bitwise_repeatable(method):
    """The assembly of the update matrices has one writer per target column
    and a fixed order (no atomics): repeated factorizations give the same
    bits, in eager launches and graph replays."""
    import torch
    A = W.small_grid("27pt", (18, 18, 18), seed=62, lo=0.1, hi=1.0, shift=1e-4)
    s = rlb.Symbolic.from_matrix(A, method=method,
                                 **({"hybrid_step_us": -1} if method == "hybrid" else {}))
    assert (s.array("launches").reshape(-1, 12)[:, 0] == 2).sum() >= 1
    num = rlb.Numeric(s)
    vals = torch.from_numpy(A.values).cuda()
    assert num.factor(vals) == 0
    # the factor storage (the update matrices' working storage after it is
    # scratch: only the lower triangles are written)
    nf = factor_elems(s)
    ref = num.workspace[:nf].cpu().numpy().copy()
    g = rlb.Numeric(s)
    g.set_graph_mode(True)
    for rep in range(3):
        assert num.factor(vals) == 0
        assert np.array_equal(bits(num.workspace[:nf].cpu().numpy()), bits(ref)), rep
        assert g.factor(vals) == 0
        assert np.array_equal(bits(g.workspace[:nf].cpu().numpy()), bits(ref)), rep
    o, f = oracle_factor(A)
    compare_factor(num.export(), f, A.n)
