"""rlb_solve_noalloc (the solve whose work vectors live in a fixed per-GPU
library array, for callers that cannot allocate) against rlb_solve, through
the C-ABI: two calls in a row, the second on a smaller input, each compared
with the allocating solve of the same factor."""
import numpy as np
import pytest

from paper_2409_13090_amd import rlb
from paper_2409_13090_amd import workloads as W

pytestmark = pytest.mark.gpu


def _setup(A):
    import torch
    s = rlb.Symbolic.from_matrix(A)
    num = rlb.Numeric(s)
    vals = torch.from_numpy(A.values).cuda()
    assert num.factor(vals) == 0
    B = torch.from_numpy(np.asfortranarray(A.rhs)).cuda()
    if B.dim() == 2:
        B = B.T.contiguous().T
    return s, num, B


def _check(num, B):
    X_ref = B.clone()
    if X_ref.dim() == 2:
        X_ref = X_ref.T.contiguous().T
    num.solve(X_ref)
    X = B.clone()
    if X.dim() == 2:
        X = X.T.contiguous().T
    num.solve_noalloc(X)
    x, xr = X.cpu().numpy(), X_ref.cpu().numpy()
    rel = np.linalg.norm(x - xr) / np.linalg.norm(xr)
    be = num.backward_error(B, X)
    print(f"[case] n={B.shape[0]} rel diff {rel:.2e} backward error {be.max():.2e}", flush=True)
    assert rel <= 1e-12, rel
    assert np.all(be <= 1e-14), be


def test_noalloc_solve_matches_solve_twice_then_smaller():
    big = W.small_grid("27pt", (15, 14, 13), seed=71, lo=0.1, hi=1.0, shift=1e-4, nrhs=6)
    small = W.small_grid("5pt", (20, 17, 1), seed=72, nrhs=1)
    s1, n1, B1 = _setup(big)
    s2, n2, B2 = _setup(small)
    _check(n1, B1)
    _check(n2, B2)  # the second call, smaller: the array keeps the first call's data
    _check(n1, B1)


def test_noalloc_solve_rejects_sizes_beyond_capacity():
    import torch
    A = W.small_grid("5pt", (400, 400, 1), seed=73)  # n = 160000: 16 RHS exceed 2^21
    s = rlb.Symbolic.from_matrix(A)
    num = rlb.Numeric(s)
    X = torch.zeros((A.n, 16), dtype=torch.float64, device="cuda").T.contiguous().T
    with pytest.raises(rlb.RlbError) as e:
        num.solve_noalloc(X)
    assert e.value.status == -1
