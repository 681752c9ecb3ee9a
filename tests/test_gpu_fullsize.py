"""Device path at the sizes of the benchmark workloads, through the C-ABI.

* A 27-point grid whose root supernode is about 1500 columns wide, compared
  with the oracle element by element (the widest supernode the oracle can
  afford in full; the 64^3 27-point workload's factor, 4.5e11 flops, takes
  the oracle several minutes and is checked through its properties).
* The 64^3 27-point workload: FP64 factor (probe residual of the whole
  factor, solves whose backward error the host recomputes) and the FP32
  update form refined to backward error <= 1e-14, recomputed on the host.
* The 40^3 three-dof elasticity workload: the BF16 and FP16 update forms
  refined to <= 1e-14, recomputed on the host.
"""
import numpy as np
import pytest

from parity_util import compare_factor, gpu_factor, oracle_factor, probe_residual
from paper_2409_13090_amd import rlb
from paper_2409_13090_amd import workloads as W
from test_gpu_parity import cpu_backward_error, solve_check

pytestmark = pytest.mark.gpu


def _cm(torch, a):
    t = torch.from_numpy(np.asfortranarray(a)).cuda()
    return t.T.contiguous().T if t.dim() == 2 else t


@pytest.mark.timeout(300)
def test_wide_root_27pt_32_every_column():
    A = W.small_grid("27pt", (32, 32, 32), seed=51, lo=0.1, hi=1.0, shift=1e-4, nrhs=2)
    print(f"[case] 27pt 32^3 n={A.n}", flush=True)
    s, num, vals, info = gpu_factor(A)
    assert info == 0
    assert np.max(np.diff(s.array("sn_ptr"))) >= 1000
    o, f = oracle_factor(A)
    err = compare_factor(num.export(), f, A.n)
    print(f"[case] rel_err={err:.3e}", flush=True)
    solve_check(num, A)


@pytest.mark.timeout(600)
def test_config4_fp64_and_fp32_refinement_full_size():
    import torch
    A = W.config4()
    print(f"[case] lap3d27_64 n={A.n}", flush=True)
    s, num, vals, info = gpu_factor(A, graph=True)
    assert info == 0 and num.factor(vals) == 0
    gpu = num.export()
    pr = probe_residual(A, s.array("perm"), gpu, nprobe=2)
    print(f"[case] FP64 probe residual {pr:.3e}", flush=True)
    assert pr < 1e-14
    assert np.all(gpu[2][gpu[0][:-1]] > 0)
    del gpu
    be = solve_check(num, A)
    print(f"[case] FP64 backward errors max {be.max():.3e}", flush=True)
    num32 = rlb.Numeric(s, rlb.RLB_PREC_FP32_UPDATES)
    assert num32.factor(vals) == 0
    B = _cm(torch, A.rhs)
    X = torch.zeros_like(B).T.contiguous().T
    rep = num32.refine(B, X, tol=1e-14, max_iter=30)
    print(f"[case] FP32+IR iterations {rep['iterations']} pcg_from {rep['pcg_from']} "
          f"be {max(rep['backward_error']):.3e}", flush=True)
    assert rep["converged"]
    be_host = cpu_backward_error(A, A.rhs, X.cpu().numpy())
    print(f"[case] FP32+IR host backward error max {be_host.max():.3e}", flush=True)
    assert np.all(be_host <= 1e-14), be_host


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,name", [(rlb.RLB_PREC_BF16_UPDATES, "bf16"),
                                       (rlb.RLB_PREC_FP16_UPDATES, "fp16")])
def test_config5_16bit_refinement_full_size(prec, name):
    import torch
    A = W.config5()
    print(f"[case] elast3_40 {name} n={A.n}", flush=True)
    s = rlb.Symbolic.from_matrix(A)
    num = rlb.Numeric(s, prec)
    vals = torch.from_numpy(A.values).cuda()
    assert num.factor(vals) == 0
    B = _cm(torch, A.rhs)
    X = torch.zeros_like(B).T.contiguous().T
    rep = num.refine(B, X, tol=1e-14, max_iter=120)
    print(f"[case] {name} patched {num.pivots_patched()} iterations {rep['iterations']} "
          f"pcg_from {rep['pcg_from']} be {max(rep['backward_error']):.3e}", flush=True)
    assert rep["converged"]
    be_host = cpu_backward_error(A, A.rhs, X.cpu().numpy())
    print(f"[case] {name} host backward error max {be_host.max():.3e}", flush=True)
    assert np.all(be_host <= 1e-14), be_host
