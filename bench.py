"""Benchmark of the RLB supernodal Cholesky hot path on one MI355X.

Default workload: 3D 27-point stencil on a 64^3 grid (n = 262144), weights
U[0.1, 1], diagonal shift 1e-4, nested dissection with reordering inside
supernodes, 8 right-hand sides (seeded synthetic data) -- the workload on
which the FP64 path and the FP32-update form with FP64 refinement are
compared. --workload lap3d7_48 (the 48^3 7-point workload), batch512 and
elast3_40 select the others.

One step = one pass of the device hot path in FP64: factor (A-load, then per
level the POTRF+TRSM of every supernode and its SYRK/GEMM updates written
straight into ancestor storage), solve of the right-hand sides, and the FP64
residual / backward error. The analysis (host symbolic phase) and the upload
of the integer plan happen once, before timing.

value = factorization GFLOP/s = F_exact / t_factor, where F_exact is the sum
over columns of (column count)^2 on the exact structure and t_factor is the
median device time of the factor over the timed steps (HIP events on the
factor's stream). The same matrix is also factored with FP32-operand updates
and refined in FP64 to backward error <= 1e-14 ("mixed_ir"); the times to
solution of both forms are medians over the same number of repetitions.

Prints ONE JSON line.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "factor GFLOP/s + % MFMA peak, FP64 vs FP32-update+IR at backward err ≤1e-14"
WORKLOAD_TEXT = {
    "lap3d7_48": "lap3d7_{side}: 3D 7-point Laplacian {side}^3 (n={n}), weights 10^U(-2,2), "
                 "shift 1e-6*max diag, nested dissection + reordering within supernodes, 4 RHS",
    "lap3d27_64": "lap3d27_64: 3D 27-point stencil 64^3 (n={n}), weights U[0.1,1], shift 1e-4, "
                  "nested dissection + reordering within supernodes, 8 RHS",
    "elast3_40": "elast3_40: 3 dofs per node on 40^3 (n={n}), 7-point coupling with 3x3 SPD "
                 "blocks E*R*diag(1,1,1e-2)*R^T, shift 1e-6*I, 16 RHS",
    "irr3d_150k": "irr3d_150k: k-nearest-neighbour (k=10) graph Laplacian of {n} random points "
                  "in the unit cube, weights U[0.5,1.5], shift 1e-2, graph nested dissection + "
                  "reordering within supernodes, 4 RHS",
}
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_16BIT_TFLOPS = 2516.6  # dense BF16/FP16 MFMA
# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs scaled by the same counters on a 256 MiB device copy; valid
# only for the kernel source they were taken on (first 16 hex digits of the
# SHA-256 of kernels.hip), otherwise the roofline reports traffic as null.
MEASURED_TRAFFIC = {
    "lap3d27_64": {"kernels_sha256": "8061a75a28f12f09", "bytes_per_launch": 1015278042,
                   "summary": "profiles/k_update_lap3d27_64_hbm_traffic.md"},
    "lap3d7_48": {"kernels_sha256": "8061a75a28f12f09", "bytes_per_launch": 179886029,
                  "summary": "profiles/k_update_lap3d7_48_hbm_traffic.md"},
}


def kernel_source_hash():
    import hashlib
    path = os.path.join(ROOT, "paper_2409_13090_amd", "csrc", "kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload, side):
    rec = MEASURED_TRAFFIC.get(workload)
    if rec is None or (workload == "lap3d7_48" and side != 48):
        return None
    if rec["kernels_sha256"] != kernel_source_hash():
        return None
    return rec["bytes_per_launch"]


def cpu_baseline(A, sym, label, budget_flops=1.0e11):
    """Time the CPU oracle (Algorithm 1, one thread) on a bounded sample of the
    same workload: the first k columns of the factored matrix, whose factor
    columns Algorithm 1 computes exactly on their own."""
    import numpy as np

    from oracle import onum, osym

    perm = sym.array("perm")
    cc = sym.array("colcount").astype(np.float64)
    cum = np.cumsum(cc * cc)
    k = int(np.searchsorted(cum, budget_flops))
    k = max(1, min(k, A.n))
    a_cp, a_ri, a_x = osym.permute_lower(A.n, A.colptr, A.rowidx, A.values, perm)
    structs, _ = osym.column_structures(A.n, a_cp, a_ri, upto=k)
    l_cp, l_ri = onum.pattern_csc(structs)
    t0 = time.perf_counter()
    _, info = onum.alg1(A.n, a_cp, a_ri, a_x, l_cp, l_ri, ncols=k)
    dt = time.perf_counter() - t0
    flops = float(cum[k - 1])
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"Algorithm 1 on the first {k} of {A.n} columns of the {label} factor "
                      f"({flops:.3e} flops, {dt:.1f} s, info={info})",
            "seconds": dt, "cpu_model": host_cpu_model(), "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0))}


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=7)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--side", type=int, default=48)
    ap.add_argument("--workload", default="lap3d27_64",
                    choices=["lap3d27_64", "lap3d7_48", "batch512", "elast3_40", "irr3d_150k"],
                    help="lap3d27_64 (default) carries the FP64 vs FP32-update+refinement "
                         "comparison; the others are the 48^3 7-point workload, the batched "
                         "form and the 3-dof elasticity workload")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 256 MiB device to device (calibrates the HBM byte counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--max-iter", type=int, default=100,
                    help="refinement steps allowed to the reduced-precision form")
    ap.add_argument("--mixed", choices=["fp32", "bf16", "fp16"], default=None,
                    help="update operands of the refined form (default: fp32, bf16 for elast3_40)")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch the factor's kernels one by one instead of replaying a HIP graph")
    ap.add_argument("--prof-reps", type=int, default=3,
                    help="factorizations timed launch by launch for the roofline")
    ap.add_argument("--mixed-reps", type=int, default=7,
                    help="timed repetitions of each time to solution (after one untimed)")
    ap.add_argument("--no-rl", action="store_true",
                    help="skip the RL (Algorithm 4) factorization of the same matrix")
    ap.add_argument("--ablations", action="store_true",
                    help="only the FP64 factor under the analysis switches one at a time "
                         "(maximal blocks, reordering, merge cap, outer blocks, atomic "
                         "splitting, RL, XCD tile order); prints one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the factorization runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding over several GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2409_13090_amd import rlb
    from paper_2409_13090_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        a = torch.ones(1 << 25, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": a.numel() * 8, "copies": 3}))
        return
    if args.workload == "batch512":
        return bench_batch(args)
    if args.ablations:
        return bench_ablations(args)
    order_kw = {}
    if args.workload == "lap3d27_64":
        A = W.config4()
    elif args.workload == "elast3_40":
        A = W.config5()
    elif args.workload == "irr3d_150k":
        A = W.irregular3d(150000)
        order_kw = {"ordering": "graph"}
    else:
        A = W.config2(side=args.side)
    t0 = time.perf_counter()
    sym = rlb.Symbolic.from_matrix(A, **order_kw)
    t_analyze = time.perf_counter() - t0
    info = sym.info()
    F = info["flops_exact"]

    vals = torch.from_numpy(A.values).to(dev)
    B = torch.from_numpy(np.asfortranarray(A.rhs)).to(dev).T.contiguous().T
    X = torch.empty_like(B).T.contiguous().T
    num = rlb.Numeric(sym, rlb.RLB_PREC_FP64)
    graph = not args.no_graph
    num.set_graph_mode(graph)
    ws = torch.empty(info["factor_bytes"] // 8 + 1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        num.factor(vals, ws, check=False)
        e1.record(stream)
        st = num.status()
        assert st == 0, f"factor reported info={st}"
        X.copy_(B)
        num.solve(X)
        be = num.backward_error(B, X)  # synchronizes
        return e0, e1, be, time.perf_counter() - t0

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    recs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    fac_ms = [r[0].elapsed_time(r[1]) for r in recs]
    be = np.max([r[2] for r in recs], axis=0)
    t_fac = statistics.median(fac_ms) / 1e3
    gflops = F / t_fac / 1e9
    tts64 = statistics.median([r[3] for r in recs])

    # per-launch HIP events on the factor's stream (eager launches of the same
    # kernels) for the roofline of the dominant kernel
    num.set_profiling(True)
    profs = []
    for _ in range(args.prof_reps):
        num.factor(vals, ws, check=True)
        profs.append(num.last_profile())
    num.set_profiling(False)
    upd_ms = [p["update_ms"] for p in profs]
    pan_ms = [p["panel_ms"] for p in profs]
    n_upd = profs[0]["n_update"]

    # dominant kernel: the SYRK/GEMM update tiles (FP64 MFMA)
    upd_s = statistics.median(upd_ms) / 1e3
    # (the algorithmic flops of the tiles these launches run; the previous
    # block's update inside the panel launches is not part of them)
    ach = info["flops_upd_launch"] / upd_s / 1e12
    roof = {"kernel": "update launches: k_update / k_update_win / k_update_pack / k_update_short "
                      "(SYRK/GEMM summed into 64x64 target tiles, MFMA f64 16x16x4), with the "
                      "k_part_reduce launches that sum the parts of split tiles",
            "bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4),
            "traffic": measured_traffic(args.workload, args.side),
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated)",
            "launches_per_factor": n_upd,
            "avg_launch_us": round(statistics.median(upd_ms) / n_upd * 1e3, 2),
            "alg_flops_per_launch": info["flops_upd_launch"] / n_upd}

    out = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_total / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT.get(args.workload, "").format(side=args.side, n=A.n),
                   "n": A.n, "nrhs": int(A.rhs.shape[1]), "graph": graph,
                   "timing": f"median of {args.steps} timed steps after {args.warmup} warm-up"},
        "pct_fp64_peak": round(gflops / 1e3 / PEAK_FP64_TFLOPS * 100, 3),
        "factor_ms": round(t_fac * 1e3, 3),
        "factor_ms_min": round(min(fac_ms), 3),
        "factor_ms_max": round(max(fac_ms), 3),
        "panel_ms": round(statistics.median(pan_ms), 3),
        "update_ms": round(statistics.median(upd_ms), 3),
        "n_panel_launches": profs[0]["n_panel"],
        "flops_exact": F,
        "backward_error": [float(f"{v:.3e}") for v in be],
        "time_to_solution_ms": round(tts64 * 1e3, 3),
        "analyze_s": round(t_analyze, 3),
        "plan": {k: info[k] for k in ("n_supernodes", "n_levels", "n_launches",
                                      "n_update_tiles", "n_panel_tiles", "n_merged_tiles", "n_split_tiles",
                                      "nnz_stored")},
        "roofline": roof,
    }

    def time_method(method, **extra):
        """FP64 factor of the same matrix with another update method (or
        another planner option), on the same symbolic phase settings (median
        of the timed steps)."""
        sym_m = rlb.Symbolic.from_matrix(A, method=method, **order_kw, **extra)
        info_m = sym_m.info()
        num_m = rlb.Numeric(sym_m, rlb.RLB_PREC_FP64)
        num_m.set_graph_mode(graph)
        ws_m = torch.empty(info_m["factor_bytes"] // 8 + 1, dtype=torch.float64, device=dev)
        assert num_m.factor(vals, ws_m) == 0
        ms_m = []
        for _ in range(args.steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            num_m.factor(vals, ws_m, check=False)
            e1.record(stream)
            e1.synchronize()
            ms_m.append(e0.elapsed_time(e1))
        assert num_m.status() == 0
        X.copy_(B)
        num_m.solve(X)
        be_m = num_m.backward_error(B, X)
        t_m = statistics.median(ms_m) / 1e3
        kinds = sym_m.array("launches").reshape(-1, 12)[:, 0]
        n_asm = int((kinds == 2).sum())
        return {"factor_ms": round(t_m * 1e3, 3), "gflops": round(F / t_m / 1e9, 2),
                "rlb_factor_ms": round(t_fac * 1e3, 3),
                "over_rlb_time": round(t_m / t_fac, 3),
                "fp_storage_bytes": info_m["factor_bytes"],
                "update_matrix_bytes": info_m["u_bytes"],
                "rlb_fp_storage_bytes": info["factor_bytes"],
                "assembly_launches": n_asm,
                "reduce_launches": int((kinds == 3).sum()),
                "split_workgroups": info_m["n_split_tiles"],
                "backward_error_max": float(f"{max(be_m):.3e}")}

    if not args.no_rl:
        # RL (Algorithm 4) on the same matrix and the same symbolic phase:
        # update matrices in working storage, assembled into the ancestors
        out["rl"] = {"method": "RL (Algorithm 4): SYRK into an update matrix per supernode, "
                               "assembled into the ancestors through relative indices "
                               "(one writer per target column, no atomics)",
                     **time_method("rl")}
        # per supernode the cheaper of the two routes by the planner's model
        out["hybrid"] = {"method": "RLB for most supernodes, RL's update matrix for those "
                                   "whose rectangles meet many target tiles (planner's "
                                   "cost model; not the paper's method)",
                         **time_method("hybrid")}
        # RLB with the launches' heaviest tiles cut into parts summed by a
        # reduce launch in a fixed order (load balance; adds part blocks of
        # working storage that Algorithm 5 does without, hence an option)
        out["split"] = {"method": "RLB with heavy target tiles cut into parts written to "
                                  "workspace blocks and summed in part order by a reduce "
                                  "launch (split_chunks < 0; deterministic; not the paper's "
                                  "method)",
                        **time_method("rlb", split_chunks=-1)}
    if not args.no_mixed:
        mixed = args.mixed or ("bf16" if args.workload == "elast3_40" else "fp32")
        prec = {"fp32": rlb.RLB_PREC_FP32_UPDATES, "bf16": rlb.RLB_PREC_BF16_UPDATES,
                "fp16": rlb.RLB_PREC_FP16_UPDATES}[mixed]
        num32 = rlb.Numeric(sym, prec)
        num32.set_graph_mode(graph)
        ws32 = torch.empty_like(ws)
        X32 = torch.zeros_like(B).T.contiguous().T
        reps = []
        info32 = 0
        # one untimed repetition (graph capture), then mixed_reps timed ones;
        # time to solution = factor + first solve + refinement to <= 1e-14
        for rep in range(1 + args.mixed_reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record(stream)
            num32.factor(vals, ws32, check=False)
            e1.record(stream)
            info32 = num32.status()
            if info32 != 0:
                break
            X32.zero_()
            r = num32.refine(B, X32, tol=1e-14, max_iter=args.max_iter)
            torch.cuda.synchronize()
            if rep > 0:
                reps.append((e0.elapsed_time(e1), time.perf_counter() - t0, r))
        peak_m = PEAK_FP32_TFLOPS if mixed == "fp32" else PEAK_16BIT_TFLOPS
        if info32 != 0 or not reps:
            out["mixed_ir"] = {"precision": mixed, "factor_info": info32, "converged": False}
        else:
            t32 = statistics.median([x[0] for x in reps]) / 1e3
            tts32 = statistics.median([x[1] for x in reps])
            be32 = max(max(x[2]["backward_error"]) for x in reps)
            its = [x[2]["iterations"] for x in reps]
            out["mixed_ir"] = {
                "precision": f"{mixed} update operands, FP32 accumulation, FP64 "
                             "POTRF/TRSM/storage, FP64 refinement",
                "factor_info": info32,
                "pivots_patched": num32.pivots_patched(),
                "converged": bool(all(x[2]["converged"] for x in reps)),
                "factor_gflops": round(F / t32 / 1e9, 2),
                "pct_update_precision_peak": round(F / t32 / 1e12 / peak_m * 100, 3),
                "pcg_from": reps[-1][2]["pcg_from"],
                "factor_ms": round(t32 * 1e3, 3),
                "ir_iterations": its[-1],
                "ir_iterations_all": its,
                "backward_error": float(f"{be32:.3e}"),
                "time_to_solution_ms": round(tts32 * 1e3, 3),
                "fp64_time_to_solution_ms": round(tts64 * 1e3, 3),
                "timing": f"medians of {len(reps)} repetitions after one untimed, both forms"}

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, sym, args.workload)
    print(json.dumps(out), flush=True)


ABLATIONS = [
    ("default", {}),
    ("maximal_blocks_off", {"maximal_blocks": False}),
    ("reordering_off", {"reorder": False}),
    ("merge_cap_0", {"merge_cap": 0.0}),
    ("merge_cap_0.0625", {"merge_cap": 0.0625}),
    ("merge_cap_0.25", {"merge_cap": 0.25}),
    ("outer_block_64", {"outer_block": 64}),
    ("outer_block_512", {"outer_block": 512}),
    ("atomic_split", {"deterministic": False}),
    ("big_tiles_128", {"big_tile_min": 256}),
    ("tall_tiles_128x64", {"tall_tile_min": 256}),
    ("method_rl", {"method": "rl"}),
    ("method_hybrid", {"method": "hybrid"}),
    ("tile_order_xcd", {"tile_order": "xcd"}),
]


def bench_ablations(args):
    """The FP64 factorization of one workload under each analysis switch
    (one at a time): median device time of the graph-replayed factor over
    args.steps runs, the plan's block and call counts (Alg. 5), stored
    entries and padded flops, and the backward error of one solve."""
    import numpy as np
    import torch

    from paper_2409_13090_amd import rlb
    from paper_2409_13090_amd import workloads as W

    dev = torch.device("cuda:0")
    A = {"lap3d27_64": W.config4, "elast3_40": W.config5}.get(args.workload,
                                                             lambda: W.config2(side=args.side))()
    vals = torch.from_numpy(A.values).to(dev)
    B = torch.from_numpy(np.asfortranarray(A.rhs)).to(dev).T.contiguous().T
    stream = torch.cuda.current_stream()
    rows = {}
    F = None
    for name, kw in ABLATIONS:
        sym = rlb.Symbolic.from_matrix(A, **kw)
        info = sym.info()
        num = rlb.Numeric(sym, rlb.RLB_PREC_FP64)
        num.set_graph_mode(True)
        assert num.factor(vals) == 0
        ms = []
        for _ in range(args.steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            num.factor(vals, check=False)
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        assert num.status() == 0
        X = B.clone().T.contiguous().T
        num.solve(X)
        be = float(max(num.backward_error(B, X)))
        F = F or info["flops_exact"]
        t = statistics.median(ms)
        rows[name] = {"factor_ms": round(t, 3), "gflops": round(info["flops_exact"] / t / 1e6, 1),
                      "n_supernodes": info["n_supernodes"], "n_blocks": info["n_blocks"],
                      "n_calls": info["n_calls"], "nnz_stored": info["nnz_stored"],
                      "flops_padded": info["flops_padded"], "n_launches": info["n_launches"],
                      "fp_storage_bytes": info["factor_bytes"], "backward_error": float(f"{be:.3e}")}
        del num
        print(json.dumps({"ablation": name, **rows[name]}), file=sys.stderr, flush=True)
    out = {"metric": METRIC, "value": rows["default"]["gflops"], "unit": "GFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 1, "ms_per_step": rows["default"]["factor_ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": WORKLOAD_TEXT.get(args.workload, "").format(side=args.side, n=A.n),
                      "mode": "ablations of the analysis switches, FP64 factor"},
           "flops_exact": F, "ablations": rows}
    print(json.dumps(out), flush=True)


def _batch_member_alg1(job):
    """Algorithm 1 on one batch member (oracle): returns (seconds of
    Algorithm 1 alone, info)."""
    n, colptr, rowidx, values, perm = job
    from oracle import onum, osym

    a_cp, a_ri, a_x = osym.permute_lower(n, colptr, rowidx, values, perm)
    structs, _ = osym.column_structures(n, a_cp, a_ri)
    l_cp, l_ri = onum.pattern_csc(structs)
    t0 = time.perf_counter()
    _, info = onum.alg1(n, a_cp, a_ri, a_x, l_cp, l_ri)
    return time.perf_counter() - t0, info


def cpu_baseline_batch(mats, syms, flops):
    """The CPU oracle (Algorithm 1, one thread) on every member of the batch,
    one after the other in this process; only Algorithm 1's own time is summed
    (as for one matrix: the oracle's symbolic structures are not timed)."""
    res = [_batch_member_alg1((A.n, A.colptr, A.rowidx, A.values, s.array("perm")))
           for A, s in zip(mats, syms)]
    dt = sum(r[0] for r in res)
    bad = sum(1 for r in res if r[1] != 0)
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"Algorithm 1 on all {len(mats)} matrices ({flops:.3e} flops, {dt:.2f} s "
                      f"summed over the matrices; {bad} failed)",
            "seconds": dt, "cpu_model": host_cpu_model(), "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0))}


def bench_batch(args):
    """The batched form: independent 9-point grid Laplacians (side ~ U{16..96})
    factored with one merged level schedule, replayed as a HIP graph."""
    import numpy as np
    import torch

    from paper_2409_13090_amd import rlb
    from paper_2409_13090_amd import workloads as W

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    mats = [W.batch_member(i, args.batch_count) for i in range(args.batch_count)]
    syms = [rlb.Symbolic.from_matrix(A) for A in mats]
    t_analyze = time.perf_counter() - t0
    F = sum(s.info()["flops_exact"] for s in syms)
    b = rlb.Batch(syms)
    b.set_graph_mode(not args.no_graph)
    vals = [torch.from_numpy(A.values).to(dev) for A in mats]
    stream = torch.cuda.current_stream()
    # level schedule chosen by timing the candidates on the device
    schedule, schedule_ms = b.autotune(vals, reps=2)
    narrow_min = b.tuning()[1]
    for _ in range(args.warmup):
        assert np.all(b.factor(vals) == 0)
    ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.factor(vals, check=False)
        e1.record(stream)
        assert np.all(b.status() == 0)
        ms.append(e0.elapsed_time(e1))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    t_fac = statistics.median(ms) / 1e3
    # backward error of every member's solve (one RHS each)
    worst = 0.0
    for i, A in enumerate(mats):
        B = torch.from_numpy(A.rhs[:, 0].copy()).to(dev)
        X = B.clone()
        b.solve(i, X)
        num = rlb.Numeric(syms[i])
        num.values = vals[i]
        worst = max(worst, float(num.backward_error(B, X)[0]))
    out = {"metric": METRIC, "value": round(F / t_fac / 1e9, 2), "unit": "GFLOP/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(t_total / args.steps * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"batch{args.batch_count}: {args.batch_count} 2D 9-point "
                                  "Laplacians, side ~ U{16..96}, weights U[0.5,1.5], shift 1e-3, "
                                  "merged level schedule and narrow-item threshold (autotuned), "
                                  "HIP graph replay",
                      "count": args.batch_count, "sum_n": int(sum(A.n for A in mats)),
                      "schedule": schedule, "narrow_min": narrow_min},
           "schedule_ms": {k: round(v, 3) for k, v in schedule_ms.items()},
           "factor_ms": round(t_fac * 1e3, 3), "flops_exact": F,
           "pct_fp64_peak": round(F / t_fac / 1e12 / PEAK_FP64_TFLOPS * 100, 3),
           "backward_error_max": float(f"{worst:.3e}"), "analyze_s": round(t_analyze, 2)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(mats, syms, F)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
