"""Benchmark: block-AMG preconditioned FGMRES solve of a 3D mortar-contact
saddle-point system on one MI355X.

One step is one pass of the whole solve path on the 40^3 / 41x41x40 hex8
contact workload (428,778 unknowns): the mixed-precision forward FGMRES
solve to relative residual 1e-8 (FP32 V-cycle hierarchy inside FP64
FGMRES), the adjoint solve A^T lam = dL/dx on the same hierarchy, and the
gradient sampling on K's pattern.  `value` is the forward solve time in
seconds (median over the timed steps, device time from hipEvents); the FP64
path is timed the same way and reported beside it.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="contact3d_40")
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--spmv-format", type=int, default=0, help="device storage of K: 0 auto, 1 CSR, 2 blocked-ELL")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many MiB (5 times) and exit; used to scale "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    return ap.parse_args()


def copy_probe(mib):
    import torch

    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": n * 4, "launches": 5}), flush=True)


def smooth_u_bytes(info0, elem):
    """Algorithmic HBM bytes of one level-0 residual+Jacobi launch.

    Blocked layout: every nonzero bs x bs block of K once (bs^2 values plus
    one 4-byte block index; slice padding not counted), G's entries (value +
    column) and row pointers, and the vectors b_u, jinv, z_u (read once),
    z_l, zn_u (written).  CSR layout: K's entries (value + column) and row
    pointers instead of the blocks."""
    n_u, n_l = info0["n_u"], info0["n_l"]
    vec = n_u * elem * 4 + n_l * elem + info0["nnz_G"] * (elem + 4) + (n_u + 1) * 4
    if info0["k_layout"] == 1:
        bs = info0["k_bs"]
        return info0["k_blocks"] * (bs * bs * elem + 4) + vec
    return info0["nnz_K"] * (elem + 4) + (n_u + 1) * 4 + vec


def vcycle_matrix_bytes(solver, elem):
    """Matrix bytes streamed by one forward V-cycle (a lower bound on its
    traffic: vectors excluded).  Per smoothing level with nu_pre + nu_post
    sweeps of nj Jacobi steps: K is read (nu_pre + nu_post) * nj times (each
    sweep but the first from zero, its extra Jacobi steps, and the residual
    before restriction); G twice per sweep plus the residual; B and C once
    per sweep plus the residual; R and P once.  K in its device layout
    (bs x bs blocks with a 4-byte block index, or CSR), P and R either CSR or
    index-free (values plus one 4-byte base column per fine row for P, one
    4-byte row index per fine row for R), the other blocks CSR (value +
    4-byte column).  The coarsest level: its dense inverse."""
    o = solver.options
    sweeps = o.nu_pre + o.nu_post
    nj = max(1, o.jacobi_sweeps)
    total = 0
    for l in range(solver.n_levels):
        info = solver.level_info(l)
        if l == solver.n_levels - 1:
            n = info["n_u"] + info["n_l"]
            total += n * n * elem
            break
        if info["k_layout"] in (1, 2):
            kb = info["k_blocks"] * (info["k_bs"] ** 2 * elem + 4)
        else:
            kb = info["nnz_K"] * (elem + 4)
        e = elem + 4
        total += sweeps * nj * kb
        total += (2 * sweeps + 1) * info["nnz_G"] * e
        total += (sweeps + 1) * (info["nnz_B"] + info["nnz_C"]) * e
        nnz_p = solver.level_matrix(l, "P_u").nnz + solver.level_matrix(l, "P_l").nnz
        if info.get("transfer_layout") == 1:
            total += 2 * (nnz_p * elem + 4 * (info["n_u"] + info["n_l"]))
        else:
            total += 2 * nnz_p * e
    return total


def time_vcycles(solver, reps=50):
    """Seconds per forward V-cycle application (graph replay, hipEvents)."""
    import torch

    r = torch.from_numpy(np.random.default_rng(0).standard_normal(solver.n)).cuda()
    for _ in range(3):
        solver.vcycle(r)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        solver.vcycle(r)
    b.record()
    b.synchronize()
    return a.elapsed_time(b) * 1e-3 / reps


PAPER_CONTEXT = ("The paper reports no GPU, per-solve or bandwidth figures for this path: its CheapSIMPLE "
                 "PA-AMG runs used GMRES to 1e-8 on 2x Xeon E5-2670 (16 cores), e.g. 20.5 GMRES iterations per "
                 "Newton step on a 6,300-unknown two-body problem (3 levels), and whole-simulation linear-solver "
                 "totals of 21,883 s (2D rings) and 16,288 s (3D tori) including a hierarchy rebuild every Newton "
                 "step.")

PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "k_smooth_u_bell_contact3d_40.md")
KERNELS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1912_09056_amd", "csrc", "kernels.hip")


def measured_traffic():
    """HBM bytes per launch of the FP32 level-0 smoother kernel from the
    committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the
    kernel source changed since those counters were taken."""
    import hashlib

    try:
        text = open(PROFILE).read()
        sha = hashlib.sha256(open(KERNELS, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines() if line.startswith(("traffic_", "kernel_source")))
    if vals.get("kernel_source_sha256_16", "").strip() != sha:
        return None
    return float(vals["traffic_bytes_per_launch_fp32"])


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    import torch

    from contactgen import make_workload
    from paper_1912_09056_amd import AMGOptions, AMGSolver
    from paper_1912_09056_amd.camg import KCLASS_SMOOTH_U

    torch.cuda.set_device(0)
    t0 = time.time()
    prob = make_workload(args.workload)
    print(f"[bench] workload {args.workload}: n={prob.n} nnz(K)={prob.K.nnz} ({time.time() - t0:.1f}s)",
          file=sys.stderr, flush=True)
    top = torch.from_numpy(prob.top_dofs).cuda()
    b = torch.from_numpy(prob.b).cuda()

    solvers, setup_s = {}, {}
    for name, prec in (("mixed", 1), ("fp64", 0)):
        t1 = time.time()
        solvers[name] = AMGSolver.from_problem(
            prob, AMGOptions(max_levels=args.levels, precision=prec, spmv_format=args.spmv_format))
        setup_s[name] = time.time() - t1
        print(f"[bench] setup {name}: {setup_s[name]:.1f}s levels={solvers[name].n_levels}", file=sys.stderr,
              flush=True)

    def step(s):
        x, fi = s.solve(b, rtol=1e-8)
        g = torch.zeros_like(x)
        g[top] = x[top]  # dL/dx for L = 0.5 ||u_top||^2
        lam, ai = s.solve(g, transpose=True, rtol=1e-8)
        dK = s.grad_K(lam, x)
        return fi, ai, dK

    results, xs = {}, {}
    for name in ("fp64", "mixed"):
        s = solvers[name]
        for _ in range(args.warmup):
            step(s)
        fwd, adj = [], []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            fi, ai, _ = step(s)
            fwd.append(fi)
            adj.append(ai)
        torch.cuda.synchronize()
        t_end = time.perf_counter()
        results[name] = dict(fwd=fwd, adj=adj, wall=(t_end - t_start) / args.steps)
        xs[name] = s.solve(b, rtol=1e-8)[0].cpu().numpy()
        results[name]["vcycle_s"] = time_vcycles(s)
        if name == "mixed":
            # per-launch durations of the level-0 smoother kernel: hipEvents
            # around every launch on the solver's stream during one more step
            # of the same work (event brackets need eager launches, so the
            # timed steps above replay the V-cycle graph instead)
            s.profile_enable(KCLASS_SMOOTH_U)
            step(s)
            torch.cuda.synchronize()
            n_launch, ms = s.profile_read(KCLASS_SMOOTH_U)
            s.profile_enable(0)
            results[name]["smooth_u"] = (n_launch, ms)
        print(f"[bench] {name}: fwd iters {[f['iters'] for f in fwd]} t {[round(f['seconds'], 5) for f in fwd]} "
              f"adj iters {[a['iters'] for a in adj]}", file=sys.stderr, flush=True)

    for name, r in results.items():
        for f in r["fwd"] + r["adj"]:
            if not f["converged"]:
                raise SystemExit(f"{name} solve did not converge: {f}")

    mixed, fp64 = results["mixed"], results["fp64"]
    solve_mixed = float(np.median([f["seconds"] for f in mixed["fwd"]]))
    solve_fp64 = float(np.median([f["seconds"] for f in fp64["fwd"]]))
    info0 = solvers["mixed"].level_info(0)
    n_launch, ms = mixed["smooth_u"]
    avg_s = ms * 1e-3 / max(n_launch, 1)
    bytes_per = smooth_u_bytes(info0, 4)
    achieved = bytes_per / avg_s / 1e9
    peak = 8000.0
    traffic = measured_traffic() if info0["k_layout"] == 1 else None
    vc_bytes = {"mixed": vcycle_matrix_bytes(solvers["mixed"], 4), "fp64": vcycle_matrix_bytes(solvers["fp64"], 8)}
    diff = float(np.linalg.norm(xs["mixed"] - xs["fp64"]) / np.linalg.norm(xs["fp64"]))

    out = {
        "metric": "solve time to rel. residual 1e-8 (s), V-cycle GB/s vs HBM peak: mixed vs FP64",
        "value": solve_mixed,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["wall"] * 1e3,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32 V-cycle / f64 FGMRES",
        "data": "synthetic (seeded structured hex8 contact problem)",
        "config": {
            "workload": f"{args.workload}: 3D hex8 two-block mortar contact, slave 40^3 over master 41x41x40, "
                        f"E=1 nu=0.3, all slave nodes active, n={prob.n}",
            "levels": solvers["mixed"].n_levels,
            "smoother": "CheapSIMPLE V(2,2), Jacobi(Atilde) prediction, diagonal Schur, alpha=omega=0.8",
            "krylov": "FGMRES(50) CGS2, rtol 1e-8",
            "step": "forward solve + adjoint solve + dL/dK sampling",
        },
        "mixed": {
            "solve_s": solve_mixed,
            "iters": int(np.median([f["iters"] for f in mixed["fwd"]])),
            "adjoint_s": float(np.median([a["seconds"] for a in mixed["adj"]])),
            "adjoint_iters": int(np.median([a["iters"] for a in mixed["adj"]])),
            "setup_s": setup_s["mixed"],
            "vcycles_per_s": 1.0 / mixed["vcycle_s"],
            "vcycle_matrix_GBps": vc_bytes["mixed"] / mixed["vcycle_s"] / 1e9,
        },
        "fp64": {
            "solve_s": solve_fp64,
            "iters": int(np.median([f["iters"] for f in fp64["fwd"]])),
            "adjoint_s": float(np.median([a["seconds"] for a in fp64["adj"]])),
            "adjoint_iters": int(np.median([a["iters"] for a in fp64["adj"]])),
            "ms_per_step": fp64["wall"] * 1e3,
            "setup_s": setup_s["fp64"],
            "vcycles_per_s": 1.0 / fp64["vcycle_s"],
            "vcycle_matrix_GBps": vc_bytes["fp64"] / fp64["vcycle_s"] / 1e9,
        },
        "vcycle_bytes_model": "matrix streams of one forward V-cycle (K in its device layout, G, B, C, R, P, the "
                              "dense coarsest inverse), vectors excluded: a lower bound on its traffic",
        "speedup_mixed_vs_fp64": solve_fp64 / solve_mixed,
        "mixed_vs_fp64_solution_rel_diff": diff,
        "paper_context": PAPER_CONTEXT,
        "roofline": {
            "kernel": "level-0 CheapSIMPLE residual+Jacobi, FP32 (k_smooth_u_bell: sliced blocked-ELL K)"
                      if info0["k_layout"] == 1 else "level-0 CheapSIMPLE residual+Jacobi, FP32 (k_smooth_u: CSR K)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": peak,
            "unit": "GB/s",
            "frac": achieved / peak,
            "traffic": traffic,
            "achieved_from_counters_GBps": traffic / avg_s / 1e9 if traffic else None,
            "bytes_per_launch": bytes_per,
            "bytes_model": "nonzero 3x3 blocks of K (9 FP32 values + 4-byte block index each) + G CSR + "
                           "5 FP32 vectors of n_u, read or written once",
            "k_blocks": info0["k_blocks"],
            "k_slots_with_padding": info0["k_slots"],
            "avg_launch_us": avg_s * 1e6,
            "launches": n_launch,
            "timing": "hipEvents around each launch on the solver stream, one profiled step after the timed ones",
        },
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"], x_ref = cpu_baseline(prob, args, out["fp64"]["iters"])
        ref = np.linalg.norm(x_ref)
        out["error_vs_oracle"] = {
            "reference": "FP64 oracle solve to relative residual 1e-12 on the host",
            "mixed": float(np.linalg.norm(xs["mixed"] - x_ref) / ref),
            "fp64": float(np.linalg.norm(xs["fp64"] - x_ref) / ref),
        }
    print(json.dumps(out), flush=True)


def cpu_baseline(prob, args, iters_to_tol):
    """The FP64 oracle on the host: a bounded sample of FGMRES iterations
    (fixed count, setup excluded), scaled to the iteration count that
    reaches 1e-8 (the GPU FP64 path's count, which matches the oracle's).
    Also returns the oracle's solution at relative residual 1e-12 (untimed),
    the reference for the GPU solutions' error."""
    from threadpoolctl import threadpool_info

    from oracle.adjoint import solve as oracle_solve
    from oracle.hierarchy import AMGOptions as OracleOptions
    from oracle.hierarchy import build_hierarchy

    opts = OracleOptions(max_levels=args.levels)
    t0 = time.time()
    lv = build_hierarchy(prob, opts)
    t_setup = time.time() - t0
    k = args.cpu_iters
    t0 = time.perf_counter()
    oracle_solve(lv, opts, prob.b, fixed_iters=k)
    t = time.perf_counter() - t0
    threads = max([1] + [p.get("num_threads", 1) for p in threadpool_info()])
    print(f"[bench] cpu oracle: setup {t_setup:.1f}s, {k} iterations {t:.1f}s", file=sys.stderr, flush=True)
    # reference solution for the error figures (not timed)
    t0 = time.time()
    x_ref = oracle_solve(lv, opts, prob.b, rtol=1e-12, max_iters=400).x
    print(f"[bench] oracle reference solve {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    return {
        "value": t / k * iters_to_tol,
        "unit": "s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{k} FGMRES(50) iterations of the FP64 numpy/scipy oracle on the same problem "
                  f"(setup excluded), scaled to {iters_to_tol} iterations",
        "setup_s": t_setup,
    }, x_ref


if __name__ == "__main__":
    main()
