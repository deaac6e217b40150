"""Benchmark: block-AMG preconditioned FGMRES solve of a 3D mortar-contact
saddle-point system on one MI355X.

One step is one pass of the whole solve path on the 100^3 / 101x101x100 hex8
contact workload with lognormal(0, 1) element moduli (6,273,918 unknowns, 4
levels): the mixed-precision forward FGMRES solve to relative residual 1e-8
(FP32 V-cycle hierarchy inside FP64 FGMRES), the adjoint solve A^T lam =
dL/dx on the same hierarchy, and the gradient sampling on A's pattern.
`value` is the forward solve time in seconds (median over the timed steps,
device time from hipEvents); the FP64 path is timed the same way on fewer
steps and reported beside it, with both iteration counts and the
mixed-vs-FP64 solution difference.

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
    ap.add_argument("--workload", default="contact3d_100_lognormal")
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="FGMRES iterations of the oracle in the CPU sample (0: sized to about 20 s)")
    ap.add_argument("--fp64-steps", type=int, default=5, help="timed steps of the FP64 comparison path")
    ap.add_argument("--spmv-format", type=int, default=0,
                    help="device storage of K: 0 auto, 1 CSR, 2 blocked-ELL; +4: no symmetric storage")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many MiB (5 times) and exit; used to scale "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    return ap.parse_args()


def copy_probe(mib):
    import torch

    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(5):
        y.copy_(x)
    b.record()
    b.synchronize()
    s = a.elapsed_time(b) * 1e-3 / 5
    print(json.dumps({"copy_probe_bytes_each_way": n * 4, "launches": 6, "us_per_copy": s * 1e6,
                      "read_plus_write_GBps": 2 * n * 4 / s / 1e9}), flush=True)


def smooth_u_bytes(info0, nnz_K_true, elem):
    """HBM bytes of one level-0 residual+Jacobi launch, as (algorithmic,
    stored).

    Both count G's entries (value + column) and row pointers, K's row
    pointers, and the vectors b_u, jinv, z_u (read once), z_l and zn_u
    (written).  Blocked layout: `algorithmic` counts K's true nonzeros
    (one value each) plus one block-column index (2 or 4 bytes, as stored)
    per nonzero bs x bs block;
    `stored` counts every value of those blocks (including the zeros a block
    holds) and is what the kernel actually streams (slice padding is in
    neither).  Symmetric storage (k_layout 3): only the blocks on and right
    of the block diagonal are stored and streamed (their true nonzeros, or
    all their values), with a 2-byte delta each, plus a 2-byte delta and a
    2-byte mirror position per block left of it (those blocks are the
    stored ones read again, transposed).  CSR layout: K's entries (value +
    column), both the same."""
    n_u, n_l = info0["n_u"], info0["n_l"]
    vec = n_u * elem * 4 + n_l * elem + info0["nnz_G"] * (elem + 4) + (n_u + 1) * 4
    if info0["k_layout"] == 3:
        bs = info0["k_bs"]
        up = info0["k_blocks"] - info0["k_lower_blocks"]
        idx = up * 2 + info0["k_lower_blocks"] * 4
        return info0["k_nnz_stored"] * elem + idx + vec, up * bs * bs * elem + idx + vec
    if info0["k_layout"] == 1:
        bs, ib = info0["k_bs"], info0["k_index_bytes"]
        return nnz_K_true * elem + info0["k_blocks"] * ib + vec, info0["k_blocks"] * (bs * bs * elem + ib) + vec
    b = info0["nnz_K"] * (elem + 4) + (n_u + 1) * 4 + vec
    return b, b


def vcycle_matrix_bytes(solver, elem, fine_k_value_bytes=None):
    """Matrix bytes streamed by one forward V-cycle (a lower bound on its
    traffic: vectors excluded).  Per smoothing level with nu_pre + nu_post
    sweeps of nj Jacobi steps: K is read (nu_pre + nu_post) * nj times (each
    sweep but the first from zero, its extra Jacobi steps, and the residual
    before restriction); G twice per sweep plus the residual; B and C once
    per sweep plus the residual; R and P once.  K in its device layout
    (bs x bs blocks with a 2- or 4-byte block index; in symmetric storage the
    blocks on and right of the diagonal plus 4 index bytes per block left of
    it; or CSR), P and R either CSR or
    index-free (values plus one 4-byte base column per fine row for P, one
    4-byte row index per fine row for R), the other blocks CSR (value +
    4-byte column).  The coarsest level: its dense inverse.  fine_k_value_bytes
    overrides the value size of a blocked-ELL level-0 K (bfloat16 storage)."""
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
        if info["k_layout"] == 3:
            ve = fine_k_value_bytes if (l == 0 and fine_k_value_bytes) else elem
            low = info["k_lower_blocks"]
            kb = (info["k_blocks"] - low) * (info["k_bs"] ** 2 * ve + 2) + low * 4
        elif info["k_layout"] in (1, 2):
            ve = fine_k_value_bytes if (l == 0 and fine_k_value_bytes and info["k_layout"] == 1) else elem
            kb = info["k_blocks"] * (info["k_bs"] ** 2 * ve + info["k_index_bytes"])
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

PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
KERNELS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1912_09056_amd", "csrc", "kernels.hip")


def measured_traffic(workload):
    """HBM bytes per launch of the FP32 level-0 smoother kernel on this
    workload from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or
    None when there is none or the kernel source changed since those
    counters were taken."""
    import hashlib

    try:
        text = open(os.path.join(PROFILES, f"k_smooth_u_bell_{workload}.md")).read()
        sha = hashlib.sha256(open(KERNELS, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines() if line.startswith(("traffic_", "kernel_source")))
    if vals.get("kernel_source_sha256_16", "").strip() != sha:
        return None
    return float(vals["traffic_bytes_per_launch_fp32"])

WORKLOAD_TEXT = {
    "contact3d_40": "3D hex8 two-block mortar contact, slave 40^3 over master 41x41x40, E=1 nu=0.3, all slave "
                    "nodes active",
    "contact3d_100_lognormal": "3D hex8 two-block mortar contact, slave 100^3 over master 101x101x100, element "
                               "E ~ lognormal(0, 1), nu=0.3, all slave nodes active",
    "contact3d_150_curved": "3D hex8 two-block mortar contact, slave 150^3 over master 151x151x150, curved "
                            "interface, element E ~ lognormal(0, 2), nu ~ U[0.25, 0.35], all slave nodes active",
}


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
    for name, prec in (("mixed", 1), ("fp64", 0), ("mixed_bf16", 2)):
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
        dA = s.grad_A(lam, x)  # dL/dA on the stored entries of K, G, B, C
        return fi, ai, dA

    results, xs = {}, {}
    for name in ("fp64", "mixed_bf16", "mixed"):
        s = solvers[name]
        # the FP64 and bfloat16-storage paths are comparisons: fewer timed steps
        n_steps = args.steps if name == "mixed" else max(1, min(args.steps, args.fp64_steps))
        n_warm = args.warmup if name == "mixed" else min(args.warmup, 1)
        for _ in range(n_warm):
            step(s)
        fwd, adj = [], []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(n_steps):
            fi, ai, _ = step(s)
            fwd.append(fi)
            adj.append(ai)
        torch.cuda.synchronize()
        t_end = time.perf_counter()
        results[name] = dict(fwd=fwd, adj=adj, wall=(t_end - t_start) / n_steps, steps=n_steps)
        x, fi = s.solve(b, rtol=1e-8)
        xs[name] = x.cpu().numpy()
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
              f"adj iters {[a['iters'] for a in adj]} t {[round(a['seconds'], 5) for a in adj]}", file=sys.stderr,
              flush=True)

    for name, r in results.items():
        for f in r["fwd"] + r["adj"]:
            if not f["converged"]:
                raise SystemExit(f"{name} solve did not converge: {f}")

    # true residuals of both solutions, recomputed on the host in FP64
    A = prob.full_matrix()
    true_res = {name: float(np.linalg.norm(prob.b - A @ x) / np.linalg.norm(prob.b)) for name, x in xs.items()}
    del A

    mixed, fp64 = results["mixed"], results["fp64"]
    solve_mixed = float(np.median([f["seconds"] for f in mixed["fwd"]]))
    solve_fp64 = float(np.median([f["seconds"] for f in fp64["fwd"]]))
    info0 = solvers["mixed"].level_info(0)
    n_launch, ms = mixed["smooth_u"]
    avg_s = ms * 1e-3 / max(n_launch, 1)
    bytes_alg, bytes_stored = smooth_u_bytes(info0, prob.K.nnz, 4)
    achieved = bytes_alg / avg_s / 1e9
    peak = 8000.0
    traffic = measured_traffic(args.workload) if info0["k_layout"] in (1, 3) else None
    sym = info0["k_layout"] == 3
    # the same operator's bytes in the full blocked layout (every nonzero block
    # stored, 2-byte deltas): what a full-storage pass would have to stream
    full_bytes = smooth_u_bytes(dict(info0, k_layout=1, k_index_bytes=2), prob.K.nnz, 4)[0] if sym else bytes_alg
    vc_bytes = {"mixed": vcycle_matrix_bytes(solvers["mixed"], 4), "fp64": vcycle_matrix_bytes(solvers["fp64"], 8),
                "mixed_bf16": vcycle_matrix_bytes(solvers["mixed_bf16"], 4, fine_k_value_bytes=2)}
    diff = float(np.linalg.norm(xs["mixed"] - xs["fp64"]) / np.linalg.norm(xs["fp64"]))
    diff16 = float(np.linalg.norm(xs["mixed_bf16"] - xs["fp64"]) / np.linalg.norm(xs["fp64"]))

    def summary(name):
        r = results[name]
        return {
            "solve_s": float(np.median([f["seconds"] for f in r["fwd"]])),
            "iters": int(np.median([f["iters"] for f in r["fwd"]])),
            "adjoint_s": float(np.median([a["seconds"] for a in r["adj"]])),
            "adjoint_iters": int(np.median([a["iters"] for a in r["adj"]])),
            "timed_steps": r["steps"],
            "ms_per_step": r["wall"] * 1e3,
            "setup_s": setup_s[name],
            "true_rel_residual": true_res[name],
            "vcycles_per_s": 1.0 / r["vcycle_s"],
            "vcycle_matrix_GBps": vc_bytes[name] / r["vcycle_s"] / 1e9,
            "vcycle_matrix_frac_of_peak": vc_bytes[name] / r["vcycle_s"] / 1e9 / peak,
        }

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
            "workload": f"{args.workload}: {WORKLOAD_TEXT.get(args.workload, 'synthetic contact problem')}, "
                        f"n={prob.n}, nnz(K)={prob.K.nnz}",
            "levels": solvers["mixed"].n_levels,
            "level_rows": [solvers["mixed"].level_info(l)["n_u"] + solvers["mixed"].level_info(l)["n_l"]
                           for l in range(solvers["mixed"].n_levels)],
            "smoother": "CheapSIMPLE V(2,2), Jacobi(Atilde) prediction, diagonal Schur, alpha=omega=0.8",
            "krylov": "FGMRES(50) CGS2, rtol 1e-8",
            "step": "mixed forward solve + adjoint solve + dL/dA sampling on K, G, B, C",
        },
        "mixed": summary("mixed"),
        "fp64": summary("fp64"),
        "mixed_bf16": dict(summary("mixed_bf16"), solution_rel_diff_vs_fp64=diff16,
                           note="option CAMG_PREC_MIXED_BF16: as mixed, with the fine level's K stored in bfloat16 "
                                "for the V-cycle (FP32 arithmetic); not the headline, which keeps the FP32 hierarchy"),
        "vcycle_bytes_model": "matrix streams of one forward V-cycle (K in its device layout, G, B, C, R, P, the "
                              "dense coarsest inverse), vectors excluded: a lower bound on its traffic",
        "speedup_mixed_vs_fp64": solve_fp64 / solve_mixed,
        "mixed_vs_fp64_solution_rel_diff": diff,
        "paper_context": PAPER_CONTEXT,
        "roofline": {
            "kernel": ("level-0 CheapSIMPLE residual+Jacobi, FP32 (k_smooth_u_bell_npl, one thread per node, on "
                       "levels of 8192 slices or more, else k_smooth_u_bell: sliced blocked-ELL K, symmetric "
                       "storage)") if sym else
                      "level-0 CheapSIMPLE residual+Jacobi, FP32 (k_smooth_u_bell: sliced blocked-ELL K)"
                      if info0["k_layout"] == 1 else "level-0 CheapSIMPLE residual+Jacobi, FP32 (k_smooth_u: CSR K)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": peak,
            "unit": "GB/s",
            "frac": achieved / peak,
            "traffic": traffic,
            "achieved_from_counters_GBps": traffic / avg_s / 1e9 if traffic else None,
            "bytes_per_launch": bytes_alg,
            "bytes_model": ("K's true nonzeros in the stored blocks (on and right of the block diagonal; one FP32 "
                            "value each) + a 2-byte delta per stored block + a 2-byte delta and a 2-byte mirror "
                            "position per block left of the diagonal + G CSR + row pointers + 5 FP32 vectors of "
                            "n_u, read or written once") if sym else
                           f"K's true nonzeros (one FP32 value each) + one {info0['k_index_bytes']}-byte block-column "
                           "index per nonzero 3x3 block + G CSR + row pointers + 5 FP32 vectors of n_u, read or "
                           "written once",
            "bytes_per_launch_stored": bytes_stored,
            "frac_stored_bytes": bytes_stored / avg_s / 1e9 / peak,
            "stored_bytes_model": "as bytes_model but every value of each nonzero 3x3 block (the zeros a block "
                                  "holds included): what the kernel streams",
            "nnz_K": prob.K.nnz,
            "full_storage_bytes_per_launch": full_bytes,
            "full_storage_equivalent_GBps": full_bytes / avg_s / 1e9,
            "full_storage_equivalent_frac": full_bytes / avg_s / 1e9 / peak,
            "k_layout": {1: "sliced blocked-ELL", 3: "sliced blocked-ELL, symmetric storage"}.get(
                info0["k_layout"], "CSR"),
            "k_blocks": info0["k_blocks"],
            "k_lower_blocks": info0["k_lower_blocks"],
            "k_nnz_stored": info0["k_nnz_stored"],
            "k_slots_with_padding": info0["k_slots"],
            "avg_launch_us": avg_s * 1e6,
            "launches": n_launch,
            "timing": "hipEvents around each launch on the solver stream, one profiled step after the timed ones",
        },
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"], x_ref = cpu_baseline(prob, args, out["fp64"]["iters"])
        if x_ref is not None:
            ref = np.linalg.norm(x_ref)
            out["error_vs_oracle"] = {
                "reference": "FP64 oracle solve to relative residual 1e-12 on the host",
                "mixed": float(np.linalg.norm(xs["mixed"] - x_ref) / ref),
                "fp64": float(np.linalg.norm(xs["fp64"] - x_ref) / ref),
            }
    print(json.dumps(out), flush=True)


def cpu_baseline(prob, args, iters_to_tol):
    """The FP64 oracle on the host, on one thread (its sparse products are
    single-threaded SciPy; the dense BLAS pool is limited to one thread so
    the count is exact): a bounded sample of FGMRES iterations (fixed count,
    setup excluded), scaled to the iteration count that reaches 1e-8 on the
    GPU's FP64 path.  Below a million unknowns it also returns the oracle's
    solution at relative residual 1e-12 (untimed), the reference for the GPU
    solutions' error; above, that solve would take minutes and is skipped."""
    from threadpoolctl import threadpool_limits

    from oracle.adjoint import solve as oracle_solve
    from oracle.hierarchy import AMGOptions as OracleOptions
    from oracle.hierarchy import build_hierarchy

    opts = OracleOptions(max_levels=args.levels)
    with threadpool_limits(limits=1):
        t0 = time.time()
        lv = build_hierarchy(prob, opts)
        t_setup = time.time() - t0
        k = args.cpu_iters
        if k <= 0:
            # size the sample to about 20 s from the cost of one iteration
            t0 = time.perf_counter()
            oracle_solve(lv, opts, prob.b, fixed_iters=1)
            t1 = time.perf_counter() - t0
            k = int(min(20, max(1, round(20.0 / max(t1, 1e-3)))))
        t0 = time.perf_counter()
        oracle_solve(lv, opts, prob.b, fixed_iters=k)
        t = time.perf_counter() - t0
        print(f"[bench] cpu oracle: setup {t_setup:.1f}s, {k} iterations {t:.1f}s", file=sys.stderr, flush=True)
        x_ref = None
        if prob.n < 1_000_000:
            t0 = time.time()
            x_ref = oracle_solve(lv, opts, prob.b, rtol=1e-12, max_iters=400).x
            print(f"[bench] oracle reference solve {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    return {
        "value": t / k * iters_to_tol,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{k} FGMRES(50) iterations of the FP64 numpy/scipy oracle on the same problem, one thread "
                  f"(setup of {t_setup:.0f} s excluded), scaled to {iters_to_tol} iterations",
        "setup_s": t_setup,
    }, x_ref


if __name__ == "__main__":
    main()
