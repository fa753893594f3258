"""Benchmark of the blocked multi-RHS quark solve on one MI355X.

A step is one blocked force evaluation (the paper's Alg. 2) for the 8^3x8
Schroedinger-functional lattice with 5 pseudo-fermions (kappa = 0.13,
links exp(i 0.3 H)): pack, one batched CG on D^+D to a 1e-10 true relative
residual per RHS (FP32 inner iteration with FP64 reliable updates), the g5 map
to X and Y, the summed force and the action.  All inputs are synthetic and
resident in device memory before the timed region.

Prints one JSON line.  Extra keys: the same solve in plain FP64 CG on the same
GPU, the FP16 path and block CG, the error of every result against the FP64
oracle (solutions, X, Y, force), the fused half-dslash bandwidth and GFLOP/s
on lattices far larger than the 256 MB Infinity Cache, and the comparison
rows (16^3x16 FP16 storage, the learned preconditioner, the 64-lattice batch).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "5-RHS D†D solve time to 1e-10 vs plain FP64 CG; dslash HBM GB/s, % peak"
# solve tolerance of the bench step per route, chosen for equal force accuracy
STEP_TOL = {"full": 1e-10, "schur": 1e-11}
HBM_PEAK_GBS = 8000.0
HOP_FLOP = 1320  # flop of the Wilson hopping term per output site per RHS


def rel_err(a, b, np):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_config1(p, u, phi, np):
    """The oracle's results for the bench workload (untimed): Alg. 2 (X, Y by
    two per-RHS FP64 CG solves to 1e-13, the literal force) and the normal
    equation solution (D^+D)^-1 Phi the solve rows compute."""
    from oracle import force as fmod
    from oracle import native, solvers
    from oracle.dirac import WilsonDirac
    d = native.NativeWilson(p.dims, p.bc, p.kappa, u)
    x, _ = solvers.solve_D(d, phi, 1e-13)
    y, _ = solvers.solve_Ddag(d, x, 1e-13)
    g = fmod.coefficients_to_matrix(fmod.force_coefficients(WilsonDirac(p.dims, p.bc, p.kappa, u), x, y))
    z, _ = solvers.cg_normal(d, phi, 1e-13)
    return {"x": x, "y": y, "g": g, "s": fmod.action(None, x), "z": z}


def oracle_first_rhs(p, u, b, tol=1e-12):
    """The oracle's (D^+D)^-1 b for the first RHS only (16^3x16 rows: one FP64
    CG with the compiled operator, untimed)."""
    from oracle import native, solvers
    d = native.NativeWilson(p.dims, p.bc, p.kappa, u)
    x, _ = solvers.cg(d.DdagD, b[:1], tol)
    return x


COUNTERS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                             "hop_kernel_counters_sf8x8x8x8_5rhs.txt")
KERNEL_SOURCES = ("hop.hip", "hop_impl.h", "device.h", "internal.h")


def kernel_source_hash() -> str:
    """SHA-256 over the sources of the hopping kernel: counter figures taken
    with other sources do not describe the kernel that runs."""
    h = hashlib.sha256()
    base = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1009_5169_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(base, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(prec: str, n_rhs: int, shape=None):
    """HBM-side bytes per launch of the roofline kernel from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by
    what the counter reads for a plain copy of known size), or None when the
    summary is missing, is for another precision / RHS count / launch shape,
    or was taken with different kernel sources."""
    try:
        with open(COUNTERS_FILE) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_sha256") != kernel_source_hash() or kv.get("prec") != prec or int(kv.get("n_rhs", 0)) != n_rhs:
        return None
    if shape is not None and [int(v) for v in kv.get("launch_shape", "").split()] != [int(v) for v in shape]:
        return None
    copy_kib = float(kv["copy_bytes"]) / 1024.0
    fetch = float(kv["fetch_kib_per_dispatch"]) * copy_kib / float(kv["copy_fetch_kib"])
    write = float(kv["write_kib_per_dispatch"]) * copy_kib / float(kv["copy_write_kib"])
    return int(round((fetch + write) * 1024))


def kernel_name(prec: str, shape) -> str:
    """The hopping kernel a launch shape (sb, nr, xcd, tc, ds) selects."""
    sb, nr, xcd, tc, ds = shape
    if ds:
        return f"hop_split_kernel<EPI_D, {ds}, {prec}> (both parities)"
    if tc:
        return f"hop_sweep_kernel<EPI_D, {prec}> (both parities, {tc} time slices per thread)"
    return f"hop_kernel<EPI_D, {prec}> (both parities)"


def hop_bytes_per_site_rhs(prec: str, n_rhs: int) -> float:
    """Algorithmic HBM bytes of the timed hopping kernel (D epilogue, both
    parities in one launch, input = self field) per lattice site per RHS: the
    input spinor read once, the output written once, and the site's 4 links
    U_mu(n) read once per launch and shared by the n_rhs RHS (every link is
    the forward link of one site and the backward link of its neighbour).
    FP64 links are 18 reals; the FP32 / FP16 copies store two rows (12 reals);
    FP16 spinors carry one FP32 norm."""
    if prec == "fp64":
        spinor, link = 24 * 8, 18 * 8
    elif prec == "fp32":
        spinor, link = 24 * 4, 12 * 4
    else:  # fp16 values + one fp32 norm per site
        spinor, link = 24 * 2 + 4, 12 * 2
    return 2 * spinor + 4 * link / n_rhs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "fp16"],
                    help="precision of the bench step's solves (default: the fastest measured on this "
                         "workload, see step_ms_by_route)")
    ap.add_argument("--route", default="schur", choices=["full", "schur"],
                    help="route of the bench step: CG on D^+D (full) or the even/odd Schur complement "
                         "(schur, the default: the fastest measured on this workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bandwidth", action="store_true")
    ap.add_argument("--bw-dims", default="32,32,32,64")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the batch, FP16 and learned-preconditioner measurements")
    ap.add_argument("--rows", default="fp16,learned,batch,routes,paper_solvers,hmc",
                    help="which comparison rows to run (comma list of fp16, learned, batch, routes, "
                         "paper_solvers, hmc)")
    ap.add_argument("--rows-only", action="store_true",
                    help="run only the comparison rows (no bench step), for kernel traces of them")
    ap.add_argument("--profile-big", action="store_true",
                    help="with --profile-kernels: also the bandwidth lattice, 1 and 5 RHS")
    ap.add_argument("--order-ab", action="store_true",
                    help="with --profile-kernels: on the bandwidth lattice, 1 RHS, time the direction-split "
                         "kernel in half-index tile order and then in z-blocked order (forced launch shapes)")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only launch the roofline kernel (solve shape) and a 1 GiB copy, for counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the pseudo-fermion "
              "sharding across GPUs is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1009_5169_amd as mfq
    import synth

    dev = "cuda:0"
    p = synth.CONFIG_1
    if args.profile_kernels:
        profile_kernels(args, synth, mfq, torch, dev, np)
        return
    if args.rows_only:
        print(json.dumps({"rows": run_rows(args, synth, mfq, torch, dev, np)}))
        return
    u = p.links()
    phi_h = p.rhs()
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, torch.from_numpy(u).to(dev))
    phi = torch.from_numpy(phi_h).to(dev)
    # route S solves D X = Phi and D^+ Y = X, each to its own tolerance, so at
    # the same tol its X, Y and force carry ~10x the error of route F's single
    # solve on D^+D; it runs at STEP_TOL["schur"] = 1e-11, where its force
    # matches route F's accuracy at 1e-10 (rel_err_vs_oracle checks it)
    params = mfq.make_params(tol=STEP_TOL[args.route], prec=args.prec, max_iter=20000, route=args.route)
    torch.cuda.synchronize()
    print(f"[bench] workload {p.name} prec={args.prec} route={args.route}", file=sys.stderr, flush=True)

    def step():
        return lat.force(phi, params=params)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g, action, stats, rc = step()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)
    # the same step once more (untimed), keeping X and Y for the oracle comparison
    g_step, action_step, stats_step, _, x_step, y_step = lat.force(phi, params=params, want_xy=True)
    # the step by every route and precision (5 timed steps each), the basis of the default
    step_ms_by_route = {}
    for rt in ("full", "schur"):
        for pr_name in ("fp64", "fp32", "fp16"):
            pr_alt = mfq.make_params(tol=STEP_TOL[rt], prec=pr_name, max_iter=20000, route=rt)
            lat.force(phi, params=pr_alt)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(5):
                lat.force(phi, params=pr_alt)
            torch.cuda.synchronize()
            step_ms_by_route[f"{rt}_{pr_name}"] = round((time.perf_counter() - t) * 200, 4)

    # dominant kernel: the fused hopping kernel with the D epilogue of the inner
    # CG (both parities in one launch), same launch shape as in the solve,
    # timed with HIP events on its stream
    n = p.n_rhs
    hop_ms = lat.time_hop(args.prec, n, iters=200)
    shape = lat.hop_shape(args.prec, n)
    vd = p.dims[0] * p.dims[1] * p.dims[2] * (p.dims[3] - 1)
    per_launch = hop_bytes_per_site_rhs(args.prec, n) * vd * n
    achieved = per_launch / (hop_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": measured_traffic(args.prec, n, shape),
                "kernel": kernel_name(args.prec, shape), "launch_us": round(hop_ms * 1e3, 3),
                "timing": "HIP events around 200 back-to-back launches on a nonzero field, solver launch shape "
                          "(route S runs the same kernel and shape on one parity at a time)",
                "residency": "cache-resident: %.1f MB per launch, inside the 256 MB Infinity Cache; "
                             "launch-latency bound (see roofline_hbm_lattice for the HBM-resident figure)"
                             % (per_launch / 1e6),
                "gflops": round(HOP_FLOP * vd * n / (hop_ms * 1e-3) / 1e9, 1),
                "shape": list(shape),
                "algorithmic_bytes_per_launch": int(per_launch)}

    # solve-only times on the same GPU: this precision and plain FP64 CG
    def solve_ms(prec, reps=5, precond="none"):
        pr = mfq.make_params(tol=1e-10, prec=prec, max_iter=20000, precond=precond)
        lat.solve(phi, params=pr)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            x, st, _ = lat.solve(phi, params=pr)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / reps, x, st

    s_ms, x_this, st_this = solve_ms("fp32")
    s64_ms, x64, st64 = solve_ms("fp64")
    s16_ms, x16, st16 = solve_ms("fp16")
    sb_ms, xb, stb = solve_ms("fp64", precond="blockcg")  # one Krylov space for all RHS
    x64h = x64.cpu().numpy()
    err = lambda a: float(np.linalg.norm(a.cpu().numpy() - x64h) / np.linalg.norm(x64h))
    # results the CPU-baseline leg compares with the oracle
    gpu_results = {"g": g_step.cpu().numpy(), "x": x_step.cpu().numpy(), "y": y_step.cpu().numpy(),
                   "s": list(action_step),
                   "z": {"fp32": x_this.cpu().numpy(), "fp64": x64h, "fp16": x16.cpu().numpy(),
                         "block_cg_fp64": xb.cpu().numpy()}}

    out = {
        "metric": METRIC, "value": round(ms_per_step, 4), "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16"}[args.prec], "data": "synthetic",
        "config": {"workload": p.name, "dims": list(p.dims), "bc": p.bc, "kappa": p.kappa,
                   "link_eps": p.eps, "n_rhs": n, "tol": STEP_TOL[args.route],
                   "step": ("blocked force (Alg. 2): D X = Phi and D^+ Y = X by CG on the even/odd Schur "
                            "complement, odd sites rebuilt, + force + action" if args.route == "schur" else
                            "blocked force: batched CG on DdagD + g5 map + force + action"),
                   "route": args.route, "precision": args.prec,
                   "step_iters": [s["iters"] for s in stats_step]},
        "step_ms_by_route": step_ms_by_route,
        # the timed step against the same step by plain FP64 CG (route F: one CG
        # on D^+D to 1e-10 + g5 map), both at the same force error vs the oracle
        "step_speedup_vs_plain_fp64_cg": round(step_ms_by_route["full_fp64"] / ms_per_step, 3),
        "roofline": roofline,
        "solve_ms": {"fp32": round(s_ms, 4), "fp64": round(s64_ms, 4), "fp16": round(s16_ms, 4),
                     "block_cg_fp64": round(sb_ms, 4)},
        "solve_speedup_fp32_vs_fp64_cg": round(s64_ms / s_ms, 3),
        "solve_speedup_fp16_vs_fp64_cg": round(s64_ms / s16_ms, 3),
        "iters": {"fp32": [s["iters"] for s in st_this], "fp64": [s["iters"] for s in st64],
                  "fp16": [s["iters"] for s in st16], "block_cg_fp64": [s["iters"] for s in stb]},
        "solution_rel_err_vs_fp64_path": {"fp32": err(x_this), "fp16": err(x16), "block_cg_fp64": err(xb)},
        "true_rel_resid_max": max(s["true_rel_resid"] for s in st_this),
    }

    if not args.no_bandwidth:
        out["dslash_bandwidth"] = bandwidth_runs(args, synth, mfq, torch, dev, np)
        main_run = out["dslash_bandwidth"].get("32x32x32x64_periodic", {}).get("runs", {}).get("fp32_n5")
        if main_run:
            out["roofline_hbm_lattice"] = {
                "bound": "hbm", "achieved": main_run["GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": main_run["frac"], "gflops": main_run["GFLOP/s"], "launch_us": main_run["us"],
                "kernel": "inner-solver hopping kernel, D epilogue, FP32, 5 RHS, both parities",
                "workload": "32^3x64 periodic, 5 RHS (HBM-resident: 2.4 GB per launch)",
                "shape": main_run["shape"]}

    row_results = {}
    if not args.no_rows:
        out["rows"] = run_rows(args, synth, mfq, torch, dev, np, row_results)

    if not args.no_cpu_baseline:
        # the CPU-baseline leg: the oracle timed on the host, and the oracle's
        # results that every GPU result above is compared with
        out["cpu_baseline"] = cpu_baseline(p, u, phi_h, np)
        out["rel_err_vs_oracle"] = oracle_errors(p, u, phi_h, gpu_results, row_results, synth, np)
    lat.close()
    print(json.dumps(out))


def oracle_errors(p, u, phi_h, gpu, rows, synth, np):
    """Errors of the GPU results against the FP64 oracle (part of the
    CPU-baseline leg; the oracle's solves are untimed here)."""
    print("[bench] oracle reference for the bench workload", file=sys.stderr, flush=True)
    ref = oracle_config1(p, u, phi_h, np)
    out = {"oracle": "FP64 CPU oracle: per-RHS CG to 1e-13 (Alg. 2's two solves for X, Y; the normal "
                     "equations for the solve rows), literal per-generator force; 16^3x16 rows: the first "
                     "RHS, CG to 1e-12",
           "step": {"force": rel_err(gpu["g"], ref["g"], np), "X": rel_err(gpu["x"], ref["x"], np),
                    "Y": rel_err(gpu["y"], ref["y"], np),
                    "action": float(max(abs(a - b) / b for a, b in zip(gpu["s"], ref["s"])))},
           "solve": {k: rel_err(v, ref["z"], np) for k, v in gpu["z"].items()}}
    for row, (q, xs) in rows.items():
        print(f"[bench] oracle CG (first RHS) for row {row}", file=sys.stderr, flush=True)
        x_or = oracle_first_rhs(q, q.links(), q.rhs())
        out[row] = {k: rel_err(v[:1], x_or, np) for k, v in xs.items()}
    return out


def cpu_baseline(p, u, phi_h, np):
    """The oracle as it stands, timed on the host: Alg. 2 for the bench
    workload (two per-RHS FP64 CG solves to 1e-10 with the compiled operator,
    then the literal force), median of 3 on all cores; then a bounded sample
    on one core (the first pseudo-fermion only, scaled by the RHS count)."""
    from oracle import force as fmod
    from oracle import native, solvers
    from oracle.dirac import WilsonDirac

    d = native.NativeWilson(p.dims, p.bc, p.kappa, u)
    wd = WilsonDirac(p.dims, p.bc, p.kappa, u)

    def alg2(phi):
        t = time.perf_counter()
        x, _ = solvers.solve_D(d, phi, 1e-10)
        y, _ = solvers.solve_Ddag(d, x, 1e-10)
        fmod.force_coefficients(wd, x, y)
        return (time.perf_counter() - t) * 1e3

    threads = native.set_threads(0)
    print(f"[bench] cpu oracle: one full step x3, {threads} threads", file=sys.stderr, flush=True)
    runs = sorted(alg2(phi_h) for _ in range(3))
    one_cg = time.perf_counter()
    solvers.cg_normal(d, phi_h, 1e-10)
    one_cg = (time.perf_counter() - one_cg) * 1e3
    native.set_threads(1)
    print("[bench] cpu oracle: first pseudo-fermion, 1 thread", file=sys.stderr, flush=True)
    single = alg2(phi_h[:1]) * phi_h.shape[0]
    native.set_threads(threads)
    return {"value": round(runs[1], 2), "unit": "ms", "cores": threads, "kind": "oracle",
            "runs_ms": [round(v, 2) for v in runs],
            "sample": "one full step of the same workload, median of 3: Alg. 2 as the oracle states it "
                      "(two per-RHS FP64 CG solves on the normal equations, tol 1e-10, compiled operator "
                      "with OpenMP over sites; then the literal per-generator force)",
            "one_core": {"value": round(single, 2), "unit": "ms", "cores": 1,
                         "sample": "the first pseudo-fermion's Alg. 2 on one thread, times the 5 RHS"},
            "one_cg_normal_ms": round(one_cg, 2),
            "one_cg_normal_note": "the oracle's single CG on D^+D for all 5 RHS (the solve the GPU step "
                                  "runs once), all cores"}


BANDWIDTH_RUNS = (
    # (dims, bc, precisions, RHS counts)
    ((32, 32, 32, 64), "periodic", ("fp64", "fp32", "fp16"), (1, 5, 8)),
    ((48, 48, 48, 48), "periodic", ("fp32",), (1, 5)),
    ((32, 32, 32, 64), "sf", ("fp32",), (5,)),
)


def bandwidth_runs(args, synth, mfq, torch, dev, np):
    """The inner solver's hopping kernel (D epilogue, both parities, tuned
    launch shape) on lattices far larger than the 256 MB Infinity Cache:
    algorithmic GB/s, fraction of the 8 TB/s HBM peak and GFLOP/s."""
    out = {}
    for dims, bc, precs, nrs in BANDWIDTH_RUNS:
        if args.bw_dims != "32,32,32,64" and dims != tuple(int(v) for v in args.bw_dims.split(",")):
            continue
        print(f"[bench] bandwidth lattice {dims} {bc}", file=sys.stderr, flush=True)
        big = bandwidth_lattice(dims, synth, mfq, torch, dev, np, bc=bc)
        vd = dims[0] * dims[1] * dims[2] * (dims[3] - 1 if bc == "sf" else dims[3])
        runs = {}
        for prec in precs:
            for nr in nrs:
                ms = big.time_hop(prec, nr, iters=20)
                gbs = hop_bytes_per_site_rhs(prec, nr) * vd * nr / (ms * 1e-3) / 1e9
                runs[f"{prec}_n{nr}"] = {"us": round(ms * 1e3, 2), "GB/s": round(gbs, 1),
                                         "frac": round(gbs / HBM_PEAK_GBS, 4),
                                         "GFLOP/s": round(HOP_FLOP * vd * nr / (ms * 1e-3) / 1e9, 1),
                                         "shape": list(big.hop_shape(prec, nr))}
                print(f"[bench] bw {prec} n={nr}: {gbs:.1f} GB/s", file=sys.stderr, flush=True)
        out["x".join(map(str, dims)) + "_" + bc] = {"dims": list(dims), "bc": bc, "runs": runs,
                                                   "kernel": "hop kernel, D epilogue, both parities"}
        big.close()
        torch.cuda.empty_cache()
    return out


def run_rows(args, synth, mfq, torch, dev, np, row_results=None):
    """The comparison rows named by --rows; row_results (if given) receives
    each 16^3x16 row's solutions for the oracle comparison."""
    rows = set(args.rows.split(","))
    out = {}
    keep = row_results if row_results is not None else {}
    if "fp16" in rows:
        out["fp16_16x16x16x16"] = bench_fp16(synth, mfq, torch, dev, np, keep)
    if "learned" in rows:
        out["learned_16x16x16x16"] = bench_learned(synth, mfq, torch, dev, np, keep)
    if "batch" in rows:
        out["batch_64_lattices"] = bench_batch(synth, mfq, torch, dev, np)
    if "routes" in rows:
        out["routes"] = bench_routes(synth, mfq, torch, dev, np)
    if "paper_solvers" in rows:
        out["paper_solvers_16x16x16x16"] = bench_paper_solvers(synth, mfq, torch, dev, np)
    if "hmc" in rows:
        out["hmc_8x8x8x8"] = bench_hmc(synth, mfq, torch, dev, np)
    return out


def _timed(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        res = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3 / reps, res


def bench_fp16(synth, mfq, torch, dev, np, keep):
    """16^3x16 SF, eps = 0.5, kappa = 0.135, 5 RHS: FP16 storage (per-site norm)
    with FP64 defect correction against FP32 and plain FP64 CG, and FP64 block
    CG (one Krylov space for the 5 RHS), all to 1e-10."""
    p = synth.CONFIG_2
    print(f"[bench] row fp16 {p.name}", file=sys.stderr, flush=True)
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, torch.from_numpy(p.links()).to(dev))
    b = torch.from_numpy(p.rhs()).to(dev)
    res = {"workload": p.name, "tol": 1e-10}
    xs = {}
    for prec in ("fp64", "fp32", "fp16"):
        pr = mfq.make_params(tol=1e-10, prec=prec, max_iter=50000)
        ms, (x, st, rc) = _timed(lambda: lat.solve(b, params=pr))
        xs[prec] = x.cpu().numpy()
        res[prec] = {"ms": round(ms, 3), "rc": rc, "iters": [s["iters"] for s in st],
                     "true_rel_resid_max": max(s["true_rel_resid"] for s in st)}
    for prec in ("fp32", "fp16"):
        res[prec]["rel_err_vs_fp64_path"] = float(np.linalg.norm(xs[prec] - xs["fp64"]) / np.linalg.norm(xs["fp64"]))
    # block CG: the 5 RHS share one Krylov space (FP64)
    pr = mfq.make_params(tol=1e-10, prec="fp64", precond="blockcg", max_iter=50000)
    ms, (x, st, rc) = _timed(lambda: lat.solve(b, params=pr))
    res["block_cg_fp64"] = {"ms": round(ms, 3), "rc": rc, "iters": [s["iters"] for s in st],
                            "true_rel_resid_max": max(s["true_rel_resid"] for s in st),
                            "rel_err_vs_fp64_path": float(np.linalg.norm(x.cpu().numpy() - xs["fp64"])
                                                          / np.linalg.norm(xs["fp64"])),
                            "iteration_ratio_vs_fp64_cg": round(st[0]["iters"] / max(res["fp64"]["iters"]), 3)}
    xs["block_cg_fp64"] = x.cpu().numpy()
    keep["fp16_16x16x16x16"] = (p, {k: v[:1] for k, v in xs.items()})
    lat.close()
    return res


def bench_learned(synth, mfq, torch, dev, np, keep):
    """16^3x16 SF, eps = 0.5, kappa = 0.1375, 5 evaluation RHS: train the PTC
    network on pairs from plain CG on b = A xi with known Gaussian solutions xi
    (seeds 6000+), then FGMRES(16) with it and without it (the cycle in FP64,
    and in FP32 with FP64 restarts), plain FP64 CG and CG with FP32 inner
    solves, all to 1e-10."""
    p = synth.CONFIG_4
    print(f"[bench] row learned {p.name}", file=sys.stderr, flush=True)
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, torch.from_numpy(p.links()).to(dev))
    b = torch.from_numpy(p.rhs()).to(dev)
    tb = torch.from_numpy(synth.gaussian_spinors(p.dims, p.bc, 4, synth.PTC_TRAIN_SEED)).to(dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    r, e = lat.precond_pairs(tb, every=5, n_snap=4)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t
    lat.precond_init(seed=1)
    t = time.perf_counter()
    hist = lat.precond_train(r, e, steps=300, lr=3e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t
    res = {"workload": p.name, "tol": 1e-10, "pairs": int(r.shape[0]), "train_steps": 300,
           "pairs_s": round(t_pairs, 3), "train_s": round(t_train, 3),
           "loss_first": float(hist[0]), "loss_last": float(hist[-1])}
    xs = {}
    for name, kw in (("cg_fp64", dict(prec="fp64")), ("cg_fp32", dict(prec="fp32")),
                     ("fgmres_identity", dict(prec="fp64", precond="identity")),
                     ("fgmres_ptc", dict(prec="fp64", precond="ptc")),
                     ("fgmres_identity_fp32", dict(prec="fp32", precond="identity")),
                     ("fgmres_ptc_fp32", dict(prec="fp32", precond="ptc"))):
        pr = mfq.make_params(tol=1e-10, max_iter=50000, **kw)
        ms, (x, st, rc) = _timed(lambda: lat.solve(b, params=pr), reps=2)
        xs[name] = x.cpu().numpy()
        res[name] = {"ms": round(ms, 3), "rc": rc, "iters": [s["iters"] for s in st],
                     "true_rel_resid_max": max(s["true_rel_resid"] for s in st)}
    ref = xs["cg_fp64"]
    for name in ("cg_fp32", "fgmres_identity", "fgmres_ptc", "fgmres_identity_fp32", "fgmres_ptc_fp32"):
        res[name]["rel_err_vs_cg"] = float(np.linalg.norm(xs[name] - ref) / np.linalg.norm(ref))
    keep["learned_16x16x16x16"] = (p, {k: v[:1] for k, v in xs.items()})
    res["ptc_iteration_gain_vs_fgmres"] = round(sum(res["fgmres_identity"]["iters"]) /
                                                max(1, sum(res["fgmres_ptc"]["iters"])), 3)
    # time ratios against plain FP64 CG (> 1: slower than CG)
    res["ptc_ms_over_cg_ms"] = round(res["fgmres_ptc"]["ms"] / res["cg_fp64"]["ms"], 3)
    res["identity_ms_over_cg_ms"] = round(res["fgmres_identity"]["ms"] / res["cg_fp64"]["ms"], 3)
    # the FGMRES cycle in FP32 (basis, operator, network input and output; FP64 restarts)
    res["ptc_fp32_ms_over_cg_ms"] = round(res["fgmres_ptc_fp32"]["ms"] / res["cg_fp64"]["ms"], 3)
    res["ptc_fp32_ms_over_cg_fp32_ms"] = round(res["fgmres_ptc_fp32"]["ms"] / res["cg_fp32"]["ms"], 3)
    lat.close()
    return res


def bench_routes(synth, mfq, torch, dev, np):
    """Route F (one CG on D^+D over every site, then X = D^+ Y) against route S
    (D X = Phi and D^+ Y = X, each by CG on the even/odd Schur complement) for
    the blocked force on the 8^3x8 and 16^3x16 workloads, FP64, FP32 and FP16
    storage inner, to 1e-10; and the even/odd action variant (one CG on D^+D^
    over the even sites).  Forces are compared with the route F force of the same
    precision (the two routes compute the same definition)."""
    res = {}
    for p in (synth.CONFIG_1, synth.CONFIG_2):
        print(f"[bench] row routes {p.name}", file=sys.stderr, flush=True)
        lat = mfq.Lattice(p.dims, p.bc, p.kappa, torch.from_numpy(p.links()).to(dev))
        phi = torch.from_numpy(p.rhs()).to(dev)
        row = {"workload": p.name, "tol": 1e-10}
        for prec in ("fp64", "fp32", "fp16"):
            gs = {}
            for route in ("full", "schur"):
                pr = mfq.make_params(tol=1e-10, prec=prec, max_iter=50000, route=route)
                ms, (g, act, st, rc) = _timed(lambda: lat.force(phi, params=pr), reps=3)
                gs[route] = g.cpu().numpy()
                row[f"{route}_{prec}"] = {"force_ms": round(ms, 3), "rc": rc, "iters": [s["iters"] for s in st]}
            row[f"schur_{prec}"]["force_rel_diff_vs_full"] = rel_err(gs["schur"], gs["full"], np)
            row[f"schur_{prec}"]["speedup_vs_full"] = round(row[f"full_{prec}"]["force_ms"]
                                                            / row[f"schur_{prec}"]["force_ms"], 3)
            pr = mfq.make_params(tol=1e-10, prec=prec, max_iter=50000)
            ms, (g, act, st, rc) = _timed(lambda: lat.force(phi, params=pr, eo_action=True), reps=3)
            row[f"eo_action_{prec}"] = {"force_ms": round(ms, 3), "rc": rc, "iters": [s["iters"] for s in st],
                                        "note": "the even/odd action variant: a different action, one CG"}
        lat.close()
        res[p.name] = row
    return res


def bench_paper_solvers(synth, mfq, torch, dev, np):
    """The paper's solver family (Sec. 3.1-3.2) on the paper's lattice shape
    (16^3x16 SF, 5 pseudo-fermions; synthetic links eps = 0.5, kappa = 0.135):
    Alg. 2's two solves (D X = Phi, D^+ Y = X) with BiCGStab per RHS, Global
    BiCGStab and Block BiCGStab in FP64 (the paper's cases A, B, C) and with
    the FP32 inner BiCGStab as preconditioner (case D1 and its block form), to
    1e-10 on the even system; against CG on D^+D (route F).  Iterations are
    outer iterations per solve (each applies D^ twice, or the inner solve twice)."""
    p = synth.CONFIG_2
    print(f"[bench] row paper solvers {p.name}", file=sys.stderr, flush=True)
    u = p.links()
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, torch.from_numpy(u).to(dev))
    phi = torch.from_numpy(p.rhs()).to(dev)
    res = {"workload": p.name, "tol": 1e-10}
    ref = None
    for name, kw in (("cg_fp64_route_f", dict(prec="fp64")),
                     ("A_bicgstab_fp64", dict(prec="fp64", precond="bicgstab")),
                     ("B_gl_bicgstab_fp64", dict(prec="fp64", precond="gl_bicgstab")),
                     ("C_bl_bicgstab_fp64", dict(prec="fp64", precond="bl_bicgstab")),
                     ("D1_gl_bicgstab_fp64_fp32_inner", dict(prec="fp32", precond="gl_bicgstab")),
                     ("bl_bicgstab_fp64_fp32_inner", dict(prec="fp32", precond="bl_bicgstab")),
                     ("bicgstab_fp64_fp32_inner", dict(prec="fp32", precond="bicgstab"))):
        pr = mfq.make_params(tol=1e-10, max_iter=20000, **kw)
        ms, (g, act, st, rc, x, y) = _timed(lambda: lat.force(phi, params=pr, want_xy=True), reps=2)
        gh = g.cpu().numpy()
        if ref is None:
            ref = gh
        res[name] = {"force_ms": round(ms, 3), "rc": rc, "iters": [s["iters"] for s in st],
                     "inner_iters": st[0]["inner_iters"], "inner_calls": st[0]["inner_calls"],
                     "force_rel_diff_vs_cg": rel_err(gh, ref, np)}
    a_it = max(res["A_bicgstab_fp64"]["iters"])
    res["block_iterations_vs_per_rhs"] = {
        "gl": round(max(res["B_gl_bicgstab_fp64"]["iters"]) / a_it, 3),
        "bl": round(max(res["C_bl_bicgstab_fp64"]["iters"]) / a_it, 3),
        "paper_bl_vs_per_rhs": 0.82, "note": "the paper's Bl-BiCGStab took 18% fewer iterations than the "
                                             "sequential BiCGStab on its thermalized 16^4 configuration"}
    lat.close()
    return res


def bench_hmc(synth, mfq, torch, dev, np):
    """One leapfrog HMC trajectory on the GPU (tau = 0.5, 10 steps, 11 force
    evaluations) on the 8^3x8 SF 5-pseudo-fermion workload, forces by route F
    (FP64 or FP32 inner solves) or route S (FP64): time per trajectory, Delta H
    (FP64) and the decision with the draw u = 0.5.  The pseudo-fermion action
    only (no gauge action)."""
    p = synth.CONFIG_1
    print(f"[bench] row hmc {p.name}", file=sys.stderr, flush=True)
    u = p.links()
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, torch.from_numpy(u).to(dev))
    phi = torch.from_numpy(p.rhs()).to(dev)
    # momenta on every link: the library moves only the links that enter D
    pm = synth.gaussian_momentum_matrices(p.dims, p.bc, 4001)
    out = {"workload": p.name, "tau": 0.5, "n_steps": 10}
    # route F (tol 1e-10) in FP64 and FP32, and route S in FP64 at the bench
    # step's tolerance (its force as accurate as route F's)
    for key, prec, route in (("fp64", "fp64", "full"), ("fp32", "fp32", "full"), ("schur_fp64", "fp64", "schur")):
        links = torch.from_numpy(u).to(dev)
        mom = torch.from_numpy(pm).to(dev)
        lat.update_links(links)
        t = time.perf_counter()
        r, rc = lat.hmc_trajectory(links, mom, phi, 0.5, 10, 0.5, tol=STEP_TOL[route], prec=prec, route=route)
        torch.cuda.synchronize()
        out[key] = {"ms": round((time.perf_counter() - t) * 1e3, 2), "rc": rc, "delta_h": r["delta_h"],
                    "accepted": r["accepted"], "solver_iters": r["solver_iters"], "force_evals": r["force_evals"]}
    lat.close()
    return out


def bench_batch(synth, mfq, torch, dev, np):
    """The 64-lattice uneven batch (8^4, 12^4, 16^3x32 SF; 1-8 RHS each;
    kappa in [0.12, 0.135]) in one persistent launch per CG phase, FP32 inner
    with FP64 reliable updates to 1e-10, against solving the lattices one by one."""
    probs = synth.batch_problems()
    print(f"[bench] row batch: generating {len(probs)} lattices", file=sys.stderr, flush=True)
    t = time.perf_counter()
    lats, bs = [], []
    for q in probs:
        lats.append(mfq.Lattice(q.dims, q.bc, q.kappa, torch.from_numpy(q.links()).to(dev)))
        bs.append(torch.from_numpy(q.rhs()).to(dev))
    gen_s = time.perf_counter() - t
    batch = mfq.Batch(lats, [q.n_rhs for q in probs], prec="fp32")
    pr = mfq.make_params(tol=1e-10, prec="fp32", max_iter=20000)
    ms, (xs, stats, rc) = _timed(lambda: batch.solve(bs, params=pr), reps=2)
    print(f"[bench] batch solve {ms:.1f} ms rc={rc}", file=sys.stderr, flush=True)
    # Same protocol as the batch: one untimed pass (each handle tunes its
    # launch shape once), then the mean of two timed passes.
    t_one, _ = _timed(lambda: [lat.solve(b, params=pr) for lat, b in zip(lats, bs)], reps=2)
    n_rhs = sum(q.n_rhs for q in probs)
    site_rhs = sum(q.n_rhs * q.dims[0] * q.dims[1] * q.dims[2] * (q.dims[3] - 1) for q in probs)
    iters = [s["iters"] for st in stats for s in st]
    res = {"lattices": len(probs), "rhs": n_rhs, "grid": batch.grid, "ms": round(ms, 2), "rc": rc,
           "one_by_one_ms": round(t_one, 2), "speedup_vs_one_by_one": round(t_one / ms, 3),
           "iters_mean": float(np.mean(iters)), "iters_max": int(max(iters)),
           "true_rel_resid_max": max(s["true_rel_resid"] for st in stats for s in st),
           "site_rhs_iterations_per_s": round(sum(q.dims[0] * q.dims[1] * q.dims[2] * (q.dims[3] - 1)
                                                  * s["iters"] for q, st in zip(probs, stats) for s in st)
                                              / (ms * 1e-3), 1),
           "site_rhs": site_rhs, "input_generation_s": round(gen_s, 2)}
    batch.close()
    for lat in lats:
        lat.close()
    return res


def bandwidth_links(dims, synth, np, bc="periodic"):
    """Links of a bandwidth lattice: random SU(3) links on a 16^3 x 8 block,
    tiled over the lattice (the values do not matter for bandwidth and
    numpy's 3x3 eigh is slow); an SF lattice gets one more time slice (its
    T + 1 stored slices), the boundary slices holding tiled random links too
    (they never enter D)."""
    blk = (min(16, dims[0]), min(16, dims[1]), min(16, dims[2]), min(8, dims[3]))
    ub = synth.random_links(blk, "periodic", 0.3, 7)
    reps = (1, dims[3] // blk[3], dims[2] // blk[2], dims[1] // blk[1], dims[0] // blk[0], 1, 1)
    u = np.tile(ub, reps)
    if bc == "sf":
        u = np.concatenate([u, u[:, :1]], axis=1)
    return np.ascontiguousarray(u)


BANDWIDTH_KAPPA = 0.12


def bandwidth_lattice(dims, synth, mfq, torch, dev, np, bc="periodic"):
    """A bandwidth lattice as a library handle."""
    ub = bandwidth_links(dims, synth, np, bc)
    return mfq.Lattice(dims, bc, BANDWIDTH_KAPPA, torch.from_numpy(ub).to(dev))


def profile_kernels(args, synth, mfq, torch, dev, np):
    """Counter run: the hopping kernel of the inner CG on the bench lattice
    (its tuned launch shape, 50 timed launches after the tuner's), a plain
    1 GiB device copy, whose FETCH_SIZE / WRITE_SIZE calibrate the counters
    against known bytes, and with --profile-big the same kernel on the
    bandwidth lattice for 1 and 5 RHS."""
    p = synth.CONFIG_1
    out = {"profile_kernels": True}
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, torch.from_numpy(p.links()).to(dev))
    out["hop_ms"] = lat.time_hop(args.prec, p.n_rhs, iters=50)
    out["shape"] = lat.hop_shape(args.prec, p.n_rhs)
    lat.close()
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    out["copy_bytes"] = src.numel() * 8
    del src, dst
    if args.profile_big or args.order_ab:
        dims = tuple(int(v) for v in args.bw_dims.split(","))
        big = bandwidth_lattice(dims, synth, mfq, torch, dev, np)
        if args.profile_big:
            for nr in (1, 5):
                out[f"big_n{nr}_ms"] = big.time_hop(args.prec, nr, iters=20)
                out[f"big_n{nr}_shape"] = big.hop_shape(args.prec, nr)
        if args.order_ab:
            # the same kernel and grid twice: half-index order, then z-blocked order
            # (each XCD walks (z, t) planes, t before the next block of z values);
            # counter summaries tell the two apart by dispatch order
            pb = {"fp64": 8, "fp32": 4, "fp16": 2}[args.prec]
            key = "gfx950 %d %d %d %d 1 1 %d" % (dims + (pb,))
            with tempfile.TemporaryDirectory() as td:
                cache = os.path.join(td, "tune.txt")
                old = os.environ.get("MFQ_AUTOTUNE_CACHE")
                os.environ["MFQ_AUTOTUNE_CACHE"] = cache
                try:
                    for name, shape in (("linear", (64, 1, 1, 0, 4)), ("zblocked", (64, 1, 3, 0, 4))):
                        with open(cache, "w") as f:
                            f.write(key + "|%d %d %d %d %d\n" % shape)
                        big.set_autotune(True)
                        out[f"order_{name}_ms"] = big.time_hop(args.prec, 1, iters=20)
                        out[f"order_{name}_shape"] = big.hop_shape(args.prec, 1)
                finally:
                    if old is None:
                        del os.environ["MFQ_AUTOTUNE_CACHE"]
                    else:
                        os.environ["MFQ_AUTOTUNE_CACHE"] = old
        big.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
