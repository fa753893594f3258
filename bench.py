"""Benchmark of the blocked multi-RHS quark solve on one MI355X.

A step is one blocked force evaluation (the paper's Alg. 2) for the 8^3x8
Schroedinger-functional lattice with 5 pseudo-fermions (kappa = 0.13,
links exp(i 0.3 H)): pack, one batched CG on D^+D to a 1e-10 true relative
residual per RHS (FP32 inner iteration with FP64 reliable updates), the g5 map
to X and Y, the summed force and the action.  All inputs are synthetic and
resident in device memory before the timed region.

Prints one JSON line.  Extra keys: the same solve in plain FP64 CG on the same
GPU, the FP16 path, the error of each against the FP64 path, and the fused
half-dslash bandwidth on a lattice far larger than the 256 MB Infinity Cache.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "5-RHS D†D solve time to 1e-10 vs plain FP64 CG; dslash HBM GB/s, % peak"
HBM_PEAK_GBS = 8000.0


def hop_bytes_per_site_rhs(prec: str, n_rhs: int) -> float:
    """Algorithmic HBM bytes of the fused half-dslash D-epilogue kernel per
    output site per RHS: the other-parity input read once, the same-parity
    input read once, the output written once, and the 8 links of the site
    (each link is read once per launch) shared by the n_rhs RHS."""
    if prec == "fp64":
        spinor, link = 24 * 8, 18 * 8
    elif prec == "fp32":
        spinor, link = 24 * 4, 18 * 4
    else:  # fp16 values + one fp32 norm per site
        spinor, link = 24 * 2 + 4, 18 * 2
    return 3 * spinor + 8 * link / n_rhs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="fp32", choices=["fp64", "fp32", "fp16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bandwidth", action="store_true")
    ap.add_argument("--bw-dims", default="32,32,32,64")
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
    u = p.links()
    phi_h = p.rhs()
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, torch.from_numpy(u).to(dev))
    phi = torch.from_numpy(phi_h).to(dev)
    params = mfq.make_params(tol=1e-10, prec=args.prec, max_iter=20000)
    torch.cuda.synchronize()
    print(f"[bench] workload {p.name} prec={args.prec}", file=sys.stderr, flush=True)

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

    # dominant kernel: the fused half-dslash (D epilogue) of the inner CG, same
    # launch shape as in the solve, timed with HIP events on its stream
    n = p.n_rhs
    hop_ms = lat.time_hop(args.prec, n, iters=200)
    vh = p.dims[0] * p.dims[1] * p.dims[2] * (p.dims[3] - 1) // 2
    per_launch = hop_bytes_per_site_rhs(args.prec, n) * vh * n
    achieved = per_launch / (hop_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "kernel": f"hop_kernel<EPI_D,{args.prec}>", "launch_us": round(hop_ms * 1e3, 3),
                "algorithmic_bytes_per_launch": int(per_launch)}

    # solve-only times on the same GPU: this precision and plain FP64 CG
    def solve_ms(prec, reps=5):
        pr = mfq.make_params(tol=1e-10, prec=prec, max_iter=20000)
        lat.solve(phi, params=pr)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            x, st, _ = lat.solve(phi, params=pr)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / reps, x, st

    s_ms, x_this, st_this = solve_ms(args.prec)
    s64_ms, x64, st64 = solve_ms("fp64")
    s16_ms, x16, st16 = solve_ms("fp16")
    x64h = x64.cpu().numpy()
    err = lambda a: float(np.linalg.norm(a.cpu().numpy() - x64h) / np.linalg.norm(x64h))

    out = {
        "metric": METRIC, "value": round(ms_per_step, 4), "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16"}[args.prec], "data": "synthetic",
        "config": {"workload": p.name, "dims": list(p.dims), "bc": p.bc, "kappa": p.kappa,
                   "link_eps": p.eps, "n_rhs": n, "tol": 1e-10,
                   "step": "blocked force: batched CG on DdagD + g5 map + force + action",
                   "inner_precision": args.prec},
        "roofline": roofline,
        "solve_ms": {args.prec: round(s_ms, 4), "fp64": round(s64_ms, 4), "fp16": round(s16_ms, 4)},
        "solve_speedup_vs_fp64_cg": round(s64_ms / s_ms, 3),
        "iters": {args.prec: [s["iters"] for s in st_this], "fp64": [s["iters"] for s in st64],
                  "fp16": [s["iters"] for s in st16]},
        "solution_rel_err_vs_fp64_path": {args.prec: err(x_this), "fp16": err(x16)},
        "true_rel_resid_max": max(s["true_rel_resid"] for s in st_this),
    }

    if not args.no_bandwidth:
        dims = tuple(int(v) for v in args.bw_dims.split(","))
        print(f"[bench] bandwidth lattice {dims}", file=sys.stderr, flush=True)
        # random SU(3) links on a 16^3 x 8 block, tiled over the lattice: the
        # values do not matter for bandwidth and numpy's 3x3 eigh is slow
        blk = (min(16, dims[0]), min(16, dims[1]), min(16, dims[2]), min(8, dims[3]))
        ub = synth.random_links(blk, "periodic", 0.3, 7)
        reps = (1, dims[3] // blk[3], dims[2] // blk[2], dims[1] // blk[1], dims[0] // blk[0], 1, 1)
        ub = np.ascontiguousarray(np.tile(ub, reps))
        big = mfq.Lattice(dims, "periodic", 0.12, torch.from_numpy(ub).to(dev))
        del ub
        bw = {}
        vhb = dims[0] * dims[1] * dims[2] * dims[3] // 2
        for prec in ("fp64", "fp32", "fp16"):
            for nr in (1, 5):
                ms = big.time_hop(prec, nr, iters=20)
                gbs = hop_bytes_per_site_rhs(prec, nr) * vhb * nr / (ms * 1e-3) / 1e9
                bw[f"{prec}_n{nr}"] = {"us": round(ms * 1e3, 2), "GB/s": round(gbs, 1),
                                       "frac": round(gbs / HBM_PEAK_GBS, 4)}
                print(f"[bench] bw {prec} n={nr}: {gbs:.1f} GB/s", file=sys.stderr, flush=True)
        out["dslash_bandwidth"] = {"dims": list(dims), "bc": "periodic",
                                   "kernel": "hop_kernel<EPI_D>", "runs": bw}
        big.close()
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        from oracle import force as fmod
        from oracle import native

        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        d = native.NativeWilson(p.dims, p.bc, p.kappa, u)
        print(f"[bench] cpu oracle: one full step, {threads} threads", file=sys.stderr, flush=True)
        t = time.perf_counter()
        from oracle import solvers
        x, _ = solvers.solve_D(d, phi_h, 1e-10)
        y, _ = solvers.solve_Ddag(d, x, 1e-10)
        from oracle.dirac import WilsonDirac
        fmod.force_coefficients(WilsonDirac(p.dims, p.bc, p.kappa, u), x, y)
        cpu_ms = (time.perf_counter() - t) * 1e3
        out["cpu_baseline"] = {"value": round(cpu_ms, 2), "unit": "ms", "cores": threads, "kind": "oracle",
                               "sample": "one full step of the same workload: Alg. 2 with two per-RHS "
                                         "FP64 CG solves (normal equations, tol 1e-10) and the force"}
    lat.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
