"""Regenerate the shipped table of tuned launch shapes (tune_gfx950.txt).

Run on the target GPU:  python -m paper_1009_5169_amd.tune_table OUT
It runs the library's autotuner (MFQ_AUTOTUNE_CACHE=OUT) for the lattice
shapes, RHS counts and precisions of the benchmark workloads; the timing of a
launch shape does not depend on the field values, so unit links are used.
Copy OUT next to libmfq.so as tune_gfx950.txt to ship it.
"""
from __future__ import annotations

import os
import sys


def workloads():
    import synth
    out = []
    for p in (synth.CONFIG_0, synth.CONFIG_1, synth.CONFIG_2, synth.CONFIG_4):
        for prec in ("fp64", "fp32", "fp16"):
            out.append((p.dims, p.bc, p.n_rhs, prec))
    for dims in ((8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32)):
        for n in range(1, 9):
            out.append((dims, "sf", n, "fp32"))
    for n in (1, 5, 8):
        for prec in ("fp64", "fp32", "fp16"):
            out.append(((32, 32, 32, 64), "periodic", n, prec))
    for n in (1, 5):
        out.append(((48, 48, 48, 48), "periodic", n, "fp32"))
    out.append(((32, 32, 32, 64), "sf", 5, "fp32"))
    return out


def main(path: str) -> None:
    os.environ["MFQ_AUTOTUNE_CACHE"] = os.path.abspath(path)
    import torch
    import synth
    import paper_1009_5169_amd as mfq
    seen = set()
    for dims, bc, n, prec in workloads():
        if (dims, bc, n, prec) in seen:
            continue
        seen.add((dims, bc, n, prec))
        lat = mfq.Lattice(dims, bc, 0.12, torch.from_numpy(synth.unit_links(dims, bc)).to("cuda:0"))
        lat.time_hop(prec, n, iters=1)
        print(dims, bc, n, prec, lat.hop_shape(prec, n), flush=True)
        lat.close()
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "tune_gfx950.txt")
