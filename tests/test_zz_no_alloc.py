"""The operator entry point that allocates nothing (mfq_dslash_noalloc),
through the C ABI, against mfq_dslash on the same inputs: every operator, two
calls in a row on one lattice (the second with fewer RHS, so stale workspace
contents from the first would show), a smaller second lattice, and the size
limit of its fixed workspace."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1009_5169_amd as mfq  # noqa: E402

DEV = "cuda:0"
OPS = ("hop_eo", "hop_oe", "D", "Ddag", "DdagD", "hop", "hop_dag", "schur", "schur_dag", "schur_normal")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def lattice(dims, bc, kappa, seed):
    u = synth.random_links(dims, bc, 0.3, seed)
    return mfq.Lattice(dims, bc, kappa, torch.from_numpy(u).to(DEV))


def check_all_ops(lat, psi):
    x = torch.from_numpy(psi).to(DEV)
    for op in OPS:
        want = lat.dslash(op, x)
        # a poisoned output buffer: every element must be overwritten
        got = torch.full_like(x, complex(np.nan, np.nan))
        lat.dslash_noalloc(op, x, out=got)
        torch.cuda.synchronize()
        g, w = got.cpu().numpy(), want.cpu().numpy()
        assert np.all(np.isfinite(g)), op
        err = rel(g, w)
        assert err < 1e-14, (op, err)


def test_noalloc_matches_dslash_twice_then_smaller():
    p = synth.CONFIG_1
    lat = lattice(p.dims, p.bc, p.kappa, 1000)
    note(f"noalloc: {p.dims} {p.bc} 5 RHS")
    check_all_ops(lat, synth.gaussian_spinors(p.dims, p.bc, 5, 2000))
    note("noalloc: same lattice, 2 RHS")
    check_all_ops(lat, synth.gaussian_spinors(p.dims, p.bc, 2, 2001))
    small = lattice((4, 2, 2, 6), "antiperiodic", 0.12, 1001)
    note("noalloc: 4x2x2x6 antiperiodic, 1 RHS")
    check_all_ops(small, synth.gaussian_spinors((4, 2, 2, 6), "antiperiodic", 1, 2002))
    small.close()
    lat.close()


def test_noalloc_rejects_inputs_beyond_its_workspace():
    dims, bc = (16, 16, 16, 16), "sf"
    lat = lattice(dims, bc, 0.13, 1002)
    psi = torch.from_numpy(synth.gaussian_spinors(dims, bc, 5, 2003)).to(DEV)
    out = torch.zeros_like(psi)
    with pytest.raises(mfq.MfqError) as e:
        lat.dslash_noalloc("D", psi, out=out)
    assert e.value.code == -1 and "64 MiB" in str(e.value)
    torch.cuda.synchronize()
    assert not torch.any(out != 0)
    # one RHS fits (two packed fields of 11.8 MB)
    got = lat.dslash_noalloc("D", psi[:1].contiguous())
    want = lat.dslash("D", psi[:1].contiguous())
    torch.cuda.synchronize()
    assert rel(got.cpu().numpy(), want.cpu().numpy()) < 1e-14
    lat.close()
