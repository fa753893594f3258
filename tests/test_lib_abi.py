"""The C-ABI library loads and exports every entry point its header declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfq.h")
LIB = os.path.join(ROOT, "paper_1009_5169_amd", "libmfq.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfq_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mfq_dslash", "mfq_solve_multi_rhs", "mfq_fermion_force", "mfq_create",
                     "mfq_destroy", "mfq_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmfq.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_signatures_cover_header():
    from paper_1009_5169_amd import _lib
    assert set(declared_functions()) <= set(_lib.exported_symbols())


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1009_5169_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _lib.lib()


def test_batch_workload_recipe():
    """The uneven batch: 64 SF lattices drawn from {8^4, 12^4, 16^3x32}, 1..8
    RHS each, kappa in [0.12, 0.135]."""
    import synth
    probs = synth.batch_problems()
    assert len(probs) == 64
    assert {p.dims for p in probs} <= {(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32)}
    assert len({p.dims for p in probs}) == 3
    assert all(1 <= p.n_rhs <= 8 and 0.12 <= p.kappa <= 0.135 and p.bc == "sf" for p in probs)
    assert len({p.link_seed for p in probs}) == 64


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmfq.so not built")
@pytest.mark.parametrize("dims,bc,kappa,why", [
    ((4, 4, 4, 5), 0, 0.125, "even"),
    ((4, 4, 4, 2), 0, 0.125, "T >= 4"),
    ((4, 4, 4, 4), 0, 0.25, "kappa"),
    ((4, 4, 4, 4), 7, 0.125, "boundary"),
    ((128, 128, 128, 24), 1, 0.125, "volume too large"),
    ((2, 2, 4096, 2560), 1, 0.125, "2^31"),
    ((4, 4, 4, 4), 0, 0.125, "links_dev is NULL"),
])
def test_create_rejects_bad_lattices_on_the_host(dims, bc, kappa, why):
    """mfq_create checks the lattice before it touches the device: odd or too
    small extents, kappa outside (0, 0.25), an unknown boundary, more than
    4.4e7 sites (one FP64 field of a (RHS, parity) must stay under 4 GiB for
    its buffer resource), and (volume / 2) * max(Lx / 2, Ly, Lz) >= 2^31 (the
    division-free site coordinates are exact below it); the last case is a
    valid lattice whose link pointer is NULL.  All return MFQ_ERR_ARG with a
    message, and no handle."""
    class Lattice(ctypes.Structure):  # mfq_lattice
        _fields_ = [("dims", ctypes.c_int * 4), ("bc", ctypes.c_int), ("kappa", ctypes.c_double)]

    lib = ctypes.CDLL(LIB)
    lib.mfq_create.restype = ctypes.c_int
    lib.mfq_create.argtypes = [ctypes.POINTER(Lattice), ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_void_p)]
    lib.mfq_last_error.restype = ctypes.c_char_p
    lat = Lattice()
    for d in range(4):
        lat.dims[d] = dims[d]
    lat.bc = bc
    lat.kappa = kappa
    out = ctypes.c_void_p(12345)
    rc = lib.mfq_create(ctypes.byref(lat), None, None, ctypes.byref(out))
    assert rc == -1
    assert not out.value
    assert why in lib.mfq_last_error().decode()
