"""Host-side checks of the benchmark's contract and bookkeeping (no GPU)."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("prec,n,want", [("fp64", 5, 499.2), ("fp32", 5, 230.4), ("fp16", 5, 123.2),
                                         ("fp32", 1, 384.0), ("fp64", 1, 960.0)])
def test_algorithmic_bytes_per_site_and_rhs(prec, n, want):
    """Input and output spinor once, 4 links per site shared by the RHS:
    2 * 24 w + 4 L w / n (FP16 spinors carry one FP32 norm)."""
    assert bench.hop_bytes_per_site_rhs(prec, n) == pytest.approx(want)


def _counters(path, sha, prec="fp32", n=5, fetch=3297.5, write=1688.8):
    with open(path, "w") as f:
        f.write("# test counters\n")
        f.write(f"source_sha256: {sha}\nprec: {prec}\nn_rhs: {n}\nlaunch_shape: 64 1 0 0 2\n")
        f.write(f"grid_threads: 35840\nfetch_kib_per_dispatch: {fetch}\nwrite_kib_per_dispatch: {write}\n")
        f.write("copy_bytes: 1073741824\ncopy_fetch_kib: 524299.5\ncopy_write_kib: 1048576.0\n")


def test_counter_traffic_needs_the_current_kernel_sources(tmp_path, monkeypatch):
    path = tmp_path / "counters.txt"
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(path))
    _counters(path, "0" * 64)
    assert bench.measured_traffic("fp32", 5) is None          # other sources
    _counters(path, bench.kernel_source_hash())
    got = bench.measured_traffic("fp32", 5)
    # FETCH_SIZE read half of a known copy, WRITE_SIZE all of it: scaled by 2 and 1
    copy_kib = 1073741824 / 1024.0
    want = (3297.5 * copy_kib / 524299.5 + 1688.8 * copy_kib / 1048576.0) * 1024
    assert got == int(round(want))
    assert bench.measured_traffic("fp32", 5, (64, 1, 0, 0, 2)) == got
    assert bench.measured_traffic("fp32", 5, (64, 5, 0, 0, 0)) is None  # another launch shape
    assert bench.measured_traffic("fp64", 5) is None          # another precision
    assert bench.measured_traffic("fp32", 1) is None          # another RHS count
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("fp32", 5) is None


def test_solver_names_match_the_header():
    from paper_1009_5169_amd import _lib
    header = open(os.path.join(ROOT, "include", "mfq.h")).read()
    enum = dict((k, int(v)) for k, v in re.findall(r"MFQ_PC_(\w+)\s*=\s*(\d+)", header))
    assert enum == {"NONE": 0, "PTC": 1, "IDENTITY": 2, "BLOCKCG": 3, "BICGSTAB": 4, "GL_BICGSTAB": 5,
                    "BL_BICGSTAB": 6}
    assert {k.upper(): v for k, v in _lib.PRECOND.items()} == enum
