"""Host logic of bench.py, without a GPU: the refusal of several GPUs, the
algorithmic byte counts behind every roofline figure (the formulas of the
kernel table, per launch), and the rule that HBM counters are reported only
for the kernel source they were measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


class StubHierarchy:
    """Level sizes and index widths of a made-up three-level hierarchy."""

    nlev = 3
    sizes = [dict(n=1000, nnz=7000, nnz_hat=7000, nnz_P=1800, n_coarse=500, gamma=0.0, bytes=0),
             dict(n=500, nnz=9000, nnz_hat=9000, nnz_P=700, n_coarse=100, gamma=0.0, bytes=0),
             dict(n=100, nnz=3000, nnz_hat=2200, nnz_P=0, n_coarse=0, gamma=0.1, bytes=0)]

    def __init__(self, widths):
        self.widths = widths

    def level_info(self, l):
        return self.sizes[l]

    def index_width(self, l, which):
        return self.widths.get((l, which), 4)


def test_more_than_one_gpu_is_refused_before_touching_a_device():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_workloads_listed():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 0
    for w in ("poisson3d", "aniso2d", "fv3d", "serve", "setup", "lumping", "methods"):
        assert w in r.stdout


@pytest.mark.parametrize("idx", [4, 2])
def test_launch_bytes_follow_the_kernel_table(idx):
    """Algorithmic bytes: FP64 values and int32 indices whatever index width
    the kernel reads."""
    h = StubHierarchy({(0, "A"): idx, (0, "AHAT"): idx, (0, "R"): idx, (0, "P"): idx, (1, "AHAT"): idx})
    e = 12
    # Jacobi: entries, row pointers, x gathered, b, dinv read, x' written
    assert bench.launch_bytes(h, "JACOBI", 0) == e * 7000 + 4 * 1001 + 32 * 1000
    # zero-guess residual: the prescaled sweep gathered, b read, r written
    assert bench.launch_bytes(h, "JACOBI_ZERO", 1) == e * 9000 + 4 * 501 + 24 * 500
    # residual of level 0 reads the Galerkin operator
    assert bench.launch_bytes(h, "RESIDUAL", 0) == e * 7000 + 4 * 1001 + 24 * 1000
    assert bench.launch_bytes(h, "SPMV_DOT", 0) == e * 7000 + 4 * 1001 + 16 * 1000
    # restriction below the coarsest level also writes omega D^-1 b_c (16 n_c more)
    assert bench.launch_bytes(h, "RESTRICT", 0) == e * 1800 + 4 * 501 + 8 * 1000 + 8 * 500 + 16 * 500
    assert bench.launch_bytes(h, "INTERP", 0) == e * 1800 + 4 * 1001 + 8 * 500 + 16 * 1000
    assert bench.launch_bytes(h, "COARSE", 0) == 0


def test_lump_share_bytes():
    h = StubHierarchy({})
    # level 2: n = 100, nnz = 3000, 2200 kept
    assert bench.lump_shares_bytes(h, 2) == 8 * 101 + 13 * 3000 + 8 * 800 + 8 * 100 + 20 * 2200


def test_traffic_reported_only_for_the_measured_source(tmp_path):
    src = tmp_path / "kernels.hip"
    src.write_text("// kernel source\n")
    sha = bench.kernel_source_sha(str(src))
    counters = tmp_path / "counters.json"
    counters.write_text(json.dumps({"kernel_source_sha": sha, "kernels": {
        "JACOBI@1": {"hbm_bytes_per_launch": 123456}, "N192:JACOBI@1": {"hbm_bytes_per_launch": 654321}}}))
    assert bench.traffic_for("JACOBI", 1, str(counters), str(src)) == 123456
    assert bench.traffic_for("JACOBI", 1, str(counters), str(src), N=192) == 654321
    assert bench.traffic_for("JACOBI", 1, str(counters), str(src), N=128) is None
    assert bench.traffic_for("JACOBI", 0, str(counters), str(src)) is None
    src.write_text("// kernel source, changed\n")
    assert bench.traffic_for("JACOBI", 1, str(counters), str(src)) is None
    assert bench.traffic_for("JACOBI", 1, str(tmp_path / "missing.json"), str(src)) is None


def test_crossing_margin_and_host_description():
    import math
    # relative residuals 0.1, 1e-5, 2e-9 against tol 1e-8: the closest is the last
    assert abs(bench.crossing_margin([1.0, 0.1, 1e-5, 2e-9], 1e-8) - abs(math.log(0.2))) < 1e-12
    assert bench.crossing_margin([1.0], 1e-8) == float("inf")
    d = bench.host_description()
    assert d["nproc"] >= 1 and d["affinity_cpus"] >= 1
    assert bench.omp_threads() >= 1


def test_fp32_cycle_launch_bytes():
    h = StubHierarchy({(1, "AHAT"): 2, (0, "R"): 2, (0, "P"): 2})
    # 4-byte values and vectors, int32 indices even where the level keeps 2-byte ones
    assert bench.launch_bytes32(h, "JACOBI", 1) == 8 * 9000 + 4 * 501 + 16 * 500
    assert bench.launch_bytes32(h, "JACOBI_ZERO", 1) == 8 * 9000 + 4 * 501 + 12 * 500
    assert bench.launch_bytes32(h, "RESTRICT", 0) == 8 * 1800 + 4 * 501 + 4 * 1000 + 4 * 500 + 8 * 500
    assert bench.launch_bytes32(h, "INTERP", 0) == 8 * 1800 + 4 * 1001 + 4 * 500 + 8 * 1000
