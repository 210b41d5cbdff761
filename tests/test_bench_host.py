"""Host-side pieces of bench.py (no GPU): the algorithmic work counts it divides
by, the gating of the measured HBM-traffic table, and the single-GPU guard."""
import hashlib
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_sigma2b_counts(bench):
    # per slice pair: 2 n^4 for the products M^(i), 8 n^3 for the epilogues and
    # the direct term; a self-paired middle slice 2 n^4 + 5 n^3
    n = 199
    assert bench.sigma2b_flops(n, 1025) == 512 * (2 * n**4 + 8 * n**3) + (2 * n**4 + 5 * n**3)
    assert bench.sigma2b_flops(n, 1024) == 512 * (2 * n**4 + 8 * n**3)
    assert abs(bench.sigma2b_flops(n, 1025) - 1.641e12) < 1e9
    # compulsory bytes: G read once, Sigma_c written once, V read once
    assert bench.sigma2b_bytes(n, 1025, 8) == 8 * (2 * 1025 * n * n + n * n)
    assert abs(bench.sigma2b_bytes(n, 1025, 8) - 0.6498e9) < 1e6


def test_dyson_count(bench):
    n, M = 199, 1024
    assert bench.dyson_flops(n, M) == (M // 2) * 8 * n**3 + 2 * (M + 1) * 2 * n**3


def test_traffic_table_only_for_its_source(bench):
    src = os.path.join(ROOT, "paper_0911_4348_amd", "csrc", "sigma2b.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    got = bench.measured_traffic("f64", 199, 1025, 0)
    if h == bench.TRAFFIC_SRC_SHA256:
        assert got == bench.TRAFFIC_F64_NB199[0]
        # the table never claims less than the compulsory bytes
        assert all(v >= bench.sigma2b_bytes(199, 1025, 8) for v in bench.TRAFFIC_F64_NB199.values())
    else:
        assert got is None
    assert bench.measured_traffic("f32", 199, 1025, 0) is None
    assert bench.measured_traffic("f64", 200, 1025, 0) is None
    assert bench.measured_traffic("f64", 199, 513, 0) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_new_modes_are_documented_in_help():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 0
    assert "--issue-probe" in r.stdout and "--scan-size" in r.stdout
