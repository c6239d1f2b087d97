"""CPU checks of bench.py's measurement model: the algorithmic work and bytes
per pair it divides by, the peak it compares against, the source hash that
ties counter summaries to the kernel, and the one-GPU rule."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_gate_count_model():
    # m=100, E=5: 100*11*9 + 100*10*8 + 100*14.25 = 19,325 gates per 32
    # pairs, plus two sequences of 7 words at 256 ops per 32 pairs
    assert bench.algorithmic_lane_ops_per_pair(100, 5) == pytest.approx((9900 + 8000 + 1425 + 2 * 7 * 256) / 32)
    assert bench.algorithmic_lane_ops_per_pair(100, 5) == pytest.approx(715.90625)
    # E=0: one candidate, no comparisons
    assert bench.algorithmic_lane_ops_per_pair(100, 0) == pytest.approx((900 + 1425 + 3584) / 32)
    # grows linearly in E: two more candidates per window, each 9 + 8 gates
    d1 = bench.algorithmic_lane_ops_per_pair(250, 11) - bench.algorithmic_lane_ops_per_pair(250, 10)
    d2 = bench.algorithmic_lane_ops_per_pair(250, 21) - bench.algorithmic_lane_ops_per_pair(250, 20)
    assert d1 == pytest.approx(d2) == pytest.approx(250 * (18 + 16) / 32)


def test_bytes_and_peak():
    assert bench.algorithmic_bytes_per_pair(100) == 57
    assert bench.VALU_PEAK_TOPS == pytest.approx(78.6432)
    assert bench.HBM_PEAK_GBS == 8000.0


def test_source_hash_ignores_comments_and_layout():
    a = "int f(int x) { // one\n  return x + 1; /* two */ }\n"
    b = "int f(int x) {\n\n return x + 1;   }"
    assert bench.strip_comments(a) == bench.strip_comments(b)
    assert bench.strip_comments("a /* x */ b") != bench.strip_comments("ab")
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash()


def test_source_hash_covers_the_plain_kernels_compile_flags(monkeypatch):
    # counters taken on one build of the kernel do not vouch for another one
    # compiled with other flags; include paths (machine-specific) are left out
    from paper_1809_07858_amd import build as hipbuild
    for src in hipbuild.EXTRA:
        assert src in hipbuild.SOURCES
    h = bench.kernel_source_hash()
    original = dict(hipbuild.EXTRA)
    # the same code built somewhere else: same hash
    flags = [f if not os.path.isabs(f) else "/elsewhere/include" for f in hipbuild.FLAGS]
    monkeypatch.setattr(hipbuild, "FLAGS", flags)
    assert bench.kernel_source_hash() == h
    # other flags for the plain kernels' source: another hash
    extra = dict(original)
    extra["csrc/shouji_plain.hip"] = []
    monkeypatch.setattr(hipbuild, "EXTRA", extra)
    assert bench.kernel_source_hash() != h


def test_committed_traffic_matches_its_summary():
    # reported only for the source the counters were taken on, and then
    # exactly the summary's figure
    path = os.path.join(ROOT, "profiles", "shouji_plain_m100_E5_n2000000_hbm_traffic.md")
    assert os.path.exists(path)
    t = bench.committed_traffic("m100_E5_n2000000")
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals["kernel_source_sha256"] == bench.kernel_source_hash():
        assert t == float(vals["hbm_bytes_per_launch"])
    else:
        assert t is None
    assert bench.committed_traffic("no_such_workload") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_planning_model():
    # m*((2E+1)*26 + 15)/32 + 1.9*m lane-ops per pair: m=100, E=5 -> 1130.625
    assert bench.planning_lane_ops_per_pair(100, 5) == pytest.approx(100 * 301 / 32 + 190)
    assert bench.planning_lane_ops_per_pair(100, 5) == pytest.approx(1130.625)
    # E=0 and m=250, E=25
    assert bench.planning_lane_ops_per_pair(100, 0) == pytest.approx(100 * 41 / 32 + 190)
    assert bench.planning_lane_ops_per_pair(250, 25) == pytest.approx(250 * (51 * 26 + 15) / 32 + 475)
    # the 57 us per 2M pairs that a half of the peak means at the headline
    t = bench.planning_lane_ops_per_pair(100, 5) * 2_000_000 / (0.5 * bench.VALU_PEAK_TOPS * 1e12)
    assert t == pytest.approx(57.5e-6, rel=1e-2)


def test_cpu_model_is_reported():
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()
