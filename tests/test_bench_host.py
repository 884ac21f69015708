"""Host-side logic of the benchmark (no GPU): the kernel-code digest that keys
the recorded counters (a stale record is reported as null, never applied to
changed code), the VALU-issue arithmetic at the measured clock, the main
kernel a plan configuration launches, the reading of rocm-smi's clock, the
method's lane-operation count, and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import numpy as np

import bench
from paper_2306_04316_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_digest_ignores_comments(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2306_04316_amd" / "csrc"
    csrc.mkdir(parents=True)
    src = {"kernels_batched.hip": "int f(int a) { return a + 1; } // one\n/* block */\n",
           "staged_exact.h": "#pragma once\nint h();\n", "ring_walk.h": "#pragma once\nint g();\n",
           "filter_bound.h": "#pragma once\nint b();\n", "kernels_wave.hip": "int w();\n"}
    for name, text in src.items():
        (csrc / name).write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.kernel_digest("k_batched")
    (csrc / "kernels_batched.hip").write_text("int f(int a) {\n    return a + 1;   // another comment\n}\n")
    assert bench.kernel_digest("k_batched") == d0, "comments and spacing must not change the digest"
    (csrc / "kernels_batched.hip").write_text("int f(int a) { return a + 2; }\n")
    assert bench.kernel_digest("k_batched") != d0, "a code change must change the digest"
    d1 = bench.kernel_digest("k_batched")
    (csrc / "filter_bound.h").write_text("#pragma once\nint b(int);\n")
    assert bench.kernel_digest("k_batched") != d1, "a change in a shared header must change the digest"


def test_kernel_names():
    assert bench.kernel_name({"kernel": 5, "mode": 1}) == "k_batched"
    assert bench.kernel_name({"kernel": 5, "mode": 0}) == "k_batched"
    assert bench.kernel_name({"kernel": 3, "mode": 1}) == "k_filtered_fp32"
    assert bench.kernel_name({"kernel": 3, "mode": 0}) == "k_staged_batched_fp64"
    assert bench.kernel_name({"kernel": 4, "mode": 0}) == "k_runs_batched_fp64"
    assert bench.kernel_name({"kernel": 4, "mode": 0, "index": 1}) == "k_runs_indexed_fp64"
    ring = W.fractal(scale=0.0001, n_vertices=70_000)
    assert bench.kernel_name({"kernel": 4, "mode": 0, "index": 0}, ring) == "k_ring_segments"
    small = W.fractal(scale=0.0001, n_vertices=60_000)
    assert bench.kernel_name({"kernel": 4, "mode": 0, "index": 0}, small) == "k_runs_batched_fp64"
    assert bench.kernel_name({"kernel": 4, "mode": 0, "index": 0}, W.footprints(scale=0.001)) == "k_runs_batched_fp64"
    assert bench.kernel_name({"kernel": 1, "mode": 0}) == "k_per_pair_fp64"


def test_valu_issue_at_measured_clock(monkeypatch):
    # 600 wavefront instructions on each of the 1024 SIMDs take 2400 cycles: 1 us at 2.4 GHz, 2 us at 1.2 GHz
    d = bench.kernel_digest("k_batched")
    monkeypatch.setattr(bench, "PROFILED", {(4, "filtered", "k_batched", d): {
        "valu_insts": 1024 * 600, "waves": 1024, "source": "test"}})
    v = bench.valu_entry(4, "filtered", "k_batched", 1e-3, 2.4e9, "test clock", 0.0)
    assert abs(v["issue_frac"] - 1.0) < 1e-12 and v["insts_per_wavefront"] == 600
    v = bench.valu_entry(4, "filtered", "k_batched", 2e-3, 1.2e9, "test clock", 0.0)
    assert abs(v["issue_frac"] - 1.0) < 1e-12 and v["clock_hz"] == 1.2e9
    # no reading under load: the nominal clock, said so
    v = bench.valu_entry(4, "filtered", "k_batched", 1e-3, None, "unused", 0.0)
    assert v["clock_hz"] == 2.4e9 and "nominal" in v["clock_source"]
    # another workload, mode or kernel has no record
    assert bench.valu_entry(2, "filtered", "k_batched", 1e-3, 2.4e9, "x", 0.0)["issue_frac"] is None
    assert bench.valu_entry(4, "exact", "k_batched", 1e-3, 2.4e9, "x", 0.0)["issue_frac"] is None
    # the method's own lane operations over the peak at that clock
    v = bench.valu_entry(4, "filtered", "k_batched", 1.0, 2.4e9, "x", 1024 * 16 * 2.4e9 * 1e-3 * 0.25)
    assert abs(v["algorithmic_frac"] - 0.25) < 1e-12


def test_hbm_roofline_traffic_tied_to_digest(monkeypatch):
    d = bench.kernel_digest("k_batched")
    monkeypatch.setattr(bench, "PROFILED", {(4, "filtered", "k_batched", d): {
        "fetch_bytes": 100, "write_bytes": 20, "source": "test"}})
    r = bench.hbm_roofline(4, "filtered", "k_batched", 8_000_000, 1.0, "test")
    assert abs(r["frac"] - 0.001) < 1e-12 and r["traffic"] == 120 and r["kernel_digest"] == d
    assert bench.hbm_roofline(4, "exact", "k_batched", 8_000_000, 1.0, "test")["traffic"] is None


def test_sclk_reading():
    j = {"card0": {"dcefclk clock speed:": "(357Mhz)", "sclk clock level:": "2", "sclk clock speed:": "(2400Mhz)",
                   "mclk clock speed:": "(1900Mhz)"}}
    assert bench.sclk_hz(j) == 2.4e9
    assert bench.sclk_hz({"card0": {"sclk clock level": "1 (2105Mhz)"}}) == 2.105e9
    assert bench.sclk_hz(None) is None
    assert bench.sclk_hz({"card0": {"fclk": "x"}}) is None


def test_alg_lane_ops():
    class Wk:
        n_tests = 1000
        n_points = 10
    assert bench.alg_lane_ops(Wk, "exact", 0.5) == 2 * 1000 + 6 * 0.5 * 1000 + 10
    assert bench.alg_lane_ops(Wk, "filtered", 0.5) == 2 * 1000 + 6 * 0.5 * 1000 + 10 + 1000


def test_straddle_fraction_of_a_square():
    from paper_2306_04316_amd import workloads as W
    # a unit square: a point inside its y range straddles exactly 2 of its 4 edges
    px = np.full(100, 0.5)
    py = np.linspace(0.01, 0.99, 100)
    w = W.Workload("sq", px, py, np.array([0, 4], dtype=np.int64), np.array([0.0, 1.0, 1.0, 0.0]),
                   np.array([0.0, 0.0, 1.0, 1.0]), None, {})
    assert abs(bench.straddle_fraction(w) - 0.5) < 1e-12


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_alu_roofline_of_an_issue_bound_kernel():
    hbm = {"bound": "hbm", "achieved": 1.0, "peak": 8000.0, "unit": "GB/s", "frac": 1.25e-4, "traffic": None,
           "traffic_unit": "bytes per launch", "kernel": "k_runs_batched_fp64", "kernel_ms": 1000.0,
           "kernel_ms_source": "test", "alg_bytes_per_launch": 1e9, "kernel_digest": "x",
           "valu": {"algorithmic_lane_ops": 2e13, "peak_lane_ops_per_s": 4e13, "algorithmic_frac": 0.5}}
    r = bench.alu_roofline(hbm)
    assert r["bound"] == "alu" and r["achieved"] == 20.0 and r["peak"] == 40.0 and r["frac"] == 0.5
    assert r["hbm"]["frac"] == 1.25e-4 and "valu" in r


def test_attach_valu_peak():
    """The measured VALU peak beside a roofline's VALU figures."""
    import bench
    v = {"algorithmic_lane_ops": 2e9, "insts_per_launch": 1e6}
    bench.attach_valu_peak(v, 1.0, 4e13)
    assert v["measured_peak_lane_ops_per_s"] == 4e13
    assert abs(v["algorithmic_frac_of_measured_peak"] - 2e9 / 1e-3 / 4e13) < 1e-12
    assert abs(v["issue_frac_of_measured_peak"] - 1e6 * 64 / 1e-3 / 4e13) < 1e-12
    w = {"algorithmic_lane_ops": 1e9, "insts_per_launch": None}
    bench.attach_valu_peak(w, 2.0, 1e13)
    assert "issue_frac_of_measured_peak" not in w
    bench.attach_valu_peak(None, 1.0, 1e13)   # no VALU figures: nothing to do
