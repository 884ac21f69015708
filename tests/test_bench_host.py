"""Host-side logic of the benchmark (no GPU): the choice of how the timed steps
are measured, the kernel-code digest that keys the recorded HBM traffic (a
stale record is reported as null, never applied to changed code), and the
refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def cfg(**kw):
    c = dict(mode=0, kernel=3, pairs_per_lane=4, lds_slots=256, persistent=0, order=0, use_graph=0, index=0)
    c.update(kw)
    return c


def test_single_kernel_step():
    # an eager binary64 step with no ordering pass and no queue: the main kernel alone
    assert bench.single_kernel_step(cfg())
    assert bench.single_kernel_step(cfg(persistent=1))          # staged persistent: fixed stride, no queue
    assert not bench.single_kernel_step(cfg(use_graph=1))       # graph launches
    assert not bench.single_kernel_step(cfg(mode=1))            # filtered: recheck kernel follows
    assert not bench.single_kernel_step(cfg(order=1))           # heaviest-first order is a prep pass
    assert not bench.single_kernel_step(cfg(index=1))           # the y-index sorts the points first
    assert not bench.single_kernel_step(cfg(kernel=4, persistent=1))   # runs kernel's queue reset


def test_kernel_digest_ignores_comments(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2306_04316_amd" / "csrc"
    csrc.mkdir(parents=True)
    src = {"kernels_exact.hip": "int f(int a) { return a + 1; } // one\n/* block */\n",
           "staged_exact.h": "#pragma once\nint h();\n",
           "ring_walk.h": "#pragma once\nint g();\n"}
    for name, text in src.items():
        (csrc / name).write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.kernel_digest()
    (csrc / "kernels_exact.hip").write_text("int f(int a) {\n    return a + 1;   // another comment\n}\n")
    assert bench.kernel_digest() == d0, "comments and spacing must not change the digest"
    (csrc / "kernels_exact.hip").write_text("int f(int a) { return a + 2; }\n")
    assert bench.kernel_digest() != d0, "a code change must change the digest"
    d1 = bench.kernel_digest()
    (csrc / "staged_exact.h").write_text("#pragma once\nint h(int);\n")
    assert bench.kernel_digest() != d1, "a change in the shared staged item must change the digest"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_valu_issue_tied_to_digest(monkeypatch):
    # 600 wavefront instructions on each of the 1024 SIMDs take 2400 cycles: 1 us at 2.4 GHz
    d = bench.kernel_digest("exact")
    monkeypatch.setattr(bench, "PROFILED_VALU", {(2, "exact", d): {"valu_insts": 1024 * 600, "waves": 1024,
                                                                     "source": "test"}})
    v = bench.valu_issue("exact", 2, 1e-3)
    assert abs(v["issue_frac"] - 1.0) < 1e-12 and v["insts_per_wavefront"] == 600
    assert bench.valu_issue("exact", 2, 2e-3)["issue_frac"] == 0.5
    # another mode, config or digest has no record
    assert bench.valu_issue("filtered", 2, 1e-3) is None
    assert bench.valu_issue("exact", 4, 1e-3) is None
    assert bench.kernel_digest("filtered") != d
