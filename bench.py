"""Throughput of the ray-casting point-in-polygon hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config 4] [--mode filtered|exact]

One step is one full pass of the hot path over one batch of the workload --
counter resets and work ordering, the main classification kernel and, in the
filtered mode, the binary64 recheck of undecided pairs -- through a plan of the
C ABI (one HIP graph launch when the tuned plan keeps its graph).  The default
workload is the batched one: 1,000,000 star polygons with ring sizes following
a power law on [3, 4096] and Poisson(100) points each (about 10^8 pairs), in
the binary32-filtered mode.  Inputs are resident in HBM before timing starts;
each step reads at least 1 GB, four times the last-level cache.

Prints one JSON line: point-edge tests/s as `value` (and points/s), the main
kernel's HBM roofline fraction from its own dispatch timestamps (HIP events on
its launch stream) with its VALU issue utilisation at the engine clock read
under load, bit-exact parity of every pair against the CPU oracle, the
recheck and ambiguity fractions, the other arithmetic mode, the staged
filtered kernel and the plain per-pair kernel on the same workload, the oracle
timed on this host's cores, entries for the other four workloads (each with
parity, roofline and oracle timing), the extensions, and the paper's own
timings with the hardware it states (context, not the target).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
SIMDS = 1024                   # 256 compute units x 4 SIMDs
LANES_PER_SIMD_CLK = 16        # a wave64 VALU instruction takes 4 cycles on a 16-lane SIMD
NOMINAL_CLOCK_HZ = 2.4e9       # peak engine clock
TUNE_CACHE = os.path.join(ROOT, "paper_2306_04316_amd", "tune_cache.txt")
METRIC = "point-edge tests/s and points/s at bit-exact match; % of HBM/VALU roofline"

WORKLOAD_TEXT = {
    1: "star: 1 star-shaped polygon, 64 vertices, 100,000 points in its bbox",
    2: "footprints: 100,000 footprint polygons (rotated rectangles / L-shapes, 4-32 vertices), "
       "10,000,000 point->polygon pairs (100 per polygon, bbox x1.2), pairs sorted by polygon",
    3: "fractal: 1 midpoint-displaced 1024-gon with 1,000,000 vertices, 10,000,000 points in its bbox",
    4: "batched: 1,000,000 star polygons, ring sizes k ~ k^-2 on [3,4096], Poisson(100) points each "
       "(about 1e8 point->polygon pairs, sorted by polygon)",
    5: "stress: the batched topology in metres (offset 5e6, 5-50 m), 3% of points on or near edges and vertices",
}

# The paper's own timings (Simulation section, Tables execution_1, Execution-times-points1 and
# the slower machine's), with the hardware it states; context only, not the target.
PAPER_CONTEXT = {
    "workload": "17,097,823 building points vs one country boundary polygon (its vertex count is not stated, "
                "so only points/s can be derived)",
    "rows": [
        {"method": "Algorithm 1 (constraint 1, numpy, one point per call)", "points": 17097823,
         "seconds": 1117.207, "points_per_s": 15304, "hardware": "Intel i7-8750H (6 cores / 12 threads), 32 GB",
         "software": "Python 3.10.8, numpy"},
        {"method": "Algorithm 4 (constraint 2, numba parallel, 12 threads): the paper's fastest",
         "points": 17097823, "seconds": 202.510, "points_per_s": 84429,
         "hardware": "Intel i7-8750H (6 cores / 12 threads), 32 GB", "software": "Python 3.10.8, numba"},
        {"method": "Algorithm 4, 4 threads", "points": 17097823, "seconds": 534.855, "points_per_s": 31967,
         "hardware": "Intel i5-4590 (4 cores / 4 threads), 8 GB", "software": "Python 3.10.8, numba"},
    ],
}

# Recorded counters of main kernels per launch (rocprofv3 --pmc runs of this benchmark, summaries
# under profiles/), keyed by (workload, mode, kernel name, digest of the kernel's sources): an entry
# stops applying when the sources change, and the figures it feeds are then reported as null.
# fetch/write: FETCH_SIZE and WRITE_SIZE scaled by their reading of a copy kernel of known size.
PROFILED: dict = {
    (4, "filtered", "k_filtered_fp32", "84956aede086"): {
        "fetch_bytes": 2413978994, "write_bytes": 100029746, "valu_insts": 498057611, "waves": 390656,
        "source": "profiles/filtered_batched.md"},
    (4, "exact", "k_staged_batched_fp64", "20bc7d20b8e6"): {
        "fetch_bytes": 2414966565, "write_bytes": 100027707, "valu_insts": 431314460, "waves": 390656,
        "source": "profiles/staged_batched_exact.md"},
    (4, "filtered", "k_batched", "ca9bc706ed9c"): {
        "fetch_bytes": 2473433098, "write_bytes": 100148905, "valu_insts": 503289813, "waves": 781308,
        "source": "profiles/batched_kernel_batched.md"},
    (4, "filtered", "k_batched+k_wave_rings", "ca9bc706ed9c"): {
        "fetch_bytes": 2623426984, "write_bytes": 101822759, "valu_insts": 603743450, "waves": 787452,
        "source": "profiles/batched_kernel_wave_ring_256_batched.md"},
    (3, "exact", "k_ring_segments", "501d20328a6a"): {
        "fetch_bytes": 1335002027, "write_bytes": 34495968, "valu_insts": 347753019004, "waves": 312512,
        "source": "profiles/ring_segments_fractal.md"},
}

KERNEL_SOURCES = {
    "k_batched": ("kernels_batched.hip", "kernels_wave.hip", "staged_exact.h", "ring_walk.h", "filter_bound.h"),
    "k_batched+k_wave_rings": ("kernels_batched.hip", "kernels_wave.hip", "staged_exact.h", "ring_walk.h",
                               "filter_bound.h"),
    "k_filtered_fp32": ("kernels_filtered.hip", "staged_exact.h", "ring_walk.h", "filter_bound.h"),
    "k_staged_batched_fp64": ("kernels_exact.hip", "staged_exact.h", "ring_walk.h"),
    "k_runs_batched_fp64": ("kernels_exact.hip", "ring_walk.h"),
    "k_ring_segments": ("kernels_exact.hip", "ring_walk.h"),
    "k_runs_indexed_fp64": ("kernels_index.hip", "sort_staged.h", "ring_walk.h"),
    "k_per_pair_fp64": ("kernels_exact.hip", "ring_walk.h"),
}


SEGMENT_MIN_VERTICES = 65536   # plans walk one ring for every point in segments from this size on


def kernel_name(cfg, w=None) -> str:
    """The main kernel a plan configuration launches (on workload w, when given:
    a plan of the runs kernel over one ring for every point walks it in
    segments from SEGMENT_MIN_VERTICES vertices on)."""
    k, mode = cfg["kernel"], cfg["mode"]
    if k == 5:
        return "k_batched+k_wave_rings" if cfg.get("wave_k", 0) > 0 else "k_batched"
    if k == 1:
        return "k_per_pair_fp64"
    if k == 4:
        if cfg.get("index"):
            return "k_runs_indexed_fp64"
        if (w is not None and w.point_poly is None and getattr(w, "poly_rings", None) is None and w.n_polys == 1
                and w.n_vertices >= SEGMENT_MIN_VERTICES):
            return "k_ring_segments"
        return "k_runs_batched_fp64"
    return "k_filtered_fp32" if mode == 1 else "k_staged_batched_fp64"


def kernel_digest(name: str) -> str:
    """Digest of the code a kernel is compiled from (comments and spacing left out)."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2306_04316_amd", "csrc")
    for f in KERNEL_SOURCES[name]:
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            code = re.sub(r"/\*.*?\*/", " ", fh.read(), flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:12]


def profiled(config: int, mode: str, name: str):
    return PROFILED.get((config, mode, name, kernel_digest(name)))


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="filtered", choices=["exact", "filtered"])
    ap.add_argument("--kernel", default="auto", choices=["auto", "per_pair", "segmented", "staged", "runs", "batched"])
    ap.add_argument("--pairs-per-lane", type=int, default=0)
    ap.add_argument("--lds-slots", type=int, default=0)
    ap.add_argument("--persistent", type=int, default=-1)
    ap.add_argument("--order", type=int, default=-1)
    ap.add_argument("--wave-k", type=int, default=0,
                    help="filtered batched plans: ring size from which the wavefront-per-ring kernel takes the "
                         "pairs (0 = the tuner's or the cache's choice, -1 = off)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip autotuning at plan creation")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="tuning cache (a listed workload class is not re-tuned; new results are appended)")
    ap.add_argument("--compare-steps", type=int, default=10,
                    help="steps of each comparison run (0 = skip them)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="oracle timing budget of the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-clocks", action="store_true", help="do not read clocks with rocm-smi")
    ap.add_argument("--no-configs", action="store_true", help="skip the entries of the other workloads")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the extensions (constraint 2, several rings, candidate pairs, y-index)")
    ap.add_argument("--probe-copy-mb", type=int, default=0,
                    help="run only the HBM calibration copy of this many MiB (for counter scaling)")
    return ap.parse_args(argv)


def progress(msg: str) -> None:
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def host_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    n = int(env) if env and env.isdigit() else (os.cpu_count() or 1)
    try:
        n = min(n, len(os.sched_getaffinity(0)))
    except AttributeError:
        pass
    return max(1, n)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------- clocks
def rocm_smi(args, timeout=20):
    """rocm-smi's JSON output (a child process), or None."""
    import shutil
    exe = shutil.which("rocm-smi") or "/opt/rocm/bin/rocm-smi"
    try:
        r = subprocess.run([exe, *args, "--json"], capture_output=True, text=True, timeout=timeout,
                           stdin=subprocess.DEVNULL)
        return json.loads(r.stdout[r.stdout.index("{"):])
    except (OSError, ValueError, subprocess.SubprocessError):
        return None


def sclk_hz(j):
    """The current engine clock in a rocm-smi --showclocks JSON (first card), or None."""
    if not j:
        return None
    import re
    for card in j.values():
        if not isinstance(card, dict):
            continue
        for key, val in card.items():
            if "sclk" in key.lower() and isinstance(val, str):
                m = re.search(r"([0-9]+(?:\.[0-9]+)?)\s*mhz", val.lower())
                if m:
                    return float(m.group(1)) * 1e6
    return None


def clock_under_load(run_steps, seconds=1.5):
    """The engine clock while the GPU runs the benchmark's own steps: rocm-smi in a
    child process, started once the loop is running.  (hz or None, raw reading)."""
    box = {}

    def read():
        time.sleep(0.3)
        box["j"] = rocm_smi(["--showclocks"])

    import torch
    t = threading.Thread(target=read)
    t0 = time.perf_counter()
    t.start()
    while t.is_alive() or time.perf_counter() - t0 < 0.5:
        run_steps()
        torch.cuda.synchronize()   # keep the queue short: the loop ends soon after the reading
        if time.perf_counter() - t0 > seconds + 20:
            break
    t.join()
    j = box.get("j")
    return sclk_hz(j), j


# ---------------------------------------------------------------- device helpers
VALU_PROBE_ITERS = 8192   # rounds of eight binary64 additions per thread (about 1 ms)


def measured_peaks(P, dev, nbytes: int = 1 << 30, reps: int = 10):
    """HBM rates of plain streaming kernels over nbytes (median of reps launches):
    a read-only stream (pip_probe_read) and a copy (pip_probe_copy); and the
    vector-ALU issue rate of independent binary64 additions (pip_probe_valu)."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    sink64 = torch.zeros(1, dtype=torch.float64, device=dev)
    lane_ops = P.probe_valu(VALU_PROBE_ITERS, sink64)
    out = {}
    for name, fn, moved in (("read_stream", lambda: P.probe_read(src, sink), nbytes),
                            ("copy", lambda: P.probe_copy(dst, src), 2 * nbytes),
                            ("valu", lambda: P.probe_valu(VALU_PROBE_ITERS, sink64), lane_ops)):
        for _ in range(3):
            fn()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b) * 1e-3)
        if name == "valu":
            out["valu_lane_ops_per_s"] = moved / float(np.median(ts))
        else:
            out[name + "_GBs"] = moved / float(np.median(ts)) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    out["probe"] = (f"pip_probe_read / pip_probe_copy over {nbytes >> 20} MiB; pip_probe_valu, {lane_ops} lane "
                    f"operations (binary64 additions, eight waves per SIMD); median of {reps} launches")
    return out


def attach_valu_peak(v, kernel_ms, measured):
    """The measured VALU issue rate beside a roofline's VALU figures: the method's
    lane operations and (when recorded) the kernel's executed lane instructions
    per second as fractions of what the probe issues."""
    if not v:
        return
    v["measured_peak_lane_ops_per_s"] = measured
    v["algorithmic_frac_of_measured_peak"] = v["algorithmic_lane_ops"] / (kernel_ms * 1e-3) / measured
    if v.get("insts_per_launch"):
        v["issue_frac_of_measured_peak"] = v["insts_per_launch"] * 64 / (kernel_ms * 1e-3) / measured


def device_copies(P, w, dev, min_bytes=1 << 30):
    """Device copies of a workload, enough that the steps rotating over them read at
    least min_bytes between two reads of the same data (the last-level cache is 256 MB)."""
    import torch
    n = max(1, math.ceil(min_bytes / max(1, w.nbytes_algorithmic())))
    cs = []
    for _ in range(n):
        d = P.to_device(w, dev)
        d["out"] = torch.empty(w.n_points, dtype=torch.uint8, device=dev)
        cs.append(d)
    return cs


class Runner:
    """Plans over rotating device copies of one workload."""

    def __init__(self, P, copies, plan_opts):
        self.plans = [P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], out=d["out"],
                             poly_rings=d.get("poly_rings"), **plan_opts) for d in copies]
        self.copies = copies

    def steps(self, n, first=0):
        for i in range(first, first + n):
            self.plans[i % len(self.plans)].execute()

    def timed(self, steps, warmup):
        """Mean ms per step over `steps` back-to-back executions after `warmup`,
        bracketed by a device synchronisation and HIP events on both sides."""
        import torch
        self.steps(warmup)
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        start.record()
        self.steps(steps, warmup)
        stop.record()
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / steps, time.perf_counter() - t0

    def phase_times(self, steps, warmup=2):
        """Per-step device times (prep, main, recheck) of plans created with timing; the
        main time is the kernel's own dispatch timestamps on its launch stream."""
        import torch
        self.steps(warmup)
        torch.cuda.synchronize()
        out = []
        n = len(self.plans)
        for i in range(steps):
            p = self.plans[i % n]
            p.execute()
            out.append(p.timing())
        return np.array(out)

    def last_out(self, i):
        return self.copies[i % len(self.copies)]["out"]

    def close(self):
        for p in self.plans:
            p.close()


# ---------------------------------------------------------------- roofline pieces
def valu_entry(config, mode, name, kernel_ms, clock_hz, clock_src, alg_lane_ops):
    """VALU issue utilisation of a main kernel: its recorded VALU instructions per
    launch x 4 cycles over all SIMD cycles of the measured duration at the clock
    read under load; beside it the method's own lane operations over the VALU peak
    at that clock.  Instruction figures are null when the kernel has changed since
    they were recorded."""
    hz = clock_hz or NOMINAL_CLOCK_HZ
    peak_lane_ops = SIMDS * LANES_PER_SIMD_CLK * hz
    e = {"clock_hz": hz, "clock_source": clock_src if clock_hz else "nominal 2.4 GHz (no reading under load)",
         "peak_lane_ops_per_s": peak_lane_ops,
         "algorithmic_lane_ops": alg_lane_ops,
         "algorithmic_frac": alg_lane_ops / (kernel_ms * 1e-3) / peak_lane_ops}
    rec = profiled(config, mode, name)
    if rec and rec.get("valu_insts"):
        e.update(insts_per_launch=rec["valu_insts"], insts_per_wavefront=rec["valu_insts"] / rec["waves"],
                 issue_frac=rec["valu_insts"] * 4 / (SIMDS * hz * kernel_ms * 1e-3),
                 insts_source=rec["source"])
    else:
        e.update(insts_per_launch=None, issue_frac=None)
    return e


def hbm_roofline(config, mode, name, alg_bytes, kernel_ms, source):
    gbs = alg_bytes / (kernel_ms * 1e-3) / 1e9
    rec = profiled(config, mode, name)
    traffic = None
    if rec and rec.get("fetch_bytes") is not None:
        traffic = rec["fetch_bytes"] + rec["write_bytes"]
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": traffic, "traffic_unit": "bytes per launch", "kernel": name, "kernel_ms": kernel_ms,
            "kernel_ms_source": source, "alg_bytes_per_launch": alg_bytes, "kernel_digest": kernel_digest(name)}


def alu_roofline(hbm):
    """Roofline of a kernel bound by vector instruction issue: the method's lane
    operations per second against the VALU lane peak at the clock read under load
    (1024 SIMDs x 16 lanes per cycle); the HBM figures move under "hbm"."""
    v = hbm.pop("valu")
    achieved = v["algorithmic_lane_ops"] / (hbm["kernel_ms"] * 1e-3) / 1e12
    r = {"bound": "alu", "achieved": achieved, "peak": v["peak_lane_ops_per_s"] / 1e12, "unit": "T lane-op/s",
         "frac": v["algorithmic_frac"], "traffic": hbm["traffic"], "traffic_unit": hbm["traffic_unit"],
         "kernel": hbm["kernel"], "kernel_ms": hbm["kernel_ms"], "kernel_ms_source": hbm["kernel_ms_source"],
         "kernel_digest": hbm["kernel_digest"], "valu": v,
         "hbm": {k: hbm[k] for k in ("achieved", "peak", "unit", "frac", "alg_bytes_per_launch")},
         "note": "every point tests every edge of one ring: bound by vector instruction issue, "
                 "2 lane operations per test (the straddle comparison); the HBM figures are beside it"}
    return r


def alg_lane_ops(w, mode, strad_frac):
    """The method's VALU lane operations: 2 per point-edge test (the straddle
    comparisons), 6 per straddling test (two differences, two products, a sum and
    a comparison), 1 per pair; the filtered mode adds one comparison per test."""
    T = w.n_tests
    ops = 2 * T + 6 * strad_frac * T + w.n_points
    if mode == "filtered":
        ops += T
    return ops


def straddle_fraction(w, sample=20000, seed=3, max_tests=20_000_000):
    """Fraction of point-edge tests whose edge straddles the point's y (a sample of
    pairs, at most about max_tests tests)."""
    rng = np.random.default_rng(seed)
    kbar = max(1.0, w.n_tests / max(1, w.n_points))
    sample = int(max(10, min(sample, max_tests / kbar)))
    idx = rng.choice(w.n_points, min(sample, w.n_points), replace=False)
    k = w.edges_per_pair()[idx]
    q = w.point_poly[idx] if w.point_poly is not None else np.zeros(idx.size, dtype=np.int64)
    tot = strad = 0
    for i, qq in zip(idx, q):
        b, e = w.offsets[qq], w.offsets[qq + 1]
        y = w.vy[b:e]
        ab = y > w.py[i]
        strad += int(np.count_nonzero(ab != np.roll(ab, 1)))
    tot = int(k.sum())
    return strad / max(1, tot)


# ---------------------------------------------------------------- oracle
def oracle_parity(w, got, th):
    """Bit-exact comparison of every pair with the oracle (the indexed mode for one ring)."""
    import oracle
    t0 = time.perf_counter()
    if w.point_poly is None and w.n_vertices > 100_000:
        want = oracle.classify_indexed(w.px, w.py, w.offsets, w.vx, w.vy, nthreads=th)
        how = "the oracle's indexed mode (exact y buckets; same bits as the plain loop)"
    else:
        want = oracle.classify_workload(w, nthreads=th)
        how = "the oracle"
    secs = time.perf_counter() - t0
    nbad = int(np.count_nonzero(got != want))
    text = "bit-exact (all pairs)" if nbad == 0 else f"MISMATCH in {nbad} pairs"
    return text, want, {"against": how, "seconds": secs}


def cpu_baseline(w, budget_s, th, sample_n=None):
    """The oracle as it stands on this host's cores, over whole passes of a bounded
    sample of the workload, plus one pass on one thread of a smaller sample."""
    import oracle
    from paper_2306_04316_amd import workloads as W
    n = w.n_points
    if sample_n is None:
        probe_n = min(n, 20_000)
        t0 = time.perf_counter()
        oracle.classify_workload(W.subsample(w, np.arange(probe_n)), nthreads=th)
        dt = max(time.perf_counter() - t0, 1e-6)
        sample_n = int(min(n, max(probe_n, probe_n * 0.5 * budget_s / dt)))
    if sample_n >= n:
        s, label = w, f"the full workload ({n} pairs)"
    else:
        idx = np.sort(np.random.default_rng(11).choice(n, sample_n, replace=False)) if w.point_poly is None \
            else np.arange(sample_n)
        s = W.subsample(w, idx)
        label = (f"{sample_n} sampled points of {n} against the whole ring" if w.point_poly is None
                 else f"the first {sample_n} of {n} pairs (contiguous, same polygons)")
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.classify_workload(s, nthreads=th)
        reps += 1
        el = time.perf_counter() - t0
        if el >= 0.5 * budget_s or reps >= 50:
            break
    per = el / reps
    out = {"value": s.n_tests / per, "unit": "tests/s", "points_per_s": s.n_points / per, "cores": th,
           "kind": "oracle", "sample": f"{label}, {reps} pass(es), {per:.4f} s per pass", "cpu_model": cpu_model()}
    n1 = int(min(s.n_points, max(200, s.n_points * 0.1 * budget_s / (per * th))))
    s1 = W.subsample(s, np.arange(n1))
    t1 = time.perf_counter()
    oracle.classify_workload(s1, nthreads=1)
    d1 = max(time.perf_counter() - t1, 1e-6)
    out["single_thread"] = {"value": s1.n_tests / d1, "unit": "tests/s",
                            "sample": f"the first {n1} pairs of that sample, one pass, {d1:.3f} s"}
    return out


# ---------------------------------------------------------------- one workload, fully
def plan_options(a, mode, kernel, **kw):
    o = dict(mode=mode, kernel=kernel, pairs_per_lane=a.pairs_per_lane, lds_slots=a.lds_slots,
             persistent=a.persistent, order=a.order, use_graph=not a.no_graph,
             tune=0 if (a.no_tune or kernel in ("per_pair", "segmented")) else 1, tune_cache=a.tune_cache,
             wave_k=a.wave_k)
    o.update(kw)
    return o


def measure(P, w, copies, opts, steps, warmup, config, mode, th, parity=True, want=None, ktimes=None):
    """One plan configuration on one workload: step time (graph or eager launches as the
    plan keeps them), the main kernel's own timestamps, the phase split, parity."""
    r = Runner(P, copies, opts)
    cfg = r.plans[0].config()
    ms, wall = r.timed(steps, warmup)
    last = r.last_out(warmup + steps - 1).cpu().numpy()
    r.close()
    tuned = dict(opts, tune=0, kernel=cfg["kernel"], pairs_per_lane=cfg["pairs_per_lane"],
                 lds_slots=cfg["lds_slots"], persistent=cfg["persistent"], order=cfg["order"],
                 wave_k=cfg["wave_k"] if cfg["wave_k"] > 0 else -1)
    rk = Runner(P, copies, dict(tuned, use_graph=False, timing=1))
    ph = rk.phase_times(ktimes or max(10, min(steps, 50)))
    rk.close()
    name = kernel_name(cfg, w)
    main_ms = float(np.mean(ph[:, 1]))
    e = {"ms_per_step": ms, "tests_per_s": w.n_tests / (ms * 1e-3), "points_per_s": w.n_points / (ms * 1e-3),
         "pairs": w.n_points, "tests": w.n_tests, "steps": steps, "warmup": warmup, "wall_s_timed": wall,
         "plan": cfg, "main_kernel": name, "main_kernel_ms": main_ms, "main_kernel_ms_min": float(np.min(ph[:, 1])),
         "phases_ms": {"prep": float(np.mean(ph[:, 0])), "main": main_ms, "recheck": float(np.mean(ph[:, 2]))}}
    if parity:
        if want is None:
            e["parity"], want, e["parity_check"] = oracle_parity(w, last, th)
        else:
            nbad = int(np.count_nonzero(last != want))
            e["parity"] = "bit-exact (all pairs)" if nbad == 0 else f"MISMATCH in {nbad} pairs"
    return e, want, tuned


def recheck_figures(P, w, copies, tuned):
    """Recheck counts of one execution of the tuned filtered plan (pairs sent to the binary64
    recheck), and the batched kernel's device counters on the same workload (point-edge tests
    counted, side tests inside its bound) from one execution of a stats plan."""
    if tuned.get("mode") != "filtered":
        return None
    d = copies[0]
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], out=d["out"],
                **dict(tuned, use_graph=False))
    pl.execute()
    own = pl.stats()
    pl.close()
    opts = dict(tuned, use_graph=False, stats=True)
    if tuned.get("kernel") != 5:
        opts.update(kernel=5, pairs_per_lane=2, lds_slots=512)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], out=d["out"], **opts)
    st = pl.execute(stats=True)
    pl.close()
    return {"rechecked_pairs": own["rechecked_pairs"], "recheck_pair_fraction": own["rechecked_pairs"] / max(1, w.n_points),
            "source": "one execution of the tuned plan (pip_plan_stats)",
            "batched_kernel_counters": {
                "tests_counted": st["tests"], "tests_expected": w.n_tests, "ambiguous_tests": st["ambiguous_tests"],
                "ambiguous_test_fraction": st["ambiguous_tests"] / max(1, w.n_tests),
                "rechecked_pairs": st["rechecked_pairs"],
                "recheck_pair_fraction": st["rechecked_pairs"] / max(1, w.n_points),
                "wave_k": opts.get("wave_k", 0),
                "source": "one execution of a batched-kernel plan with device counters (pip_stats)"}}


def config_entry(P, W, a, config, dev, th, clock):
    """Parity, throughput, roofline and the oracle's rate for one of the other workloads."""
    import torch
    w = W.make(config, seed=a.seed)
    copies = device_copies(P, w, dev)
    if config == 3:
        # one ring of 10^6 vertices for every point: the exact runs kernel streams the ring
        # wave-uniformly; bound by vector instruction issue (2 lane operations per test)
        mode = "exact"
        opts = plan_options(a, "exact", "auto", use_graph=False, tune=0, pairs_per_lane=0, lds_slots=0,
                            persistent=-1, order=-1)
        e, want, tuned = measure(P, w, copies, opts, 3, 1, config, mode, th, ktimes=3)
    else:
        mode = a.mode
        opts = plan_options(a, mode, "auto", pairs_per_lane=0, lds_slots=0, persistent=-1, order=-1)
        e, want, tuned = measure(P, w, copies, opts, 50 if w.n_points > 1e6 else 200, 20, config, mode, th)
    e["workload"] = WORKLOAD_TEXT[config]
    e["mode"] = mode
    e["dtype"] = "f64" if mode == "exact" else "f32+f64"
    name = e["main_kernel"]
    e["roofline"] = hbm_roofline(config, mode, name, w.nbytes_algorithmic(), e["main_kernel_ms"],
                                 "the main kernel's own dispatch timestamps (HIP events on its launch stream)")
    sf = straddle_fraction(w)
    e["roofline"]["valu"] = valu_entry(config, mode, name, e["main_kernel_ms"], clock[0], clock[1],
                                       alg_lane_ops(w, mode, sf))
    e["straddle_fraction"] = sf
    if config == 3:
        e["roofline"] = alu_roofline(e["roofline"])
        e["cpu_baseline"] = cpu_baseline(w, 4.0, th, sample_n=2000)
    else:
        e["cpu_baseline"] = cpu_baseline(w, 4.0, th)
    rf = recheck_figures(P, w, copies, tuned)
    if rf:
        e["recheck"] = rf
    del copies
    torch.cuda.empty_cache()
    return e


# ---------------------------------------------------------------- extensions beyond the hot path
def extensions(P, W, a, dev, th):
    """Parity and timing of the extensions, each on its own synthetic workload."""
    import torch
    import oracle
    out = {}

    def cpu_entry(work, unit, secs, sample):
        return {"value": work / secs, "unit": unit, "cores": th, "kind": "oracle",
                "sample": f"{sample}, {secs:.3f} s"}

    def run(w, opts, steps=10, config=0, mode="exact"):
        copies = device_copies(P, w, dev)
        e, want, _ = measure(P, w, copies, opts, steps, 2, config, mode, th, ktimes=steps)
        e["roofline"] = hbm_roofline(config, mode, e["main_kernel"], w.nbytes_algorithmic(), e["main_kernel_ms"],
                                     "the main kernel's own dispatch timestamps")
        del copies
        torch.cuda.empty_cache()
        return e

    base = dict(mode="exact", kernel="auto", pairs_per_lane=0, lds_slots=0, persistent=-1, order=-1,
                use_graph=False, tune=0)
    # constraint 2 (the paper's second crossing test) on the footprints workload
    progress("extension: constraint-2 predicate")
    w = W.footprints(seed=a.seed)
    t0 = time.perf_counter()
    oracle.classify_workload(w, nthreads=th, predicate=2)
    secs = time.perf_counter() - t0
    copies = device_copies(P, w, dev)
    e, _, _ = measure(P, w, copies, dict(base, predicate="intersection"), 10, 2, 0, "exact", th, parity=False,
                      ktimes=10)
    got = copies[(2 + 10 - 1) % len(copies)]["out"].cpu().numpy()
    want = oracle.classify_workload(w, nthreads=th, predicate=2)
    e["parity"] = "bit-exact (all pairs)" if np.array_equal(got, want) else "MISMATCH"
    del copies
    e["roofline"] = hbm_roofline(0, "exact", e["main_kernel"], w.nbytes_algorithmic(), e["main_kernel_ms"],
                                 "the main kernel's own dispatch timestamps")
    e["cpu_baseline"] = cpu_entry(w.n_tests, "tests/s", secs, f"the whole workload ({w.n_points} pairs), one pass")
    out["constraint2_footprints"] = e
    # polygons of several rings
    progress("extension: polygons with holes and detached parts")
    w = W.holes(seed=a.seed)
    t0 = time.perf_counter()
    oracle.classify_workload(w, nthreads=th)
    secs = time.perf_counter() - t0
    e = run(w, dict(base))
    e.update(polygons=w.n_polys, rings=w.n_rings)
    e["cpu_baseline"] = cpu_entry(w.n_tests, "tests/s", secs, f"the whole workload ({w.n_points} pairs), one pass")
    out["rings_holes"] = e
    # candidate pairs by bounding box (raw points of the footprints workload)
    progress("extension: candidate pairs by bounding box")
    w = W.raw_points(W.footprints(seed=a.seed))
    d = P.to_device(w, dev)
    walls, kern = [], []
    for rep in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tm = {}
        c = P.candidate_pairs(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], timing=tm)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        kern.append(tm["ms_count"] + tm["ms_fill"])
    m = int(c["point"].numel())
    idx = np.sort(np.random.default_rng(5).choice(w.n_points, 3000, replace=False))
    t0 = time.perf_counter()
    wp, wq = oracle.bbox_join(w.px[idx], w.py[idx], w.offsets, w.vx, w.vy, nthreads=th)
    secs = time.perf_counter() - t0
    gp, gq = c["point"].cpu().numpy(), c["poly"].cpu().numpy()
    sel = np.isin(gp, idx)
    order = np.lexsort((gp[sel], gq[sel]))
    ok = np.array_equal(gq[sel][order], wq) and np.array_equal(gp[sel][order], idx[wp])
    t = float(np.min(walls[1:]))
    km = float(np.min(kern[1:]))
    nbytes = 16 * w.n_points + 16 * w.n_vertices + 8 * (w.n_polys + 1) + 28 * m
    gbs = nbytes / (km * 1e-3) / 1e9
    out["candidate_pairs"] = {
        "kernel_ms": km, "ms_wall_incl_host_sync": t * 1e3, "points": w.n_points, "polygons": w.n_polys,
        "pairs": m, "points_per_s": w.n_points / (km * 1e-3),
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                     "traffic": None, "kernel": "the join's kernels (pip_join_timing: device time of both count "
                     "phases and the fill, without its host synchronisations and allocations)", "kernel_ms": km,
                     "alg_bytes_per_launch": nbytes},
        "parity": "exact pair set (3000 sampled points)" if ok else "MISMATCH",
        "cpu_baseline": cpu_entry(idx.size, "points/s", secs, f"{idx.size} sampled points against every polygon's box")}
    del c, d
    torch.cuda.empty_cache()
    # y-index for one large polygon (the fractal workload)
    progress("extension: y-index on the 10^6-vertex polygon")
    w = W.make(3, seed=a.seed)
    e = run(w, dict(mode="exact", kernel="auto", index=True, use_graph=False, tune=0), steps=5, config=3)
    e["note"] = ("tests_per_s counts every point-edge test the method defines; the index skips most of them "
                 "(points_per_s is the comparable figure)")
    e["method_equivalent_tests_per_s"] = e.pop("tests_per_s")
    e["roofline"]["note"] = "a tree walk and leaf edge tests bound by latency; the bytes it must move are few"
    out["yindex_fractal"] = e
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                                   "(the pairs are independent: a multi-GPU split is a partition "
                                   "of polygons with their points, with no exchange)"}), flush=True)
        sys.exit(2)
    clocks_idle = None
    if not a.no_clocks and not a.probe_copy_mb:
        progress("device clocks and power cap at idle (rocm-smi)")
        clocks_idle = rocm_smi(["--showclocks", "--showmaxpower"])
    import torch
    import paper_2306_04316_amd as P
    from paper_2306_04316_amd import workloads as W

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    th = host_threads()

    if a.probe_copy_mb:
        nb = a.probe_copy_mb << 20
        src = torch.empty(nb, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty(nb, dtype=torch.uint8, device=dev)
        for _ in range(3):
            P.probe_copy(dst, src)
        torch.cuda.synchronize()
        print(json.dumps({"probe_copy_bytes": nb}), flush=True)
        return

    t_gen = time.perf_counter()
    w = W.make(a.config, seed=a.seed)
    t_gen = time.perf_counter() - t_gen
    copies = device_copies(P, w, dev)
    torch.cuda.synchronize()
    T, N = w.n_tests, w.n_points
    progress(f"workload {a.config}: N={N} P={w.n_polys} V={w.n_vertices} T={T}; {len(copies)} device copies")

    # ---- the headline: timed steps, main-kernel timestamps, parity
    opts = plan_options(a, a.mode, a.kernel)
    progress("headline plan and timed steps")
    head, want, tuned = measure(P, w, copies, opts, a.steps, a.warmup, a.config, a.mode, th,
                                parity=not a.no_parity)
    name = head["main_kernel"]
    # ---- the engine clock under load (the VALU issue figures use it)
    clock = (None, None)
    clock_raw = None
    if not a.no_clocks:
        progress("engine clock under load (rocm-smi while steps run)")
        r = Runner(P, copies, dict(tuned, use_graph=bool(head["plan"]["use_graph"])))
        hz, clock_raw = clock_under_load(lambda: r.steps(20))
        torch.cuda.synchronize()
        r.close()
        clock = (hz, "rocm-smi sclk read while the benchmark's steps ran")
    alg_bytes = w.nbytes_algorithmic()
    main_ms = head["main_kernel_ms"]
    roof = hbm_roofline(a.config, a.mode, name, alg_bytes, main_ms,
                        "the main kernel's own dispatch timestamps (HIP events recorded by its dispatch on its "
                        f"launch stream), mean of {a.steps if a.steps < 50 else 50} eager executions after the "
                        "timed steps")
    sf = straddle_fraction(w)
    roof["valu"] = valu_entry(a.config, a.mode, name, main_ms, clock[0], clock[1], alg_lane_ops(w, a.mode, sf))
    if a.config == 3:   # every point tests every edge of one ring: bound by vector issue
        roof = alu_roofline(roof)
    rf = recheck_figures(P, w, copies, tuned)

    # ---- the same workload: the other mode, the staged filtered kernel, the per-pair kernel
    compare = {}
    if a.compare_steps > 0:
        other = "filtered" if a.mode == "exact" else "exact"
        runs = [("mode_" + other, plan_options(a, other, "auto", pairs_per_lane=0, lds_slots=0)),
                ("staged_filtered_kernel", plan_options(a, "filtered", "staged", pairs_per_lane=0, lds_slots=0)),
                ("batched_kernel", plan_options(a, "filtered", "batched", pairs_per_lane=0, lds_slots=0,
                                                wave_k=-1)),
                ("batched_kernel_wave_ring_256", plan_options(a, "filtered", "batched", pairs_per_lane=0,
                                                              lds_slots=0, wave_k=256)),
                ("per_pair_baseline", plan_options(a, "exact", "per_pair", use_graph=False)),
                # the headline's tuned plan replayed as one HIP graph per step (the tuner may keep eager
                # launches when they issue the sequence as fast)
                ("tuned_plan_as_graph", dict(tuned, use_graph=True, tune=0, tune_cache=None))]
        for label, o in runs:
            progress(f"comparison: {label}")
            e, _, _ = measure(P, w, copies, o, a.compare_steps, 2, a.config, o["mode"], th, want=want,
                              parity=want is not None, ktimes=a.compare_steps)
            e["roofline"] = hbm_roofline(a.config, o["mode"], e["main_kernel"], alg_bytes, e["main_kernel_ms"],
                                         "the main kernel's own dispatch timestamps")
            e["roofline"]["valu"] = valu_entry(a.config, o["mode"], e["main_kernel"], e["main_kernel_ms"], clock[0],
                                               clock[1], alg_lane_ops(w, o["mode"], sf))
            compare[label] = e
        pp = compare["per_pair_baseline"]["main_kernel_ms"]
        compare["main_kernel_speedup_vs_per_pair"] = pp / main_ms
        compare["step_speedup_vs_per_pair"] = compare["per_pair_baseline"]["ms_per_step"] / head["ms_per_step"]

    cpu = None
    if not a.no_cpu_baseline:
        progress("cpu baseline (the oracle on this host's cores)")
        cpu = cpu_baseline(w, a.cpu_seconds, th)
    del copies
    torch.cuda.empty_cache()

    configs = {}
    if not a.no_configs:
        for c in (1, 2, 3, 5):
            if c == a.config:
                continue
            progress(f"workload {c}")
            configs[str(c)] = config_entry(P, W, a, c, dev, th, clock)

    ext = None
    if not a.no_extensions:
        ext = extensions(P, W, a, dev, th)

    progress("bandwidth probes")
    peaks = measured_peaks(P, dev)
    hbm_gbs = roof["hbm"]["achieved"] if roof["bound"] == "alu" else roof["achieved"]
    peaks["frac_of_read_stream"] = hbm_gbs / peaks["read_stream_GBs"]
    roof["measured_peaks"] = peaks
    attach_valu_peak(roof.get("valu"), roof["kernel_ms"], peaks["valu_lane_ops_per_s"])
    if roof["bound"] == "alu":
        roof["frac_of_measured_peak"] = roof["valu"]["algorithmic_frac_of_measured_peak"]
    for e in list((configs or {}).values()) + list(compare.values() if isinstance(compare, dict) else []):
        r = e.get("roofline") if isinstance(e, dict) else None
        if r:
            attach_valu_peak(r.get("valu"), r["kernel_ms"], peaks["valu_lane_ops_per_s"])
            if r.get("bound") == "alu":
                r["frac_of_measured_peak"] = r["valu"]["algorithmic_frac_of_measured_peak"]
    rec = {
        "metric": METRIC,
        "value": T / (head["ms_per_step"] * 1e-3),
        "unit": "tests/s",
        "points_per_s": N / (head["ms_per_step"] * 1e-3),
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.mode == "exact" else "f32+f64",
        "data": "synthetic",
        "parity": head.get("parity", "not checked"),
        "config": {"workload": WORKLOAD_TEXT[a.config], "config_id": a.config, "seed": a.seed, "pairs": N,
                   "polygons": w.n_polys, "vertices": w.n_vertices, "tests": T, "mode": a.mode,
                   "plan": head["plan"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "recheck": rf,
        "step": {"phases_ms": head["phases_ms"], "main_kernel_ms_min": head["main_kernel_ms_min"],
                 "wall_s_timed": head["wall_s_timed"], "parity_check": head.get("parity_check"),
                 "straddle_fraction": sf},
        "compare": compare,
        "configs": configs,
        "extensions": ext,
        "paper_context": PAPER_CONTEXT,
        "device_clocks": {"idle": clocks_idle, "under_load": clock_raw},
        "gen_s": t_gen,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
