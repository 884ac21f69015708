"""Throughput of the ray-casting point-in-polygon hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config 2] [--mode exact|filtered] [--no-tune]

One step is one full pass of the hot path over one batch of the workload
(default: the footprint workload, 100,000 building-footprint polygons and 10M
point->polygon pairs) through a plan of the C ABI: counter resets and
heaviest-first work ordering, the main kernel, and (filtered mode) the binary64
recheck, launched as one HIP graph.  Inputs are resident in HBM before timing
starts; the steps rotate over four device copies of the batch (one plan each) so
that no step reads data the previous step left in the caches (the copies total
more than the 256 MB last-level cache).

Prints one JSON line: throughput (point-edge tests/s as `value`, points/s), the
dominant kernel's HBM roofline fraction with its duration taken from HIP events
recorded by its own dispatches on the launch stream during the timed steps, the bit-exact
parity result against the CPU oracle, the same path in the other arithmetic
mode and the plain per-pair baseline kernel for comparison, and the oracle's own
speed on this host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# Tuned plan configurations shipped with the package (written by the plan autotuner on MI355X);
# a plan whose workload class is listed there is created without re-tuning.
TUNE_CACHE = os.path.join(ROOT, "paper_2306_04316_amd", "tune_cache.txt")
METRIC = "point-edge tests/s and points/s at bit-exact match; % of HBM/VALU roofline"

WORKLOAD_TEXT = {
    1: "star: 1 star-shaped polygon, 64 vertices, 100,000 points in its bbox",
    2: "footprints: 100,000 footprint polygons (rotated rectangles / L-shapes, 4-32 vertices), "
       "10,000,000 point->polygon pairs (100 per polygon, bbox x1.2), pairs sorted by polygon",
    3: "fractal: 1 midpoint-displaced 1024-gon with 1,000,000 vertices, 10,000,000 points in its bbox",
    4: "batched: 1,000,000 star polygons, k ~ k^-2 on [3,4096], Poisson(100) points each (~1e8 pairs)",
    5: "stress: batched topology in metres (offset 5e6, 5-50 m), 3% of points on/near edges and vertices",
}

# HBM traffic of the main kernel per launch, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs
# of this benchmark (bytes, after scaling by the counters' reading of a copy kernel of known size).
# Keyed by (config, mode, kernel-source digest): an entry stops applying as soon as the kernel
# sources change, and the benchmark then reports traffic as null.
PROFILED_TRAFFIC: dict = {
    # footprints, exact mode, k_staged_batched_fp64<0, 4, false, false, false>
    # (profiles/staged_footprints_exact.md: FETCH_SIZE and WRITE_SIZE scaled by the copy calibration)
    (2, "exact", "3490bb00a683"): {"fetch_bytes": 220034029, "write_bytes": 10000000},
    # footprints, filtered mode, k_filtered_fp32<4, false> (profiles/filtered_footprints.md)
    (2, "filtered", "ef05df756c55"): {"fetch_bytes": 220086121, "write_bytes": 10001760},
    # batched, both modes (profiles/staged_batched_exact.md, profiles/filtered_batched.md)
    (4, "exact", "3490bb00a683"): {"fetch_bytes": 2415001030, "write_bytes": 100027584},
    (4, "filtered", "ef05df756c55"): {"fetch_bytes": 2413919385, "write_bytes": 100029552},
}

# VALU instructions of the main kernel per launch (rocprofv3 --pmc SQ_INSTS_VALU, SQ_WAVES; median
# over launches), keyed like PROFILED_TRAFFIC.
PROFILED_VALU: dict = {
    (2, "exact", "3490bb00a683"): {"valu_insts": 19025260, "waves": 39064,
                                   "source": "profiles/staged_footprints_exact.md"},
    (2, "filtered", "ef05df756c55"): {"valu_insts": 26096941, "waves": 39064,
                                      "source": "profiles/filtered_footprints.md"},
    (4, "exact", "3490bb00a683"): {"valu_insts": 431314460, "waves": 390656,
                                   "source": "profiles/staged_batched_exact.md"},
    (4, "filtered", "ef05df756c55"): {"valu_insts": 498057611, "waves": 390656,
                                      "source": "profiles/filtered_batched.md"},
}
SIMDS = 1024          # 256 compute units x 4 SIMDs
CLOCK_HZ = 2.4e9      # peak engine clock


DIGEST_SOURCES = {"exact": ("kernels_exact.hip", "staged_exact.h", "ring_walk.h"),
                  "filtered": ("kernels_filtered.hip", "staged_exact.h", "ring_walk.h")}


def kernel_digest(mode: str = "exact") -> str:
    """Digest of the code a mode's main kernel is compiled from (its sources,
    comments and spacing left out); a change there invalidates the recorded
    traffic and instruction counts."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2306_04316_amd", "csrc")
    for f in DIGEST_SOURCES[mode]:
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            code = re.sub(r"/\*.*?\*/", " ", fh.read(), flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:12]


def valu_issue(mode: str, config: int, kernel_ms: float):
    """VALU issue utilisation of a mode's main kernel: its recorded VALU
    instruction count per launch (rocprofv3 SQ_INSTS_VALU) times 4 cycles (a
    wavefront instruction on a 16-lane SIMD) over all SIMD cycles of the
    measured duration (1024 SIMDs at 2.4 GHz).  None when the kernel has
    changed since the count was taken."""
    rec = PROFILED_VALU.get((config, mode, kernel_digest(mode)))
    if rec is None:
        return None
    cycles = kernel_ms * 1e-3 * SIMDS * CLOCK_HZ
    return {"insts_per_launch": rec["valu_insts"], "insts_per_wavefront": rec["valu_insts"] / rec["waves"],
            "issue_frac": rec["valu_insts"] * 4 / cycles, "peak": "1 wavefront instruction per 4 cycles per SIMD",
            "source": rec["source"]}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="exact", choices=["exact", "filtered"])
    ap.add_argument("--kernel", default="auto", choices=["auto", "per_pair", "segmented", "staged", "runs", "batched"])
    ap.add_argument("--pairs-per-lane", type=int, default=0)
    ap.add_argument("--lds-slots", type=int, default=0)
    ap.add_argument("--persistent", type=int, default=-1)
    ap.add_argument("--order", type=int, default=-1)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--index", action="store_true",
                    help="one polygon: y-indexed path (edges skipped by y-range tree, points in y order)")
    ap.add_argument("--no-tune", action="store_true", help="skip autotuning at plan creation")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="tuning cache (a listed workload class is not re-tuned; new results are appended)")
    ap.add_argument("--copies", type=int, default=4, help="device copies the steps rotate over")
    ap.add_argument("--compare-steps", type=int, default=10,
                    help="steps for the other-mode and per-pair comparison runs (0 = skip them)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target oracle timing budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-clocks", action="store_true", help="skip reading clocks and power cap with rocm-smi")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the extension measurements (constraint 2, several rings, candidate pairs, y-index)")
    ap.add_argument("--probe-copy-mb", type=int, default=0,
                    help="run only the HBM calibration copy of this many MiB (for counter scaling)")
    return ap.parse_args()


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


def cpu_baseline(w, budget_s: float):
    """The oracle as it stands, on this host's cores, over whole passes of a bounded sample."""
    import oracle
    from paper_2306_04316_amd import workloads as W
    th = host_threads()
    n = w.n_points
    probe_n = min(n, 20_000)
    t0 = time.perf_counter()
    oracle.classify_workload(W.subsample(w, np.arange(probe_n)), nthreads=th)
    dt = max(time.perf_counter() - t0, 1e-6)
    want = int(min(n, max(probe_n, probe_n * 0.5 * budget_s / dt)))
    if want >= n:
        s, label = w, f"the full workload ({n} pairs)"
    else:
        s = W.subsample(w, np.arange(want))
        label = f"the first {want} of {n} pairs (contiguous, same polygons)"
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.classify_workload(s, nthreads=th)
        reps += 1
        el = time.perf_counter() - t0
        if el >= 0.5 * budget_s:
            break
    per = el / reps
    # one thread, on a sample sized for about a tenth of the budget
    n1 = int(min(s.n_points, max(1000, s.n_points * 0.1 * budget_s / (per * th))))
    s1 = W.subsample(w, np.arange(n1))
    t1 = time.perf_counter()
    oracle.classify_workload(s1, nthreads=1)
    d1 = max(time.perf_counter() - t1, 1e-6)
    return {"value": s.n_tests / per, "unit": "tests/s", "points_per_s": s.n_points / per, "cores": th,
            "kind": "oracle", "sample": f"{label}, {reps} pass(es), {per:.4f} s per pass",
            "cpu_model": cpu_model(),
            "single_thread": {"value": s1.n_tests / d1, "unit": "tests/s",
                              "sample": f"the first {n1} pairs, one pass, {d1:.3f} s"}}


def device_clocks():
    """The GPU's current clocks and power cap as rocm-smi reports them (a child
    process; None when the tool is missing, fails or prints no JSON)."""
    import shutil
    import subprocess
    exe = shutil.which("rocm-smi") or "/opt/rocm/bin/rocm-smi"
    try:
        r = subprocess.run([exe, "--showclocks", "--showmaxpower", "--json"], capture_output=True, text=True,
                           timeout=20, stdin=subprocess.DEVNULL)
        j = r.stdout[r.stdout.index("{"):]
        return json.loads(j)
    except (OSError, ValueError, subprocess.SubprocessError):
        return None


def measured_peaks(P, dev, nbytes: int = 1 << 30, reps: int = 10):
    """HBM rates this device reaches with plain streaming kernels over nbytes
    (median of reps launches, HIP events on the current stream): a read-only
    stream (pip_probe_read) and a copy (pip_probe_copy, read plus write)."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    out = {}
    for name, fn, moved in (("read_stream", lambda: P.probe_read(src, sink), nbytes),
                            ("copy", lambda: P.probe_copy(dst, src), 2 * nbytes)):
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
        out[name + "_GBs"] = moved / float(np.median(ts)) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    out["probe"] = f"pip_probe_read / pip_probe_copy over {nbytes >> 20} MiB, median of {reps} launches"
    return out


def single_kernel_step(cfg) -> bool:
    """An eager step that launches the main kernel alone: binary64 mode (no recheck), no
    y-index, no per-execution item order, no work-queue reset."""
    return (not cfg["use_graph"] and cfg["mode"] == 0 and not cfg["index"] and cfg["order"] != 1
            and not (cfg["persistent"] and cfg["kernel"] == 4))


class Runner:
    """Plans over rotating device copies of one workload; times every step with HIP events
    recorded on the launch stream just before and after the plan's (graph) launch."""

    def __init__(self, P, copies, plan_opts, timed_copies=None):
        """timed_copies: indices of the copies whose plans take plan_opts' timing (default:
        all); the others run with none, so their steps put nothing but their kernels in the stream."""
        timing = plan_opts.get("timing", 0)
        on = set(range(len(copies))) if timed_copies is None else set(timed_copies)
        self.plans = [P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], out=d["out"],
                             poly_rings=d.get("poly_rings"), **dict(plan_opts, timing=timing if c in on else 0))
                      for c, d in enumerate(copies)]
        self.timed = [bool(timing) and c in on for c in range(len(copies))]

    def run(self, steps, warmup, step_events=True):
        """step_events: HIP events around every launch (off when the plans record the
        main kernel's own timestamps, so the stream carries nothing but the steps)."""
        import torch
        n = len(self.plans)
        for i in range(warmup):
            self.plans[i % n].execute()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps if step_events else 0)]
        phase = []
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        start.record()
        for i in range(steps):
            if self.timed[i % n] and i >= n:
                # before this plan runs again, read the phase events of its previous execution
                # (enqueued n steps ago; waits for that execution only, n - 1 steps stay queued)
                phase.append(self.plans[i % n].timing())
            if step_events:
                ev[i][0].record()
            self.plans[i % n].execute()
            if step_events:
                ev[i][1].record()
        stop.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        for i in range(max(0, steps - n), steps):
            if self.timed[i % n]:
                phase.append(self.plans[i % n].timing())
        step_ms = np.array([a.elapsed_time(b) for a, b in ev]) if step_events else None
        return start.elapsed_time(stop) / steps, step_ms, (np.array(phase) if phase else None), wall

    def close(self):
        for p in self.plans:
            p.close()


def extensions(P, W, a, cfg, dev):
    """Parity and timing of the extensions beyond the hot path, each on its own
    synthetic workload (two device copies, so the 256 MB last-level cache does not
    hold a whole step's inputs)."""
    import torch
    import oracle
    out = {}
    th = host_threads()

    def copies_of(w, n=2):
        cs = []
        for _ in range(n):
            d = P.to_device(w, dev)
            d["out"] = torch.empty(w.n_points, dtype=torch.uint8, device=dev)
            cs.append(d)
        return cs

    def roofline(kernel, alg_bytes, ms, note=None):
        gbs = alg_bytes / (ms * 1e-3) / 1e9
        r = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
             "traffic": None, "kernel": kernel, "kernel_ms": ms, "alg_bytes_per_launch": alg_bytes}
        if note:
            r["note"] = note
        return r

    def oracle_timed(fn, *args, **kw):
        t0 = time.perf_counter()
        r = fn(*args, **kw)
        return r, time.perf_counter() - t0

    def cpu_entry(work, unit, secs, sample):
        return {"value": work / secs, "unit": unit, "cores": th, "kind": "oracle",
                "sample": f"{sample}, {secs:.3f} s"}

    def plan_entry(w, cs, opts, want, steps=10, kernel="main classification kernel", note=None, warm=2):
        r = Runner(P, cs, dict(opts, timing=True, tune=0))
        ms, _, ph, _ = r.run(steps, warm)
        main_ms = float(np.mean(ph[:, 1]))
        got = cs[(2 + steps - 1) % len(cs)]["out"].cpu().numpy()
        e = {"ms_per_step_eager": ms, "main_kernel_ms": main_ms, "prep_ms": float(np.mean(ph[:, 0])),
             "tests_per_s": w.n_tests / (ms * 1e-3), "pairs": w.n_points, "tests": w.n_tests,
             "config": r.plans[0].config(),
             "roofline": roofline(kernel, w.nbytes_algorithmic(), main_ms, note)}
        if opts.get("mode") == "filtered":
            e["recheck_fraction"] = r.plans[0].stats()["rechecked_pairs"] / max(1, w.n_points)
            e["recheck_ms"] = float(np.mean(ph[:, 2]))
        if isinstance(want, tuple):   # sampled
            idx, ws = want
            e["parity"] = ("bit-exact (%d sampled pairs)" % idx.size) if np.array_equal(got[idx], ws) else "MISMATCH"
        else:
            e["parity"] = "bit-exact (all pairs)" if np.array_equal(got, want) else \
                "MISMATCH in %d pairs" % int(np.count_nonzero(got != want))
        r.close()
        return e

    base = dict(mode="exact", kernel="auto", pairs_per_lane=cfg["pairs_per_lane"], lds_slots=cfg["lds_slots"],
                persistent=0, order=0, use_graph=False)
    # constraint 2 (the paper's second crossing test) on the footprints workload
    progress("extension: constraint-2 predicate")
    w = W.footprints(seed=a.seed)
    cs = copies_of(w)
    want, secs = oracle_timed(oracle.classify_workload, w, nthreads=th, predicate=2)
    e = plan_entry(w, cs, dict(base, predicate="intersection"), want)
    e["cpu_baseline"] = cpu_entry(w.n_tests, "tests/s", secs, f"the whole workload ({w.n_points} pairs), one pass")
    out["constraint2_footprints"] = e
    del cs
    # polygons of several rings
    progress("extension: polygons with holes and detached parts")
    w = W.holes(seed=a.seed)
    cs = copies_of(w)
    want, secs = oracle_timed(oracle.classify_workload, w, nthreads=th)
    e = plan_entry(w, cs, dict(base), want)
    e.update(polygons=w.n_polys, rings=w.n_rings)
    e["cpu_baseline"] = cpu_entry(w.n_tests, "tests/s", secs, f"the whole workload ({w.n_points} pairs), one pass")
    out["rings_holes"] = e
    del cs
    # candidate pairs by bounding box (raw points of the footprints workload)
    progress("extension: candidate pairs by bounding box")
    w = W.raw_points(W.footprints(seed=a.seed))
    d = P.to_device(w, dev)
    times = []
    for rep in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = P.candidate_pairs(d["px"], d["py"], d["offsets"], d["vx"], d["vy"])
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    m = int(c["point"].numel())
    idx = np.sort(np.random.default_rng(5).choice(w.n_points, 3000, replace=False))
    (wp, wq), secs = oracle_timed(oracle.bbox_join, w.px[idx], w.py[idx], w.offsets, w.vx, w.vy, nthreads=th)
    gp, gq = c["point"].cpu().numpy(), c["poly"].cpu().numpy()
    sel = np.isin(gp, idx)
    order = np.lexsort((gp[sel], gq[sel]))
    ok = np.array_equal(gq[sel][order], wq) and np.array_equal(gp[sel][order], idx[wp])
    t = float(np.min(times[1:]))
    nbytes = 16 * w.n_points + 16 * w.n_vertices + 8 * (w.n_polys + 1) + 28 * m
    out["candidate_pairs"] = {"ms_wall_incl_host_sync": t * 1e3, "points": w.n_points, "polygons": w.n_polys,
                              "pairs": m, "points_per_s": w.n_points / t,
                              "roofline": roofline("the whole join (every kernel, allocations and two host "
                                                   "synchronisations, wall time)", nbytes, t * 1e3),
                              "parity": "exact pair set (3000 sampled points)" if ok else "MISMATCH",
                              "cpu_baseline": cpu_entry(idx.size, "points/s", secs,
                                                        f"{idx.size} sampled points against every polygon's box")}
    del c, d
    # y-index for one large polygon (config 3 shape)
    progress("extension: y-index on the 10^6-vertex polygon")
    w = W.make(3, seed=a.seed)
    cs = copies_of(w, 1)
    idx = np.sort(np.random.default_rng(1).choice(w.n_points, 2000, replace=False))
    ws, secs = oracle_timed(oracle.classify_workload, W.subsample(w, idx), nthreads=th)
    e = plan_entry(w, cs, dict(mode="exact", kernel="auto", index=True, use_graph=False), (idx, ws), steps=5,
                   kernel="indexed runs kernel",
                   note="issue-bound tree walk and leaf edge tests; the bytes it must move are few")
    e["note"] = "tests_per_s counts every point-edge test the method defines (the index skips most of them)"
    e["cpu_baseline"] = cpu_entry(idx.size * w.n_vertices, "tests/s", secs,
                                  f"{idx.size} sampled pairs against the whole ring")
    out["yindex_fractal"] = e
    del cs
    # the batched workload (power-law ring sizes, ~10^8 pairs): both modes with the plan shape the
    # tuner keeps for it, against the plain per-pair kernel; these kernels are bound by vector
    # instruction issue, so each carries its recorded VALU issue utilisation beside the HBM figure
    progress("extension: batched workload, both modes and the per-pair kernel")
    w = W.make(4, seed=a.seed)
    cs = copies_of(w)
    idx = np.sort(np.random.default_rng(2).choice(w.n_points, 20000, replace=False))
    ws = oracle.classify_workload(W.subsample(w, idx), nthreads=th)
    _, secs = oracle_timed(oracle.classify_workload, w, nthreads=th)   # the oracle's rate: one whole pass
    shape = dict(kernel="staged", pairs_per_lane=4, lds_slots=256, persistent=0, order=1, use_graph=False)
    b = {}
    for label, opts in (("filtered", dict(shape, mode="filtered")), ("exact", dict(shape, mode="exact")),
                        ("per_pair_baseline", dict(mode="exact", kernel="per_pair", use_graph=False))):
        progress(f"extension: batched workload, {label}")
        e = plan_entry(w, cs, opts, (idx, ws), steps=20, warm=20)
        if label != "per_pair_baseline":
            e["roofline"]["valu"] = valu_issue(opts["mode"], 4, e["main_kernel_ms"])
        b[label] = e
    pp = b["per_pair_baseline"]["main_kernel_ms"]
    b["filtered_main_kernel_speedup_vs_per_pair"] = pp / b["filtered"]["main_kernel_ms"]
    b["exact_main_kernel_speedup_vs_per_pair"] = pp / b["exact"]["main_kernel_ms"]
    b["cpu_baseline"] = cpu_entry(int(w.n_tests), "tests/s", secs, f"the whole workload ({w.n_points} pairs), one pass")
    out["batched"] = b
    del cs
    return out


def progress(msg: str) -> None:
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                                   "(the pairs are independent: a multi-GPU split is a partition "
                                   "of polygons with their points, with no exchange)"}), flush=True)
        sys.exit(2)
    clocks = None
    if not a.no_clocks and not a.probe_copy_mb:
        progress("device clocks (rocm-smi)")
        clocks = device_clocks()
    import torch
    import paper_2306_04316_amd as P
    from paper_2306_04316_amd import workloads as W

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

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
    copies = []
    for _ in range(max(1, a.copies)):
        d = P.to_device(w, dev)
        d["out"] = torch.empty(w.n_points, dtype=torch.uint8, device=dev)
        copies.append(d)
    torch.cuda.synchronize()

    def plan_opts(mode, kernel, index=False):
        return dict(mode=mode, kernel=kernel, pairs_per_lane=a.pairs_per_lane, lds_slots=a.lds_slots,
                    persistent=a.persistent, order=a.order, use_graph=not a.no_graph, index=index,
                    tune=0 if (a.no_tune or index or kernel in ("per_pair", "segmented")) else 1,
                    tune_cache=a.tune_cache)


    T, N = w.n_tests, w.n_points
    progress(f"workload {a.config}: N={N} P={w.n_polys} V={w.n_vertices}; creating plans"
             + ("" if a.no_tune or a.index else " (autotuning)"))
    runner = Runner(P, copies, plan_opts(a.mode, a.kernel, a.index))
    cfg = runner.plans[0].config()
    tuned_opts = dict(plan_opts(a.mode, a.kernel, a.index), tune=0, kernel=cfg["kernel"],
                      pairs_per_lane=cfg["pairs_per_lane"], lds_slots=cfg["lds_slots"],
                      persistent=cfg["persistent"], order=cfg["order"])
    kernel_ts = None
    single = single_kernel_step(cfg)
    if not cfg["use_graph"]:
        # eager launches: the timed steps carry the main kernel's own start/end timestamps
        # (events recorded by its dispatch, no extra commands in the stream).  When a step is
        # that kernel alone, only the steps over the first device copy record them, which keeps
        # the cost of those events off the other steps.
        runner.close()
        runner = Runner(P, copies, dict(tuned_opts, use_graph=False, timing=2),
                        timed_copies=[0] if single else None)
    progress(f"plan config {cfg}; timed run of {a.steps} steps")
    ms_per_step, step_ms, ts, wall = runner.run(a.steps, a.warmup, step_events=cfg["use_graph"] != 0)
    if ts is not None:
        kernel_ts = ts[:, 1]
        step_ms = kernel_ts
    runner.close()
    # Phase breakdown from eager executions with events between the phases (same plan options,
    # not graph-launched); when the graph holds the main kernel alone, the per-step events of the
    # timed region above bracket exactly that kernel.
    progress("phase timing run")
    rt = Runner(P, copies, dict(tuned_opts, timing=True))
    _, _, phase, _ = rt.run(max(8, min(a.steps, 20)), 2)
    rt.close()
    if kernel_ts is not None:
        main_ms = float(np.mean(kernel_ts))
        main_src = ("the main kernel's own start/end timestamps (HIP events recorded by its dispatch) on "
                    + (f"one step in {len(copies)} (those over the first device copy)" if single else "every step")
                    + " of the timed region, on the launch stream")
    else:
        main_ms = float(np.mean(phase[:, 1]))
        main_src = ("the main kernel's own start/end timestamps (HIP events recorded by its dispatch) in eager "
                    "executions after the timed graph launches")
    alg_bytes = w.nbytes_algorithmic()
    achieved = alg_bytes / (main_ms * 1e-3) / 1e9
    last = copies[(a.warmup + a.steps - 1) % len(copies)]["out"]

    parity = "not checked"
    want = None
    if not a.no_parity:
        progress("parity against the oracle")
        import oracle
        got = last.cpu().numpy()
        if T <= 5_000_000_000:
            want = oracle.classify_workload(w, nthreads=host_threads())
            nbad = int(np.count_nonzero(got != want))
            parity = "bit-exact (all pairs)" if nbad == 0 else f"MISMATCH in {nbad} pairs"
        else:
            idx = np.sort(np.random.default_rng(1).choice(N, 2000, replace=False))
            ws = oracle.classify_workload(W.subsample(w, idx), nthreads=host_threads())
            nbad = int(np.count_nonzero(got[idx] != ws))
            parity = ("bit-exact (2000 sampled pairs)" if nbad == 0
                      else f"MISMATCH in {nbad} of 2000 sampled pairs")

    compare = {}
    if a.compare_steps > 0:
        other = "filtered" if a.mode == "exact" else "exact"
        runs = [("mode_" + other, plan_opts(other, "auto")), ("per_pair_baseline", plan_opts("exact", "per_pair"))]
        if a.index:
            runs = [("unindexed", plan_opts("exact", "auto"))]
        for label, opts in runs:
            progress(f"comparison run: {label}")
            r = Runner(P, copies, dict(opts, timing=True))
            st = r.plans[0]
            ms, _, ph, _ = r.run(a.compare_steps, 2)
            entry = {"ms_per_step_eager": ms, "main_kernel_ms": float(np.mean(ph[:, 1])),
                     "prep_ms": float(np.mean(ph[:, 0])), "config": st.config()}
            if opts["mode"] == "filtered":
                s = st.stats()
                entry["recheck_fraction"] = s["rechecked_pairs"] / max(1, N)
                entry["recheck_ms"] = float(np.mean(ph[:, 2]))
            if opts["mode"] != a.mode and label.startswith("mode_"):
                kms = entry["main_kernel_ms"]
                gbs = alg_bytes / (kms * 1e-3) / 1e9
                tr2 = PROFILED_TRAFFIC.get((a.config, opts["mode"], kernel_digest(opts["mode"])))
                entry["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": gbs / HBM_PEAK_GBS,
                                     "traffic": None if tr2 is None else tr2["fetch_bytes"] + tr2["write_bytes"],
                                     "kernel": "main classification kernel", "kernel_ms": kms,
                                     "alg_bytes_per_launch": alg_bytes, "kernel_digest": kernel_digest(opts["mode"]),
                                     "valu": valu_issue(opts["mode"], a.config, kms)}
            if want is not None:
                got = copies[(2 + a.compare_steps - 1) % len(copies)]["out"].cpu().numpy()
                entry["parity"] = "bit-exact" if np.array_equal(got, want) else "MISMATCH"
            r.close()
            compare[label] = entry
        if "per_pair_baseline" in compare:
            compare["main_kernel_speedup_vs_per_pair"] = compare["per_pair_baseline"]["main_kernel_ms"] / main_ms
        if "unindexed" in compare:
            compare["speedup_vs_unindexed"] = compare["unindexed"]["main_kernel_ms"] / main_ms

    if not a.no_cpu_baseline:
        progress("cpu baseline (oracle)")
    cpu = None if a.no_cpu_baseline else cpu_baseline(w, a.cpu_seconds)

    ext = None
    n_copies = len(copies)
    if not a.no_extensions and a.config == 2:
        del copies, last, runner, rt
        torch.cuda.empty_cache()
        ext = extensions(P, W, a, cfg, dev)

    progress("bandwidth probes")
    peaks = measured_peaks(P, dev)
    peaks["frac_of_read_stream"] = achieved / peaks["read_stream_GBs"]
    digest = kernel_digest(a.mode)
    tr = PROFILED_TRAFFIC.get((a.config, a.mode, digest))
    traffic = None if tr is None else tr["fetch_bytes"] + tr["write_bytes"]
    rec = {
        "metric": METRIC,
        "value": T / (ms_per_step * 1e-3),
        "unit": "tests/s",
        "points_per_s": N / (ms_per_step * 1e-3),
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.mode == "exact" else "f32+f64",
        "data": "synthetic",
        "parity": parity,
        "config": {"workload": WORKLOAD_TEXT[a.config], "config_id": a.config, "seed": a.seed, "pairs": N,
                   "polygons": w.n_polys, "vertices": w.n_vertices, "tests": T, "mode": a.mode,
                   "plan": cfg, "device_copies": n_copies},
        "phases_ms_eager": {"prep": float(np.mean(phase[:, 0])), "main": float(np.mean(phase[:, 1])),
                            "recheck": float(np.mean(phase[:, 2]))},
        "step_ms_events": {"mean": float(np.mean(step_ms)), "min": float(np.min(step_ms)),
                           "source": "main kernel timestamps" if kernel_ts is not None else "events around launches"},
        "kernel_ms_timestamps": None if kernel_ts is None else {
            "mean": float(np.mean(kernel_ts)), "min": float(np.min(kernel_ts)), "steps": int(kernel_ts.size),
            "steps_sampled": "those over the first device copy" if single else "all"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_unit": "bytes per launch",
                     "kernel": "main classification kernel", "kernel_ms": main_ms, "kernel_ms_source": main_src,
                     "alg_bytes_per_launch": alg_bytes, "kernel_digest": digest,
                     "valu": valu_issue(a.mode, a.config, main_ms), "measured_peaks": peaks},
        "compare": compare,
        "extensions": ext,
        "cpu_baseline": cpu,
        "device_clocks": clocks,
        "wall_s_timed": wall,
        "gen_s": t_gen,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
