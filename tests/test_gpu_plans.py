"""GPU parity of plans (pip_plan_*): exact and binary32-filtered modes, work
ordering, persistent queues, graph replays and the autotuner -- every mask
compared bit for bit with the CPU oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same_mask, note, to_dev
from paper_2306_04316_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2306_04316_amd as P
    return P


def plan_run(P, w, **opts):
    import torch
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], **opts)
    pl.execute()
    torch.cuda.synchronize()
    got = pl.out.cpu().numpy()
    st = pl.stats()
    cfg = pl.config()
    pl.close()
    return got, st, cfg


def check_plan(P, w, what, **opts):
    note(f"plan {what} {opts} N={w.n_points} P={w.n_polys} V={w.n_vertices}")
    got, st, cfg = plan_run(P, w, **opts)
    want = oracle.classify_workload(w)
    assert_same_mask(got, want, f"plan {what} {opts}", w.px, w.py, w.point_poly)
    return st, cfg


SMALL = {
    "star": lambda: W.star(),
    "footprints": lambda: W.footprints(scale=0.0123),
    "batched": lambda: W.batched(scale=0.01),
    "stress": lambda: W.stress(scale=0.02),
    "fractal": lambda: W.fractal(scale=0.001, n_vertices=20_000),
}


@pytest.mark.parametrize("mode", ["exact", "filtered"])
@pytest.mark.parametrize("name", list(SMALL))
def test_plan_small(P, mode, name):
    st, cfg = check_plan(P, SMALL[name](), name, mode=mode)
    assert cfg["use_graph"] == 1


@pytest.mark.parametrize("mode", ["exact", "filtered"])
@pytest.mark.parametrize("name", ["star", "batched", "fractal"])
def test_plan_small_tuned(P, mode, name):
    check_plan(P, SMALL[name](), name, mode=mode, tune=1)


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("mode", ["exact", "filtered"])
def test_plan_scheduling_variants(P, persistent, order, mode):
    check_plan(P, W.batched(scale=0.01), "batched", mode=mode, persistent=persistent, order=order)


@pytest.mark.parametrize("ppl", [1, 2, 4])
@pytest.mark.parametrize("lds", [64, 256, 2048])
def test_plan_tiles(P, ppl, lds):
    check_plan(P, W.stress(scale=0.005), "stress", mode="filtered", pairs_per_lane=ppl, lds_slots=lds)
    check_plan(P, W.stress(scale=0.005), "stress", mode="exact", pairs_per_lane=ppl, lds_slots=lds)


def test_filtered_recheck_fraction(P):
    w = W.stress(scale=0.02)
    st, _ = check_plan(P, w, "stress", mode="filtered")
    frac = st["rechecked_pairs"] / w.n_points
    note(f"stress recheck fraction {frac:.4f}")
    # the special classes (on vertices, level with a horizontal edge, within 1e-9 m) are 3%
    assert 0.01 < frac < 0.2


def test_filtered_force_recheck(P):
    w = W.batched(scale=0.01)
    st, _ = check_plan(P, w, "batched", mode="filtered", force_recheck=True)
    # every staged pair goes through the binary64 recheck; pairs of rings too
    # large to stage are decided by the binary64 wave-uniform walk anyway
    assert st["rechecked_pairs"] >= 0.5 * w.n_points


@pytest.mark.parametrize("kernel", ["staged", "batched"])
def test_filtered_levels_equal_in_binary32(P, kernel):
    """Points level with a vertex to within a binary64 ulp or two, far from the
    vertex in x: after re-centring their binary32 y equals the vertex's.  The
    staged kernel's binary32 straddle order is then undecided and every such
    pair must be rechecked; the batched kernel compares y in binary64 (exact)
    and decides them.  Both must match the oracle."""
    base = 1.0e6
    rel = [(0.0, 0.0), (4.0, 0.3), (4.5, 1.7), (2.0, 1.1), (0.5, 2.9), (-0.5, 1.4)]
    vx = np.array([base + a for a, _ in rel])
    vy = np.array([base + b for _, b in rel])
    px, py = [], []
    for yv in vy:
        for d in (-3.5e-10, -1.2e-10, 0.0, 1.2e-10, 3.5e-10):
            for xr in (-2.0, 1.0, 2.5, 6.0):
                px.append(base + xr)
                py.append(yv + d)
    px, py = np.array(px), np.array(py)
    w = W.Workload("levels", px, py, np.array([0, len(vx)], dtype=np.int64), vx, vy, None, {})
    # binary32 y of the points and vertices re-centred on the box's centre
    cy = 0.5 * vy.min() + 0.5 * vy.max()
    level = np.isin(np.float32(py - cy), np.float32(vy - cy))
    assert level.sum() >= len(vy) * 12
    st, _ = check_plan(P, w, "levels", mode="filtered", kernel=kernel)
    if kernel == "staged":
        assert st["rechecked_pairs"] >= int(level.sum())
    rx = np.array([-0.0, 1e-300, 1e-300, -0.0])
    ry = np.array([-0.0, -0.0, 1e-300, 1e-300])
    tx = np.array([0.0, -0.0, 5e-301, 1e-300, 2e-300, 0.0, -1e-300])
    ty = np.array([0.0, -0.0, 5e-301, 5e-301, 5e-301, 1e-300, -1e-300])
    bx = np.array([-1e300, 1e300, 1e300, -1e300])
    by = np.array([-1e300, -1e300, 1e300, 1e300])
    for ringx, ringy, name in ((rx, ry, "tiny square"), (bx, by, "huge square")):
        w = W.Workload(name, tx, ty, np.array([0, 4], dtype=np.int64), ringx, ringy, None, {})
        check_plan(P, w, name, mode="filtered", kernel=kernel)


def test_filtered_negative_control(P):
    """With the error bound switched off (bound_scale=0) the binary32 filter alone
    must get some stress pairs wrong: the recheck is load-bearing."""
    import torch
    w = W.stress(scale=0.02)
    note("negative control: filtered with bound_scale=0")
    got, st, _ = plan_run(P, w, mode="filtered", bound_scale=0.0)
    want = oracle.classify_workload(w)
    nbad = int(np.count_nonzero(got != want))
    assert nbad > 0, "the unbounded binary32 filter matched the oracle everywhere"
    note(f"negative control mismatches: {nbad}")


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("mode", ["exact", "filtered"])
@pytest.mark.parametrize("name", ["footprints", "batched", "stress"])
def test_plan_other_seeds(P, name, mode, seed):
    """The same generators at other seeds, tuned plans, both modes."""
    make = {"footprints": lambda: W.footprints(seed=seed, scale=0.01),
            "batched": lambda: W.batched(seed=seed, scale=0.005),
            "stress": lambda: W.stress(seed=seed, scale=0.01)}[name]
    check_plan(P, make(), f"{name} seed {seed}", mode=mode, tune=1)


@pytest.mark.parametrize("mode", ["exact", "filtered"])
def test_graph_replays(P, mode):
    """Several replays of one captured graph, with eager work between them."""
    import torch
    w = W.stress(scale=0.01)
    want = oracle.classify_workload(w)
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], mode=mode)
    assert pl.config()["use_graph"] == 1
    for r in range(4):
        note(f"graph replay {r} mode={mode}")
        pl.out.fill_(7)
        tmp = torch.ones(1 << 20, device="cuda").cumsum(0)   # unrelated eager work
        pl.execute()
        torch.cuda.synchronize()
        assert_same_mask(pl.out.cpu().numpy(), want, f"replay {r}")
        assert tmp[-1].item() == float(1 << 20)
    pl.close()


def test_plan_sees_new_data_in_same_buffers(P):
    import torch
    w1 = W.footprints(scale=0.01, seed=1)
    d = to_dev(w1)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], mode="filtered")
    pl.execute()
    torch.cuda.synchronize()
    assert_same_mask(pl.out.cpu().numpy(), oracle.classify_workload(w1), "first data")
    # new points, same polygons, same buffers
    rng = np.random.default_rng(5)
    w1.px = w1.px + rng.uniform(-1e-4, 1e-4, w1.n_points)
    d["px"].copy_(torch.from_numpy(w1.px))
    pl.execute()
    torch.cuda.synchronize()
    assert_same_mask(pl.out.cpu().numpy(), oracle.classify_workload(w1), "second data")
    pl.close()


def test_plan_eager_mode(P):
    check_plan(P, W.batched(scale=0.005), "batched", mode="filtered", use_graph=False)
    check_plan(P, W.batched(scale=0.005), "batched", mode="exact", use_graph=False)


def test_plan_baseline_kernels(P):
    check_plan(P, W.footprints(scale=0.01), "footprints", kernel="per_pair")
    check_plan(P, W.footprints(scale=0.01), "footprints", kernel="segmented")


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("persistent", [0, 1])
def test_plan_runs_kernel(P, name, persistent):
    check_plan(P, SMALL[name](), name, kernel="runs", persistent=persistent)


@pytest.mark.parametrize("ppl", [1, 2, 4])
def test_plan_runs_tiles(P, ppl):
    check_plan(P, W.stress(scale=0.01), "stress", kernel="runs", pairs_per_lane=ppl)


def test_plan_unsorted_pairs(P):
    w = W.footprints(scale=0.01)
    s = W.subsample(w, np.random.default_rng(3).permutation(w.n_points))
    for mode in ("exact", "filtered"):
        check_plan(P, s, "shuffled", mode=mode)


def test_plan_empty(P):
    import torch
    w = W.footprints(scale=0.001)
    d = to_dev(w)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    pl = P.Plan(e, e, d["offsets"], d["vx"], d["vy"], torch.empty(0, dtype=torch.int32, device="cuda"),
                mode="filtered")
    pl.execute()
    torch.cuda.synchronize()
    assert pl.stats()["pairs"] == 0
    pl.close()


def test_autotune_and_cache(P, tmp_path):
    cache = str(tmp_path / "tune.txt")
    w = W.batched(scale=0.005)
    st, cfg = check_plan(P, w, "batched", mode="exact", tune=1, tune_cache=cache)
    assert cfg["tuned"] == 1 and cfg["tune_ms"] > 0
    text = open(cache).read().split()
    assert len(text) == 9 and text[-1] == "0"     # exact mode: no wave kernel
    st, cfg2 = check_plan(P, w, "batched", mode="exact", tune=1, tune_cache=cache)
    assert cfg2["tuned"] == 2
    for k in ("kernel", "pairs_per_lane", "lds_slots", "persistent", "order", "use_graph", "wave_k"):
        assert cfg2[k] == cfg[k]
    # filtered: the tuner also picks the wave kernel's ring size (off, 256 or 1024), kept by the cache
    st, cfg = check_plan(P, w, "batched", mode="filtered", tune=1, tune_cache=cache)
    assert cfg["tuned"] == 1 and cfg["wave_k"] in (0, 256, 1024)
    st, cfg2 = check_plan(P, w, "batched", mode="filtered", tune=1, tune_cache=cache)
    assert cfg2["tuned"] == 2 and cfg2["wave_k"] == cfg["wave_k"] and cfg2["kernel"] == cfg["kernel"]
    # an old cache line without the field keeps the wave kernel off
    with open(cache, "w") as f:
        f.write(" ".join(text[:-1]) + "\n")
    st, cfg3 = check_plan(P, w, "batched", mode="exact", tune=1, tune_cache=cache)
    assert cfg3["tuned"] == 2 and cfg3["wave_k"] == 0


@pytest.mark.parametrize("mode", ["exact", "filtered"])
def test_plan_full_batched(P, mode):
    check_plan(P, W.batched(), "batched full", mode=mode)


@pytest.mark.parametrize("mode", ["exact", "filtered"])
def test_plan_full_stress(P, mode):
    st, _ = check_plan(P, W.stress(), "stress full", mode=mode)
    if mode == "filtered":
        note(f"stress full rechecked pairs {st['rechecked_pairs']}")


@pytest.mark.parametrize("mode", ["exact", "filtered"])
def test_plan_full_footprints(P, mode):
    check_plan(P, W.footprints(), "footprints full", mode=mode)


# ---------------------------------------------------------------- y-indexed single polygon
@pytest.mark.parametrize("name", ["star", "fractal"])
def test_plan_index_small(P, name):
    st, cfg = check_plan(P, SMALL[name](), name, index=True)
    assert cfg["index"] == 1


def test_plan_index_fractal_full_sampled(P):
    import torch
    w = W.fractal()
    note("index fractal full")
    got, st, cfg = plan_run(P, w, index=True)
    idx = np.sort(np.random.default_rng(12).choice(w.n_points, 2000, replace=False))
    s = W.subsample(w, idx)
    assert_same_mask(got[idx], oracle.classify_workload(s), "index fractal full (sampled)", s.px, s.py)


def test_plan_index_degenerate(P):
    rng = np.random.default_rng(4)
    px = rng.uniform(-2, 2, 5000)
    py = rng.uniform(-2, 2, 5000)
    py[:50] = 0.0
    py[50:100] = 1.0
    for ring in ([(0.0, 0.0)], [(0.0, 0.0), (1.0, 1.0)], [(0, 0), (1, 0), (1, 1), (0, 1), (0, 0)],
                 [(float(np.cos(t)), float(np.sin(t))) for t in np.linspace(0, 6.2, 3000)]):
        vx = np.array([a for a, _ in ring], dtype=np.float64)
        vy = np.array([b for _, b in ring], dtype=np.float64)
        w = W.Workload("ring", px, py, np.array([0, vx.size], dtype=np.int64), vx, vy, None, {})
        check_plan(P, w, f"index ring k={vx.size}", index=True)


@pytest.mark.parametrize("layout", ["one_bucket", "one_piece", "piece_plus_one", "wide_sparse", "clustered",
                                    "descending", "three_pieces_wide"])
def test_plan_index_point_layouts(P, layout):
    """Point sets that stress the y-index's banded sort: every point in one
    bucket, a single piece (2048 points) and one point more, fewer points
    than coarse digits spread over the whole range (pieces spanning many
    coarse digits), half the points in a band of 1e-9, points in descending
    y.  The output is prefilled, so a point lost or duplicated by the sort
    shows as a mismatch."""
    import torch
    rng = np.random.default_rng(61)
    t = np.sort(rng.uniform(0, 2 * np.pi, 3000))
    r = 1.0 + 0.2 * rng.uniform(-1, 1, 3000)
    vx, vy = r * np.cos(t), r * np.sin(t)
    n = {"one_piece": 2048, "piece_plus_one": 2049, "wide_sparse": 700, "three_pieces_wide": 3 * 2048 + 5}.get(layout,
                                                                                                              20_000)
    px = rng.uniform(-1.3, 1.3, n)
    py = rng.uniform(-1.3, 1.3, n)
    if layout == "one_bucket":
        py[:] = 0.25
    elif layout == "clustered":
        py[: n // 2] = 0.1 + rng.uniform(0, 1e-9, n // 2)
    elif layout == "descending":
        py = np.sort(py)[::-1].copy()
    elif layout == "three_pieces_wide":
        py[:5] = [-1e3, 1e3, -1.25, 1.25, 0.0]
    w = W.Workload("index-layout", px, py, np.array([0, vx.size], dtype=np.int64), vx, vy, None, {})
    note(f"index layout {layout} N={n}")
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], index=True)
    assert pl.config()["index"] == 1
    for _ in range(2):
        pl.out.fill_(7)
        pl.execute()
        torch.cuda.synchronize()
        assert_same_mask(pl.out.cpu().numpy(), oracle.classify_workload(w), f"index layout {layout}", w.px, w.py)
    pl.close()


def one_ring(k, n, seed):
    """A star-like ring of k vertices and n points over its box, some level
    with vertices and some on them."""
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0, 2 * np.pi, k))
    r = 1.0 + 0.3 * rng.uniform(-1, 1, k)
    vx, vy = r * np.cos(t), r * np.sin(t)
    px = rng.uniform(-1.4, 1.4, n)
    py = rng.uniform(-1.4, 1.4, n)
    j = rng.integers(0, k, n // 10)
    py[: n // 10] = vy[j]
    px[n // 10: n // 5], py[n // 10: n // 5] = vx[j[: n // 5 - n // 10]], vy[j[: n // 5 - n // 10]]
    return W.Workload("one-ring", px, py, np.array([0, k], dtype=np.int64), vx, vy, None, {})


@pytest.mark.parametrize("k", [65_535, 65_536, 65_537, 131_072 * 8, 131_072 * 8 + 1, 300_001])
@pytest.mark.parametrize("pred", ["side", "intersection"])
def test_plan_one_ring_segments(P, k, pred):
    """One ring for every point (no pair index): from 65,536 vertices on, plans
    walk the ring in segments laid out over the XCDs (one and two segment
    groups here), combining each 64-point run's segment parities; every point
    of a ragged count against the oracle, eager and over graph replays."""
    import torch
    w = one_ring(k, 2_111, seed=k % 97)
    want = oracle.classify_workload(w, predicate=2 if pred == "intersection" else 1)
    d = to_dev(w)
    for graph in (False, True):
        note(f"one ring k={k} pred={pred} graph={graph}")
        pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], None, predicate=pred, use_graph=graph)
        for _ in range(3 if graph else 1):
            pl.out.fill_(7)
            pl.execute()
            torch.cuda.synchronize()
            assert_same_mask(pl.out.cpu().numpy(), want, f"one ring k={k} {pred} graph={graph}", w.px, w.py)
        pl.close()


def test_plan_one_ring_changes_between_executions(P):
    """The segmented walk reads the ring's size on the device: a plan made for
    a ring of 200,000 vertices stays exact when the buffers then hold a ring
    of 1,000 vertices (offsets rewritten) and one of 150,000."""
    import torch
    w = one_ring(200_000, 1_500, seed=3)
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], None)
    for kk in (200_000, 1_000, 150_000):
        sub = W.Workload("one-ring prefix", w.px, w.py, np.array([0, kk], dtype=np.int64), w.vx[:kk], w.vy[:kk],
                         None, {})
        d["offsets"].copy_(torch.tensor([0, kk], dtype=torch.int64, device="cuda"))
        note(f"one ring changed to k={kk}")
        pl.out.fill_(7)
        pl.execute()
        torch.cuda.synchronize()
        assert_same_mask(pl.out.cpu().numpy(), oracle.classify_workload(sub), f"ring of {kk}", w.px, w.py)
    pl.close()


def test_plan_index_rejects_pair_index(P):
    w = W.footprints(scale=0.001)
    d = to_dev(w)
    with pytest.raises(P.PipError) as e:
        P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], index=True)
    assert e.value.code == -1


# ---------------------------------------------------------------- the benchmark's own launch configuration
@pytest.mark.parametrize("config", [2, 4, 5])
def test_bench_configuration_full(P, config):
    """Full-size workloads with the plan built exactly as the benchmark builds it
    (autotuning with the shipped cache): every pair of the last of several
    executions against the oracle."""
    import os
    import torch
    cache = os.path.join(os.path.dirname(P.__file__), "tune_cache.txt")
    w = W.make(config)
    note(f"bench configuration, workload {config}: N={w.n_points}")
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], mode="exact", tune=1,
                tune_cache=cache)
    note(f"config {pl.config()}")
    for _ in range(3):
        pl.execute()
    torch.cuda.synchronize()
    got = pl.out.cpu().numpy()
    pl.close()
    assert_same_mask(got, oracle.classify_workload(w), f"bench configuration {config}", w.px, w.py, w.point_poly)


def test_plan_index_more_than_64_top_nodes(P):
    """A ring of 2.2 million vertices has 68 top-level nodes, more than one
    wavefront tests at once: the walk's second group of top nodes, sampled."""
    rng = np.random.default_rng(31)
    k = 2_200_000
    t = np.sort(rng.uniform(0, 2 * np.pi, k))
    r = 1.0 + 0.05 * rng.uniform(-1, 1, k)
    vx, vy = r * np.cos(t), r * np.sin(t)
    n = 20_000
    px = rng.uniform(-1.1, 1.1, n)
    py = rng.uniform(-1.1, 1.1, n)
    py[:200] = vy[rng.integers(0, k, 200)]
    w = W.Workload("big-ring", px, py, np.array([0, k], dtype=np.int64), vx, vy, None, {})
    note("index ring of 2.2M vertices")
    got, st, cfg = plan_run(P, w, index=True)
    assert cfg["index"] == 1
    idx = np.sort(rng.choice(n, 600, replace=False))
    s = W.subsample(w, idx)
    assert_same_mask(got[idx], oracle.classify_workload(s), "index 2.2M-vertex ring (sampled)", s.px, s.py)
