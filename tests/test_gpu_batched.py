"""GPU parity of the batched kernel (PIP_KERNEL_BATCHED) in both arithmetic
modes: LDS tiles of every size against rings that end inside, at and across
tile and 32-vertex chunk boundaries, degenerate rings, rings and points outside
the binary32 filter's range, items that take the binary64 fallback, the
device-side test counters, pip_classify's filtered mode, graph replays and the
full-size batched workload -- every mask compared bit for bit with the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same_mask, note, to_dev
from paper_2306_04316_amd import workloads as W
from test_gpu_edges import KS, star_polys

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2306_04316_amd as P
    return P


def run_plan(P, w, execs=1, **opts):
    import torch
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], kernel="batched", **opts)
    cfg = pl.config()
    assert cfg["kernel"] == 5, cfg
    st = None
    for _ in range(execs):
        pl.out.fill_(7)
        st = pl.execute(stats=True)
    torch.cuda.synchronize()
    got = pl.out.cpu().numpy()
    pl.close()
    return got, st, cfg


def check(P, w, what, **opts):
    note(f"batched {what} {opts} N={w.n_points} P={w.n_polys} V={w.n_vertices}")
    got, st, cfg = run_plan(P, w, **opts)
    assert_same_mask(got, oracle.classify_workload(w), f"batched {what} {opts}", w.px, w.py, w.point_poly)
    return st, cfg


def ring_sizes(w):
    k = np.diff(w.offsets)
    q = w.point_poly if w.point_poly is not None else np.zeros(w.n_points, dtype=np.int64)
    return k, q


SMALL = {
    "star": lambda: W.star(),
    "footprints": lambda: W.footprints(scale=0.0123),
    "batched": lambda: W.batched(scale=0.01),
    "stress": lambda: W.stress(scale=0.02),
}


@pytest.mark.parametrize("tile", [32, 512])
@pytest.mark.parametrize("ppl", [1, 2, 4])
@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("mode", ["exact", "filtered"])
def test_batched_small(P, mode, name, ppl, tile):
    check(P, SMALL[name](), name, mode=mode, pairs_per_lane=ppl, lds_slots=tile)


@pytest.mark.parametrize("tile", [32, 64, 512, 1024])
@pytest.mark.parametrize("mode", ["exact", "filtered"])
def test_batched_ring_sizes(P, mode, tile):
    """Rings of 3 .. 5000 vertices (around 32-vertex chunks, the threshold of
    64, the tiles and 4096), points on vertices and level with them."""
    w = star_polys(KS + [4095, 4096, 4097, 5000], 300, seed=3)
    check(P, w, "ring sizes", mode=mode, lds_slots=tile, pairs_per_lane=2)


@pytest.mark.parametrize("mode", ["exact", "filtered"])
def test_batched_ring_sizes_few_points(P, mode):
    """Few pairs per polygon: many rings per item, large rings shared by few lanes."""
    w = star_polys([3, 70, 5, 4096, 9, 33, 64, 65, 1000, 4, 2049] * 6, 5, seed=4)
    for tile in (32, 256):
        check(P, w, "few points", mode=mode, lds_slots=tile, pairs_per_lane=4)


def degenerate_workload():
    """Rings with 0, 1 and 2 vertices, repeated vertices, a closing duplicate,
    horizontal edges, collinear runs and a spike, points on and next to them."""
    rings = [
        [],
        [(0.0, 0.0)],
        [(0.0, 0.0), (1.0, 1.0)],
        [(0.0, 0.0), (2.0, 0.0), (2.0, 0.0), (2.0, 1.0), (0.0, 1.0), (0.0, 0.0)],
        [(0.0, 0.0), (1.0, 0.0), (2.0, 0.0), (2.0, 2.0), (1.0, 2.0), (0.0, 2.0), (0.0, 1.0)],
        [(0.0, 0.0), (3.0, 0.0), (3.0, 1.0), (1.5, 1.0), (1.5, 3.0), (1.5, 1.0), (0.0, 1.0)],
        [(0.0, 0.0), (2.0, 2.0), (0.0, 2.0), (2.0, 0.0)],   # self-intersecting bow tie
    ]
    rng = np.random.default_rng(11)
    vx, vy, off, px, py, pp = [], [], [0], [], [], []
    for q, r in enumerate(rings):
        for a, b in r:
            vx.append(a + 10.0 * q)
            vy.append(b)
        off.append(off[-1] + len(r))
        pts = [(x + 10.0 * q, y) for x in np.arange(-0.5, 3.51, 0.25) for y in np.arange(-0.5, 3.51, 0.25)]
        pts += [(10.0 * q + rng.uniform(-0.5, 3.5), rng.uniform(-0.5, 3.5)) for _ in range(200)]
        for x, y in pts:
            px.append(x)
            py.append(y)
            pp.append(q)
    return W.Workload("degenerate", np.array(px), np.array(py), np.array(off, dtype=np.int64),
                      np.array(vx, dtype=np.float64), np.array(vy, dtype=np.float64),
                      np.array(pp, dtype=np.int32), {})


@pytest.mark.parametrize("tile", [32, 512])
@pytest.mark.parametrize("mode", ["exact", "filtered"])
def test_batched_degenerate_rings(P, mode, tile):
    check(P, degenerate_workload(), "degenerate", mode=mode, lds_slots=tile)


def test_batched_outside_filter_range(P):
    """Rings with normals or coordinates outside the binary32 filter's range
    (coordinates near 1e300 and 1e-300, a point 2^61 away) are undecided and
    go through the binary64 recheck; the bits still match the oracle."""
    rings = [
        ([-1e300, 1e300, 1e300, -1e300], [-1e300, -1e300, 1e300, 1e300]),
        ([-0.0, 1e-300, 1e-300, -0.0], [-0.0, -0.0, 1e-300, 1e-300]),
        ([0.0, 4.0, 4.0, 0.0], [0.0, 0.0, 4.0, 4.0]),
    ]
    pts = [
        [(0.0, 0.0), (-0.0, -0.0), (5e299, 5e299), (1e300, 0.0), (2e300, 1.0), (-1e300, -1e300)],
        [(0.0, 0.0), (-0.0, -0.0), (5e-301, 5e-301), (1e-300, 5e-301), (2e-300, 5e-301), (0.0, 1e-300)],
        [(1.0, 1.0), (2.0 ** 62, 1.0), (-(2.0 ** 62), 1.0), (1.0, 2.0 ** 62), (4.0, 2.0), (0.0, 0.0)],
    ]
    vx, vy, off, px, py, pp = [], [], [0], [], [], []
    for q, ((rx, ry), ps) in enumerate(zip(rings, pts)):
        vx += rx
        vy += ry
        off.append(off[-1] + len(rx))
        for x, y in ps:
            px.append(x)
            py.append(y)
            pp.append(q)
    w = W.Workload("filter range", np.array(px), np.array(py), np.array(off, dtype=np.int64), np.array(vx),
                   np.array(vy), np.array(pp, dtype=np.int32), {})
    st, _ = check(P, w, "filter range", mode="filtered")
    # the huge and tiny rings (12 pairs) and the far points (3) cannot be filtered
    assert st["rechecked_pairs"] >= 15
    check(P, w, "filter range", mode="exact")


@pytest.mark.parametrize("mode", ["exact", "filtered"])
def test_batched_fallbacks(P, mode):
    """Items whose pairs are not sorted by polygon, and items with more polygons
    than the ring table holds (one pair per polygon), take the staged binary64
    item; the bits are the same."""
    w = W.footprints(scale=0.01)
    s = W.subsample(w, np.random.default_rng(3).permutation(w.n_points))
    check(P, s, "shuffled", mode=mode)
    one = star_polys([3 + (q % 40) for q in range(3000)], 1, seed=5)
    for ppl in (1, 2, 4):
        check(P, one, "one pair per polygon", mode=mode, pairs_per_lane=ppl)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 511, 512, 513, 1023, 1025, 4097])
def test_batched_ragged_counts(P, n):
    base = W.batched(scale=0.002, seed=7)
    s = W.subsample(base, np.arange(min(n, base.n_points)))
    for mode in ("exact", "filtered"):
        check(P, s, f"ragged n={n}", mode=mode)


def test_batched_counters(P):
    """Device-side counts: tests = the sum over pairs of the tested ring's
    vertex count (exact in both modes); the stress set has undecided side
    tests in the filtered mode and none are counted in the exact mode."""
    w = W.stress(scale=0.01)
    k, q = ring_sizes(w)
    tests = int(k[q].sum())
    st, _ = check(P, w, "stress counters", mode="filtered", stats=True)
    note(f"counters {st}")
    assert st["tests"] == tests
    assert st["ambiguous_tests"] > 0
    assert st["rechecked_pairs"] > 0
    # every pair with an undecided side test is rechecked (and only those, here)
    assert st["ambiguous_tests"] >= st["rechecked_pairs"]
    st, _ = check(P, w, "stress counters", mode="exact", stats=True)
    assert st["tests"] == tests and st["ambiguous_tests"] == 0 and st["rechecked_pairs"] == 0
    # counters restart at every execution
    got, st2, _ = run_plan(P, w, execs=3, mode="filtered", stats=True)
    assert st2["tests"] == tests


def test_batched_force_recheck(P):
    w = W.batched(scale=0.005)
    st, _ = check(P, w, "force recheck", mode="filtered", force_recheck=True, stats=True)
    assert st["rechecked_pairs"] == w.n_points


def test_batched_negative_control(P):
    """With the bound switched off (bound_scale = 0) the binary32 side values
    alone must get some stress pairs wrong: the recheck is load-bearing."""
    w = W.stress(scale=0.02)
    note("batched negative control")
    got, st, _ = run_plan(P, w, mode="filtered", bound_scale=0.0)
    nbad = int(np.count_nonzero(got != oracle.classify_workload(w)))
    note(f"batched negative control mismatches: {nbad}")
    assert nbad > 0


@pytest.mark.parametrize("name", ["footprints", "stress", "batched"])
def test_classify_filtered(P, name):
    """pip_classify in the filtered mode (pooled workspace), twice in a row on
    the same stream, and with the exact batched kernel."""
    import torch
    w = SMALL[name]()
    d = to_dev(w)
    want = oracle.classify_workload(w)
    for rep in range(2):
        note(f"pip_classify filtered {name} rep {rep}")
        got = P.classify(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], mode="filtered")
        torch.cuda.synchronize()
        assert_same_mask(got.cpu().numpy(), want, f"pip_classify filtered {name}", w.px, w.py, w.point_poly)
    got = P.classify(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], kernel="batched")
    torch.cuda.synchronize()
    assert_same_mask(got.cpu().numpy(), want, f"pip_classify batched exact {name}", w.px, w.py, w.point_poly)


@pytest.mark.parametrize("stats", [False, True])
def test_batched_graph_replays(P, stats):
    import torch
    w = W.stress(scale=0.01)
    want = oracle.classify_workload(w)
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], mode="filtered",
                kernel="batched", stats=stats)
    assert pl.config()["use_graph"] == 1
    for r in range(4):
        note(f"batched graph replay {r} stats={stats}")
        pl.out.fill_(7)
        tmp = torch.ones(1 << 20, device="cuda").cumsum(0)
        st = pl.execute(stats=True)
        assert_same_mask(pl.out.cpu().numpy(), want, f"batched replay {r}")
        assert tmp[-1].item() == float(1 << 20)
        assert st["rechecked_pairs"] > 0
    pl.close()


@pytest.mark.parametrize("mode", ["exact", "filtered"])
def test_batched_full_workload(P, mode):
    """The full batched workload (10^8 pairs, rings of 3 .. 4096 vertices), every pair."""
    w = W.batched()
    st, cfg = check(P, w, "batched full", mode=mode, stats=True)
    k, q = ring_sizes(w)
    assert st["tests"] == int(k[q].sum())
    note(f"batched full {mode}: {st}")


def test_batched_full_stress(P):
    st, _ = check(P, W.stress(), "stress full", mode="filtered")
    note(f"stress full (batched kernel) rechecked pairs {st['rechecked_pairs']}")


@pytest.mark.parametrize("kernel", ["batched", "staged"])
@pytest.mark.parametrize("family", ["near-edge", "pow2", "vertex-level", "subnormal"])
def test_filtered_adversarial_families(P, family, kernel):
    """The filtered mode on the adversarial (point, edge) families that the CPU
    soundness test of the bound uses: bit-exact, and the first mismatch named."""
    import torch
    from adversarial import FAMILIES
    w = FAMILIES[family]()
    note(f"adversarial family {family} kernel={kernel} N={w.n_points}")
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], mode="filtered", kernel=kernel)
    pl.execute()
    torch.cuda.synchronize()
    got = pl.out.cpu().numpy()
    st = pl.stats()
    pl.close()
    assert_same_mask(got, oracle.classify_workload(w), f"adversarial {family} {kernel}", w.px, w.py, w.point_poly)
    note(f"adversarial {family} {kernel}: {st['rechecked_pairs']} of {w.n_points} pairs rechecked")
