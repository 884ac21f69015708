"""GPU parity of candidate-pair generation by bounding box (pip_join_*): the
pair set equals the oracle's brute-force join exactly, grouped by polygon."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same_mask, note
from paper_2306_04316_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2306_04316_amd as P
    return P


def gpu_join(P, px, py, offsets, vx, vy, poly_rings=None):
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = P.candidate_pairs(t(px), t(py), t(offsets), t(vx), t(vy), None if poly_rings is None else t(poly_rings))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def check_join(got, px, py, want_p, want_q, what):
    assert got["point"].size == want_p.size, f"{what}: {got['point'].size} pairs vs {want_p.size}"
    assert np.all(np.diff(got["poly"]) >= 0), f"{what}: not grouped by polygon"
    a = np.lexsort((got["point"], got["poly"]))
    assert np.array_equal(got["poly"][a], want_q), what
    assert np.array_equal(got["point"][a], want_p), what
    assert np.array_equal(got["px"], px[got["point"]]) and np.array_equal(got["py"], py[got["point"]]), what


@pytest.mark.parametrize("scale", [0.002, 0.02])
def test_join_footprints(P, scale):
    w = W.raw_points(W.footprints(scale=scale, seed=2))
    note(f"join footprints N={w.n_points} P={w.n_polys}")
    got = gpu_join(P, w.px, w.py, w.offsets, w.vx, w.vy)
    wp, wq = oracle.bbox_join(w.px, w.py, w.offsets, w.vx, w.vy)
    check_join(got, w.px, w.py, wp, wq, "join footprints")


def test_join_rings(P):
    w = W.raw_points(W.holes(scale=0.01, seed=3, p_part=0.5))
    got = gpu_join(P, w.px, w.py, w.offsets, w.vx, w.vy, w.poly_rings)
    wp, wq = oracle.bbox_join(w.px, w.py, w.offsets, w.vx, w.vy, poly_rings=w.poly_rings)
    check_join(got, w.px, w.py, wp, wq, "join rings")


def test_join_degenerate(P):
    """Points on box edges (integer lattice), empty polygons, a point polygon, a
    segment, polygons outside the points' extent, one polygon over everything,
    duplicate points."""
    g = np.arange(-20, 21) / 2.0
    X, Y = np.meshgrid(g, g)
    px = np.concatenate([X.ravel(), np.full(50, 1.0)])
    py = np.concatenate([Y.ravel(), np.full(50, 2.0)])
    rings = [[(0, 0), (4, 0), (4, 3), (0, 3)], [], [(1, 2)], [(-3, 1), (5, 1)], [(100, 100), (101, 100), (101, 101)],
             [(-50, -50), (50, -50), (50, 50)], [(2.5, -1.5), (3.5, -1.5), (3, 9)], []]
    off = np.zeros(len(rings) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(r) for r in rings])
    vx = np.array([a for r in rings for a, _ in r], dtype=np.float64)
    vy = np.array([b for r in rings for _, b in r], dtype=np.float64)
    got = gpu_join(P, px, py, off, vx, vy)
    wp, wq = oracle.bbox_join(px, py, off, vx, vy)
    check_join(got, px, py, wp, wq, "join degenerate")
    # all points identical
    got = gpu_join(P, np.full(1000, 0.5), np.full(1000, 0.5), off, vx, vy)
    wp, wq = oracle.bbox_join(np.full(1000, 0.5), np.full(1000, 0.5), off, vx, vy)
    check_join(got, np.full(1000, 0.5), np.full(1000, 0.5), wp, wq, "join identical points")
    # no points
    got = gpu_join(P, np.zeros(0), np.zeros(0), off, vx, vy)
    assert got["point"].size == 0


def test_join_clustered_points(P):
    """Most points in one grid cell, many times a sort piece (4,096 points in
    the coarse pass, 2,048 in the fine pass) and across several 16,384-point
    chunks, beside a tight cluster and a spread; boxes over the cluster,
    beside it and over everything."""
    rng = np.random.default_rng(8)
    px = np.concatenate([np.full(40_000, 0.25), 0.25 + rng.uniform(-1e-7, 1e-7, 10_000), rng.uniform(-5, 5, 20_000)])
    py = np.concatenate([np.full(40_000, -0.5), -0.5 + rng.uniform(-1e-7, 1e-7, 10_000), rng.uniform(-5, 5, 20_000)])
    perm = rng.permutation(px.size)
    px, py = px[perm], py[perm]
    rings = [[(0.2, -0.6), (0.3, -0.6), (0.3, -0.4), (0.2, -0.4)], [(0.25, -0.5), (0.26, -0.5), (0.26, -0.49)],
             [(1.0, 1.0), (2.0, 1.0), (2.0, 2.0)], [(-6, -6), (6, -6), (6, 6), (-6, 6)],
             [(0.25 - 1e-8, -0.5 - 1e-8), (0.25 + 1e-8, -0.5 - 1e-8), (0.25, -0.5 + 1e-8)]]
    off = np.zeros(len(rings) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(r) for r in rings])
    vx = np.array([a for r in rings for a, _ in r], dtype=np.float64)
    vy = np.array([b for r in rings for _, b in r], dtype=np.float64)
    note(f"join clustered N={px.size}")
    got = gpu_join(P, px, py, off, vx, vy)
    wp, wq = oracle.bbox_join(px, py, off, vx, vy)
    check_join(got, px, py, wp, wq, "join clustered")


def test_join_one_large_polygon(P):
    """The paper's preparation step: many points against one large polygon's box."""
    w = W.fractal(scale=0.01, n_vertices=50_000)
    rng = np.random.default_rng(4)
    px = rng.uniform(-4, 4, 200_000)
    py = rng.uniform(4, 12, 200_000)
    got = gpu_join(P, px, py, w.offsets, w.vx, w.vy)
    wp, wq = oracle.bbox_join(px, py, w.offsets, w.vx, w.vy)
    check_join(got, px, py, wp, wq, "join one polygon")


def test_join_full_footprints_sampled(P):
    """10^7 raw points x 10^5 polygons: every sampled point's candidate polygons
    equal the brute-force join of that point."""
    w = W.raw_points(W.footprints())
    note(f"join full N={w.n_points} P={w.n_polys}")
    got = gpu_join(P, w.px, w.py, w.offsets, w.vx, w.vy)
    assert np.all(np.diff(got["poly"]) >= 0)
    idx = np.sort(np.random.default_rng(5).choice(w.n_points, 3000, replace=False))
    wp, wq = oracle.bbox_join(w.px[idx], w.py[idx], w.offsets, w.vx, w.vy)
    sel = np.isin(got["point"], idx)
    gp, gq = got["point"][sel], got["poly"][sel]
    a = np.lexsort((gp, gq))
    assert np.array_equal(gq[a], wq) and np.array_equal(gp[a], idx[wp])
    note(f"join full pairs {got['point'].size}")


def test_join_then_classify(P):
    """Candidate pairs straight into a plan: the masks match the oracle's."""
    import torch
    w = W.raw_points(W.holes(scale=0.02, seed=6))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    d = dict(offsets=t(w.offsets), vx=t(w.vx), vy=t(w.vy), poly_rings=t(w.poly_rings))
    c = P.candidate_pairs(t(w.px), t(w.py), d["offsets"], d["vx"], d["vy"], d["poly_rings"])
    pl = P.Plan(c["px"], c["py"], d["offsets"], d["vx"], d["vy"], c["poly"], poly_rings=d["poly_rings"])
    pl.execute()
    torch.cuda.synchronize()
    got = pl.out.cpu().numpy()
    pl.close()
    want = oracle.classify_rings(c["px"].cpu().numpy(), c["py"].cpu().numpy(), w.poly_rings, w.offsets, w.vx, w.vy,
                                 c["poly"].cpu().numpy())
    assert_same_mask(got, want, "join then classify")
    assert want.mean() > 0.3
