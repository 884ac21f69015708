"""GPU parity for polygons of several rings (holes, detached parts): the staged
and per-pair kernels, one-shot and as plans, against the oracle bit for bit."""
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


def run_classify(P, w, **kw):
    import torch
    d = to_dev(w)
    got = P.classify_rings(d["px"], d["py"], d["poly_rings"], d["offsets"], d["vx"], d["vy"], d["point_poly"], **kw)
    torch.cuda.synchronize()
    return got.cpu().numpy()


def run_plan(P, w, **kw):
    import torch
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], poly_rings=d["poly_rings"], **kw)
    pl.execute()
    torch.cuda.synchronize()
    got = pl.out.cpu().numpy()
    cfg = pl.config()
    pl.close()
    return got, cfg


def pred_num(predicate):
    return 2 if predicate == "intersection" else 1


@pytest.mark.parametrize("predicate", ["side", "intersection"])
@pytest.mark.parametrize("kernel", ["auto", "staged", "per_pair"])
@pytest.mark.parametrize("scale", [0.003, 0.05])
def test_rings_classify(P, kernel, predicate, scale):
    w = W.holes(scale=scale, seed=1)
    note(f"rings classify kernel={kernel} predicate={predicate} P={w.n_polys} R={w.n_rings}")
    got = run_classify(P, w, kernel=kernel, predicate=predicate)
    assert_same_mask(got, oracle.classify_workload(w, predicate=pred_num(predicate)), f"rings {kernel}",
                     w.px, w.py, w.point_poly)


@pytest.mark.parametrize("ppl", [1, 2, 4])
@pytest.mark.parametrize("lds", [16, 64, 512])
def test_rings_tiles_and_fallback(P, ppl, lds):
    """Small LDS budgets send items to the scalar-load group walk."""
    w = W.holes(scale=0.01, seed=2)
    note(f"rings tiles ppl={ppl} lds={lds}")
    got = run_classify(P, w, kernel="staged", pairs_per_lane=ppl, lds_slots=lds)
    assert_same_mask(got, oracle.classify_workload(w), f"rings ppl={ppl} lds={lds}", w.px, w.py, w.point_poly)


def test_rings_one_ring_each_matches_classify(P):
    import torch
    w = W.footprints(scale=0.01, seed=3)
    d = to_dev(w)
    pr = torch.arange(w.n_polys + 1, dtype=torch.int64, device="cuda")
    a = P.classify_rings(d["px"], d["py"], pr, d["offsets"], d["vx"], d["vy"], d["point_poly"], kernel="staged")
    b = P.classify(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], kernel="staged")
    torch.cuda.synchronize()
    assert_same_mask(a.cpu().numpy(), b.cpu().numpy(), "one ring each")
    assert_same_mask(a.cpu().numpy(), oracle.classify_workload(w), "one ring each vs oracle")


@pytest.mark.parametrize("opts", [dict(), dict(persistent=1), dict(order=1), dict(persistent=1, order=1),
                                  dict(use_graph=False), dict(kernel="per_pair"), dict(predicate="intersection")])
def test_rings_plan(P, opts):
    w = W.holes(scale=0.02, seed=4)
    note(f"rings plan {opts}")
    got, cfg = run_plan(P, w, **opts)
    want = oracle.classify_workload(w, predicate=pred_num(opts.get("predicate", "side")))
    assert_same_mask(got, want, f"rings plan {opts}", w.px, w.py, w.point_poly)


def test_rings_plan_tuned(P, tmp_path):
    w = W.holes(scale=0.02, seed=5)
    got, cfg = run_plan(P, w, tune=1, tune_cache=str(tmp_path / "t.txt"))
    assert cfg["kernel"] == 3
    assert_same_mask(got, oracle.classify_workload(w), "rings tuned", w.px, w.py, w.point_poly)
    assert ":rings" in open(tmp_path / "t.txt").read()


def test_rings_full(P):
    w = W.holes()
    note(f"rings full N={w.n_points} P={w.n_polys} R={w.n_rings}")
    got, cfg = run_plan(P, w)
    assert_same_mask(got, oracle.classify_workload(w), "rings full", w.px, w.py, w.point_poly)


def test_rings_degenerate(P):
    """Polygons with no ring, rings of 0..2 vertices, a large ring with a hole
    (too large to stage), repeated and level vertices."""
    rng = np.random.default_rng(8)
    rings = [
        [],                                                     # polygon 0: no ring
        [[(0, 0), (4, 0), (4, 4), (0, 4)], [(1, 1), (1, 3), (3, 3), (3, 1)]],
        [[(0, 0)], [(0, 0), (2, 2)], [], [(0, 0), (4, 0), (4, 4), (0, 4)]],
        [[(float(np.cos(t)) * 3, float(np.sin(t)) * 3) for t in np.linspace(0, 6.2, 3000)],
         [(-1, -1), (-1, 1), (1, 1), (1, -1)], [(0, 0), (0.5, 0), (0.5, 0.5)]],
        [[(0, 0), (2, 0), (2, 2), (0, 2)], [(0, 0), (2, 0), (2, 2), (0, 2)]],   # a ring and its copy
    ]
    vx, vy, roff, prings = [], [], [0], [0]
    for poly in rings:
        for ring in poly:
            vx += [float(a) for a, _ in ring]
            vy += [float(b) for _, b in ring]
            roff.append(roff[-1] + len(ring))
        prings.append(prings[-1] + len(poly))
    n = 20000
    pp = np.sort(rng.integers(0, len(rings), n)).astype(np.int32)
    px = rng.uniform(-4, 5, n)
    py = rng.uniform(-4, 5, n)
    py[::7] = np.round(py[::7])          # level with vertices and horizontal edges
    px[::11] = np.round(px[::11])
    w = W.Workload("rings-degenerate", px, py, np.array(roff, dtype=np.int64), np.array(vx), np.array(vy), pp, {},
                   poly_rings=np.array(prings, dtype=np.int64))
    want = oracle.classify_workload(w)
    for kernel in ("staged", "per_pair"):
        for lds in (64, 4096):
            got = run_classify(P, w, kernel=kernel, lds_slots=lds)
            assert_same_mask(got, want, f"rings degenerate {kernel} lds={lds}", w.px, w.py, w.point_poly)
    got, _ = run_plan(P, w)
    assert_same_mask(got, want, "rings degenerate plan", w.px, w.py, w.point_poly)


def test_rings_rejections(P):
    import torch
    w = W.holes(scale=0.002)
    d = to_dev(w)
    for kernel in ("segmented", "runs"):
        with pytest.raises(P.PipError) as e:
            P.classify_rings(d["px"], d["py"], d["poly_rings"], d["offsets"], d["vx"], d["vy"], d["point_poly"],
                             kernel=kernel)
        assert e.value.code == -6
    with pytest.raises(P.PipError) as e:
        P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], poly_rings=d["poly_rings"],
               mode="filtered")
    assert e.value.code == -6
    bad = d["poly_rings"].clone()
    bad[1] = bad[2] + 1   # not monotone
    with pytest.raises(P.PipError) as e:
        P.classify_rings(d["px"], d["py"], bad, d["offsets"], d["vx"], d["vy"], d["point_poly"], validate=True)
    assert e.value.code == -2


@pytest.mark.parametrize("predicate", ["side", "intersection"])
@pytest.mark.parametrize("lds", [64, 256])
def test_rings_one_pass_boundary(P, predicate, lds):
    """Polygons whose rings together hold 31, 32 and 33 vertices (one-pass path
    on both sides of the chunk size), rings of 1-3 vertices among them, and
    points on and level with vertices: one pass or ring by ring, same bits."""
    rng = np.random.default_rng(21)
    vx, vy, roff, prings, px, py, pp = [], [], [0], [0], [], [], []
    q = 0
    for total in (31, 32, 33, 30, 32, 34):
        sizes = []
        left = total
        while left > 0:
            s = int(min(left, rng.integers(1, 12)))
            sizes.append(s)
            left -= s
        cx = 5.0 * q
        for r, s in enumerate(sizes):
            t = np.sort(rng.uniform(0, 2 * np.pi, s))
            rad = rng.uniform(0.3, 1.0, s) * (1.0 if r == 0 else 0.4)
            x, y = cx + rad * np.cos(t), rad * np.sin(t)
            vx += list(x)
            vy += list(y)
            roff.append(roff[-1] + s)
        prings.append(prings[-1] + len(sizes))
        m = 700
        qx = rng.uniform(cx - 1.1, cx + 1.1, m)
        qy = rng.uniform(-1.1, 1.1, m)
        lo, hi = roff[prings[q]], roff[prings[q + 1]]
        j = rng.integers(lo, hi, m // 5)
        qy[: m // 5] = np.array(vy)[j]                          # level with vertices
        qx[: m // 10] = np.array(vx)[j[: m // 10]]              # on vertices
        px.append(qx)
        py.append(qy)
        pp.append(np.full(m, q, dtype=np.int32))
        q += 1
    w = W.Workload("rings-one-pass", np.concatenate(px), np.concatenate(py), np.array(roff, dtype=np.int64),
                   np.array(vx), np.array(vy), np.concatenate(pp), {}, poly_rings=np.array(prings, dtype=np.int64))
    note(f"rings one pass predicate={predicate} lds={lds}")
    want = oracle.classify_workload(w, predicate=pred_num(predicate))
    got = run_classify(P, w, kernel="staged", lds_slots=lds, predicate=predicate)
    assert_same_mask(got, want, f"rings one pass {predicate} lds={lds}", w.px, w.py, w.point_poly)
