"""GPU parity at the kernels' structural boundaries: ring sizes around the
32-vertex chunk and the LDS edge budget, work items holding exactly as many
rings as a workgroup stages (and one more), ragged pair counts -- every
kernel and both crossing tests, bit for bit against the oracle."""
import math

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


def star_polys(ks, pts_each, seed=0):
    """Star-shaped rings of the given sizes (one polygon each), pts_each points per
    polygon uniform in its bbox x1.2, a few of them on vertices and level with them."""
    rng = np.random.default_rng(seed)
    vx, vy, off, px, py, pp = [], [], [0], [], [], []
    for q, k in enumerate(ks):
        th = np.sort(rng.uniform(0, 2 * math.pi, k))
        r = rng.uniform(0.5, 1.0, k)
        cx, cy = 10.0 * q, 3.0
        x, y = cx + r * np.cos(th), cy + r * np.sin(th)
        vx.append(x)
        vy.append(y)
        off.append(off[-1] + k)
        m = pts_each
        qx = rng.uniform(x.min() - 0.1, x.max() + 0.1, m)
        qy = rng.uniform(y.min() - 0.1, y.max() + 0.1, m)
        j = rng.integers(0, k, m // 8)
        qx[: m // 8], qy[: m // 8] = x[j], y[j]                 # on vertices
        qy[m // 8: m // 4] = y[rng.integers(0, k, m // 4 - m // 8)]   # level with vertices
        px.append(qx)
        py.append(qy)
        pp.append(np.full(m, q, dtype=np.int32))
    return W.Workload("stars", np.concatenate(px), np.concatenate(py), np.array(off, dtype=np.int64),
                      np.concatenate(vx), np.concatenate(vy), np.concatenate(pp), {})


KS = [3, 4, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 2047, 2048]


@pytest.mark.parametrize("predicate", ["side", "intersection"])
@pytest.mark.parametrize("kernel,lds", [("staged", 64), ("staged", 512), ("staged", 2048), ("runs", 0),
                                        ("per_pair", 0), ("segmented", 0)])
def test_ring_sizes_at_boundaries(P, kernel, lds, predicate):
    import torch
    w = star_polys(KS, 300, seed=1)
    note(f"ring sizes kernel={kernel} lds={lds} predicate={predicate}")
    d = to_dev(w)
    got = P.classify(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], kernel=kernel,
                     lds_slots=lds, predicate=predicate)
    torch.cuda.synchronize()
    want = oracle.classify_workload(w, predicate=2 if predicate == "intersection" else 1)
    assert_same_mask(got.cpu().numpy(), want, f"ring sizes {kernel} lds={lds}", w.px, w.py, w.point_poly)


@pytest.mark.parametrize("ppl", [1, 4])
@pytest.mark.parametrize("lds", [16, 64, 256, 1024, 2048])
def test_ring_sizes_at_boundaries_filtered(P, lds, ppl):
    """The filtered mode across the same ring sizes: items that fit its binary32
    layout are filtered, larger ones take the binary64 tile walk in the same LDS."""
    import torch
    w = star_polys(KS, 300, seed=2)
    note(f"ring sizes filtered lds={lds} ppl={ppl}")
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], mode="filtered",
                kernel="staged", lds_slots=lds, pairs_per_lane=ppl, persistent=0, order=0, use_graph=False)
    pl.execute()
    torch.cuda.synchronize()
    got = pl.out.cpu().numpy()
    pl.close()
    want = oracle.classify_workload(w)
    assert_same_mask(got, want, f"ring sizes filtered lds={lds} ppl={ppl}", w.px, w.py, w.point_poly)


@pytest.mark.parametrize("pairs_per_poly", [8, 7])
@pytest.mark.parametrize("ppl", [1, 2, 4])
def test_rings_per_item_limit(P, pairs_per_poly, ppl):
    """256*ppl pairs per item with 8 pairs per polygon fill an item with exactly
    32*ppl rings (128 at ppl = 4, the staging limit); 7 pairs per polygon put one
    more ring in some items."""
    import torch
    n_polys = 4096
    w = star_polys([4 + (q % 5) for q in range(n_polys)], pairs_per_poly, seed=2)
    note(f"rings per item: {pairs_per_poly} pairs per polygon, ppl={ppl}")
    d = to_dev(w)
    got = P.classify(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], kernel="staged",
                     pairs_per_lane=ppl, lds_slots=2048)
    torch.cuda.synchronize()
    assert_same_mask(got.cpu().numpy(), oracle.classify_workload(w), "rings per item", w.px, w.py, w.point_poly)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025, 4095, 4097])
def test_ragged_pair_counts(P, n):
    import torch
    base = W.footprints(scale=0.002, seed=7)
    s = W.subsample(base, np.arange(min(n, base.n_points)))
    d = to_dev(s)
    for kernel in ("staged", "runs", "segmented", "per_pair"):
        got = P.classify(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], kernel=kernel)
        torch.cuda.synchronize()
        assert_same_mask(got.cpu().numpy(), oracle.classify_workload(s), f"ragged n={n} {kernel}")
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], mode="filtered")
    pl.execute()
    torch.cuda.synchronize()
    assert_same_mask(pl.out.cpu().numpy(), oracle.classify_workload(s), f"ragged n={n} filtered")
    pl.close()
