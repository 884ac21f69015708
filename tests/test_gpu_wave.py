"""GPU parity of the wavefront-per-large-ring form of the filtered batched
step: rings at and around the size threshold (63/64/65 and the larger ones),
4096-vertex rings, a ring whose pairs span several work items, pairs of
several large rings in one item, the form switched off, the device counters,
forced rechecks, graph replays and the adversarial families -- every mask
compared bit for bit with the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same_mask, note, to_dev
from paper_2306_04316_amd import workloads as W
from test_gpu_edges import star_polys

pytestmark = pytest.mark.gpu

AROUND = [3, 8, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 4095, 4096, 4097]


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2306_04316_amd as P
    return P


def run(P, w, execs=1, **opts):
    import torch
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], kernel="batched",
                mode="filtered", **opts)
    cfg = pl.config()
    st = None
    for _ in range(execs):
        pl.out.fill_(7)
        st = pl.execute(stats=True)
    torch.cuda.synchronize()
    got = pl.out.cpu().numpy()
    pl.close()
    return got, st, cfg


def check(P, w, what, **opts):
    note(f"wave {what} {opts} N={w.n_points} P={w.n_polys} V={w.n_vertices}")
    got, st, cfg = run(P, w, **opts)
    assert_same_mask(got, oracle.classify_workload(w), f"wave {what} {opts}", w.px, w.py, w.point_poly)
    return st, cfg


@pytest.mark.parametrize("ppl", [1, 2, 4])
@pytest.mark.parametrize("wave_k", [64, 128, 256, 1024])
def test_wave_threshold_sizes(P, wave_k, ppl):
    w = star_polys(AROUND, 150, seed=11)
    st, cfg = check(P, w, "threshold sizes", wave_k=wave_k, pairs_per_lane=ppl, stats=True)
    assert cfg["wave_k"] == wave_k
    k = np.diff(w.offsets)
    assert st["tests"] == int(k[w.point_poly].sum())


def test_wave_default_and_off(P):
    w = star_polys(AROUND, 150, seed=12)
    _, cfg = check(P, w, "default")
    assert cfg["wave_k"] == 0          # untuned and uncached: off
    _, cfg = check(P, w, "off", wave_k=-1)
    assert cfg["wave_k"] == 0
    _, cfg = check(P, w, "low value", wave_k=5)
    assert cfg["wave_k"] == 64


def test_wave_exact_mode_ignores_threshold(P):
    import torch
    w = star_polys(AROUND, 100, seed=13)
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], kernel="batched", mode="exact",
                wave_k=64)
    assert pl.config()["wave_k"] == 0
    pl.execute()
    torch.cuda.synchronize()
    assert_same_mask(pl.out.cpu().numpy(), oracle.classify_workload(w), "wave exact mode")
    pl.close()


@pytest.mark.parametrize("pts", [1, 63, 64, 65, 300, 1100, 2600])
def test_wave_ring_across_items(P, pts):
    """One 4096-vertex ring and one 200-vertex ring with `pts` points each: the
    large ring's pairs span 1 .. 6 work items and share items with the other."""
    w = star_polys([200, 4096, 70, 4096], pts, seed=pts)
    check(P, w, f"across items pts={pts}", wave_k=128, pairs_per_lane=2)


def test_wave_many_large_rings_per_item(P):
    """Many large rings with few pairs each: several tasks per work item."""
    w = star_polys([64, 300, 65, 700, 128, 2000, 97] * 12, 9, seed=5)
    check(P, w, "many large rings", wave_k=64, pairs_per_lane=4)


def test_wave_counters_and_recheck(P):
    w = W.stress(scale=0.01)
    k = np.diff(w.offsets)
    st, _ = check(P, w, "stress counters", wave_k=64, stats=True)
    assert st["tests"] == int(k[w.point_poly].sum())
    assert st["ambiguous_tests"] > 0 and st["rechecked_pairs"] > 0
    st, _ = check(P, w, "force recheck", wave_k=64, force_recheck=True, stats=True)
    assert st["rechecked_pairs"] == w.n_points


def test_wave_negative_control(P):
    """Bound switched off: the wave form's binary32 side values alone get some
    stress pairs wrong (the recheck is load-bearing there too)."""
    w = W.stress(scale=0.02)
    k = np.diff(w.offsets)
    keep = k[w.point_poly] >= 64
    got, _, _ = run(P, w, wave_k=64, bound_scale=0.0)
    bad = got != oracle.classify_workload(w)
    note(f"wave negative control: {int(bad.sum())} mismatches, {int((bad & keep).sum())} on large rings")
    assert int((bad & keep).sum()) > 0


def test_wave_graph_replays(P):
    import torch
    w = W.stress(scale=0.01)
    want = oracle.classify_workload(w)
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], mode="filtered",
                kernel="batched", wave_k=64)
    assert pl.config()["use_graph"] == 1
    for r in range(4):
        note(f"wave graph replay {r}")
        pl.out.fill_(7)
        tmp = torch.ones(1 << 20, device="cuda").cumsum(0)
        pl.execute()
        torch.cuda.synchronize()
        assert_same_mask(pl.out.cpu().numpy(), want, f"wave replay {r}")
        assert tmp[-1].item() == float(1 << 20)
    pl.close()


def test_wave_unsorted_pairs(P):
    """Pairs not sorted by polygon take the batched kernel's binary64 fallback
    items; sorted runs inside still hand large rings to the wave kernel."""
    w = star_polys(AROUND, 120, seed=21)
    rng = np.random.default_rng(4)
    idx = np.arange(w.n_points)
    cut = w.n_points // 2
    idx[:cut] = rng.permutation(idx[:cut])
    check(P, W.subsample(w, idx), "half shuffled", wave_k=64)


def near_edge_rings(k, n_rings, pts, offset, seed):
    """Star rings of k vertices (offset by `offset`), each with `pts` points a
    few ulps (1 .. 10^4, either side, in x) from a point of a random edge,
    and some exactly on vertices or level with them."""
    import math
    rng = np.random.default_rng(seed)
    vx, vy, off, px, py, pp = [], [], [0], [], [], []
    for q in range(n_rings):
        th = np.sort(rng.uniform(0, 2 * math.pi, k))
        r = rng.uniform(0.5, 1.0, k)
        x, y = offset + 10.0 * q + r * np.cos(th), offset + r * np.sin(th)
        vx.append(x)
        vy.append(y)
        off.append(off[-1] + k)
        j = rng.integers(0, k, pts)
        t = rng.uniform(0.0, 1.0, pts)
        ax, ay, bx, by = x[j - 1], y[j - 1], x[j], y[j]
        qx, qy = ax + t * (bx - ax), ay + t * (by - ay)
        m = np.round(np.exp(rng.uniform(0, math.log(1e4), pts))) * rng.choice([-1, 1], pts)
        qx = qx + m * np.spacing(qx)
        v = rng.integers(0, k, pts // 8)
        qx[: pts // 8], qy[: pts // 8] = x[v], y[v]
        qy[pts // 8: pts // 4] = y[rng.integers(0, k, pts // 4 - pts // 8)]
        px.append(qx)
        py.append(qy)
        pp.append(np.full(pts, q, dtype=np.int32))
    return W.Workload("near-edge rings", np.concatenate(px), np.concatenate(py), np.array(off, dtype=np.int64),
                      np.concatenate(vx), np.concatenate(vy), np.concatenate(pp), {})


@pytest.mark.parametrize("offset", [0.0, 5e6])
@pytest.mark.parametrize("k", [64, 300, 4096])
def test_wave_near_edge_points(P, k, offset):
    """Points within 1 .. 10^4 ulps of edges of large rings (and on vertices,
    level with them), near the origin and offset by 5e6: bit-exact."""
    w = near_edge_rings(k, 12, 400, offset, seed=k)
    st, _ = check(P, w, f"near-edge k={k} offset={offset}", wave_k=64, stats=True)
    note(f"wave near-edge k={k} offset={offset}: {st['rechecked_pairs']} of {w.n_points} rechecked, "
         f"{st['ambiguous_tests']} ambiguous tests")


def test_wave_full_workload(P):
    w = W.batched()
    k = np.diff(w.offsets)
    st, cfg = check(P, w, "batched full", stats=True, wave_k=128)
    assert st["tests"] == int(k[w.point_poly].sum())
    note(f"wave full: {st}")
