"""Pins for the oracle's polygons of several rings (holes, detached parts): the
even-odd rule over all edges of all rings, each ring closed on itself."""
import numpy as np
import pytest

import exact_geom as X
import pins
from paper_2306_04316_amd import workloads as W


def multi_ring_cases(seed=31, n=40):
    """Small integer polygons of 2..4 rings drawn from the single-ring kinds."""
    rings = pins.small_integer_polygons(seed=seed, n=4 * n)
    rng = np.random.default_rng(seed)
    out, i = [], 0
    for _ in range(n):
        m = int(rng.integers(2, 5))
        out.append(rings[i:i + m])
        i += m
    return out


def pack(rings):
    xs = np.concatenate([r[0] for r in rings]).astype(np.float64)
    ys = np.concatenate([r[1] for r in rings]).astype(np.float64)
    off = np.zeros(len(rings) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(r[0]) for r in rings])
    return xs, ys, off


def pin_rings_winding(oracle, mutant=0):
    """Off every ring's boundary, the parity is (sum of the rings' exact winding
    numbers) mod 2; on a boundary, the XOR of the exact integer rule per ring."""
    fails = []
    for rings in multi_ring_cases():
        allx = np.concatenate([r[0] for r in rings])
        ally = np.concatenate([r[1] for r in rings])
        gx = np.arange(2 * (allx.min() - 1), 2 * (allx.max() + 1) + 1)
        gy = np.arange(2 * (ally.min() - 1), 2 * (ally.max() + 1) + 1)
        GX, GY = np.meshgrid(gx, gy)
        qx2, qy2 = GX.ravel(), GY.ravel()
        wsum = np.zeros(qx2.shape, dtype=np.int64)
        onb = np.zeros(qx2.shape, dtype=bool)
        rule = np.zeros(qx2.shape, dtype=np.int64)
        for (rx, ry) in rings:
            wsum += X.winding_int(qx2, qy2, 2 * rx, 2 * ry)
            onb |= X.on_boundary_int(qx2, qy2, 2 * rx, 2 * ry)
            rule ^= X.halfopen_rule_int(qx2, qy2, 2 * rx, 2 * ry).astype(np.int64)
        want = np.where(onb, rule, np.abs(wsum) % 2).astype(np.uint8)
        vx, vy, off = pack(rings)
        got = oracle.classify_rings(qx2 / 2.0, qy2 / 2.0, np.array([0, len(rings)]), off, vx, vy, nthreads=4,
                                    mutant=mutant)
        if not np.array_equal(got, want):
            fails.append(len(rings))
    return fails


def test_rings_winding(oracle_mod):
    assert pin_rings_winding(oracle_mod) == []


def test_rings_mutant_caught(oracle_mod):
    """A planted mistake -- the rings walked as one chain -- fails the pin."""
    assert pin_rings_winding(oracle_mod, mutant=8) != []


def test_one_ring_per_polygon_is_the_single_ring_rule(oracle_mod):
    w = W.footprints(scale=0.01, seed=4)
    a = oracle_mod.classify_workload(w)
    b = oracle_mod.classify_rings(w.px, w.py, np.arange(w.n_polys + 1), w.offsets, w.vx, w.vy, w.point_poly)
    assert np.array_equal(a, b)
    c2a = oracle_mod.classify_workload(w, predicate=2)
    c2b = oracle_mod.classify_rings(w.px, w.py, np.arange(w.n_polys + 1), w.offsets, w.vx, w.vy, w.point_poly,
                                    predicate=2)
    assert np.array_equal(c2a, c2b)


def test_ring_order_and_start_vertex_do_not_matter(oracle_mod):
    """Bit-exact for any float64 input: each edge is evaluated identically."""
    w = W.holes(scale=0.005, seed=2)
    want = oracle_mod.classify_workload(w)
    rng = np.random.default_rng(7)
    vx, vy, off, pr = [], [], [0], [0]
    for q in range(w.n_polys):
        rs = list(range(w.poly_rings[q], w.poly_rings[q + 1]))
        rng.shuffle(rs)
        for r in rs:
            x = w.vx[w.offsets[r]:w.offsets[r + 1]]
            y = w.vy[w.offsets[r]:w.offsets[r + 1]]
            s = int(rng.integers(0, x.size))
            vx.append(np.roll(x, s))
            vy.append(np.roll(y, s))
            off.append(off[-1] + x.size)
        pr.append(pr[-1] + len(rs))
    got = oracle_mod.classify_rings(w.px, w.py, np.array(pr), np.array(off), np.concatenate(vx),
                                    np.concatenate(vy), w.point_poly)
    assert np.array_equal(got, want)


def test_holes_exact_rational(oracle_mod):
    """On a sample of the holes workload, the exact-rational even-odd rule over all
    rings agrees wherever every straddling edge is certified by the float64 bound."""
    w = W.holes(scale=0.01, seed=5)
    got = oracle_mod.classify_workload(w)
    idx = np.random.default_rng(3).choice(w.n_points, 3000, replace=False)
    unc = 0
    for i in idx:
        q = int(w.point_poly[i])
        par, cert = 0, True
        for r in range(w.poly_rings[q], w.poly_rings[q + 1]):
            b, e = w.offsets[r], w.offsets[r + 1]
            p, c = X.exact_rule_parity_f64(float(w.px[i]), float(w.py[i]), w.vx[b:e], w.vy[b:e])
            par ^= p
            cert &= c
        if cert:
            assert got[i] == par, i
        else:
            unc += 1
    assert unc < 30


def test_holes_workload_shape():
    w = W.holes(scale=0.01, seed=0)
    assert w.poly_rings[0] == 0 and w.poly_rings[-1] == w.n_rings
    assert np.all(np.diff(w.poly_rings) >= 1) and np.all(np.diff(w.offsets) >= 4)
    frac_multi = np.mean(np.diff(w.poly_rings) > 1)
    assert 0.45 < frac_multi < 0.75
    assert w.n_tests == int(np.sum(w.edges_per_pair()))


def test_rings_rejects_bad_arguments(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.classify_rings(np.zeros(2), np.zeros(2), np.array([0, 5]), np.array([0, 4]),
                                  np.zeros(4), np.zeros(4))
