"""Seeded generators: shapes, determinism and the properties each recipe promises."""
import numpy as np

from paper_2306_04316_amd import workloads as W


def test_star_recipe():
    w = W.star()
    assert w.n_points == 100_000 and w.n_vertices == 64 and w.point_poly is None
    th = np.arctan2(w.vy, w.vx) % (2 * np.pi)
    assert np.all(np.diff(th) > 0)
    r = np.hypot(w.vx, w.vy)
    assert r.min() >= 0.5 and r.max() <= 1.0
    assert w.px.min() >= w.vx.min() and w.px.max() <= w.vx.max()


def test_deterministic():
    a, b = W.footprints(scale=0.01), W.footprints(scale=0.01)
    for f in ("px", "py", "offsets", "vx", "vy", "point_poly"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = W.footprints(scale=0.01, seed=1)
    assert not np.array_equal(a.px, c.px)


def test_footprints_recipe():
    w = W.footprints(scale=0.05)
    k = np.diff(w.offsets)
    assert k.min() >= 4 and k.max() <= 32
    assert w.n_points == 100 * w.n_polys
    assert np.all(np.diff(w.point_poly) >= 0)
    assert w.vx.min() > -0.01 and w.vx.max() < 2.01 and w.vy.min() > 4.99 and w.vy.max() < 7.01


def test_fractal_exact_vertex_count():
    w = W.fractal(scale=0.001, n_vertices=5000)
    assert w.n_vertices == 5000 and w.n_points == 10_000
    full = W.fractal(scale=0.0)
    assert full.n_vertices == 1_000_000


def test_batched_power_law():
    w = W.batched(scale=0.02)
    k = np.diff(w.offsets)
    assert k.min() >= 3 and k.max() <= 4096
    assert 14 < k.mean() < 24          # E[k] = 18.7 for the discrete k^-2 law on [3, 4096]
    assert np.all(np.diff(w.point_poly) >= 0)
    assert abs(w.n_points / w.n_polys - 100) < 3


def test_stress_classes():
    w = W.stress(scale=0.01)
    s = w.offsets[:-1]
    assert np.all(w.vy[s] == w.vy[s + 1])                    # edge 0 horizontal
    assert w.vx.min() > 4.99e6
    n = w.params["n_class"]
    assert sum(n) == w.n_points and n[2] > 0 and n[3] > 0
    # class 2 points are bitwise copies of vertices
    verts = set(zip(w.vx.tolist(), w.vy.tolist()))
    hits = sum((x, y) in verts for x, y in zip(w.px.tolist(), w.py.tolist()))
    assert hits >= n[2]
