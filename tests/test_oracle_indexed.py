"""The oracle's indexed mode for one ring (edges that cannot straddle a point's
ray skipped through an exact y index) against the plain double loop: the same
bits on every pair, on rings with horizontal edges, repeated vertices, a
degenerate y range, points level with vertices and outside the ring's y
range, and on samples of the fractal workload (the one it is used for)."""
import numpy as np
import pytest

import oracle
from paper_2306_04316_amd import workloads as W


def both(px, py, vx, vy, nthreads=4):
    off = np.array([0, len(vx)], dtype=np.int64)
    plain = oracle.classify(px, py, off, vx, vy, None, nthreads=nthreads)
    idx = oracle.classify_indexed(px, py, off, vx, vy, nthreads=nthreads)
    return plain, idx


def test_indexed_equals_plain_on_small_rings():
    rng = np.random.default_rng(21)
    rings = [
        ([0.0], [0.0]),
        ([0.0, 1.0], [0.0, 1.0]),
        ([0.0, 2.0, 2.0, 0.0], [0.0, 0.0, 0.0, 0.0]),   # no y range at all
        ([0.0, 3.0, 3.0, 1.5, 1.5, 1.5, 0.0], [0.0, 0.0, 1.0, 1.0, 3.0, 1.0, 1.0]),
        ([0.0, 1.0, 2.0, 2.0, 1.0, 0.0, 0.0], [0.0, 0.0, 0.0, 2.0, 2.0, 2.0, 0.0]),
        ([0.0, 2.0, 0.0, 2.0], [0.0, 2.0, 2.0, 0.0]),
    ]
    for rx, ry in rings:
        vx, vy = np.array(rx), np.array(ry)
        px = rng.uniform(-1, 4, 4000)
        py = rng.uniform(-1, 4, 4000)
        py[:1000] = rng.choice(vy, 1000)          # level with vertices
        px[1000:1200] = rng.choice(vx, 200)
        py[1000:1200] = rng.choice(vy, 200)
        plain, idx = both(px, py, vx, vy)
        assert np.array_equal(plain, idx), (rx, ry)


@pytest.mark.parametrize("k", [3, 64, 1000, 20000])
def test_indexed_equals_plain_on_stars(k):
    rng = np.random.default_rng(k)
    th = np.sort(rng.uniform(0, 2 * np.pi, k))
    r = rng.uniform(0.5, 1.0, k)
    vx, vy = 5e6 + r * np.cos(th), 5e6 + r * np.sin(th)
    px = 5e6 + rng.uniform(-1.2, 1.2, 20000)
    py = 5e6 + rng.uniform(-1.2, 1.2, 20000)
    py[:3000] = vy[rng.integers(0, k, 3000)]
    px[3000:4000] = vx[rng.integers(0, k, 1000)]
    py[3000:4000] = vy[rng.integers(0, k, 1000)]
    plain, idx = both(px, py, vx, vy)
    assert np.array_equal(plain, idx)


def test_indexed_equals_plain_on_fractal_sample():
    w = W.fractal(scale=0.0005, n_vertices=200_000)
    plain, idx = both(w.px, w.py, w.vx, w.vy, nthreads=8)
    assert np.array_equal(plain, idx)
    assert 0 < plain.sum() < plain.size


def test_indexed_mode_catches_planted_mistakes():
    """The indexed mode applies the same per-edge rule: a planted mistake in the
    rule shows up in it too (here the dropped-orientation mutant on a square)."""
    vx = np.array([0.0, 1.0, 1.0, 0.0])
    vy = np.array([0.0, 0.0, 1.0, 1.0])
    px = np.array([0.5, 2.0, -1.0])
    py = np.array([0.5, 0.5, 0.5])
    off = np.array([0, 4], dtype=np.int64)
    good = oracle.classify_indexed(px, py, off, vx, vy, nthreads=1)
    assert good.tolist() == [1, 0, 0]
    oracle.build(3, force=False)
    bad = oracle.classify_indexed(px, py, off, vx, vy, nthreads=1, mutant=3)
    assert bad.tolist() != good.tolist()
