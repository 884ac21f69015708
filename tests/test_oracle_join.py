"""Pins for the oracle's candidate-pair generation by bounding box (the paper's
data preparation restricted the points to the polygon's bounding box,
Simulation section; here for many polygons at once)."""
import numpy as np

import pins


def lattice(lo, hi):
    g = np.arange(2 * lo, 2 * hi + 1) / 2.0
    X, Y = np.meshgrid(g, g)
    return X.ravel(), Y.ravel()


def int_polys(seed):
    """Small integer rings (several kinds) plus degenerate ones: a point, a
    horizontal segment, an empty polygon."""
    rings = [(xs, ys) for (xs, ys) in pins.small_integer_polygons(seed=seed, n=30)]
    rings += [(np.array([3]), np.array([-2])), (np.array([-5, 5]), np.array([1, 1])),
              (np.array([], dtype=np.int64), np.array([], dtype=np.int64))]
    off = np.zeros(len(rings) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(r[0]) for r in rings])
    vx = np.concatenate([r[0] for r in rings]).astype(np.float64)
    vy = np.concatenate([r[1] for r in rings]).astype(np.float64)
    return rings, off, vx, vy


def pin_join_integer(oracle, mutant=0):
    """Closed boxes of small integer polygons, computed in Python integers, on
    every integer and half-integer point: exact, listed by polygon then index."""
    rings, off, vx, vy = int_polys(seed=41)
    px, py = lattice(-9, 9)
    pp, pq = oracle.bbox_join(px, py, off, vx, vy, nthreads=4, mutant=mutant)
    want_p, want_q = [], []
    for q, (xs, ys) in enumerate(rings):
        if len(xs) == 0:
            continue
        x0, x1, y0, y1 = min(xs), max(xs), min(ys), max(ys)
        for i in range(px.size):
            if x0 <= px[i] <= x1 and y0 <= py[i] <= y1:
                want_p.append(i)
                want_q.append(q)
    return np.array_equal(pp, np.array(want_p)) and np.array_equal(pq, np.array(want_q))


def test_join_integer_closed_form(oracle_mod):
    assert pin_join_integer(oracle_mod)


def test_join_mutant_caught(oracle_mod):
    assert not pin_join_integer(oracle_mod, mutant=9)


def test_join_contains_every_inside_pair(oracle_mod):
    """On integer polygons (exact float64 arithmetic) the classification oracle's
    inside points of a polygon are a subset of its candidates."""
    rings, off, vx, vy = int_polys(seed=43)
    px, py = lattice(-9, 9)
    pp, pq = oracle_mod.bbox_join(px, py, off, vx, vy)
    cand = set(zip(pp.tolist(), pq.tolist()))
    for q in range(len(rings)):
        inside = oracle_mod.classify(px, py, off, vx, vy, np.full(px.size, q, dtype=np.int32))
        for i in np.nonzero(inside)[0]:
            assert (int(i), q) in cand


def test_join_rings_use_every_ring(oracle_mod):
    """A polygon's box covers all its rings (a detached part widens it)."""
    from paper_2306_04316_amd import workloads as W
    w = W.holes(scale=0.002, seed=3, p_part=1.0)
    pp, pq = oracle_mod.bbox_join(w.px, w.py, w.offsets, w.vx, w.vy, poly_rings=w.poly_rings)
    for q in range(w.n_polys):
        b, e = w.offsets[w.poly_rings[q]], w.offsets[w.poly_rings[q + 1]]
        x0, x1, y0, y1 = w.vx[b:e].min(), w.vx[b:e].max(), w.vy[b:e].min(), w.vy[b:e].max()
        mine = (w.point_poly == q)
        want = np.nonzero((w.px >= x0) & (w.px <= x1) & (w.py >= y0) & (w.py <= y1))[0]
        assert np.array_equal(np.sort(pp[pq == q]), want)
        # the points drawn for q inside its box are all candidates of q
        assert set(np.nonzero(mine & (w.px >= x0) & (w.px <= x1) & (w.py >= y0) & (w.py <= y1))[0]) <= set(want)


def test_join_point_permutation(oracle_mod):
    """Permuting the points permutes the candidates (the same pairs)."""
    rings, off, vx, vy = int_polys(seed=45)
    px, py = lattice(-6, 6)
    perm = np.random.default_rng(1).permutation(px.size)
    a_p, a_q = oracle_mod.bbox_join(px, py, off, vx, vy)
    b_p, b_q = oracle_mod.bbox_join(px[perm], py[perm], off, vx, vy)
    assert sorted(zip(a_q.tolist(), a_p.tolist())) == sorted(zip(b_q.tolist(), perm[b_p].tolist()))
