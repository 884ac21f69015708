"""Pins for the oracle's constraint-2 predicate (parametric intersection; paper,
Method section, eqs. lamda_eq1 / lambda / find_x, and Algorithm 2)."""
import math

import numpy as np

import exact_geom as X
import pins
from paper_2306_04316_amd import workloads as W


def cls2(oracle, px, py, rx, ry):
    off = np.array([0, len(rx)], dtype=np.int64)
    return oracle.classify(np.asarray(px, float), np.asarray(py, float), off, np.asarray(rx, float),
                           np.asarray(ry, float), nthreads=4, predicate=2)


def test_c2_rectangles_closed_form(oracle_mod):
    """x_new is exactly the vertical edge's x, so the closed form of constraint 1 holds:
    inside iff x0 < p_x <= x1 and y0 <= p_y < y1 (with the text's x >= p_x reading)."""
    rng = np.random.default_rng(21)
    for _ in range(40):
        mag = 10.0 ** rng.uniform(-5, 5)
        x0, x1 = np.sort(rng.uniform(-1, 1, 2)) * mag
        y0, y1 = np.sort(rng.uniform(-1, 1, 2)) * mag
        xs = np.array([x0, x1, np.nextafter(x0, np.inf), np.nextafter(x1, -np.inf), np.nextafter(x1, np.inf)])
        ys = np.array([y0, y1, np.nextafter(y0, np.inf), np.nextafter(y1, -np.inf), 0.5 * (y0 + y1)])
        gx, gy = np.meshgrid(xs, ys)
        px = np.concatenate([gx.ravel(), rng.uniform(x0 - mag, x1 + mag, 200)])
        py = np.concatenate([gy.ravel(), rng.uniform(y0 - mag, y1 + mag, 200)])
        want = ((x0 < px) & (px <= x1) & (y0 <= py) & (py < y1)).astype(np.uint8)
        for ring in ([(x0, y0), (x1, y0), (x1, y1), (x0, y1)], [(x1, y1), (x1, y0), (x0, y0), (x0, y1)]):
            got = cls2(oracle_mod, px, py, [v[0] for v in ring], [v[1] for v in ring])
            assert np.array_equal(got, want)


def test_c2_winding_off_boundary(oracle_mod):
    """Off the boundary on small integer rings the intersection is far (>= 1/(2|d_y|))
    from a half-integer p_x, so rounding cannot flip a crossing: parity = winding mod 2."""
    for (xs, ys) in pins.small_integer_polygons(seed=23, n=60):
        gx = np.arange(2 * (xs.min() - 1), 2 * (xs.max() + 1) + 1)
        gy = np.arange(2 * (ys.min() - 1), 2 * (ys.max() + 1) + 1)
        GX, GY = np.meshgrid(gx, gy)
        qx2, qy2 = GX.ravel(), GY.ravel()
        onb = X.on_boundary_int(qx2, qy2, 2 * xs, 2 * ys)
        w = X.winding_int(qx2, qy2, 2 * xs, 2 * ys)
        got = cls2(oracle_mod, qx2 / 2.0, qy2 / 2.0, xs, ys)
        bad = np.nonzero(~onb & (got != (np.abs(w) % 2)))[0]
        assert bad.size == 0, f"ring {list(zip(xs, ys))} point {qx2[bad[0]] / 2, qy2[bad[0]] / 2}"


def paper_alg2(qx, qy, rxc, ryc):
    """Algorithm 2's computation, vectorised over points: product-form candidates,
    d = r_{i+1} - r_i, l = (y - y_i)/d_y, x_new = x_i + l d_x, strict x_new > x."""
    f = ryc[None, :] - qy[:, None]
    prod = f[:, 1:] * f[:, :-1]
    cand = prod <= 0
    dx = np.broadcast_to(rxc[1:] - rxc[:-1], prod.shape)
    dy = np.broadcast_to(ryc[1:] - ryc[:-1], prod.shape)
    with np.errstate(divide="ignore", invalid="ignore"):
        lam = (qy[:, None] - ryc[None, :-1]) / dy
        xn = rxc[None, :-1] + lam * dx
    cnt = np.count_nonzero(cand & (xn > qx[:, None]), axis=1)
    tie = np.any(cand & (xn == qx[:, None]), axis=1)
    return (cnt % 2).astype(np.uint8), np.any(f == 0, axis=1), tie


def test_c2_paper_algorithm2_bit_exact(oracle_mod):
    """Where no vertex is level with the point and no intersection equals p_x exactly,
    the half-open rule with x >= p_x and Algorithm 2's listing evaluate the same
    rounded operations and must agree bit for bit."""
    rng = np.random.default_rng(24)
    for t in range(12):
        k = int(rng.integers(3, 65))
        ang = np.sort(rng.uniform(0, 2 * math.pi, k))
        r = rng.uniform(0.5, 1.0, k)
        c, sc = [(0.0, 1.0), (1.3, 2e-4), (5e6, 25.0)][t % 3]
        rx, ry = c + sc * r * np.cos(ang), c + sc * r * np.sin(ang)
        qx, qy = pins._near_edge_points(rng, rx, ry, 3000, rel=4e-16)
        got = cls2(oracle_mod, qx, qy, rx, ry)
        want, zero, tie = paper_alg2(qx, qy, np.append(rx, rx[0]), np.append(ry, ry[0]))
        ok = ~zero & ~tie
        assert np.array_equal(got[ok], want[ok])
        assert ok.mean() > 0.9


def test_c2_agrees_with_c1_off_the_band(oracle_mod):
    """Both predicates decide the same exact geometric fact; on footprints they agree
    except on pairs within rounding of an edge (bounded fraction)."""
    w = W.footprints(scale=0.01)
    a = oracle_mod.classify_workload(w)
    b = oracle_mod.classify_workload(w, predicate=2)
    assert np.count_nonzero(a != b) <= 2
