"""Pins for the CPU oracle: checks against facts that the paper and mathematics fix.

Each ``pin_*`` function runs the oracle (optionally a build with a planted
mistake, ``mutant``) on inputs whose correct classification is known by other
means, and returns a list of failure descriptions (empty == pinned).  The
test module asserts the real oracle passes every pin and that every planted
mistake fails at least one.

Pins (the rule is the paper's Method section, constraint 1, Algorithm 1, with
the half-open straddle reading):
  P1  axis-aligned rectangles: closed form  x0 < px <= x1  and  y0 <= py < y1
  P2  convex integer polygons: inside iff strictly left of every CCW edge
  P3  small integer polygons (self-intersecting, repeated vertices, collinear
      runs, horizontal edges, spikes): parity == winding number mod 2 off the
      boundary (quadrant-walk winding, not ray casting); exact rule on it
  P4  invariants: start-vertex rotation and a repeated closing vertex
      (bit-exact, any float64 input); reversal and integer translation (integer
      input); triangulated area-sum inclusion for simple polygons
  P5  the paper's own product-form straddle test with its operation order,
      vectorised independently, bit-exact where no vertex is level with the
      point (where the two straddle forms coincide)
  P6  star polygon closed form: a point in the angular sector of edge j is
      inside iff it is strictly on the centre's side of edge j (exact
      rationals), on float64 pairs certified by the binary64 error bound
  P7  footprint polygons: exact-rational evaluation of the rule on a seeded
      sample, certified pairs only
  G   hand-derived cases in tests/golden/hand_cases.txt
"""
from __future__ import annotations

import math
import os

import numpy as np

import exact_geom as X

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_cases.txt")


def _cls(oracle, px, py, rx, ry, mutant):
    off = np.array([0, len(rx)], dtype=np.int64)
    return oracle.classify(np.asarray(px, dtype=np.float64), np.asarray(py, dtype=np.float64), off,
                           np.asarray(rx, dtype=np.float64), np.asarray(ry, dtype=np.float64),
                           nthreads=4, mutant=mutant)


# ------------------------------------------------------------------ P1
def pin_rectangles(oracle, mutant=0, seed=1, n_rect=60):
    rng = np.random.default_rng(seed)
    fails = []
    for r in range(n_rect):
        mag = 10.0 ** rng.uniform(-6, 6)
        off = rng.uniform(-1e3, 1e3) * (1 if r % 2 else 0)
        x0, x1 = np.sort(rng.uniform(-1, 1, 2)) * mag + off
        y0, y1 = np.sort(rng.uniform(-1, 1, 2)) * mag - off
        if not (x0 < x1 and y0 < y1):
            continue
        xs = np.array([x0, x1, np.nextafter(x0, -np.inf), np.nextafter(x0, np.inf),
                       np.nextafter(x1, -np.inf), np.nextafter(x1, np.inf), 0.5 * (x0 + x1)])
        ys = np.array([y0, y1, np.nextafter(y0, -np.inf), np.nextafter(y0, np.inf),
                       np.nextafter(y1, -np.inf), np.nextafter(y1, np.inf), 0.5 * (y0 + y1)])
        gx, gy = np.meshgrid(xs, ys)
        px = np.concatenate([gx.ravel(), rng.uniform(x0 - mag, x1 + mag, 200)])
        py = np.concatenate([gy.ravel(), rng.uniform(y0 - mag, y1 + mag, 200)])
        want = ((x0 < px) & (px <= x1) & (y0 <= py) & (py < y1)).astype(np.uint8)
        ccw = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
        for order in (ccw, ccw[::-1]):
            for s in range(4):
                ring = order[s:] + order[:s]
                for closed in (False, True):
                    rr = ring + ring[:1] if closed else ring
                    got = _cls(oracle, px, py, [v[0] for v in rr], [v[1] for v in rr], mutant)
                    bad = np.nonzero(got != want)[0]
                    if bad.size:
                        i = bad[0]
                        fails.append(f"P1 rect ({x0},{y0})-({x1},{y1}) start={s} closed={closed} "
                                     f"p=({px[i]!r},{py[i]!r}) got={got[i]} want={want[i]}")
    return fails


# ------------------------------------------------------------------ P2
def pin_convex(oracle, mutant=0, seed=2, n_poly=40):
    rng = np.random.default_rng(seed)
    fails = []
    for t in range(n_poly):
        R = 2 ** int(rng.integers(3, 21))
        pts = rng.integers(-R, R + 1, size=(int(rng.integers(3, 40)), 2))
        hull = X.convex_hull_ccw(pts.tolist())
        if len(hull) < 3:
            continue
        hx = np.array([p[0] for p in hull], dtype=np.int64)
        hy = np.array([p[1] for p in hull], dtype=np.int64)
        qx = rng.integers(hx.min() - 2, hx.max() + 3, 400)
        qy = rng.integers(hy.min() - 2, hy.max() + 3, 400)
        qx = np.concatenate([qx, hx, (hx + np.roll(hx, -1)) // 2])
        qy = np.concatenate([qy, hy, (hy + np.roll(hy, -1)) // 2])
        k = len(hull)
        allpos = np.ones(qx.shape, dtype=bool)
        anyzero = np.zeros(qx.shape, dtype=bool)
        for i in range(k):
            ax, ay, bx, by = int(hx[i]), int(hy[i]), int(hx[(i + 1) % k]), int(hy[(i + 1) % k])
            o = (bx - ax) * (qy - ay) - (by - ay) * (qx - ax)
            allpos &= o > 0
            anyzero |= o == 0
        onb = X.on_boundary_int(qx, qy, hx, hy)
        off_b = ~onb
        for rev in (False, True):
            rx, ry = (hx[::-1], hy[::-1]) if rev else (hx, hy)
            got = _cls(oracle, qx, qy, rx, ry, mutant)
            bad = np.nonzero(off_b & (got != allpos.astype(np.uint8)))[0]
            if bad.size:
                i = bad[0]
                fails.append(f"P2 convex k={k} R={R} rev={rev} p=({qx[i]},{qy[i]}) got={got[i]}")
    # float64 regular n-gons: certified points only
    for n in (3, 5, 17, 64, 257):
        ang = 2 * math.pi * np.arange(n) / n + 0.1
        rx, ry = 2.5 * np.cos(ang) + 0.3, 2.5 * np.sin(ang) - 0.7
        m = max(100, 3000 // n)
        qx = rng.uniform(-3, 3.6, m)
        qy = rng.uniform(-3.7, 2.4, m)
        got = _cls(oracle, qx, qy, rx, ry, mutant)
        for i in range(qx.shape[0]):
            want = 1
            cert = True
            for j in range(n):
                s = X.side_exact(qx[i], qy[i], rx[j], ry[j], rx[(j + 1) % n], ry[(j + 1) % n])
                # (p-a).(dy,-dx) < 0  <=>  p strictly left of a CCW edge
                if -s <= 0:
                    want = 0
                if abs(s) <= X.side_bound64(qx[i], qy[i], rx[j], ry[j], rx[(j + 1) % n], ry[(j + 1) % n]):
                    cert = False
            if cert and got[i] != want:
                fails.append(f"P2 n-gon n={n} p=({qx[i]!r},{qy[i]!r}) got={got[i]} want={want}")
                break
    return fails


# ------------------------------------------------------------------ P3
def small_integer_polygons(seed=3, n=80):
    """Random small integer rings of several kinds (coordinates in [-8, 8])."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(n):
        kind = t % 6
        k = int(rng.integers(3, 13))
        if kind == 0:      # arbitrary (usually self-intersecting)
            xs, ys = rng.integers(-8, 9, k), rng.integers(-8, 9, k)
        elif kind == 1:    # repeated vertices
            xs, ys = rng.integers(-8, 9, k), rng.integers(-8, 9, k)
            j = int(rng.integers(0, k))
            xs = np.insert(xs, j, xs[j])
            ys = np.insert(ys, j, ys[j])
        elif kind == 2:    # horizontal edges and collinear runs on a few levels
            xs = rng.integers(-8, 9, k)
            ys = rng.choice([-4, 0, 3], k)
        elif kind == 3:    # star-shaped (simple) around the origin
            ang = np.sort(rng.uniform(0, 2 * math.pi, k))
            r = rng.integers(2, 9, k)
            xs, ys = np.rint(r * np.cos(ang)).astype(np.int64), np.rint(r * np.sin(ang)).astype(np.int64)
        elif kind == 4:    # spikes: vertex pairs that touch a level from one side
            xs = rng.integers(-8, 9, k)
            ys = np.where(np.arange(k) % 2 == 0, 0, rng.integers(-6, 7, k))
        else:              # axis-parallel staircase (many collinear and level vertices)
            steps = rng.integers(-3, 4, (k, 2))
            xs = np.cumsum(np.where(np.arange(k) % 2 == 0, steps[:, 0], 0))
            ys = np.cumsum(np.where(np.arange(k) % 2 == 1, steps[:, 1], 0))
            xs = np.clip(xs, -8, 8)
            ys = np.clip(ys, -8, 8)
        out.append((np.asarray(xs, dtype=np.int64), np.asarray(ys, dtype=np.int64)))
    return out


def pin_winding(oracle, mutant=0, seed=3):
    fails = []
    for (xs, ys) in small_integer_polygons(seed):
        # every integer and half-integer point of the bbox grown by 1: work in 2x units
        gx = np.arange(2 * (xs.min() - 1), 2 * (xs.max() + 1) + 1)
        gy = np.arange(2 * (ys.min() - 1), 2 * (ys.max() + 1) + 1)
        GX, GY = np.meshgrid(gx, gy)
        qx2, qy2 = GX.ravel(), GY.ravel()
        rx2, ry2 = 2 * xs, 2 * ys
        got = _cls(oracle, qx2 / 2.0, qy2 / 2.0, xs.astype(np.float64), ys.astype(np.float64), mutant)
        onb = X.on_boundary_int(qx2, qy2, rx2, ry2)
        w = X.winding_int(qx2, qy2, rx2, ry2)
        want_off = (np.abs(w) % 2).astype(np.uint8)
        bad = np.nonzero(~onb & (got != want_off))[0]
        if bad.size:
            i = bad[0]
            fails.append(f"P3 winding ring={list(zip(xs.tolist(), ys.tolist()))} "
                         f"p=({qx2[i] / 2},{qy2[i] / 2}) got={got[i]} winding={w[i]}")
        want_on = X.halfopen_rule_int(qx2, qy2, rx2, ry2)
        bad = np.nonzero(onb & (got != want_on))[0]
        if bad.size:
            i = bad[0]
            fails.append(f"P3 boundary ring={list(zip(xs.tolist(), ys.tolist()))} "
                         f"p=({qx2[i] / 2},{qy2[i] / 2}) got={got[i]} want={want_on[i]}")
    return fails


# ------------------------------------------------------------------ P4
def _near_edge_points(rng, rx, ry, n, rel=1e-15):
    k = len(rx)
    e = rng.integers(0, k, n)
    t = rng.random(n)
    ax, ay = rx[e], ry[e]
    bx, by = rx[(e + 1) % k], ry[(e + 1) % k]
    d = rng.uniform(-1, 1, n) * rel * (np.abs(ax) + np.abs(ay) + 1.0)
    ln = np.hypot(bx - ax, by - ay)
    ln[ln == 0] = 1.0
    return ax + t * (bx - ax) - d * (by - ay) / ln, ay + t * (by - ay) + d * (bx - ax) / ln


def pin_invariants(oracle, mutant=0, seed=4):
    rng = np.random.default_rng(seed)
    fails = []
    # (a) rotation of the start vertex / repeated closing vertex: bit-exact on float64 input
    for t in range(12):
        k = int(rng.integers(3, 40))
        ang = np.sort(rng.uniform(0, 2 * math.pi, k))
        r = rng.uniform(0.5, 1.0, k)
        c = 5e6 if t % 2 else 0.0
        rx, ry = c + 20 * r * np.cos(ang), c - 20 * r * np.sin(ang)
        qx, qy = _near_edge_points(rng, rx, ry, 1500)
        qx = np.concatenate([qx, rx, rng.uniform(rx.min(), rx.max(), 500)])
        qy = np.concatenate([qy, ry, np.full(500, ry[0])])
        base = _cls(oracle, qx, qy, rx, ry, mutant)
        for s in range(1, k):
            got = _cls(oracle, qx, qy, np.roll(rx, -s), np.roll(ry, -s), mutant)
            if np.any(got != base):
                fails.append(f"P4 rotation k={k} shift={s}")
                break
        got = _cls(oracle, qx, qy, np.append(rx, rx[0]), np.append(ry, ry[0]), mutant)
        if np.any(got != base):
            fails.append(f"P4 closing-duplicate k={k}")
    # (b) reversal and integer translation: exact on integer inputs
    for (xs, ys) in small_integer_polygons(seed + 1, n=30):
        gx = np.arange(2 * (xs.min() - 1), 2 * (xs.max() + 1) + 1)
        gy = np.arange(2 * (ys.min() - 1), 2 * (ys.max() + 1) + 1)
        GX, GY = np.meshgrid(gx, gy)
        qx, qy = GX.ravel() / 2.0, GY.ravel() / 2.0
        base = _cls(oracle, qx, qy, xs, ys, mutant)
        rev = _cls(oracle, qx, qy, xs[::-1], ys[::-1], mutant)
        if np.any(rev != base):
            fails.append(f"P4 reversal ring={list(zip(xs.tolist(), ys.tolist()))}")
        dx, dy = int(rng.integers(-1000, 1000)), int(rng.integers(-1000, 1000))
        tr = _cls(oracle, qx + dx, qy + dy, xs + dx, ys + dy, mutant)
        if np.any(tr != base):
            fails.append(f"P4 translation ({dx},{dy})")
    # (c) simple polygons: agreement with triangulated area-sum inclusion off the boundary
    for t in range(25):
        k = int(rng.integers(3, 14))
        ang = np.sort(rng.choice(np.arange(0, 360, 7), k, replace=False)) * math.pi / 180
        r = rng.integers(3, 12, k)
        xs = np.rint(r * np.cos(ang)).astype(np.int64)
        ys = np.rint(r * np.sin(ang)).astype(np.int64)
        pts = list(zip(xs.tolist(), ys.tolist()))
        if len(set(pts)) < k:
            continue
        try:
            tris = X.ear_clip(xs, ys)
        except ValueError:
            continue
        gx = np.arange(2 * (xs.min() - 1), 2 * (xs.max() + 1) + 1)
        gy = np.arange(2 * (ys.min() - 1), 2 * (ys.max() + 1) + 1)
        GX, GY = np.meshgrid(gx, gy)
        qx2, qy2 = GX.ravel(), GY.ravel()
        tris2 = [tuple((2 * a, 2 * b) for (a, b) in tri) for tri in tris]
        inside_tri = X.in_some_triangle(qx2, qy2, tris2)
        onb = X.on_boundary_int(qx2, qy2, 2 * xs, 2 * ys)
        w = X.winding_int(qx2, qy2, 2 * xs, 2 * ys)
        if np.any(~onb & (inside_tri != (w % 2 == 1))):
            continue   # not simple after rounding; the area-sum test does not apply
        got = _cls(oracle, qx2 / 2.0, qy2 / 2.0, xs, ys, mutant)
        bad = np.nonzero(~onb & (got != inside_tri.astype(np.uint8)))[0]
        if bad.size:
            i = bad[0]
            fails.append(f"P4 area-sum ring={pts} p=({qx2[i] / 2},{qy2[i] / 2}) got={got[i]}")
    return fails


# ------------------------------------------------------------------ P5
def paper_product_form(qx, qy, rx_closed, ry_closed):
    """Constraint 1 as the paper computes it, vectorised over points (numpy, float64).

    Rows are query points, columns are edges i -> i+1 of the explicitly closed
    ring.  Candidate edges: f_i * f_{i+1} <= 0 with f = r_y - p_y.  Normal
    (y_{i+1}-y_i, x_i-x_{i+1}) negated where its x part is negative.  The edge
    counts when (p_x - x_i)*n_x + (p_y - y_i)*n_y <= 0 (numpy rounds each
    operation separately).  Returns (parity, f_has_zero, f_product_tiny).
    """
    f = ry_closed[None, :] - qy[:, None]
    prod = f[:, 1:] * f[:, :-1]
    cand = prod <= 0
    nx = np.broadcast_to(ry_closed[1:] - ry_closed[:-1], prod.shape).copy()
    ny = np.broadcast_to(rx_closed[:-1] - rx_closed[1:], prod.shape).copy()
    flip = nx < 0
    nx[flip] = -nx[flip]
    ny[flip] = -ny[flip]
    side = (qx[:, None] - rx_closed[None, :-1]) * nx + (qy[:, None] - ry_closed[None, :-1]) * ny
    count = np.count_nonzero(cand & (side <= 0), axis=1)
    zero = np.any(f == 0, axis=1)
    tiny = np.any((np.abs(prod) < 1e-290) | ~np.isfinite(prod), axis=1)
    return (count % 2).astype(np.uint8), zero, tiny


def pin_paper_form(oracle, mutant=0, seed=5):
    rng = np.random.default_rng(seed)
    fails = []
    for t in range(16):
        k = int(rng.integers(3, 65))
        ang = np.sort(rng.uniform(0, 2 * math.pi, k))
        r = rng.uniform(0.5, 1.0, k)
        if t % 3 == 0:
            cx, cy, sc = 0.0, 0.0, 1.0
        elif t % 3 == 1:
            cx, cy, sc = 1.3, 6.1, 2e-4
        else:
            cx, cy, sc = 5.0e6, 5.1e6, 25.0
        rx, ry = cx + sc * r * np.cos(ang), cy + sc * r * np.sin(ang)
        qx, qy = _near_edge_points(rng, rx, ry, 4000, rel=4e-16)
        qx = np.concatenate([qx, rng.uniform(rx.min(), rx.max(), 2000)])
        qy = np.concatenate([qy, rng.uniform(ry.min(), ry.max(), 2000)])
        got = _cls(oracle, qx, qy, rx, ry, mutant)
        want, zero, tiny = paper_product_form(qx, qy, np.append(rx, rx[0]), np.append(ry, ry[0]))
        ok = ~zero & ~tiny
        bad = np.nonzero(ok & (got != want))[0]
        if bad.size:
            i = bad[0]
            fails.append(f"P5 paper form t={t} k={k} p=({qx[i]!r},{qy[i]!r}) got={got[i]} want={want[i]} "
                         f"({bad.size} of {int(ok.sum())})")
    return fails


# ------------------------------------------------------------------ P6
def pin_star_closed_form(oracle, star_workload, mutant=0, n_sample=3000, seed=6):
    """Star polygon (angles sorted around the origin, radii > 0): a point whose polar
    angle falls in [theta_j, theta_{j+1}) is inside iff it is strictly on the origin's
    side of edge j.  Sector and side are decided with exact rationals."""
    from fractions import Fraction
    w = star_workload
    rx, ry = w.vx, w.vy
    k = rx.shape[0]
    rng = np.random.default_rng(seed)
    idx = rng.choice(w.n_points, size=min(n_sample, w.n_points), replace=False)
    qx, qy = w.px[idx], w.py[idx]
    got = _cls(oracle, qx, qy, rx, ry, mutant)
    theta = np.arctan2(ry, rx) % (2 * math.pi)
    assert np.all(np.diff(theta) > 0), "star vertices must be sorted by angle"
    fails = []
    n_cert = 0
    for i in range(qx.shape[0]):
        x, y = float(qx[i]), float(qy[i])
        if x == 0.0 and y == 0.0:
            continue
        ang = math.atan2(y, x) % (2 * math.pi)
        j0 = int(np.searchsorted(theta, ang, side="right")) - 1
        # confirm the sector exactly: cross(v_j, p) >= 0 and cross(p, v_{j+1}) > 0
        sector = None
        for j in (j0 - 1, j0, j0 + 1):
            j %= k
            a = (Fraction(rx[j]), Fraction(ry[j]))
            b = (Fraction(rx[(j + 1) % k]), Fraction(ry[(j + 1) % k]))
            P = (Fraction(x), Fraction(y))
            c1 = a[0] * P[1] - a[1] * P[0]
            c2 = P[0] * b[1] - P[1] * b[0]
            if c1 >= 0 and c2 > 0:
                sector = j
                break
        if sector is None:
            continue
        j = sector
        ax, ay, bx, by = rx[j], ry[j], rx[(j + 1) % k], ry[(j + 1) % k]
        s = X.side_exact(x, y, ax, ay, bx, by)      # = -orient(a, b, p): < 0 on the origin's side
        want = 1 if s < 0 else 0
        _, cert = X.exact_rule_parity_f64(x, y, rx, ry)
        if not cert or s == 0:
            continue
        n_cert += 1
        if got[i] != want:
            fails.append(f"P6 star p=({x!r},{y!r}) sector={j} got={got[i]} want={want}")
            break
    if n_cert < 0.9 * qx.shape[0]:
        fails.append(f"P6 too few certified points ({n_cert})")
    return fails


# ------------------------------------------------------------------ P7
def pin_footprints_exact(oracle, fp_workload, mutant=0, n_sample=4000, seed=7):
    w = fp_workload
    rng = np.random.default_rng(seed)
    idx = rng.choice(w.n_points, size=min(n_sample, w.n_points), replace=False)
    got = oracle.classify(w.px[idx], w.py[idx], w.offsets, w.vx, w.vy, w.point_poly[idx],
                          nthreads=4, mutant=mutant)
    fails = []
    n_cert = 0
    for t, i in enumerate(idx):
        q = int(w.point_poly[i])
        b, e = int(w.offsets[q]), int(w.offsets[q + 1])
        par, cert = X.exact_rule_parity_f64(float(w.px[i]), float(w.py[i]), w.vx[b:e], w.vy[b:e])
        if not cert:
            continue
        n_cert += 1
        if got[t] != par:
            fails.append(f"P7 footprint pair {i} poly {q} got={got[t]} want={par}")
            break
    if n_cert < 0.95 * idx.shape[0]:
        fails.append(f"P7 too few certified pairs ({n_cert})")
    return fails


# ------------------------------------------------------------------ G
def load_golden(path=GOLDEN):
    """Parse hand_cases.txt: 'ring x0 y0 x1 y1 ...' blocks followed by 'p x y expected' lines."""
    cases = []
    ring = None
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "ring":
                v = [float(t) for t in tok[1:]]
                ring = (v[0::2], v[1::2])
            elif tok[0] == "p":
                cases.append((ring, float(tok[1]), float(tok[2]), int(tok[3])))
    return cases


def pin_golden(oracle, mutant=0):
    fails = []
    for (ring, x, y, want) in load_golden():
        got = _cls(oracle, [x], [y], ring[0], ring[1], mutant)[0]
        if got != want:
            fails.append(f"G ring={list(zip(*ring))} p=({x},{y}) got={got} want={want}")
    return fails
