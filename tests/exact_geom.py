"""Exact-arithmetic geometry used to pin the CPU oracle (tests only).

Nothing here shares code with the oracle or with the GPU library.  Integer
inputs use numpy int64 (exact for the small coordinates used) or Python ints;
float64 inputs are lifted to exact rationals with ``fractions.Fraction``.

Provided:
  * winding numbers by the quadrant-walk method (no ray casting involved),
  * point-on-boundary tests,
  * the half-open straddle / non-positive side rule evaluated exactly,
  * ear-clipping triangulation and the triangle area-sum inclusion test,
  * a first-order binary64 error bound for the side value, used to certify
    that a float64 evaluation cannot have a different sign from the exact one.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

U64 = 2.0 ** -53


# ---------------------------------------------------------------- integer, vectorised over points
def quadrant(dx: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """Quadrant 0..3 of a nonzero vector (dx, dy); half-open so every vector has one."""
    q = np.full(dx.shape, -1, dtype=np.int64)
    q[(dx > 0) & (dy >= 0)] = 0
    q[(dx <= 0) & (dy > 0)] = 1
    q[(dx < 0) & (dy <= 0)] = 2
    q[(dx >= 0) & (dy < 0)] = 3
    return q


def winding_int(px: np.ndarray, py: np.ndarray, rx, ry) -> np.ndarray:
    """Winding number of an integer ring around integer points by quadrant walking.

    Valid for points not on the ring.  Each edge adds the signed number of
    quarter turns its endpoints' quadrants differ by; a jump of two quadrants
    is resolved by the sign of the cross product.  Sum / 4 is the winding number.
    """
    px = np.asarray(px, dtype=np.int64)
    py = np.asarray(py, dtype=np.int64)
    k = len(rx)
    total = np.zeros(px.shape, dtype=np.int64)
    for i in range(k):
        ax, ay = int(rx[i]), int(ry[i])
        bx, by = int(rx[(i + 1) % k]), int(ry[(i + 1) % k])
        qa = quadrant(ax - px, ay - py)
        qb = quadrant(bx - px, by - py)
        d = (qb - qa) % 4
        cross = (ax - px) * (by - py) - (ay - py) * (bx - px)
        step = np.where(d == 1, 1, np.where(d == 3, -1, 0))
        step = np.where(d == 2, np.where(cross > 0, 2, -2), step)
        total += step
    return total // 4


def on_boundary_int(px, py, rx, ry) -> np.ndarray:
    """True where the integer point lies on some edge of the integer ring."""
    px = np.asarray(px, dtype=np.int64)
    py = np.asarray(py, dtype=np.int64)
    k = len(rx)
    on = np.zeros(px.shape, dtype=bool)
    for i in range(k):
        ax, ay = int(rx[i]), int(ry[i])
        bx, by = int(rx[(i + 1) % k]), int(ry[(i + 1) % k])
        cross = (bx - ax) * (py - ay) - (by - ay) * (px - ax)
        inx = (np.minimum(ax, bx) <= px) & (px <= np.maximum(ax, bx))
        iny = (np.minimum(ay, by) <= py) & (py <= np.maximum(ay, by))
        on |= (cross == 0) & inx & iny
    return on


def halfopen_rule_int(px, py, rx, ry) -> np.ndarray:
    """The constraint-1 rule with the half-open straddle test, in exact integers.

    Edge (a,b) counts iff exactly one endpoint has y > p_y and
    (p-a).n <= 0 with n = (b_y-a_y, a_x-b_x) oriented so n_x > 0.
    """
    px = np.asarray(px, dtype=np.int64)
    py = np.asarray(py, dtype=np.int64)
    k = len(rx)
    cnt = np.zeros(px.shape, dtype=np.int64)
    for i in range(k):
        ax, ay = int(rx[i]), int(ry[i])
        bx, by = int(rx[(i + 1) % k]), int(ry[(i + 1) % k])
        st = (ay > py) != (by > py)
        nx, ny = by - ay, ax - bx
        if nx < 0:
            nx, ny = -nx, -ny
        s = (px - ax) * nx + (py - ay) * ny
        cnt += (st & (s <= 0)).astype(np.int64)
    return (cnt & 1).astype(np.uint8)


def convex_hull_ccw(pts):
    """Monotone-chain convex hull of integer points, CCW, no collinear points."""
    pts = sorted(set(map(tuple, pts)))
    if len(pts) < 3:
        return pts

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    return lower[:-1] + upper[:-1]


def ear_clip(rx, ry):
    """Triangulate a simple integer polygon (either orientation) by ear clipping."""
    idx = list(range(len(rx)))
    pts = [(int(rx[i]), int(ry[i])) for i in idx]
    area2 = sum(pts[i][0] * pts[(i + 1) % len(pts)][1] - pts[(i + 1) % len(pts)][0] * pts[i][1]
                for i in range(len(pts)))
    if area2 < 0:
        idx.reverse()

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    def in_tri(p, a, b, c):
        return cross(a, b, p) >= 0 and cross(b, c, p) >= 0 and cross(c, a, p) >= 0

    tris = []
    guard = 0
    while len(idx) > 3 and guard < 10000:
        guard += 1
        n = len(idx)
        clipped = False
        for j in range(n):
            i0, i1, i2 = idx[(j - 1) % n], idx[j], idx[(j + 1) % n]
            a, b, c = pts[i0], pts[i1], pts[i2]
            if cross(a, b, c) <= 0:
                continue
            if any(in_tri(pts[m], a, b, c) for m in idx if m not in (i0, i1, i2)):
                continue
            tris.append((a, b, c))
            del idx[j]
            clipped = True
            break
        if not clipped:
            raise ValueError("ear clipping failed (polygon not simple?)")
    a, b, c = (pts[i] for i in idx)
    if cross(a, b, c) > 0:
        tris.append((a, b, c))
    return tris


def in_some_triangle(px, py, tris) -> np.ndarray:
    """Area-sum test: p is in the closed triangle ABC iff |A1|+|A2|+|A3| == |A|."""
    px = np.asarray(px, dtype=np.int64)
    py = np.asarray(py, dtype=np.int64)
    res = np.zeros(px.shape, dtype=bool)
    for (a, b, c) in tris:
        def area2(u, v, wx, wy):
            return np.abs((v[0] - u[0]) * (wy - u[1]) - (v[1] - u[1]) * (wx - u[0]))
        A = abs((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]))
        s = area2(a, b, px, py) + area2(b, c, px, py) + area2(c, a, px, py)
        res |= (s == A)
    return res


# ---------------------------------------------------------------- float64 inputs, exact rationals
def side_exact(x: float, y: float, ax: float, ay: float, bx: float, by: float) -> Fraction:
    """Exact (p - a) . (b_y - a_y, a_x - b_x) for float64 inputs (no orientation flip)."""
    X, Y = Fraction(x), Fraction(y)
    AX, AY, BX, BY = Fraction(ax), Fraction(ay), Fraction(bx), Fraction(by)
    return (X - AX) * (BY - AY) + (Y - AY) * (AX - BX)


def side_bound64(x, y, ax, ay, bx, by) -> float:
    """Bound on |fl64 side value - exact side value| for the rule's evaluation order.

    t1 = x-ax, t2 = y-ay, nx = by-ay, ny = ax-bx are each rounded once, then
    two rounded products and one rounded sum: every term carries at most
    (1+u)^4 - 1 < 4.01u relative error, so 5u * (|t1 nx| + |t2 ny|) bounds it
    (computed with 10% slack in float64 from the exact magnitudes).
    """
    t1 = abs(x - ax)
    t2 = abs(y - ay)
    nx = abs(by - ay)
    ny = abs(ax - bx)
    return 1.1 * 5.0 * U64 * (t1 * nx + t2 * ny) + 1e-300


def exact_rule_parity_f64(x, y, rx, ry):
    """(parity, certified): exact-rational evaluation of the half-open rule on float64 input.

    certified is True when every straddling edge has |exact side| > the float64
    error bound, i.e. a float64 evaluation in the rule's order must agree.
    """
    k = len(rx)
    cnt = 0
    cert = True
    for i in range(k):
        ax, ay = float(rx[i]), float(ry[i])
        bx, by = float(rx[(i + 1) % k]), float(ry[(i + 1) % k])
        if (ay > y) == (by > y):
            continue
        s = side_exact(x, y, ax, ay, bx, by)
        if by < ay:           # orientation flip n -> -n (exact)
            s = -s
        if abs(s) <= Fraction(side_bound64(x, y, ax, ay, bx, by)):
            cert = False
        if s <= 0:
            cnt += 1
    return cnt & 1, cert
