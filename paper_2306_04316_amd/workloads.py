"""Seeded synthetic workloads for the point-in-polygon hot path.

This module only *draws* inputs: polygons in a CSR layout (offsets plus SoA
vertex arrays), query points (SoA), and an optional point->polygon pair index.
It contains none of the classification arithmetic, so both the CPU oracle
tests and the GPU path can take their inputs from here without sharing any
part of the method.

The paper evaluates its ray-casting test on ~17.1 million building points
against one country boundary polygon (Simulation section).  That dataset is
not available here, so five synthetic workloads stand in for it:

  1  star        one 64-vertex star-shaped polygon, 100,000 points in its bbox
  2  footprints  100,000 building-footprint-like polygons (rotated rectangles
                 and L-shapes, 4..32 vertices), 100 points per polygon
  3  fractal     one 1,000,000-vertex midpoint-displaced 1024-gon, 10M points
  4  batched     1,000,000 star polygons with k ~ discrete power law k^-2 on
                 [3, 4096] and Poisson(100) points per polygon
  5  stress      the topology of 4 in projected metres (offset ~5e6, extents
                 5..50 m) with points on vertices, within 1e-9 m of edges and
                 level with a horizontal edge

and one more for polygons of several rings (country and building shapes
have holes and detached parts):

     holes       footprints of 2 with courtyard holes and detached parts

Every workload accepts ``scale`` (fraction of polygons / points kept) so the
same recipe yields the small cases used by parity tests.  All coordinates are
float64; offsets are int64; the pair index is int32 and sorted by polygon.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = ["Workload", "make", "CONFIG_NAMES", "star", "footprints", "fractal",
           "batched", "stress", "holes", "raw_points", "subsample"]

CONFIG_NAMES = {1: "star", 2: "footprints", 3: "fractal", 4: "batched", 5: "stress"}


@dataclasses.dataclass
class Workload:
    name: str
    px: np.ndarray                 # float64 [N]
    py: np.ndarray                 # float64 [N]
    offsets: np.ndarray            # int64 [P+1], offsets[0] == 0
    vx: np.ndarray                 # float64 [V]
    vy: np.ndarray                 # float64 [V]
    point_poly: np.ndarray | None  # int32 [N] or None (every point vs polygon 0)
    params: dict
    # polygons of several rings: polygon q owns rings poly_rings[q] .. poly_rings[q+1]-1
    # and `offsets` is then the ring CSR (ring r = vertices offsets[r] .. offsets[r+1]-1);
    # None: one ring per polygon, `offsets` is the polygon CSR
    poly_rings: np.ndarray | None = None

    @property
    def n_points(self) -> int:
        return int(self.px.shape[0])

    @property
    def n_polys(self) -> int:
        if self.poly_rings is not None:
            return int(self.poly_rings.shape[0] - 1)
        return int(self.offsets.shape[0] - 1)

    @property
    def n_rings(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_vertices(self) -> int:
        return int(self.vx.shape[0])

    def poly_vertex_counts(self) -> np.ndarray:
        """Edges of each polygon (all rings)."""
        if self.poly_rings is None:
            return np.diff(self.offsets)
        return np.diff(self.offsets[self.poly_rings])

    def edges_per_pair(self) -> np.ndarray:
        """Number of edges each pair tests (= the polygon's stored vertex count)."""
        k = self.poly_vertex_counts()
        if self.point_poly is None:
            return np.full(self.n_points, int(k[0]), dtype=np.int64)
        return k[self.point_poly]

    @property
    def n_tests(self) -> int:
        """T = sum over pairs of the number of edges tested."""
        k = self.poly_vertex_counts()
        if self.point_poly is None:
            return int(k[0]) * self.n_points
        counts = np.bincount(self.point_poly, minlength=self.n_polys)
        return int(np.dot(counts.astype(np.int64), k.astype(np.int64)))

    def nbytes_algorithmic(self) -> int:
        """Bytes the method must move once: points, pair index, mask, vertices, offsets."""
        b = 16 * self.n_points + 1 * self.n_points + 16 * self.n_vertices + 8 * (self.n_rings + 1)
        if self.poly_rings is not None:
            b += 8 * (self.n_polys + 1)
        if self.point_poly is not None:
            b += 4 * self.n_points
        return b


def _csr_from_counts(counts: np.ndarray) -> np.ndarray:
    off = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return off


def _seg_ids(counts: np.ndarray) -> np.ndarray:
    return np.repeat(np.arange(counts.shape[0], dtype=np.int64), counts)


def _points_in_inflated_bbox(rng, offsets, vx, vy, npts, inflate=1.2):
    """Uniform points in each polygon's bbox scaled by `inflate` about its centre."""
    starts = offsets[:-1]
    xmin = np.minimum.reduceat(vx, starts)
    xmax = np.maximum.reduceat(vx, starts)
    ymin = np.minimum.reduceat(vy, starts)
    ymax = np.maximum.reduceat(vy, starts)
    cx, cy = 0.5 * (xmin + xmax), 0.5 * (ymin + ymax)
    hx, hy = 0.5 * inflate * (xmax - xmin), 0.5 * inflate * (ymax - ymin)
    pp = np.repeat(np.arange(npts.shape[0], dtype=np.int32), npts)
    ux = rng.random(pp.shape[0])
    uy = rng.random(pp.shape[0])
    px = (cx[pp] - hx[pp]) + (2.0 * hx[pp]) * ux
    py = (cy[pp] - hy[pp]) + (2.0 * hy[pp]) * uy
    return px, py, pp


# --------------------------------------------------------------------------- 1
def star(seed: int = 0, n_vertices: int = 64, n_points: int = 100_000, scale: float = 1.0) -> Workload:
    """One star-shaped polygon: sorted uniform polar angles, radius U[0.5, 1.0]."""
    rng = np.random.default_rng(seed)
    n_points = max(0, int(round(n_points * scale)))
    theta = np.sort(rng.uniform(0.0, 2.0 * math.pi, n_vertices))
    r = rng.uniform(0.5, 1.0, n_vertices)
    vx = r * np.cos(theta)
    vy = r * np.sin(theta)
    px = rng.uniform(vx.min(), vx.max(), n_points)
    py = rng.uniform(vy.min(), vy.max(), n_points)
    off = np.array([0, n_vertices], dtype=np.int64)
    return Workload("star", px, py, off, vx, vy, None,
                    dict(config=1, seed=seed, n_vertices=n_vertices, n_points=n_points))


# --------------------------------------------------------------------------- 2
def footprints(seed: int = 0, n_polys: int = 100_000, pts_per_poly: int = 100,
               scale: float = 1.0, kmax: int = 32) -> Workload:
    """Building-footprint-like polygons: rotated rectangles or L-shapes, 4..32 vertices.

    Vertex count k = clip(round(lognormal(ln 6, 0.5)), 4, 32).  Half the polygons
    are L-shapes (a rectangle with a corner notch of U[0.3,0.7] of each side)
    when k >= 6.  Further vertices are added by splitting the longest edge at
    U[0.2, 0.8] with a perpendicular jitter of +-1% of that edge.  Width and
    height are log-uniform in [5e-5, 5e-4] degrees, rotation U[0, pi), centres
    lon U[0, 2], lat U[5, 7].  Each polygon gets `pts_per_poly` points uniform in
    its bbox inflated by 20%; the pair index is sorted by polygon.
    """
    rng = np.random.default_rng(seed)
    P = max(1, int(round(n_polys * scale)))
    X, Y, cnt, _, _ = _footprint_local(rng, P, kmax)
    phi = rng.uniform(0.0, math.pi, P)
    cxs = rng.uniform(0.0, 2.0, P)
    cys = rng.uniform(5.0, 7.0, P)
    cph, sph = np.cos(phi)[:, None], np.sin(phi)[:, None]
    RX = cxs[:, None] + (X * cph - Y * sph)
    RY = cys[:, None] + (X * sph + Y * cph)
    valid = np.arange(kmax)[None, :] < cnt[:, None]
    vx = RX[valid]
    vy = RY[valid]
    off = _csr_from_counts(cnt)
    npts = np.full(P, int(pts_per_poly), dtype=np.int64)
    px, py, pp = _points_in_inflated_bbox(rng, off, vx, vy, npts)
    return Workload("footprints", px, py, off, vx, vy, pp,
                    dict(config=2, seed=seed, n_polys=P, pts_per_poly=pts_per_poly))


def _footprint_local(rng, P, kmax):
    """Footprint rings in local coordinates (centred, unrotated): X, Y [P, kmax],
    vertex counts, widths, heights (the draws of `footprints` before placement)."""
    k = np.clip(np.rint(rng.lognormal(math.log(6.0), 0.5, P)), 4, kmax).astype(np.int64)
    is_L = (rng.random(P) < 0.5) & (k >= 6)
    w = np.exp(rng.uniform(math.log(5e-5), math.log(5e-4), P))
    h = np.exp(rng.uniform(math.log(5e-5), math.log(5e-4), P))
    na = rng.uniform(0.3, 0.7, P)
    nb = rng.uniform(0.3, 0.7, P)

    X = np.zeros((P, kmax))
    Y = np.zeros((P, kmax))
    hw, hh = 0.5 * w, 0.5 * h
    # rectangle, counter-clockwise
    X[:, 0], Y[:, 0] = -hw, -hh
    X[:, 1], Y[:, 1] = hw, -hh
    X[:, 2], Y[:, 2] = hw, hh
    X[:, 3], Y[:, 3] = -hw, hh
    cnt = np.full(P, 4, dtype=np.int64)
    # L-shape: notch out the top-right corner
    L = np.nonzero(is_L)[0]
    X[L, 0], Y[L, 0] = -hw[L], -hh[L]
    X[L, 1], Y[L, 1] = hw[L], -hh[L]
    X[L, 2], Y[L, 2] = hw[L], hh[L] - nb[L] * h[L]
    X[L, 3], Y[L, 3] = hw[L] - na[L] * w[L], hh[L] - nb[L] * h[L]
    X[L, 4], Y[L, 4] = hw[L] - na[L] * w[L], hh[L]
    X[L, 5], Y[L, 5] = -hw[L], hh[L]
    cnt[L] = 6

    cols = np.arange(kmax)[None, :]
    while True:
        act = np.nonzero(cnt < k)[0]
        if act.size == 0:
            break
        c = cnt[act]
        xa, ya = X[act], Y[act]
        nxt = (cols + 1) % c[:, None]
        xb = np.take_along_axis(xa, nxt, axis=1)
        yb = np.take_along_axis(ya, nxt, axis=1)
        dx, dy = xb - xa, yb - ya
        ln = np.hypot(dx, dy)
        ln[cols >= c[:, None]] = -1.0
        e = np.argmax(ln, axis=1)
        t = rng.uniform(0.2, 0.8, act.size)
        jit = rng.uniform(-0.01, 0.01, act.size)
        r = np.arange(act.size)
        ex, ey = dx[r, e], dy[r, e]
        el = ln[r, e]
        mx = xa[r, e] + t * ex + jit * (-ey)   # left normal times edge length = (-dy, dx)
        my = ya[r, e] + t * ey + jit * ex
        # shift columns after e one step right, insert the new vertex at e+1
        src = np.where(cols <= e[:, None], cols, cols - 1)
        src = np.clip(src, 0, kmax - 1)
        nx_ = np.take_along_axis(xa, src, axis=1)
        ny_ = np.take_along_axis(ya, src, axis=1)
        nx_[r, e + 1] = mx
        ny_[r, e + 1] = my
        X[act], Y[act] = nx_, ny_
        cnt[act] += 1
    return X, Y, cnt, w, h


def holes(seed: int = 0, n_polys: int = 100_000, pts_per_poly: int = 100, scale: float = 1.0,
          p_hole: float = 0.5, p_part: float = 0.2, kmax: int = 32) -> Workload:
    """Footprints made of several rings: courtyards (holes) and detached parts.

    Each polygon's outer ring is drawn as in `footprints`.  With probability
    `p_hole` it gets a rectangular hole (clockwise) of half-sizes U[0.04, 0.08]
    of the width and height, centred at (-0.3 w, -0.3 h) in the footprint's
    frame (inside both rectangles and L-shapes, whose notch never reaches
    x < -0.2 w and y < -0.2 h); with probability `p_part` a detached
    rectangular part (counter-clockwise) of half-sizes U[0.1, 0.2] of w and h
    centred at (0.8 w, 0).  Rings of a polygon are stored outer, hole, part;
    points are uniform in the polygon's bbox (all rings) inflated by 20%.
    """
    rng = np.random.default_rng(seed)
    P = max(1, int(round(n_polys * scale)))
    X, Y, cnt, w, h = _footprint_local(rng, P, kmax)
    has_hole = rng.random(P) < p_hole
    ha, hb = rng.uniform(0.04, 0.08, P) * w, rng.uniform(0.04, 0.08, P) * h
    has_part = rng.random(P) < p_part
    pa, pb = rng.uniform(0.1, 0.2, P) * w, rng.uniform(0.1, 0.2, P) * h
    phi = rng.uniform(0.0, math.pi, P)
    cxs = rng.uniform(0.0, 2.0, P)
    cys = rng.uniform(5.0, 7.0, P)

    hx0, hy0 = -0.3 * w, -0.3 * h
    HX = np.stack([hx0 - ha, hx0 - ha, hx0 + ha, hx0 + ha], axis=1)   # clockwise
    HY = np.stack([hy0 - hb, hy0 + hb, hy0 + hb, hy0 - hb], axis=1)
    px0 = 0.8 * w
    QX = np.stack([px0 - pa, px0 + pa, px0 + pa, px0 - pa], axis=1)   # counter-clockwise
    QY = np.stack([-pb, -pb, pb, pb], axis=1)
    AX = np.concatenate([X, HX, QX], axis=1)
    AY = np.concatenate([Y, HY, QY], axis=1)
    valid = np.concatenate([np.arange(kmax)[None, :] < cnt[:, None],
                            np.repeat(has_hole[:, None], 4, axis=1),
                            np.repeat(has_part[:, None], 4, axis=1)], axis=1)
    cph, sph = np.cos(phi)[:, None], np.sin(phi)[:, None]
    RX = cxs[:, None] + (AX * cph - AY * sph)
    RY = cys[:, None] + (AX * sph + AY * cph)
    vx = RX[valid]
    vy = RY[valid]
    ring_counts = np.stack([cnt, 4 * has_hole, 4 * has_part], axis=1).ravel()
    ring_counts = ring_counts[ring_counts > 0]
    ring_off = _csr_from_counts(ring_counts)
    poly_rings = _csr_from_counts(1 + has_hole.astype(np.int64) + has_part.astype(np.int64))
    poly_off = _csr_from_counts(cnt + 4 * has_hole + 4 * has_part)
    npts = np.full(P, int(pts_per_poly), dtype=np.int64)
    px, py, pp = _points_in_inflated_bbox(rng, poly_off, vx, vy, npts)
    return Workload("holes", px, py, ring_off, vx, vy, pp,
                    dict(seed=seed, n_polys=P, pts_per_poly=pts_per_poly, p_hole=p_hole, p_part=p_part),
                    poly_rings=poly_rings)


def raw_points(w: Workload, seed: int = 1) -> Workload:
    """The pairs' points of `w` as raw points (shuffled, no pair index) with the
    same polygons: the input of candidate-pair generation."""
    perm = np.random.default_rng(seed).permutation(w.n_points)
    return Workload(w.name + "[raw]", np.ascontiguousarray(w.px[perm]), np.ascontiguousarray(w.py[perm]),
                    w.offsets, w.vx, w.vy, None, dict(w.params, raw_points=True), poly_rings=w.poly_rings)


# --------------------------------------------------------------------------- 3
def fractal(seed: int = 0, n_vertices: int = 1_000_000, n_points: int = 10_000_000,
            base: int = 1024, radius: float = 3.0, centre=(0.0, 8.0), scale: float = 1.0,
            scale_vertices: bool = False) -> Workload:
    """A regular `base`-gon refined by midpoint displacement to exactly n_vertices.

    Each refinement level replaces edge (a, b) by (a, m), (m, b) with
    m = (a+b)/2 + d*|b-a|*n_left, d ~ U[-0.25, 0.25], n_left the unit left
    normal of b-a.  Full levels are applied while they fit; the last level is
    applied to the first edges only, so the ring ends with exactly n_vertices.
    Points are uniform in the final bbox.  `scale` scales the point count (and
    the vertex count too when `scale_vertices`).
    """
    rng = np.random.default_rng(seed)
    n_points = max(0, int(round(n_points * scale)))
    if scale_vertices:
        n_vertices = max(base, int(round(n_vertices * scale)))
    ang = 2.0 * math.pi * np.arange(base) / base
    x = centre[0] + radius * np.cos(ang)
    y = centre[1] + radius * np.sin(ang)
    while x.shape[0] < n_vertices:
        n = x.shape[0]
        m = min(n, n_vertices - n)          # edges refined at this level
        xb, yb = np.roll(x, -1)[:m], np.roll(y, -1)[:m]
        xa, ya = x[:m], y[:m]
        d = rng.uniform(-0.25, 0.25, m)
        # (b-a) rotated +90deg has length |b-a|: d*|b-a|*n_left == d*(-(yb-ya), xb-xa)
        mx = 0.5 * (xa + xb) - d * (yb - ya)
        my = 0.5 * (ya + yb) + d * (xb - xa)
        nx = np.empty(n + m)
        ny = np.empty(n + m)
        nx[0:2 * m:2], ny[0:2 * m:2] = xa, ya
        nx[1:2 * m:2], ny[1:2 * m:2] = mx, my
        nx[2 * m:], ny[2 * m:] = x[m:], y[m:]
        x, y = nx, ny
    px = rng.uniform(x.min(), x.max(), n_points)
    py = rng.uniform(y.min(), y.max(), n_points)
    off = np.array([0, x.shape[0]], dtype=np.int64)
    return Workload("fractal", px, py, off, x, y, None,
                    dict(config=3, seed=seed, n_vertices=int(x.shape[0]), n_points=n_points))


# --------------------------------------------------------------------------- 4/5
def _power_law_k(rng, P, kmin=3, kmax=4096, alpha=2.0):
    ks = np.arange(kmin, kmax + 1, dtype=np.float64)
    pmf = ks ** (-alpha)
    pmf /= pmf.sum()
    cdf = np.cumsum(pmf)
    u = rng.random(P)
    idx = np.searchsorted(cdf, u, side="right")
    return np.minimum(idx, ks.shape[0] - 1).astype(np.int64) + kmin


def _star_topology(rng, P, kmax=4096, mean_pts=100.0):
    """Unit-scale star polygons: k, sorted angles (order statistics), radii, point counts."""
    k = _power_law_k(rng, P, kmax=kmax)
    V = int(k.sum())
    # sorted uniforms on [0,1) per polygon: normalised prefix sums of k+1 exponentials
    e = rng.standard_exponential(V + P)
    seg = np.repeat(np.arange(P), k + 1)
    cs = np.cumsum(e)
    ends = np.cumsum(k + 1) - 1
    totals = cs[ends] - np.concatenate(([0.0], cs[ends[:-1]]))
    base = np.concatenate(([0.0], cs[ends[:-1]]))
    u = (cs - base[seg]) / totals[seg]
    keep = np.ones(V + P, dtype=bool)
    keep[ends] = False                 # drop the last (== 1.0) entry of each segment
    theta = 2.0 * math.pi * u[keep]
    r = rng.uniform(0.5, 1.0, V)
    npts = rng.poisson(mean_pts, P).astype(np.int64)
    return k, theta, r, npts


def batched(seed: int = 0, n_polys: int = 1_000_000, scale: float = 1.0, kmax: int = 4096,
            mean_pts: float = 100.0) -> Workload:
    """Star polygons with power-law vertex counts in degrees (footprint scale).

    k ~ P(k) proportional to k^-2 on {3..kmax}; shapes as the `star` workload with
    half-extents log-uniform in [2.5e-5, 2.5e-4] degrees; centres lon U[0,2],
    lat U[5,7]; Poisson(mean_pts) points per polygon uniform in the bbox x1.2.
    """
    rng = np.random.default_rng(seed)
    P = max(1, int(round(n_polys * scale)))
    k, theta, r, npts = _star_topology(rng, P, kmax, mean_pts)
    hext = np.exp(rng.uniform(math.log(2.5e-5), math.log(2.5e-4), P))
    cx = rng.uniform(0.0, 2.0, P)
    cy = rng.uniform(5.0, 7.0, P)
    seg = _seg_ids(k)
    vx = cx[seg] + hext[seg] * r * np.cos(theta)
    vy = cy[seg] + hext[seg] * r * np.sin(theta)
    off = _csr_from_counts(k)
    px, py, pp = _points_in_inflated_bbox(rng, off, vx, vy, npts)
    return Workload("batched", px, py, off, vx, vy, pp,
                    dict(config=4, seed=seed, n_polys=P, kmax=kmax, mean_pts=mean_pts))


def stress(seed: int = 0, n_polys: int = 1_000_000, scale: float = 1.0, kmax: int = 4096,
           mean_pts: float = 100.0, class_p=(0.97, 0.02, 0.005, 0.005)) -> Workload:
    """The `batched` topology in projected metres with adversarial point classes.

    Centres 5.0e6 + U[0, 2.2e5] m in x and y, extents log-uniform in [5, 50] m,
    edge 0 of every polygon made horizontal (y1 := y0).  Each pair draws a class:
    0 uniform in the bbox x1.2; 1 within 1e-9 m of a random edge; 2 a bitwise copy
    of a random vertex; 3 level with the horizontal edge (p_y = y0, p_x uniform
    over that edge's x-span widened by 50% on each side).
    """
    rng = np.random.default_rng(seed)
    P = max(1, int(round(n_polys * scale)))
    k, theta, r, npts = _star_topology(rng, P, kmax, mean_pts)
    ext = np.exp(rng.uniform(math.log(5.0), math.log(50.0), P))
    cx = 5.0e6 + rng.uniform(0.0, 2.2e5, P)
    cy = 5.0e6 + rng.uniform(0.0, 2.2e5, P)
    seg = _seg_ids(k)
    off = _csr_from_counts(k)
    vx = cx[seg] + 0.5 * ext[seg] * r * np.cos(theta)
    vy = cy[seg] + 0.5 * ext[seg] * r * np.sin(theta)
    s0 = off[:-1]
    vy[s0 + 1] = vy[s0]                     # edge 0 horizontal
    px, py, pp = _points_in_inflated_bbox(rng, off, vx, vy, npts)
    N = pp.shape[0]
    cls = rng.choice(4, size=N, p=np.asarray(class_p, dtype=np.float64))
    kk = k[pp]
    base = off[pp]
    # class 1: near a random edge
    i1 = np.nonzero(cls == 1)[0]
    e = (rng.random(i1.size) * kk[i1]).astype(np.int64)
    e = np.minimum(e, kk[i1] - 1)
    a = base[i1] + e
    b = base[i1] + (e + 1) % kk[i1]
    t = rng.random(i1.size)
    dlt = rng.uniform(-1e-9, 1e-9, i1.size)
    ex, ey = vx[b] - vx[a], vy[b] - vy[a]
    el = np.hypot(ex, ey)
    el[el == 0.0] = 1.0
    px[i1] = vx[a] + t * ex + dlt * (-ey / el)
    py[i1] = vy[a] + t * ey + dlt * (ex / el)
    # class 2: exactly on a vertex
    i2 = np.nonzero(cls == 2)[0]
    v = base[i2] + np.minimum((rng.random(i2.size) * kk[i2]).astype(np.int64), kk[i2] - 1)
    px[i2] = vx[v]
    py[i2] = vy[v]
    # class 3: level with the horizontal edge 0
    i3 = np.nonzero(cls == 3)[0]
    x0, x1 = vx[base[i3]], vx[base[i3] + 1]
    lo, hi = np.minimum(x0, x1), np.maximum(x0, x1)
    wdt = hi - lo
    px[i3] = rng.uniform(lo - 0.5 * wdt, hi + 0.5 * wdt)
    py[i3] = vy[base[i3]]
    return Workload("stress", px, py, off, vx, vy, pp,
                    dict(config=5, seed=seed, n_polys=P, kmax=kmax, mean_pts=mean_pts,
                         class_p=list(class_p), n_class=[int((cls == c).sum()) for c in range(4)]))


_MAKERS = {1: star, 2: footprints, 3: fractal, 4: batched, 5: stress}


def make(config: int, seed: int = 0, scale: float = 1.0, **kw) -> Workload:
    """Build workload `config` (1..5) with the given seed and scale."""
    return _MAKERS[int(config)](seed=seed, scale=scale, **kw)


def subsample(w: Workload, idx: np.ndarray) -> Workload:
    """The pairs `idx` of `w` (same polygons), e.g. for sampled oracle checks."""
    pp = None if w.point_poly is None else np.ascontiguousarray(w.point_poly[idx])
    return Workload(w.name + "[sample]", np.ascontiguousarray(w.px[idx]), np.ascontiguousarray(w.py[idx]),
                    w.offsets, w.vx, w.vy, pp, dict(w.params, sample=int(idx.shape[0])), poly_rings=w.poly_rings)
