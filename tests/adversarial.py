"""Adversarial inputs for the binary32 filter (tests only; no arithmetic of the
method): triangles whose first vertex is the re-centring point, and points a
few binary64 ulps off an edge, at large offsets, tiny extents and with
re-centred coordinates on both sides of powers of two.

Each family yields a Workload of triangle polygons (three vertices each, the
first one the centre the filter re-centres on) with one point per polygon,
so the CPU emulation of the filter and the GPU parity test see the same
(point, edge) configurations.
"""
from __future__ import annotations

import numpy as np

from paper_2306_04316_amd import workloads as W

OFFSETS = [0.0, 1.0, 1.0e3, 5.0e6, 1.0e7]
EXTENTS = [1.0e-9, 1.0e-6, 1.0e-3, 1.0, 50.0, 1.0e4]
ULPS = [1, 2, 5, 10, 100, 1000, 10000]


def _workload(name, cx, cy, ax, ay, bx, by, px, py):
    n = px.size
    vx = np.stack([cx, ax, bx], axis=1).reshape(-1)
    vy = np.stack([cy, ay, by], axis=1).reshape(-1)
    off = np.arange(0, 3 * n + 1, 3, dtype=np.int64)
    return W.Workload(name, np.ascontiguousarray(px), np.ascontiguousarray(py), off, vx, vy,
                      np.arange(n, dtype=np.int32), {})


def near_edge(seed=0, per_cell=60):
    """Points p = a + t (b - a), then moved j ulps of p_x in x (both signs), for
    every offset, extent and ulp count; edges in random directions, with
    nearly horizontal and nearly vertical ones over-represented."""
    rng = np.random.default_rng(seed)
    cols = {k: [] for k in ("cx", "cy", "ax", "ay", "bx", "by", "px", "py")}
    for off in OFFSETS:
        for ext in EXTENTS:
            for j in ULPS:
                m = per_cell
                ang = rng.uniform(0, 2 * np.pi, m)
                ang[: m // 6] = rng.choice([0.0, np.pi], m // 6) + rng.uniform(-1e-6, 1e-6, m // 6)
                ang[m // 6: m // 3] = np.pi / 2 + rng.uniform(-1e-6, 1e-6, m // 3 - m // 6)
                ax = off + rng.uniform(-ext, ext, m)
                ay = off + rng.uniform(-ext, ext, m)
                bx = ax + ext * np.cos(ang)
                by = ay + ext * np.sin(ang)
                # the centre: another vertex of the ring, up to a few extents away
                cx = ax + ext * rng.uniform(-3, 3, m)
                cy = ay + ext * rng.uniform(-3, 3, m)
                t = rng.uniform(0.05, 0.95, m)
                px = ax + t * (bx - ax)
                py = ay + t * (by - ay)
                sgn = rng.choice([-1.0, 1.0], m)
                px = px + sgn * j * np.spacing(np.abs(px) + 1e-300)
                for k, v in zip(cols, (cx, cy, ax, ay, bx, by, px, py)):
                    cols[k].append(v)
    c = {k: np.concatenate(v) for k, v in cols.items()}
    return _workload("near-edge", **c)


def power_of_two_straddle(seed=1, m=4000):
    """Re-centred coordinates just below and just above powers of two (the
    binary32 grid changes spacing there), for the anchor and for the point."""
    rng = np.random.default_rng(seed)
    e = rng.integers(-30, 30, m).astype(np.float64)
    p2 = np.ldexp(1.0, e.astype(np.int64))
    off = rng.choice(OFFSETS, m)
    cx = off + rng.uniform(-1, 1, m)
    cy = off + rng.uniform(-1, 1, m)
    eps = p2 * 2.0 ** -20 * rng.uniform(-1, 1, m)
    ax = cx + p2 + eps * rng.uniform(-1, 1, m)
    ay = cy - p2 + eps * rng.uniform(-1, 1, m)
    ang = rng.uniform(0, 2 * np.pi, m)
    bx = ax + p2 * np.cos(ang)
    by = ay + p2 * np.sin(ang)
    t = rng.uniform(0.1, 0.9, m)
    px = ax + t * (bx - ax)
    py = ay + t * (by - ay)
    j = rng.choice(ULPS, m) * rng.choice([-1.0, 1.0], m)
    px = px + j * np.spacing(np.abs(px) + 1e-300)
    return _workload("pow2", cx, cy, ax, ay, bx, by, px, py)


def vertex_and_level(seed=2, m=3000):
    """Points on the anchor, on the far vertex, and level with either (y equal,
    x a few ulps to several extents away)."""
    rng = np.random.default_rng(seed)
    off = rng.choice(OFFSETS, m)
    ext = rng.choice(EXTENTS, m)
    cx = off + ext * rng.uniform(-2, 2, m)
    cy = off + ext * rng.uniform(-2, 2, m)
    ax = cx + ext * rng.uniform(-1, 1, m)
    ay = cy + ext * rng.uniform(-1, 1, m)
    bx = ax + ext * rng.uniform(-1, 1, m)
    by = ay + ext * rng.uniform(-1, 1, m)
    kind = rng.integers(0, 4, m)
    px = np.where(kind == 0, ax, np.where(kind == 1, bx, ax + ext * rng.uniform(-2, 2, m)))
    py = np.where(kind == 0, ay, np.where(kind == 1, by, np.where(kind == 2, ay, by)))
    j = rng.choice(ULPS, m) * rng.choice([-1.0, 1.0], m)
    px = np.where(kind >= 2, px + j * np.spacing(np.abs(px) + 1e-300), px)
    return _workload("vertex-level", cx, cy, ax, ay, bx, by, px, py)


def subnormal_scale(seed=3, m=4000):
    """Points within 1e-36 .. 1e-45 of a ring's first vertex (the re-centring
    point), on edges of ordinary length: the re-centred point, its differences
    and products are binary32 subnormals (or flush to zero), where the bound's
    absolute term decides."""
    rng = np.random.default_rng(seed)
    base = rng.choice([0.0, 1e-30, -3e-25], m)
    a_x = base * rng.uniform(0.5, 1.5, m)
    a_y = base * rng.uniform(0.5, 1.5, m)
    L = rng.choice([1e-10, 1e-3, 1.0], m)
    ang = rng.uniform(0, 2 * np.pi, m)
    b_x = a_x + L * np.cos(ang)
    b_y = a_y + L * np.sin(ang)
    ang2 = ang + rng.uniform(0.5, 2.5, m)
    d_x = a_x + L * np.cos(ang2)
    d_y = a_y + L * np.sin(ang2)
    delta = rng.choice([1e-36, 1e-38, 1e-39, 1e-40, 1e-42, 1e-44, 1e-45], m)
    px = a_x + delta * rng.uniform(-1, 1, m)
    py = a_y + delta * rng.uniform(-1, 1, m)
    # ring (a, b, d): a is the first vertex, so the re-centring point
    return _workload("subnormal", a_x, a_y, b_x, b_y, d_x, d_y, px, py)


FAMILIES = {"near-edge": near_edge, "pow2": power_of_two_straddle, "vertex-level": vertex_and_level,
            "subnormal": subnormal_scale}
