"""CPU oracle for the ray-casting point-in-polygon test -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The GPU library (``paper_2306_04316_amd``) never imports it and
the two share no code.

``pip_oracle.c`` holds the definition (paper, Method section, constraint 1 and
Algorithm 1, with the half-open straddle rule; constraint 2 and Algorithm 2;
polygons of several rings as the XOR of their rings' parities); this module
only compiles it with gcc (binary64, no contraction, no fast-math) and
marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pip_oracle.c")
_BUILD = os.path.join(_HERE, "_build")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fno-unsafe-math-optimizations",
          "-std=c11", "-shared", "-fPIC", "-pthread", "-Wall", "-Wextra"]

_libs: dict = {}


def lib_path(mutant: int = 0) -> str:
    name = "libpiporacle.so" if not mutant else f"libpiporacle_mutant{int(mutant)}.so"
    return os.path.join(_BUILD, name)


def build(mutant: int = 0, force: bool = True) -> str:
    """Compile the oracle (optionally with a planted mistake, for pin tests)."""
    out = lib_path(mutant)
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
        return out
    os.makedirs(_BUILD, exist_ok=True)
    tmp = out + f".tmp{os.getpid()}"
    cmd = ["gcc", *CFLAGS, f"-DPIP_ORACLE_MUTANT={int(mutant)}", _SRC, "-o", tmp]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(tmp, out)
    return out


def load(mutant: int = 0) -> ctypes.CDLL:
    if mutant in _libs:
        return _libs[mutant]
    path = build(mutant, force=False)
    lib = ctypes.CDLL(path)
    for name in ("pip_oracle_classify", "pip_oracle_classify_c2"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                      ctypes.c_void_p, ctypes.c_int64,
                      ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    f = lib.pip_oracle_classify_rings
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    f = lib.pip_oracle_classify_indexed
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    f = lib.pip_oracle_bbox_join
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    _libs[mutant] = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def classify(px, py, offsets, vx, vy, point_poly=None, nthreads: int | None = None,
             mutant: int = 0, predicate: int = 1) -> np.ndarray:
    """inside[i] in {0,1} for point (px[i], py[i]) against polygon point_poly[i] (or 0).

    predicate 1: constraint 1 (normal-side test); 2: constraint 2 (parametric intersection)."""
    px = np.ascontiguousarray(px, dtype=np.float64)
    py = np.ascontiguousarray(py, dtype=np.float64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    vx = np.ascontiguousarray(vx, dtype=np.float64)
    vy = np.ascontiguousarray(vy, dtype=np.float64)
    if point_poly is not None:
        point_poly = np.ascontiguousarray(point_poly, dtype=np.int32)
    n = px.shape[0]
    if py.shape[0] != n or vx.shape[0] != vy.shape[0] or offsets[-1] > vx.shape[0]:
        raise ValueError("inconsistent array sizes")
    out = np.empty(n, dtype=np.uint8)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    fn = load(mutant).pip_oracle_classify_c2 if predicate == 2 else load(mutant).pip_oracle_classify
    rc = fn(_ptr(px), _ptr(py), n, _ptr(offsets), offsets.shape[0] - 1,
            _ptr(vx), _ptr(vy), _ptr(point_poly), _ptr(out), int(nthreads))
    if rc != 0:
        raise ValueError(f"pip_oracle_classify rejected its arguments (rc={rc})")
    return out


def classify_indexed(px, py, offsets, vx, vy, nthreads: int | None = None, mutant: int = 0) -> np.ndarray:
    """One ring against many points, with the edges that cannot straddle a point's
    ray skipped through an exact y index (pip_oracle_classify_indexed): the same
    bits as classify(), in time proportional to the straddling edges."""
    px = np.ascontiguousarray(px, dtype=np.float64)
    py = np.ascontiguousarray(py, dtype=np.float64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    vx = np.ascontiguousarray(vx, dtype=np.float64)
    vy = np.ascontiguousarray(vy, dtype=np.float64)
    if offsets.shape[0] != 2 or py.shape[0] != px.shape[0] or offsets[-1] > vx.shape[0]:
        raise ValueError("the indexed mode takes one ring and matching point arrays")
    out = np.empty(px.shape[0], dtype=np.uint8)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    rc = load(mutant).pip_oracle_classify_indexed(_ptr(px), _ptr(py), px.shape[0], _ptr(offsets), 1, _ptr(vx),
                                                  _ptr(vy), _ptr(out), int(nthreads))
    if rc != 0:
        raise ValueError(f"pip_oracle_classify_indexed failed (rc={rc})")
    return out


def classify_rings(px, py, poly_rings, ring_offsets, vx, vy, point_poly=None, nthreads: int | None = None,
                   mutant: int = 0, predicate: int = 1) -> np.ndarray:
    """Polygons of several rings: polygon q owns rings poly_rings[q]..poly_rings[q+1]-1,
    ring r the vertices ring_offsets[r]..ring_offsets[r+1]-1 (parity XORed over rings)."""
    px = np.ascontiguousarray(px, dtype=np.float64)
    py = np.ascontiguousarray(py, dtype=np.float64)
    poly_rings = np.ascontiguousarray(poly_rings, dtype=np.int64)
    ring_offsets = np.ascontiguousarray(ring_offsets, dtype=np.int64)
    vx = np.ascontiguousarray(vx, dtype=np.float64)
    vy = np.ascontiguousarray(vy, dtype=np.float64)
    if point_poly is not None:
        point_poly = np.ascontiguousarray(point_poly, dtype=np.int32)
    n = px.shape[0]
    if (py.shape[0] != n or vx.shape[0] != vy.shape[0] or ring_offsets[-1] > vx.shape[0]
            or poly_rings[-1] > ring_offsets.shape[0] - 1):
        raise ValueError("inconsistent array sizes")
    out = np.empty(n, dtype=np.uint8)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    rc = load(mutant).pip_oracle_classify_rings(
        _ptr(px), _ptr(py), n, _ptr(poly_rings), poly_rings.shape[0] - 1, _ptr(ring_offsets),
        ring_offsets.shape[0] - 1, _ptr(vx), _ptr(vy), _ptr(point_poly), _ptr(out), int(nthreads), int(predicate))
    if rc != 0:
        raise ValueError(f"pip_oracle_classify_rings rejected its arguments (rc={rc})")
    return out


def classify_workload(w, nthreads: int | None = None, mutant: int = 0, predicate: int = 1) -> np.ndarray:
    if getattr(w, "poly_rings", None) is not None:
        return classify_rings(w.px, w.py, w.poly_rings, w.offsets, w.vx, w.vy, w.point_poly, nthreads=nthreads,
                              mutant=mutant, predicate=predicate)
    return classify(w.px, w.py, w.offsets, w.vx, w.vy, w.point_poly, nthreads=nthreads, mutant=mutant,
                    predicate=predicate)


def classify_one(x: float, y: float, ring_x, ring_y, mutant: int = 0) -> int:
    """One point against one ring (convenience for small exact tests)."""
    rx = np.asarray(ring_x, dtype=np.float64)
    ry = np.asarray(ring_y, dtype=np.float64)
    off = np.array([0, rx.shape[0]], dtype=np.int64)
    return int(classify(np.array([x], dtype=np.float64), np.array([y], dtype=np.float64), off, rx, ry,
                        nthreads=1, mutant=mutant)[0])


def bbox_join(px, py, offsets, vx, vy, poly_rings=None, nthreads: int | None = None, mutant: int = 0):
    """Candidate pairs by closed bounding box: (pair_point int64[M], pair_poly int32[M]),
    listed by polygon, then by point index."""
    px = np.ascontiguousarray(px, dtype=np.float64)
    py = np.ascontiguousarray(py, dtype=np.float64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    vx = np.ascontiguousarray(vx, dtype=np.float64)
    vy = np.ascontiguousarray(vy, dtype=np.float64)
    if poly_rings is not None:
        poly_rings = np.ascontiguousarray(poly_rings, dtype=np.int64)
        n_polys = poly_rings.shape[0] - 1
    else:
        n_polys = offsets.shape[0] - 1
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    counts = np.zeros(max(n_polys, 1), dtype=np.int64)
    lib = load(mutant)
    args = (_ptr(px), _ptr(py), px.shape[0], _ptr(poly_rings), n_polys, _ptr(offsets), _ptr(vx), _ptr(vy))
    if lib.pip_oracle_bbox_join(*args, _ptr(counts), None, int(nthreads)) != 0:
        raise ValueError("pip_oracle_bbox_join rejected its arguments")
    counts = counts[:n_polys]
    pair_point = np.empty(max(int(counts.sum()), 1), dtype=np.int64)
    if lib.pip_oracle_bbox_join(*args, _ptr(counts), _ptr(pair_point), int(nthreads)) != 0:
        raise ValueError("pip_oracle_bbox_join rejected its arguments")
    m = int(counts.sum())
    return pair_point[:m], np.repeat(np.arange(n_polys, dtype=np.int32), counts)
