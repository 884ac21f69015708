"""MI355X (gfx950) ray-casting point-in-polygon (arxiv 2306.04316, constraint 1).

The work runs in ``libpip.so`` (hand-written HIP kernels behind a C ABI,
``include/pip.h``).  This package only marshals torch device tensors and
streams into that ABI:

    inside = classify(px, py, offsets, vx, vy, point_poly=None)

Inputs are CUDA (HIP) tensors: px, py, vx, vy float64; offsets int64 CSR
(offsets[0] = 0, offsets[-1] = len(vx)); point_poly int32 or None.  The result
is a uint8 tensor (1 = inside).  Work is enqueued on the current torch stream.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import PipError  # noqa: F401

__all__ = ["classify", "classify_rings", "candidate_pairs", "Plan", "PipError", "abi_version", "probe_copy",
           "probe_read", "probe_valu", "to_device"]


def _require(t, dtype, name, numel=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def options(mode="exact", kernel="auto", validate=False, pairs_per_lane=0, block=0, lds_slots=0,
            persistent=-1, order=-1, use_graph=True, tune=0, force_recheck=False, bound_scale=1.0,
            tune_cache=None, timing=False, index=False, predicate="side", stats=False,
            wave_k=0) -> _lib.pip_options:
    o = _lib.pip_options()
    _lib.load().pip_options_init(ctypes.byref(o))
    o.mode = _lib.MODES[mode] if isinstance(mode, str) else int(mode)
    o.kernel = _lib.KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    o.validate = 1 if validate else 0
    o.pairs_per_lane = int(pairs_per_lane)
    o.block = int(block)
    o.lds_slots = int(lds_slots)
    o.persistent = int(persistent)
    o.order = int(order)
    o.use_graph = 1 if use_graph else 0
    o.tune = int(tune)
    o.force_recheck = 1 if force_recheck else 0
    o.bound_scale = float(bound_scale)
    o.tune_cache = tune_cache.encode() if tune_cache else None
    # timing: True/1 = phase times, 2 or "kernel" = the main kernel's own timestamps only
    o.timing = 2 if (timing == 2 or timing == "kernel") else (1 if timing else 0)
    o.index = 1 if index else 0
    o.predicate = _lib.PREDICATES[predicate] if isinstance(predicate, str) else int(predicate)
    o.stats = 1 if stats else 0
    # filtered batched plans: ring size from which the wavefront-per-ring kernel takes
    # the pairs (0 = the tuner's or the cache's choice, off without them; -1 = off)
    o.wave_k = int(wave_k)
    return o


def _check_inputs(px, py, offsets, vx, vy, point_poly, out):
    import torch
    n = px.numel()
    _require(px, torch.float64, "px")
    _require(py, torch.float64, "py", n)
    _require(offsets, torch.int64, "offsets")
    _require(vx, torch.float64, "vx")
    _require(vy, torch.float64, "vy", vx.numel())
    if point_poly is not None:
        _require(point_poly, torch.int32, "point_poly", n)
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=px.device)
    else:
        _require(out, torch.uint8, "out", n)
    return out


class Plan:
    """A prepared classification of fixed device tensors (pip_plan_* in the C ABI).

    plan = Plan(px, py, offsets, vx, vy, point_poly, mode="filtered", tune=1)
    plan.execute()          # enqueue on the current stream; result in plan.out
    plan.stats()            # waits; figures of the last execution
    The tensors must stay alive (and at the same addresses) while the plan exists.
    """

    def __init__(self, px, py, offsets, vx, vy, point_poly=None, *, out=None, stream=None, poly_rings=None,
                 **opts):
        """With `poly_rings` (int64, n_polys+1), polygons have several rings and
        `offsets` is the ring CSR (pip_plan_create_rings)."""
        import torch
        self._lib = _lib.load()
        self.out = _check_inputs(px, py, offsets, vx, vy, point_poly, out)
        if poly_rings is not None:
            _require(poly_rings, torch.int64, "poly_rings")
        self._keep = (px, py, offsets, vx, vy, point_poly, poly_rings, self.out)
        self._opts = options(**opts)
        self.device = px.device
        h = ctypes.c_void_p()
        with torch.cuda.device(px.device):
            if poly_rings is None:
                rc = self._lib.pip_plan_create(ctypes.byref(h), _ptr(px), _ptr(py), px.numel(), _ptr(offsets),
                                               offsets.numel() - 1, _ptr(vx), _ptr(vy), vx.numel(),
                                               _ptr(point_poly), _ptr(self.out), ctypes.byref(self._opts),
                                               _stream_handle(stream))
            else:
                rc = self._lib.pip_plan_create_rings(ctypes.byref(h), _ptr(px), _ptr(py), px.numel(),
                                                     _ptr(poly_rings), poly_rings.numel() - 1, _ptr(offsets),
                                                     offsets.numel() - 1, _ptr(vx), _ptr(vy), vx.numel(),
                                                     _ptr(point_poly), _ptr(self.out), ctypes.byref(self._opts),
                                                     _stream_handle(stream))
        _lib.check(rc)
        self._h = h

    def execute(self, stream=None, stats=False):
        """Enqueue one execution; with stats=True wait for it and return its
        figures (a dict, as stats()) instead of the output tensor."""
        import torch
        st = _lib.pip_stats() if stats else None
        with torch.cuda.device(self.device):
            _lib.check(self._lib.pip_plan_execute(self._h, ctypes.byref(st) if stats else None,
                                                  _stream_handle(stream)))
        if stats:
            return {f: getattr(st, f) for f, _ in _lib.pip_stats._fields_}
        return self.out

    def stats(self) -> dict:
        st = _lib.pip_stats()
        _lib.check(self._lib.pip_plan_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _lib.pip_stats._fields_}

    def timing(self):
        """(ms_prep, ms_main, ms_recheck) of the last execution; waits for that execution only."""
        a, b, c = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
        _lib.check(self._lib.pip_plan_timing(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def config(self) -> dict:
        c = _lib.pip_plan_config()
        _lib.check(self._lib.pip_plan_get_config(self._h, ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in _lib.pip_plan_config._fields_ if f != "struct_size"}

    def close(self):
        if getattr(self, "_h", None):
            _lib.check(self._lib.pip_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def classify(px, py, offsets, vx, vy, point_poly=None, *, kernel="auto", validate=False, out=None,
             stream=None, pairs_per_lane=0, block=0, lds_slots=0, predicate="side", mode="exact",
             force_recheck=False, bound_scale=1.0):
    """inside[i] for point i against polygon point_poly[i] (or polygon 0).
    mode="filtered": binary32 side values with the binary64 recheck (pip_classify's
    filtered mode, workspace from the library's device-memory pool)."""
    import torch
    lib = _lib.load()
    n = px.numel()
    out = _check_inputs(px, py, offsets, vx, vy, point_poly, out)
    o = options(mode, kernel, validate, pairs_per_lane, block, lds_slots, predicate=predicate,
                force_recheck=force_recheck, bound_scale=bound_scale)
    with torch.cuda.device(px.device):
        rc = lib.pip_classify(_ptr(px), _ptr(py), n, _ptr(offsets), offsets.numel() - 1, _ptr(vx), _ptr(vy),
                              vx.numel(), _ptr(point_poly), _ptr(out), ctypes.byref(o), _stream_handle(stream))
    _lib.check(rc)
    return out


def classify_rings(px, py, poly_rings, ring_offsets, vx, vy, point_poly=None, *, kernel="auto", validate=False,
                   out=None, stream=None, pairs_per_lane=0, lds_slots=0, predicate="side"):
    """inside[i] for point i against polygon point_poly[i] (or 0) made of the rings
    poly_rings[q] .. poly_rings[q+1]-1, ring r = vertices ring_offsets[r] .. ring_offsets[r+1]-1."""
    import torch
    lib = _lib.load()
    n = px.numel()
    out = _check_inputs(px, py, ring_offsets, vx, vy, point_poly, out)
    _require(poly_rings, torch.int64, "poly_rings")
    o = options("exact", kernel, validate, pairs_per_lane, 0, lds_slots, predicate=predicate)
    with torch.cuda.device(px.device):
        rc = lib.pip_classify_rings(_ptr(px), _ptr(py), n, _ptr(poly_rings), poly_rings.numel() - 1,
                                    _ptr(ring_offsets), ring_offsets.numel() - 1, _ptr(vx), _ptr(vy), vx.numel(),
                                    _ptr(point_poly), _ptr(out), ctypes.byref(o), _stream_handle(stream))
    _lib.check(rc)
    return out


def candidate_pairs(px, py, offsets, vx, vy, poly_rings=None, *, stream=None, timing=None):
    """Candidate pairs by closed bounding box (pip_join_*): a dict of device tensors
    point (int64), poly (int32), px, py (float64), grouped by polygon in ascending
    order -- ready to classify as Plan(px, py, offsets, vx, vy, poly, ...).
    timing: a dict that receives the join kernels' device time (ms_count, ms_fill)."""
    import torch
    lib = _lib.load()
    _require(px, torch.float64, "px")
    _require(py, torch.float64, "py", px.numel())
    _require(offsets, torch.int64, "offsets")
    _require(vx, torch.float64, "vx")
    _require(vy, torch.float64, "vy", vx.numel())
    if poly_rings is not None:
        _require(poly_rings, torch.int64, "poly_rings")
        n_polys, n_rings = poly_rings.numel() - 1, offsets.numel() - 1
    else:
        n_polys, n_rings = offsets.numel() - 1, offsets.numel() - 1
    h = ctypes.c_void_p()
    m = ctypes.c_int64()
    with torch.cuda.device(px.device):
        _lib.check(lib.pip_join_create(ctypes.byref(h), _ptr(px), _ptr(py), px.numel(), _ptr(poly_rings), n_polys,
                                       _ptr(offsets), n_rings, _ptr(vx), _ptr(vy), vx.numel(), ctypes.byref(m),
                                       _stream_handle(stream)))
        try:
            n = int(m.value)
            out = dict(point=torch.empty(n, dtype=torch.int64, device=px.device),
                       poly=torch.empty(n, dtype=torch.int32, device=px.device),
                       px=torch.empty(n, dtype=torch.float64, device=px.device),
                       py=torch.empty(n, dtype=torch.float64, device=px.device))
            _lib.check(lib.pip_join_fill(h, _ptr(out["point"]), _ptr(out["poly"]), _ptr(out["px"]), _ptr(out["py"]),
                                         _stream_handle(stream)))
            if timing is not None:
                c, f = ctypes.c_float(), ctypes.c_float()
                _lib.check(lib.pip_join_timing(h, ctypes.byref(c), ctypes.byref(f)))
                timing.update(ms_count=c.value, ms_fill=f.value)
        finally:
            lib.pip_join_destroy(h)
    return out


def probe_copy(dst, src, stream=None):
    """Plain streaming copy of src into dst (same byte size, multiple of 16)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    _lib.check(_lib.load().pip_probe_copy(_ptr(dst), _ptr(src), nbytes, _stream_handle(stream)))


def probe_read(src, sink, stream=None):
    """Plain streaming read of src (byte size a multiple of 16); sink: a device
    tensor of at least 4 bytes that may receive one meaningless word."""
    if sink.numel() * sink.element_size() < 4:
        raise ValueError("sink must hold at least 4 bytes")
    nbytes = src.numel() * src.element_size()
    _lib.check(_lib.load().pip_probe_read(_ptr(src), nbytes, _ptr(sink), _stream_handle(stream)))


def probe_valu(iterations, sink, stream=None) -> int:
    """Vector-ALU issue probe (binary64 additions); sink: a device tensor of at
    least 8 bytes that may receive one meaningless word.  Returns the lane
    operations the launch performs."""
    if sink.numel() * sink.element_size() < 8:
        raise ValueError("sink must hold at least 8 bytes")
    n = ctypes.c_int64(0)
    _lib.check(_lib.load().pip_probe_valu(int(iterations), _ptr(sink), ctypes.byref(n), _stream_handle(stream)))
    return int(n.value)


def abi_version() -> int:
    return int(_lib.load().pip_abi_version())


def to_device(w, device="cuda"):
    """Copy a workloads.Workload's arrays to device tensors (dict of tensors)."""
    import torch
    d = dict(px=torch.from_numpy(w.px).to(device), py=torch.from_numpy(w.py).to(device),
             offsets=torch.from_numpy(w.offsets).to(device), vx=torch.from_numpy(w.vx).to(device),
             vy=torch.from_numpy(w.vy).to(device))
    d["point_poly"] = None if w.point_poly is None else torch.from_numpy(w.point_poly).to(device)
    if getattr(w, "poly_rings", None) is not None:
        d["poly_rings"] = torch.from_numpy(w.poly_rings).to(device)
    return d
