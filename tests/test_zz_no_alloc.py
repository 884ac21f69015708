"""pip_classify_noalloc (the entry point for callers that cannot allocate device
memory) through the C ABI: its masks equal pip_classify's in the filtered
mode, bit for bit and against the oracle, on two calls in a row (the second
with a smaller input, on the same static scratch array), in the exact mode on
the batched kernel (its item descriptors in the array) and by default;
an input beyond the array's capacity is rejected before any device call."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import assert_same_mask, note, to_dev
from paper_2306_04316_amd import workloads as W


def call(lib, fn, d, out, mode, stream, kernel=0):
    from paper_2306_04316_amd import _lib
    o = _lib.pip_options()
    lib.pip_options_init(ctypes.byref(o))
    o.mode = mode
    o.kernel = kernel
    pp = d["point_poly"]
    rc = getattr(lib, fn)(ctypes.c_void_p(d["px"].data_ptr()), ctypes.c_void_p(d["py"].data_ptr()),
                          d["px"].numel(), ctypes.c_void_p(d["offsets"].data_ptr()), d["offsets"].numel() - 1,
                          ctypes.c_void_p(d["vx"].data_ptr()), ctypes.c_void_p(d["vy"].data_ptr()),
                          d["vx"].numel(), None if pp is None else ctypes.c_void_p(pp.data_ptr()),
                          ctypes.c_void_p(out.data_ptr()), ctypes.byref(o), stream)
    _lib.check(rc)


@pytest.mark.gpu
def test_noalloc_matches_classify():
    import torch
    from paper_2306_04316_amd import _lib
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    lib = _lib.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # the second input is smaller than the first: the array keeps the first call's list
    for w in (W.stress(scale=0.03), W.stress(scale=0.004, seed=2)):
        assert w.n_points <= _lib.PIP_NOALLOC_MAX_POINTS
        d = to_dev(w)
        want = oracle.classify_workload(w)
        # filtered (batched kernel), exact batched kernel (descriptors in the array), exact default
        for mode, kernel in ((1, 0), (0, 5), (0, 0)):
            a = torch.full((w.n_points,), 7, dtype=torch.uint8, device="cuda")
            b = torch.full((w.n_points,), 9, dtype=torch.uint8, device="cuda")
            note(f"noalloc mode={mode} kernel={kernel} N={w.n_points}")
            call(lib, "pip_classify", d, a, mode, stream, kernel)
            call(lib, "pip_classify_noalloc", d, b, mode, stream, kernel)
            torch.cuda.synchronize()
            ga, gb = a.cpu().numpy(), b.cpu().numpy()
            assert np.array_equal(ga, gb), f"noalloc differs from pip_classify (mode {mode}, N={w.n_points})"
            assert_same_mask(gb, want, f"noalloc mode {mode} kernel {kernel}", w.px, w.py, w.point_poly)


def test_noalloc_rejects_oversized_input():
    """Checked on the host before any device call (runs without a GPU)."""
    from paper_2306_04316_amd import _lib
    lib = _lib.load()
    o = _lib.pip_options()
    lib.pip_options_init(ctypes.byref(o))
    o.mode = 1
    dummy = ctypes.c_void_p(16)
    n = _lib.PIP_NOALLOC_MAX_POINTS + 1
    rc = lib.pip_classify_noalloc(dummy, dummy, n, dummy, 1, dummy, dummy, 4, None, dummy, ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL and b"static scratch" in lib.pip_last_error()
    # the exact mode on the batched kernel keeps its item descriptors in the same array
    o.mode = 0
    o.kernel = 5
    rc = lib.pip_classify_noalloc(dummy, dummy, n, dummy, 1, dummy, dummy, 4, None, dummy, ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL and b"static scratch" in lib.pip_last_error()
