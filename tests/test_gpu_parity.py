"""GPU parity: the HIP kernels through the C ABI against the CPU oracle, bit for bit.

Every comparison is element by element on the same seeded inputs; there is
no tolerance (the inside bit is decided in binary64 on both sides).
Full-size workloads are compared in full where the oracle finishes in
seconds (star, footprints, batched, stress) and on a seeded sample of points
for the 1,000,000-vertex fractal polygon.
"""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same_mask, note, to_dev
from paper_2306_04316_amd import workloads as W

pytestmark = pytest.mark.gpu

KERNELS = ["per_pair", "segmented", "staged", "runs"]


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2306_04316_amd as P
    return P


def run(P, w, kernel, **kw):
    import torch
    d = to_dev(w)
    out = P.classify(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], kernel=kernel, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(P, w, kernel, what):
    note(f"{what} kernel={kernel} N={w.n_points} P={w.n_polys} V={w.n_vertices}")
    got = run(P, w, kernel)
    want = oracle.classify_workload(w)
    assert_same_mask(got, want, f"{what}/{kernel}", w.px, w.py, w.point_poly)
    return got


@pytest.mark.parametrize("kernel", KERNELS)
def test_star_full(P, kernel):
    check(P, W.star(), kernel, "star full")


@pytest.mark.parametrize("kernel", KERNELS)
def test_footprints_small(P, kernel):
    # several blocks and a ragged tail
    check(P, W.footprints(scale=0.0123), kernel, "footprints small")


@pytest.mark.parametrize("kernel", KERNELS)
def test_footprints_full(P, kernel):
    check(P, W.footprints(), kernel, "footprints full")


@pytest.mark.parametrize("kernel", KERNELS)
def test_batched_small(P, kernel):
    check(P, W.batched(scale=0.01), kernel, "batched small")


@pytest.mark.parametrize("kernel", KERNELS)
def test_stress_small(P, kernel):
    check(P, W.stress(scale=0.02), kernel, "stress small")


def test_batched_full(P):
    check(P, W.batched(), "staged", "batched full")


def test_stress_full(P):
    check(P, W.stress(), "staged", "stress full")


@pytest.mark.parametrize("kernel", KERNELS)
def test_fractal_reduced(P, kernel):
    check(P, W.fractal(scale=0.001, n_vertices=20_000), kernel, "fractal 20k vertices")


def test_fractal_full_sampled(P):
    import torch
    w = W.fractal()
    note(f"fractal full sampled N={w.n_points} V={w.n_vertices}")
    got = run(P, w, "runs")
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(w.n_points, 1500, replace=False))
    s = W.subsample(w, idx)
    want = oracle.classify_workload(s)
    assert_same_mask(got[idx], want, "fractal full (sampled)", s.px, s.py)
    assert 0.2 < got.mean() < 0.9


def test_unsorted_pairs(P):
    w = W.footprints(scale=0.01)
    rng = np.random.default_rng(3)
    perm = rng.permutation(w.n_points)
    s = W.subsample(w, perm)
    for k in KERNELS:
        check(P, s, k, "footprints shuffled")


def test_degenerate_rings(P):
    # rings with 0, 1, 2 vertices, repeated vertices, a closing duplicate, collinear runs
    rings = [[], [(1.0, 1.0)], [(0.0, 0.0), (2.0, 2.0)], [(0, 0), (0, 0), (4, 0), (4, 0), (4, 4), (0, 4)],
             [(0, 0), (4, 0), (4, 4), (0, 4), (0, 0)], [(0, 0), (1, 0), (2, 0), (3, 0), (3, 3), (0, 3)],
             [(0, 0), (4, 4), (4, 0), (0, 4)]]
    vx, vy, off = [], [], [0]
    for r in rings:
        vx += [float(a) for a, _ in r]
        vy += [float(b) for _, b in r]
        off.append(len(vx))
    g = np.arange(-1.0, 5.01, 0.25)
    GX, GY = np.meshgrid(g, g)
    m = GX.size
    px = np.tile(GX.ravel(), len(rings))
    py = np.tile(GY.ravel(), len(rings))
    pp = np.repeat(np.arange(len(rings), dtype=np.int32), m)
    w = W.Workload("degenerate", px, py, np.array(off, dtype=np.int64), np.array(vx), np.array(vy), pp, {})
    for k in KERNELS:
        check(P, w, k, "degenerate rings")


def test_signed_zero_and_extremes(P):
    rx = np.array([-0.0, 1e-300, 1e-300, -0.0])
    ry = np.array([-0.0, -0.0, 1e-300, 1e-300])
    big = np.array([-1e300, 1e300, 1e300, -1e300])
    bigy = np.array([-1e300, -1e300, 1e300, 1e300])
    px = np.array([0.0, -0.0, 5e-301, 1e-300, 2e-300, 0.0, 1e299, -1e300, 0.0])
    py = np.array([0.0, -0.0, 5e-301, 5e-301, 5e-301, 1e-300, 0.0, 0.0, 1e300])
    for ringx, ringy, name in ((rx, ry, "tiny square"), (big, bigy, "huge square")):
        w = W.Workload(name, px, py, np.array([0, 4], dtype=np.int64), ringx, ringy, None, {})
        for k in KERNELS:
            check(P, w, k, name)


def test_empty_input(P):
    import torch
    note("empty input")
    w = W.footprints(scale=0.001)
    d = to_dev(w)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    out = P.classify(e, e, d["offsets"], d["vx"], d["vy"], torch.empty(0, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    assert out.numel() == 0


def test_deterministic_repeat(P):
    w = W.batched(scale=0.005)
    a = run(P, w, "segmented")
    b = run(P, w, "segmented")
    assert np.array_equal(a, b)


def test_validation_errors(P):
    import torch
    note("validation errors")
    w = W.footprints(scale=0.001)
    d = to_dev(w)
    args = lambda **o: {**d, **o}
    # clean data passes validation
    out = P.classify(**args(), validate=True)
    torch.cuda.synchronize()
    assert_same_mask(out.cpu().numpy(), oracle.classify_workload(w), "validated run")
    bad = d["point_poly"].clone()
    bad[7] = w.n_polys
    with pytest.raises(P.PipError) as e:
        P.classify(**args(point_poly=bad), validate=True)
    assert e.value.code == -2
    badoff = d["offsets"].clone()
    badoff[3] = badoff[5]
    with pytest.raises(P.PipError) as e:
        P.classify(**args(offsets=badoff), validate=True)
    assert e.value.code == -2
    badx = d["px"].clone()
    badx[11] = float("nan")
    with pytest.raises(P.PipError) as e:
        P.classify(**args(px=badx), validate=True)
    assert e.value.code == -3
    badv = d["vy"].clone()
    badv[0] = float("inf")
    with pytest.raises(P.PipError) as e:
        P.classify(**args(vy=badv), validate=True)
    assert e.value.code == -3
    with pytest.raises(P.PipError) as e:
        P.classify(**args(point_poly=None))
    assert e.value.code == -1


def test_bandwidth_probes(P):
    """The copy and read-stream probes the measurement uses: the copy is exact,
    the read leaves its sink word alone or writes one word, sizes are checked."""
    import torch
    src = torch.arange(1 << 20, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    P.probe_copy(dst, src)
    P.probe_read(src, sink)
    P.probe_read(src[:0], sink)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    with pytest.raises(P.PipError):
        P.probe_read(src[:3], sink)   # 12 bytes: not a multiple of 16
    # VALU probe: eight 256-thread workgroups per compute unit, eight
    # additions per round; the sink is not written (the sum cannot be -1)
    sink64 = torch.zeros(1, dtype=torch.float64, device="cuda")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    n = P.probe_valu(100, sink64)
    torch.cuda.synchronize()
    assert n == cus * 8 * 256 * 100 * 8
    assert sink64.item() == 0.0
    with pytest.raises(P.PipError):
        P.probe_valu(0, sink64)
    with pytest.raises(ValueError):
        P.probe_valu(10, sink)   # 4 bytes: too small
