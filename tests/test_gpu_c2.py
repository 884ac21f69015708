"""GPU parity of the second crossing test (constraint 2, Algorithm 2: the
parametric intersection x = a_x + lambda (b_x - a_x) compared with p_x), for
every exact kernel, the plans and the y-index -- bit for bit against the
oracle's constraint-2 function."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same_mask, note, to_dev
from paper_2306_04316_amd import workloads as W

pytestmark = pytest.mark.gpu

KERNELS = ["per_pair", "segmented", "staged", "runs"]

SMALL = {
    "star": lambda: W.star(),
    "footprints": lambda: W.footprints(scale=0.0123),
    "batched": lambda: W.batched(scale=0.01),
    "stress": lambda: W.stress(scale=0.02),
    "fractal": lambda: W.fractal(scale=0.001, n_vertices=20_000),
}


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2306_04316_amd as P
    return P


def want_c2(w):
    return oracle.classify_workload(w, predicate=2)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name", list(SMALL))
def test_classify_c2(P, kernel, name):
    import torch
    w = SMALL[name]()
    note(f"c2 classify {name} kernel={kernel} N={w.n_points} V={w.n_vertices}")
    d = to_dev(w)
    got = P.classify(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], kernel=kernel,
                     predicate="intersection")
    torch.cuda.synchronize()
    assert_same_mask(got.cpu().numpy(), want_c2(w), f"c2 {name} {kernel}", w.px, w.py, w.point_poly)


def test_c2_differs_from_c1_somewhere(P):
    """On points placed exactly on edges the two tests round differently, so
    the constraint-2 path must not silently run constraint 1."""
    import torch
    w = W.stress(scale=0.02)
    c1, c2 = oracle.classify_workload(w), want_c2(w)
    assert np.count_nonzero(c1 != c2) > 0
    d = to_dev(w)
    got = P.classify(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], kernel="staged",
                     predicate="intersection").cpu().numpy()
    assert_same_mask(got, c2, "c2 stress staged")


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("persistent", [0, 1])
def test_plan_c2(P, name, persistent):
    import torch
    w = SMALL[name]()
    note(f"c2 plan {name} persistent={persistent}")
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], predicate="intersection",
                persistent=persistent)
    pl.execute()
    torch.cuda.synchronize()
    assert_same_mask(pl.out.cpu().numpy(), want_c2(w), f"c2 plan {name}", w.px, w.py, w.point_poly)
    pl.close()


def test_plan_c2_full_footprints(P):
    import torch
    w = W.footprints()
    note("c2 plan footprints full")
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], predicate="intersection")
    pl.execute()
    torch.cuda.synchronize()
    assert_same_mask(pl.out.cpu().numpy(), want_c2(w), "c2 footprints full", w.px, w.py, w.point_poly)
    pl.close()


@pytest.mark.parametrize("name", ["star", "fractal"])
def test_plan_c2_index(P, name):
    import torch
    w = SMALL[name]()
    note(f"c2 index {name}")
    d = to_dev(w)
    pl = P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], predicate="intersection",
                index=True)
    pl.execute()
    torch.cuda.synchronize()
    assert_same_mask(pl.out.cpu().numpy(), want_c2(w), f"c2 index {name}", w.px, w.py)
    pl.close()


def test_c2_rejected_in_filtered_mode(P):
    w = W.footprints(scale=0.001)
    d = to_dev(w)
    with pytest.raises(P.PipError) as e:
        P.Plan(d["px"], d["py"], d["offsets"], d["vx"], d["vy"], d["point_poly"], mode="filtered",
               predicate="intersection")
    assert e.value.code == -1
