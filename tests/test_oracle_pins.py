"""The CPU oracle against its pins (no GPU).  See pins.py for what each pin fixes."""
import numpy as np
import pytest

import pins
from paper_2306_04316_amd import workloads as W

PIN_NAMES = ["golden", "rectangles", "convex", "winding", "invariants", "paper_form", "star", "footprints"]


@pytest.fixture(scope="module")
def star_w():
    return W.star()


@pytest.fixture(scope="module")
def fp_w():
    return W.footprints(scale=0.01)


def run_pin(name, oracle, mutant, star_w, fp_w):
    if name == "golden":
        return pins.pin_golden(oracle, mutant)
    if name == "rectangles":
        return pins.pin_rectangles(oracle, mutant)
    if name == "convex":
        return pins.pin_convex(oracle, mutant)
    if name == "winding":
        return pins.pin_winding(oracle, mutant)
    if name == "invariants":
        return pins.pin_invariants(oracle, mutant)
    if name == "paper_form":
        return pins.pin_paper_form(oracle, mutant)
    if name == "star":
        return pins.pin_star_closed_form(oracle, star_w, mutant)
    if name == "footprints":
        return pins.pin_footprints_exact(oracle, fp_w, mutant)
    raise KeyError(name)


@pytest.mark.parametrize("name", PIN_NAMES)
def test_oracle_pinned(name, oracle_mod, star_w, fp_w):
    fails = run_pin(name, oracle_mod, 0, star_w, fp_w)
    assert not fails, "\n".join(fails[:5])


# Planted mistakes (compiled into the oracle with PIP_ORACLE_MUTANT):
#  1 boundary strictness s < 0     2 anchor at b instead of a   3 no normal flip
#  4 closing edge dropped          5 straddle with >=           6 wrong sign of n_y
#  7 n_x and n_y transposed
@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5, 6, 7])
def test_planted_mistake_is_caught(mutant, oracle_mod, star_w, fp_w):
    caught = []
    for name in PIN_NAMES:
        if run_pin(name, oracle_mod, mutant, star_w, fp_w):
            caught.append(name)
    assert caught, f"mutant {mutant} passed every pin"


def test_area_sum_pin_is_exercised():
    """The triangulation pin must actually triangulate some polygons."""
    import exact_geom as X
    xs = np.array([0, 4, 4, 2, 0])
    ys = np.array([0, 0, 3, 1, 3])
    tris = X.ear_clip(xs, ys)
    assert len(tris) == 3
    inside = X.in_some_triangle(np.array([2, 2, 1]), np.array([2, 0, 1]), tris)
    assert inside.tolist() == [False, True, True]


def test_quadrant_winding_closed_forms():
    import exact_geom as X
    sq = (np.array([0, 2, 2, 0]), np.array([0, 0, 2, 2]))
    assert X.winding_int([1], [1], *sq).tolist() == [1]
    assert X.winding_int([1], [1], sq[0][::-1], sq[1][::-1]).tolist() == [-1]
    assert X.winding_int([3], [1], *sq).tolist() == [0]
    # a ring wound twice around the origin
    ang = np.arange(8) * (2 * np.pi / 4)
    xs = np.rint(5 * np.cos(ang)).astype(np.int64)
    ys = np.rint(5 * np.sin(ang)).astype(np.int64)
    assert X.winding_int([0], [1], xs, ys).tolist() == [2]


def test_oracle_threads_do_not_change_results(oracle_mod):
    w = W.footprints(scale=0.02)
    a = oracle_mod.classify_workload(w, nthreads=1)
    b = oracle_mod.classify_workload(w, nthreads=7)
    assert np.array_equal(a, b)
    assert 0.3 < a.mean() < 0.7


def test_oracle_rejects_bad_arguments(oracle_mod):
    w = W.footprints(scale=0.001)
    bad = w.point_poly.copy()
    bad[0] = w.n_polys
    with pytest.raises(ValueError):
        oracle_mod.classify(w.px, w.py, w.offsets, w.vx, w.vy, bad)
    with pytest.raises(ValueError):
        oracle_mod.classify(w.px, w.py, w.offsets, w.vx, w.vy, None)   # several polygons, no index
    assert oracle_mod.classify(w.px[:0], w.py[:0], w.offsets, w.vx, w.vy, w.point_poly[:0]).shape == (0,)
