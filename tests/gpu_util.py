"""Helpers for GPU parity tests: device copies and mask comparison against the oracle."""
from __future__ import annotations

import sys

import numpy as np


def note(msg: str) -> None:
    """Name the case before a GPU step, so a fault can be traced to it."""
    sys.stdout.write(f"[gpu-case] {msg}\n")
    sys.stdout.flush()
    sys.stderr.write(f"[gpu-case] {msg}\n")
    sys.stderr.flush()


def to_dev(w):
    import paper_2306_04316_amd as P
    return P.to_device(w, "cuda")


def assert_same_mask(got: np.ndarray, want: np.ndarray, what: str, px=None, py=None, pp=None):
    got = np.asarray(got, dtype=np.uint8)
    want = np.asarray(want, dtype=np.uint8)
    assert got.shape == want.shape, f"{what}: shape {got.shape} vs {want.shape}"
    bad = np.nonzero(got != want)[0]
    if bad.size:
        i = int(bad[0])
        extra = ""
        if px is not None:
            extra = f" first at {i}: p=({px[i]!r},{py[i]!r})"
            if pp is not None:
                extra += f" poly={int(pp[i])}"
        raise AssertionError(f"{what}: {bad.size} of {got.size} bits differ from the oracle;{extra} "
                             f"gpu={got[i]} oracle={want[i]}")
