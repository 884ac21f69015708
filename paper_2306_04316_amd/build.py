"""Build libpip.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2306_04316_amd.build [--save-temps DIR]

All device code is compiled with -ffp-contract=off (the exact binary64 path
must round every operation separately) and with packed FP32 instructions
disabled.  Symbols are hidden except those pip.h marks PIP_API.
"""
from __future__ import annotations

import argparse
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpip.so")

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fvisibility=hidden",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _compile_objects(objdir: str, verbose: bool) -> list:
    """One hipcc per source, in parallel; returns the object files."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(objdir, exist_ok=True)
    cflags = [f for f in FLAGS if f != "-shared"]

    def one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = ["hipcc", *cflags, f"-I{INCLUDE}", f"-I{CSRC}", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True, cwd=PKG)
        return src, obj, r

    jobs = max(1, min(8, os.cpu_count() or 1))
    objs = []
    with ThreadPoolExecutor(jobs) as ex:
        for src, obj, r in ex.map(one, sources()):
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError(f"hipcc failed compiling {src}")
            objs.append(obj)
    return objs


def build(save_temps: str | None = None, verbose: bool = False) -> str:
    tmp = LIB + f".tmp{os.getpid()}"
    if not save_temps:
        # compile the sources in parallel, then link them into the library
        objdir = os.path.join(PKG, "_build", f"obj{os.getpid()}")
        try:
            objs = _compile_objects(objdir, verbose)
            cmd = ["hipcc", *FLAGS, *objs, "-o", tmp]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True, cwd=PKG)
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError(f"hipcc failed linking {LIB}")
        finally:
            import shutil
            shutil.rmtree(objdir, ignore_errors=True)
        os.replace(tmp, LIB)
        return LIB
    cmd = ["hipcc", *FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", *sources(), "-o", tmp]
    if save_temps:
        os.makedirs(save_temps, exist_ok=True)
        cmd.insert(1, f"-save-temps={'obj'}")
        cmd = [c for c in cmd if c != "-o"]
        cmd = cmd[:-1] + ["-o", os.path.join(save_temps, "libpip.so")]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=save_temps or PKG)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed building {LIB}")
    if save_temps:
        return os.path.join(save_temps, "libpip.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--save-temps", default=None, help="directory for intermediate files (ISA inspection)")
    a = ap.parse_args()
    print(build(a.save_temps, verbose=True))
