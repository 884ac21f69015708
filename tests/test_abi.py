"""The C-ABI library (no GPU needed): it loads, exports exactly what include/pip.h declares,
and rejects bad host-side arguments before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pip.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"PIP_API\s+[\w\s\*]+?\b(pip_\w+)\s*\(", src)))


def exported(path):
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True, check=True).stdout
    return sorted({ln.split()[-1] for ln in out.splitlines() if " T " in ln})


@pytest.fixture(scope="module")
def lib():
    from paper_2306_04316_amd import _lib
    return _lib.load()


def test_header_declares_api():
    names = declared()
    assert "pip_classify" in names and "pip_last_error" in names and len(names) >= 5


def test_exports_match_header(lib):
    from paper_2306_04316_amd import _lib
    exp = exported(_lib.LIB_PATH)
    assert exp == declared(), f"exported {exp} vs declared {declared()}"
    for name in declared():
        assert hasattr(lib, name)
    assert set(_lib.declared_symbols()) == set(declared())


def test_abi_version(lib):
    src = open(HEADER).read()
    v = int(re.search(r"#define PIP_ABI_VERSION (\d+)", src).group(1))
    assert lib.pip_abi_version() == v


def test_options_struct_matches_header(lib):
    from paper_2306_04316_amd import _lib
    o = _lib.pip_options()
    lib.pip_options_init(ctypes.byref(o))
    assert o.struct_size == ctypes.sizeof(_lib.pip_options)
    assert o.mode == 0 and o.kernel == 0 and o.validate == 0


def test_host_argument_errors(lib):
    """Checked on the host before any device call, so they work without a GPU."""
    from paper_2306_04316_amd import _lib
    o = _lib.pip_options()
    lib.pip_options_init(ctypes.byref(o))
    dummy = ctypes.c_void_p(16)
    # negative count
    rc = lib.pip_classify(dummy, dummy, -1, dummy, 1, dummy, dummy, 4, None, dummy, ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL and b"negative" in lib.pip_last_error()
    # several polygons without a pair index
    rc = lib.pip_classify(dummy, dummy, 10, dummy, 3, dummy, dummy, 12, None, dummy, ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL and b"point_poly" in lib.pip_last_error()
    # wrong struct size
    o2 = _lib.pip_options()
    lib.pip_options_init(ctypes.byref(o2))
    o2.struct_size = 3
    rc = lib.pip_classify(dummy, dummy, 10, dummy, 1, dummy, dummy, 4, None, dummy, ctypes.byref(o2), None)
    assert rc == _lib.PIP_EINVAL and b"struct_size" in lib.pip_last_error()
    # unknown kernel
    o.kernel = 99
    rc = lib.pip_classify(dummy, dummy, 10, dummy, 1, dummy, dummy, 4, None, dummy, ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL
    # NULL offsets
    o.kernel = 0
    rc = lib.pip_classify(dummy, dummy, 10, None, 1, dummy, dummy, 4, None, dummy, ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL
    # unknown predicate
    o.predicate = 7
    rc = lib.pip_classify(dummy, dummy, 10, dummy, 1, dummy, dummy, 4, None, dummy, ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL and b"predicate" in lib.pip_last_error()
    # constraint 2 is not offered by the binary32 filter
    o.predicate = 1
    o.mode = 1
    plan = ctypes.c_void_p()
    rc = lib.pip_plan_create(ctypes.byref(plan), dummy, dummy, 10, dummy, 1, dummy, dummy, 4, None, dummy,
                             ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL and b"filtered" in lib.pip_last_error()
    o.predicate = 0
    o.mode = 0
    # polygons of several rings: the ring index is required
    rc = lib.pip_classify_rings(dummy, dummy, 10, None, 1, dummy, 1, dummy, dummy, 4, None, dummy,
                                ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL and b"poly_rings" in lib.pip_last_error()
    rc = lib.pip_classify_rings(dummy, dummy, 10, dummy, 1, dummy, -1, dummy, dummy, 4, None, dummy,
                                ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL and b"n_rings" in lib.pip_last_error()
    o.mode = 1
    rc = lib.pip_plan_create_rings(ctypes.byref(plan), dummy, dummy, 10, dummy, 1, dummy, 1, dummy, dummy, 4, None,
                                   dummy, ctypes.byref(o), None)
    assert rc == _lib.PIP_ENOTSUP
    o.mode = 0
    # copy probe with a size that is not a multiple of 16
    rc = lib.pip_probe_copy(dummy, dummy, 17, None)
    assert rc == _lib.PIP_EINVAL
    rc = lib.pip_probe_read(dummy, 17, dummy, None)
    assert rc == _lib.PIP_EINVAL
    rc = lib.pip_probe_read(dummy, 16, None, None)
    assert rc == _lib.PIP_EINVAL
    # VALU probe: iterations out of range, NULL sink or count
    n = ctypes.c_int64(-1)
    for it, sk, cnt in ((0, dummy, ctypes.byref(n)), ((1 << 24) + 1, dummy, ctypes.byref(n)),
                        (16, None, ctypes.byref(n)), (16, dummy, None)):
        rc = lib.pip_probe_valu(it, sk, cnt, None)
        assert rc == _lib.PIP_EINVAL and b"pip_probe_valu" in lib.pip_last_error()
    assert n.value == -1


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2306_04316_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libpip.so"))
    with pytest.raises(ImportError):
        _lib.load()


def test_filtered_and_batched_argument_errors(lib):
    """Host-side checks of the filtered pip_classify, the batched kernel and the
    plans' int32 pair limit (no device call is made)."""
    from paper_2306_04316_amd import _lib
    o = _lib.pip_options()
    lib.pip_options_init(ctypes.byref(o))
    dummy = ctypes.c_void_p(16)
    plan = ctypes.c_void_p()
    # the filtered mode of pip_classify: batched kernel, constraint 1, one ring per polygon
    o.mode = 1
    o.kernel = 3
    rc = lib.pip_classify(dummy, dummy, 10, dummy, 1, dummy, dummy, 4, None, dummy, ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL and b"batched" in lib.pip_last_error()
    o.kernel = 0
    o.predicate = 1
    rc = lib.pip_classify(dummy, dummy, 10, dummy, 1, dummy, dummy, 4, None, dummy, ctypes.byref(o), None)
    assert rc == _lib.PIP_ENOTSUP
    o.predicate = 0
    rc = lib.pip_classify_rings(dummy, dummy, 10, dummy, 1, dummy, 1, dummy, dummy, 4, None, dummy,
                                ctypes.byref(o), None)
    assert rc == _lib.PIP_ENOTSUP
    big = (1 << 31)
    rc = lib.pip_classify(dummy, dummy, big, dummy, 1, dummy, dummy, 4, None, dummy, ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL and b"2^31" in lib.pip_last_error()
    # plans: fewer than 2^31 pairs in either mode (int32 pair ids in the recheck list and the item order)
    for mode in (0, 1):
        o.mode = mode
        rc = lib.pip_plan_create(ctypes.byref(plan), dummy, dummy, big, dummy, 1, dummy, dummy, 4, None, dummy,
                                 ctypes.byref(o), None)
        assert rc == _lib.PIP_EINVAL and b"2^31" in lib.pip_last_error()
        assert not plan.value
    # the batched kernel: constraint 1 only
    o.mode = 0
    o.kernel = 5
    o.predicate = 1
    rc = lib.pip_classify(dummy, dummy, 10, dummy, 1, dummy, dummy, 4, None, dummy, ctypes.byref(o), None)
    assert rc == _lib.PIP_ENOTSUP
    rc = lib.pip_plan_create(ctypes.byref(plan), dummy, dummy, 10, dummy, 1, dummy, dummy, 4, None, dummy,
                             ctypes.byref(o), None)
    assert rc == _lib.PIP_ENOTSUP
    o.predicate = 0
    # stats counting: 0 or 1, and only with the batched kernel
    o.stats = 2
    rc = lib.pip_plan_create(ctypes.byref(plan), dummy, dummy, 10, dummy, 1, dummy, dummy, 4, None, dummy,
                             ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL and b"stats" in lib.pip_last_error()
    o.stats = 1
    o.kernel = 3
    rc = lib.pip_plan_create(ctypes.byref(plan), dummy, dummy, 10, dummy, 1, dummy, dummy, 4, None, dummy,
                             ctypes.byref(o), None)
    assert rc == _lib.PIP_EINVAL and b"batched" in lib.pip_last_error()
    # pip_plan_execute / pip_plan_stats with a NULL plan
    st = _lib.pip_stats()
    assert lib.pip_plan_execute(None, ctypes.byref(st), None) == _lib.PIP_EINVAL
    assert lib.pip_plan_stats(None, ctypes.byref(st)) == _lib.PIP_EINVAL


def test_stats_struct_layout():
    """pip_stats as the header lays it out: four 64-bit counters, then three floats."""
    from paper_2306_04316_amd import _lib
    names = [f for f, _ in _lib.pip_stats._fields_]
    assert names == ["pairs", "tests", "ambiguous_tests", "rechecked_pairs", "ms_prep", "ms_main", "ms_recheck"]
    src = open(HEADER).read()
    body = re.search(r"typedef struct \{([^{}]*?)\} pip_stats;", src, re.S).group(1)
    hdr = re.findall(r"^\s*(?:uint64_t|float)\s+(\w+);", body, re.M)
    assert hdr == names
