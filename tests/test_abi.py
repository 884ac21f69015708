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


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2306_04316_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libpip.so"))
    with pytest.raises(ImportError):
        _lib.load()
