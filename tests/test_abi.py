"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every entry point the header declares, and rejects bad arguments before
touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gravfft.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(gf_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2005_10160_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.fail("libgravfft.so is not built; run __graft_entry__.build()")
    return _native.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("gf_plan_create", "gf_forward", "gf_adjoint", "gf_plan_destroy", "gf_workspace_bytes",
              "gf_plan_bytes", "gf_status_string", "gf_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2005_10160_amd import _native
    names = declared_functions()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_native.EXPORTED)


_CTYPES = {"int": ctypes.c_int, "unsigned": ctypes.c_uint, "size_t": ctypes.c_size_t, "double": ctypes.c_double}


def test_plan_info_binding_matches_header():
    """The binding's PlanInfo mirrors gf_plan_info_t field by field (names,
    order, C types), so the library writes every field where the binding
    reads it."""
    from paper_2005_10160_amd import _native
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct\s*\{(.*?)\}\s*gf_plan_info_t;", text, flags=re.S).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        fields += [(n.strip(), _CTYPES[ctype]) for n in names.split(",")]
    assert [(n, t) for n, t in _native.PlanInfo._fields_] == fields


def test_status_strings(lib):
    from paper_2005_10160_amd import _native
    for s in range(6):
        assert lib.gf_status_string(s).decode() == _native.status_name(s)


@pytest.mark.parametrize("args,what", [
    ((0, 16, 8, 50.0, 50.0, 50.0, 25.0, 0x3F, 0, 0), "nx"),
    ((16, 16, 0, 50.0, 50.0, 50.0, 25.0, 0x3F, 0, 0), "nz"),
    ((16, 16, 8, -1.0, 50.0, 50.0, 25.0, 0x3F, 0, 0), "dx"),
    ((16, 16, 8, 50.0, 50.0, 50.0, 0.0, 0x3F, 0, 0), "h"),
    ((16, 16, 8, 50.0, 50.0, 50.0, float("nan"), 0x3F, 0, 0), "h nan"),
    ((16, 16, 8, 50.0, 50.0, 50.0, 25.0, 0, 0, 0), "mask"),
    ((16, 16, 8, 50.0, 50.0, 50.0, 25.0, 0x200, 0, 0), "mask bits"),
    ((16, 16, 8, 50.0, 50.0, 50.0, 25.0, 0x3F, 7, 0), "precision"),
    ((16, 16, 8, 50.0, 50.0, 50.0, 25.0, 0x3F, 0, -1), "max_batch"),
])
def test_plan_rejects_bad_arguments(lib, args, what):
    from paper_2005_10160_amd import _native
    h = ctypes.c_void_p(123)
    st = lib.gf_plan_create(*args[:7], ctypes.c_uint(args[7]), args[8], args[9], None, ctypes.byref(h))
    assert st == _native.GF_EINVAL, what
    assert h.value is None
    assert lib.gf_last_error().decode() != ""


def test_plan_rejects_oversize(lib):
    from paper_2005_10160_amd import _native
    h = ctypes.c_void_p()
    st = lib.gf_plan_create(4096, 16, 8, 50.0, 50.0, 50.0, 25.0, ctypes.c_uint(0x3F), 0, 0, None, ctypes.byref(h))
    assert st == _native.GF_EUNSUPPORTED


def test_null_arguments(lib):
    from paper_2005_10160_amd import _native
    assert lib.gf_forward(None, None, None, 1, None, 0, None) == _native.GF_EINVAL
    assert lib.gf_adjoint(None, None, None, 1, None, 0, None) == _native.GF_EINVAL
    assert lib.gf_plan_bytes(None) == 0
    assert lib.gf_plan_destroy(None) == _native.GF_OK
    sz = ctypes.c_size_t()
    assert lib.gf_workspace_bytes(None, 0, 1, ctypes.byref(sz)) == _native.GF_EINVAL
    assert lib.gf_plan_create(16, 16, 8, 50.0, 50.0, 50.0, 25.0, ctypes.c_uint(0x3F), 0, 0, None, None) == _native.GF_EINVAL


@pytest.mark.parametrize("edges,what", [
    (None, "null edges"),
    ([0.0, 10.0, 10.0, 30.0, 40.0], "repeated edge"),
    ([0.0, 10.0, 5.0, 30.0, 40.0], "decreasing"),
    ([-1.0, 10.0, 20.0, 30.0, 40.0], "top above the surface"),
    ([0.0, 10.0, float("nan"), 30.0, 40.0], "nan"),
    ([0.0, 10.0, 20.0, 30.0, float("inf")], "inf"),
])
def test_layered_plan_rejects_bad_edges(lib, edges, what):
    from paper_2005_10160_amd import _native
    h = ctypes.c_void_p(123)
    z = None if edges is None else (ctypes.c_double * len(edges))(*edges)
    st = lib.gf_plan_create_layered(16, 16, 4, 50.0, 50.0, z, 25.0, ctypes.c_uint(0x3F), 0, 0, None,
                                    ctypes.byref(h))
    assert st == _native.GF_EINVAL, what
    assert h.value is None
    assert lib.gf_last_error().decode() != ""


@pytest.mark.parametrize("levels,dz,what", [(0, 50.0, "no level"), (-3, 50.0, "negative"), (4, 0.0, "dz")])
def test_levels_plan_rejects_bad_arguments(lib, levels, dz, what):
    from paper_2005_10160_amd import _native
    h = ctypes.c_void_p(123)
    st = lib.gf_plan_create_levels(16, 16, 4, 50.0, 50.0, dz, 25.0, levels, ctypes.c_uint(0x3F), 0, 0, None,
                                   ctypes.byref(h))
    assert st == _native.GF_EINVAL, what
    assert h.value is None


def test_levels_plan_rejects_oversize(lib):
    from paper_2005_10160_amd import _native
    h = ctypes.c_void_p()
    st = lib.gf_plan_create_levels(1024, 1024, 100, 20.0, 20.0, 20.0, 10.0, 2147483600, ctypes.c_uint(0x1), 0, 0,
                                   None, ctypes.byref(h))
    assert st == _native.GF_EUNSUPPORTED
    assert h.value is None
