"""CPU-side checks of the C ABI: the library loads, exports every entry point
declared in include/rayramses.h, and rejects bad arguments on the host before
touching the GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rayramses.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rr_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def abi():
    from paper_1601_02012_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("librayramses.so is not built (run __graft_entry__.build())")
    return _abi


def test_header_declares_the_three_entry_points():
    names = _declared()
    for n in ("rr_build_tidal_tensor", "rr_trace_rays", "rr_trace_rays_adjoint"):
        assert n in names


def test_library_exports_every_declared_symbol(abi):
    lib = abi.lib()
    for n in _declared():
        assert hasattr(lib, n), n
    assert {s[0] for s in abi.SIGNATURES} == set(_declared())


def test_struct_layouts_match_header(abi):
    assert C.sizeof(abi.FieldDesc) == 56
    assert C.sizeof(abi.Bundle) == 56
    assert C.sizeof(abi.TraceParams) == 88
    assert abi.TraceParams.max_crossings.offset == 48
    assert abi.Bundle.chi_s.offset == 32


def test_host_validation_without_gpu(abi):
    lib = abi.lib()
    h = C.c_void_p()
    assert lib.rr_tensor_create(None, 1, C.byref(h)) == -1
    assert "NULL" in abi.last_error()
    d = abi.FieldDesc()
    d.kind, d.field, d.boundary, d.dtype = 0, 0, 0, 0
    d.n_base, d.box_size, d.values = 2, 1.0, C.c_void_p(16)
    assert lib.rr_tensor_create(C.byref(d), 1, C.byref(h)) == -1
    assert "n_base" in abi.last_error()
    d.n_base = 64
    d.field, d.kind = 1, 1
    assert lib.rr_tensor_create(C.byref(d), 1, C.byref(h)) == -2      # Method A on an octree
    d.field, d.kind = 2, 1
    assert lib.rr_tensor_create(C.byref(d), 1, C.byref(h)) == -2      # ISW on an octree
    d.field, d.kind = 5, 0
    assert lib.rr_tensor_create(C.byref(d), 1, C.byref(h)) == -1      # unknown field kind
    d.field = 0
    d.box_size = -1.0
    assert lib.rr_tensor_create(C.byref(d), 1, C.byref(h)) == -1
    d.box_size = 1.0
    d.boundary, d.n_base = 1, 5
    assert lib.rr_tensor_create(C.byref(d), 1, C.byref(h)) == -6      # open grid too small
    d.boundary, d.kind = 0, 1
    d.n_cells = 64 ** 3 + 3
    d.child_oct = C.c_void_p(16)
    assert lib.rr_tensor_create(C.byref(d), 1, C.byref(h)) == -5      # malformed octree
    assert lib.rr_trace_rays(None, None, None, None, 0, None, None, None, None) == -1
    assert lib.rr_graph_launch(None, None) == -1
    lo = (C.c_int32 * 3)(0, 0, 0)
    assert lib.rr_build_tidal_tensor_box(None, None, lo, lo, None) == -1
    assert "NULL" in abi.last_error()
    assert lib.rr_rays_vertex_box(None, None, None, None, 0, lo, lo, None) == -1
    src = (C.c_double * 2)(5.0, 3.0)
    assert lib.rr_trace_rays_sources(None, None, None, None, 0, src, 2, None, None, None,
                                     None) == -1
    assert lib.rr_kappa_from_pieces(None, None, src, 2, 1, None, None, None, None) == -1
    assert "plan" in abi.last_error()
    assert lib.rr_build_isw_field(None, None, None, 1.0, None) == -1
    assert lib.rr_version() >= 10000
