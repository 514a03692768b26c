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
    assert C.sizeof(abi.Bundle) == 96
    assert C.sizeof(abi.TraceParams) == 88
    assert abi.TraceParams.max_crossings.offset == 48
    assert abi.Bundle.chi_s.offset == 32
    assert abi.Bundle.center_dir.offset == 56
    assert abi.Bundle.fov_x.offset == 80
    assert abi.Bundle.fov_y.offset == 88


def _lib_directions(abi, center, fx, fy, nx, ny):
    import numpy as np
    c = (C.c_double * 3)(*center)
    out = np.full((nx * ny, 3), np.nan)
    st = abi.lib().rr_fov_directions(c, fx, fy, nx, ny, out.ctypes.data_as(C.c_void_p))
    assert st == 0, abi.last_error()
    return out


FOV_CASES = [((0.0, 0.0, 1.0), 0.08, 0.08, 16, 16), ((0.0, 0.0, -2.0), 0.05, 0.03, 9, 7),
             ((0.15, -0.1, 1.0), 0.07, 0.025, 37, 13), ((1.0, 0.0, 0.0), 0.17, 0.17, 8, 8),
             ((0.3, 0.4, 0.866), 0.2, 0.1, 1, 5), ((-0.5, 0.2, 0.4), 0.5, 0.5, 6, 1),
             ((0.0, 1.0, 0.0), 1.0, 2.0, 11, 11), ((0.2, 0.1, -0.97), 3.0, 0.01, 5, 3)]


def test_fov_directions_equal_input_generator(abi):
    """rr_fov_directions (Sec. III E, Eq. txty, gnomonic reading) gives the same
    bits as the seeded-input generator, which evaluates the same formula in
    the same order with one rounding per operation (tan from the C library)."""
    import numpy as np
    from paper_1601_02012_amd import inputs as I
    for center, fx, fy, nx, ny in FOV_CASES:
        got = _lib_directions(abi, center, fx, fy, nx, ny)
        ref = I.fov_directions(center, fx, fy, nx, ny)
        assert got.tobytes() == ref.tobytes(), (center, fx, fy, nx, ny)


def test_fov_directions_geometry(abi):
    """Eq. txty spacing Upsilon/(N-1) with the end points at +-Upsilon/2, unit
    norms, row-major ray ids (Eq. rayid: id = iy*nx + ix) and the centre ray
    on the map axis, recovered from the directions with an independently
    built frame (atan of the projections on e1, e2 over e3)."""
    import math

    import numpy as np
    for center, fx, fy, nx, ny in FOV_CASES:
        d = _lib_directions(abi, center, fx, fy, nx, ny)
        assert np.all(np.abs(np.sum(d * d, axis=1) - 1.0) <= 1e-15)
        c = np.asarray(center, dtype=float)
        e3 = c / np.linalg.norm(c)
        if e3[0] == 0.0 and e3[1] == 0.0:
            e1, e2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, math.copysign(1.0, e3[2]), 0.0])
        else:
            h = np.array([0.0, 0.0, 1.0]) if abs(e3[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
            e1 = np.cross(h, e3)
            e1 /= np.linalg.norm(e1)
            e2 = np.cross(e3, e1)
        assert abs(np.dot(np.cross(e1, e2), e3) - 1.0) < 1e-14   # right-handed frame
        tx = np.arctan2(d @ e1, d @ e3).reshape(ny, nx)
        ty = np.arctan2(d @ e2, d @ e3).reshape(ny, nx)
        want_x = (np.arange(nx) * (fx / (nx - 1)) - fx / 2) if nx > 1 else np.zeros(1)
        want_y = (np.arange(ny) * (fy / (ny - 1)) - fy / 2) if ny > 1 else np.zeros(1)
        np.testing.assert_allclose(tx, np.broadcast_to(want_x[None, :], (ny, nx)), rtol=0,
                                   atol=2e-15)
        np.testing.assert_allclose(ty, np.broadcast_to(want_y[:, None], (ny, nx)), rtol=0,
                                   atol=2e-15)
        if nx > 1:
            np.testing.assert_allclose(np.diff(tx, axis=1), fx / (nx - 1), rtol=1e-12)
            assert abs(tx[0, 0] + fx / 2) < 2e-15 and abs(tx[0, -1] - fx / 2) < 2e-15
        if nx % 2 == 1 and ny % 2 == 1:
            mid = (ny // 2) * nx + nx // 2
            np.testing.assert_allclose(d[mid], e3, rtol=0, atol=2.3e-16)
        else:   # an even map has no ray on the axis (Eq. txty)
            assert np.all(np.abs(d @ e3 - 1.0) > 0.0)


def test_fov_directions_rejections(abi):
    import numpy as np
    lib = abi.lib()
    out = np.zeros((16, 3))
    p = out.ctypes.data_as(C.c_void_p)
    c = (C.c_double * 3)(0.0, 0.0, 1.0)
    z = (C.c_double * 3)(0.0, 0.0, 0.0)
    nan = (C.c_double * 3)(float("nan"), 0.0, 1.0)
    assert lib.rr_fov_directions(None, 0.1, 0.1, 4, 4, p) == -1
    assert lib.rr_fov_directions(c, 0.1, 0.1, 4, 4, None) == -1
    assert lib.rr_fov_directions(z, 0.1, 0.1, 4, 4, p) == -1
    assert lib.rr_fov_directions(nan, 0.1, 0.1, 4, 4, p) == -7
    assert lib.rr_fov_directions(c, float("inf"), 0.1, 4, 4, p) == -7
    assert lib.rr_fov_directions(c, 3.2, 0.1, 4, 4, p) == -1     # beyond pi
    assert lib.rr_fov_directions(c, -0.1, 0.1, 4, 4, p) == -1
    assert lib.rr_fov_directions(c, 0.0, 0.1, 4, 4, p) == -1     # several rays, no angle
    assert lib.rr_fov_directions(c, 0.1, 0.1, 0, 4, p) == -1
    assert lib.rr_fov_directions(c, 0.1, 0.1, 4, 70000, p) == -1
    assert np.all(out == 0.0)                                    # nothing written
    assert lib.rr_fov_directions(c, 0.0, 0.1, 1, 4, p) == 0      # one ray on x: no angle needed


def test_python_binding_rejects_bad_buffers_before_any_launch():
    """The binding checks dtype, contiguity and length of every caller-supplied
    buffer before it touches the device (these run on the CPU: a rejection
    here means no kernel could have been launched)."""
    import types

    import pytest as _pt
    import torch
    from paper_1601_02012_amd import api
    b = api.RayBundle(torch.zeros((64, 3), dtype=torch.float64), 8, 8, 10.0, 10.0, 0.0,
                      ray_offset=16)
    fp32 = types.SimpleNamespace(precision=1, handle=None)
    fp64 = types.SimpleNamespace(precision=0, handle=None)
    with _pt.raises(ValueError, match="kappa holds"):
        api.trace(None, fp32, [b], (0, 0, 0), kappa=torch.zeros(79))
    with _pt.raises(ValueError, match="kappa must be"):
        api.trace(None, fp32, [b], (0, 0, 0), kappa=torch.zeros(80, dtype=torch.float64))
    with _pt.raises(ValueError, match="kappa must be"):
        api.trace(None, fp64, [b], (0, 0, 0), kappa=torch.zeros(80, dtype=torch.float32))
    with _pt.raises(ValueError, match="kappa_comp holds"):
        api.trace(None, fp32, [b], (0, 0, 0), kappa=torch.zeros(80),
                  kappa_comp=torch.zeros(10))
    with _pt.raises(ValueError, match="status must be"):
        api.trace(None, fp32, [b], (0, 0, 0), kappa=torch.zeros(80),
                  status=torch.zeros(80, dtype=torch.int64))
    with _pt.raises(ValueError, match="contiguous"):
        api.trace(None, fp32, [b], (0, 0, 0), kappa=torch.zeros(160)[::2])
    grid = types.SimpleNamespace(n=8, values=torch.zeros((8, 8, 8)))
    with _pt.raises(ValueError, match="dl_dkappa"):
        api.trace_adjoint(None, fp32, grid, [b], (0, 0, 0), torch.zeros(50))
    with _pt.raises(ValueError, match="dl_dphi must be"):
        api.trace_adjoint(None, fp32, grid, [b], (0, 0, 0), torch.zeros(80),
                          dl_dphi=torch.zeros((8, 8, 8), dtype=torch.float64))
    with _pt.raises(ValueError, match="dl_dphi holds"):
        api.trace_adjoint(None, fp32, grid, [b], (0, 0, 0), torch.zeros(80),
                          dl_dphi=torch.zeros((8, 8, 7)))
    st = api.SourcesOutput(torch.zeros((80, 4)), torch.zeros((80, 3, 2), dtype=torch.float64),
                           torch.zeros(80, dtype=torch.int32))
    with _pt.raises(ValueError, match="pieces"):
        api.trace_sources(None, fp32, [b], (0, 0, 0), [5.0, 4.0], state=st)
    st.moments = torch.zeros((80, 2))
    with _pt.raises(ValueError, match="moments holds"):
        api.trace_sources(None, fp32, [b], (0, 0, 0), [5.0, 4.0, 3.0], state=st)


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
    assert lib.rr_version() >= 10100
