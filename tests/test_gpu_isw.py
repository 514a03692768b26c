"""GPU parity of the ISW integrand (Sec. VII, Eq. I1 with Q = dPhi/dt)
against the FP64 oracle.

Bars: vertex scalars to 1e-13 (FP64) / 2e-7 (FP32, one rounding of an FP64
mean) of the field's scale; crossing hashes and counts bit-exact; FP64
integrals to 1e-11 of the map's scale; FP32-Kahan integrals within
max(1e-5 |I|, 1e-7) per ray, with the rate scaled so that the map's rms is
~1e-2 (the size of a convergence map, for which that bar is stated)."""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I
from tests._cases import gpu_bundle, hashes_u64, kappa_tolerance_ok

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1601_02012_amd import api as A
    return A


@pytest.fixture(scope="module")
def plan(api):
    return api.Plan()


def _grids(api, curr, prev, box, boundary="periodic"):
    import torch
    gc = api.Grid(torch.as_tensor(np.ascontiguousarray(curr)).cuda(), box, boundary=boundary)
    gp = api.Grid(torch.as_tensor(np.ascontiguousarray(prev)).cuda(), box, boundary=boundary)
    gd = api.Grid(gc.values, box, boundary=boundary, field="phi_dot")
    return gc, gp, gd


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-7)])
@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_isw_vertex_field_matches_oracle(api, oracle, prec, tol, boundary):
    rng = np.random.default_rng(7)
    for n in (8, 33):
        prev = rng.normal(size=(n, n, n))
        curr = prev + 0.01 * rng.normal(size=(n, n, n))
        if prec == "fp32":
            prev, curr = prev.astype(np.float32), curr.astype(np.float32)
        gc, gp, gd = _grids(api, curr, prev, float(n), boundary)
        t = api.TidalTensor(gd, prec).build_isw(gc, gp, 40.0)
        got = t.to_torch()[:, 0].double().cpu().numpy()
        ref = oracle.isw_vertex_field(curr.astype(np.float64), prev.astype(np.float64), 40.0,
                                      open_boundary=boundary == "open")
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        ok = ~np.isnan(ref)
        np.testing.assert_allclose(got[ok], ref[ok], rtol=0, atol=tol * np.abs(ref[ok]).max())
        t.close()


def _case(seed=11, n=32, box=96.0):
    rng = np.random.default_rng(seed)
    phi0 = I.poisson_phi(I.gaussian_field(n, box, rng, slope=-2.0), box)
    prev = 0.98 * phi0
    curr = phi0 + 0.02 * I.poisson_phi(I.gaussian_field(n, box, rng, slope=-2.0), box)
    fov = math.radians(8.0)
    dirs = I.fov_directions((0.1, -0.05, 1.0), fov, fov * 13 / 37, 37, 13)
    return curr, prev, dirs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_isw_trace_matches_oracle(api, oracle, plan, prec):
    n, box = 32, 96.0
    curr, prev, dirs = _case()
    dt = np.float64 if prec == "fp64" else np.float32
    curr, prev = curr.astype(dt), prev.astype(dt)
    gc, gp, gd = _grids(api, curr, prev, box)
    inv_dt = 1.0
    qv = oracle.isw_vertex_field(curr.astype(np.float64), prev.astype(np.float64), inv_dt)
    obs = (5.0, 7.0, 1.0)
    windows = [(250.0, 160.0), (160.0, 0.0)]
    # scale the map to an rms of ~1e-2 (the size the tolerance is stated for)
    probe = oracle.trace_uniform_isw(n, box, obs, dirs, 250.0, 0.0, qv=qv)
    scale = 1e-2 / np.sqrt(np.mean(probe.kappa ** 2))
    t = api.TidalTensor(gd, prec).build_isw(gc, gp, inv_dt)
    out = None
    ref_total = np.zeros(len(dirs))
    for hi, lo in windows:
        gb = gpu_bundle(api, dirs, 37, 13, 250.0, hi, lo)
        out = api.trace(plan, t, [gb], obs, kappa=None if out is None else out.kappa,
                        kappa_comp=None if out is None else out.kappa_comp, quantity="scalar",
                        kappa_scale=scale, debug=True)
        ref = oracle.trace_uniform_isw(n, box, obs, dirs, hi, lo, qv=qv, scale=scale)
        assert np.all(out.status.cpu().numpy() == 0)
        assert np.array_equal(out.count.cpu().numpy(), ref.ncross)
        assert np.array_equal(hashes_u64(out.hash), ref.hash)
        ref_total += ref.kappa
    got = out.kappa.double().cpu().numpy()
    if prec == "fp64":
        np.testing.assert_allclose(got, ref_total, rtol=0, atol=1e-11 * np.abs(ref_total).max())
    else:
        ok, worst = kappa_tolerance_ok(got, ref_total)
        assert ok, worst
    # the same rays through the tidal tensor follow the same cells
    tk = api.TidalTensor(gc, prec).build()
    gb = gpu_bundle(api, dirs, 37, 13, 250.0, 250.0, 160.0)
    o2 = api.trace(plan, tk, [gb], obs, debug=True)
    o3 = api.trace(plan, t, [gb], obs, quantity="scalar", debug=True)
    assert np.array_equal(hashes_u64(o2.hash), hashes_u64(o3.hash))
    t.close()
    tk.close()


def test_isw_rejections(api, plan):
    import torch
    n, box = 16, 32.0
    rng = np.random.default_rng(3)
    curr, prev = rng.normal(size=(2, n, n, n))
    gc, gp, gd = _grids(api, curr, prev, box)
    t = api.TidalTensor(gd, "fp64").build_isw(gc, gp, 1.0)
    tk = api.TidalTensor(gc, "fp64").build()
    dirs = I.fov_directions((0.0, 0.0, 1.0), 0.1, 0.1, 8, 8)
    gb = gpu_bundle(api, dirs, 8, 8, 20.0, 20.0, 0.0)
    with pytest.raises(api.RRError):
        api.trace(plan, t, [gb], (1.0, 1.0, 1.0))                      # kappa on an ISW tensor
    with pytest.raises(api.RRError):
        api.trace(plan, tk, [gb], (1.0, 1.0, 1.0), quantity="scalar")  # scalar on a tidal one
    with pytest.raises(api.RRError):
        api.trace(plan, t, [gb], (1.0, 1.0, 1.0), quantity="scalar", integral="ngp")
    with pytest.raises(api.RRError):
        t.build(gc)                                                    # not a tidal tensor
    with pytest.raises(api.RRError):
        tk.build_isw(gc, gp, 1.0)                                      # not an ISW tensor
    with pytest.raises(api.RRError):
        api.trace_sources(plan, t, [gb], (1.0, 1.0, 1.0), [20.0, 10.0], quantity="scalar")
    with pytest.raises(api.RRError):
        t.build_isw(gc, api.Grid(torch.zeros((8, 8, 8), dtype=torch.float64).cuda(), box), 1.0)
    t.close()
    tk.close()
