"""GPU parity of Method A (Eq. kappa2: density term, gradient term with
dg/dchi, per-step surface term) against the FP64 oracle: vertex fields,
crossing lists bit-exact, kappa to 1e-11 of the map's scale (FP64) or within
max(1e-5 |kappa|, 1e-7) (FP32-Kahan); the quadratic-potential identity with
Method B; segments adding up to one pass."""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I
from tests._cases import gpu_bundle, hashes_u64, kappa_tolerance_ok, small_periodic_case

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


def _grids(api, phi, delta, box, dtype, boundary="periodic"):
    import torch
    gp = api.Grid(torch.as_tensor(phi.astype(dtype)).cuda(), box, boundary=boundary)
    gd = api.Grid(torch.as_tensor(delta.astype(dtype)).cuda(), box, boundary=boundary,
                  field="delta")
    return gd, gp


def _case(seed, n, box):
    rng = np.random.default_rng(seed)
    delta = I.gaussian_field(n, box, rng, slope=-2.0)
    phi = I.poisson_phi(delta, box)
    return phi, 0.1 * delta


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_method_a_vertex_fields_match_oracle(api, oracle, prec, tol, boundary):
    n, box = 28, 56.0
    phi, delta = _case(41, n, box)
    dt = np.float64 if prec == "fp64" else np.float32
    cd = 3.7e-5
    gd, gp = _grids(api, phi, delta, box, dt, boundary)
    t = api.TidalTensor(gd, prec).build_method_a(gd, gp, cd)
    got = t.to_torch().double().cpu().numpy()
    ref = oracle.method_a_vertex_fields(phi.astype(dt), delta.astype(dt),
                                        open_boundary=boundary == "open")
    ref[:, 0] *= cd * (box / n) ** 2      # the library stores delta_coeff delta in cell units
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    for c in range(4):
        fin = ~nan[:, c]
        scale = np.abs(ref[fin, c]).max()
        np.testing.assert_allclose(got[fin, c], ref[fin, c], rtol=0, atol=tol * scale)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_method_a_trace_matches_oracle(api, oracle, plan, prec):
    n, box = 32, 64.0
    phi, delta = _case(42, n, box)
    _, dirs = small_periodic_case(seed=42, n=n, box=box, nx=23, ny=19)
    dt = np.float64 if prec == "fp64" else np.float32
    cd = 2.5e-4
    gd, gp = _grids(api, phi, delta, box, dt)
    t = api.TidalTensor(gd, prec).build_method_a(gd, gp, cd)
    obs = (2.3, -1.1, 0.6)
    chis, hi, lo = 160.0, 120.0, 7.5
    out = api.trace(plan, t, [gpu_bundle(api, dirs, 23, 19, chis, hi, lo)], obs, debug=True)
    ref = oracle.trace_uniform_method_a(n, box, obs, dirs, chis, hi, lo, delta_coeff=cd,
                                        phi=phi.astype(dt), delta=delta.astype(dt))
    assert np.array_equal(out.count.cpu().numpy(), ref.ncross)
    assert np.array_equal(hashes_u64(out.hash), ref.hash)
    k = out.kappa.double().cpu().numpy()
    if prec == "fp64":
        np.testing.assert_allclose(k, ref.kappa, rtol=0, atol=1e-11 * np.abs(ref.kappa).max())
    else:
        ok, worst = kappa_tolerance_ok(k, ref.kappa)
        assert ok, worst


def test_method_a_quadratic_equals_method_b(api, plan):
    """Quadratic potential, delta_coeff delta = tr M: Method A on the GPU gives
    the Method B closed form on every chi window (open grid)."""
    import torch
    n, box = 24, 24.0
    rng = np.random.default_rng(43)
    M = rng.normal(size=(3, 3)); M = M + M.T
    idx = np.arange(n) + 0.5
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    X = [x, y, z]
    phi = sum(0.5 * M[a, b] * X[a] * X[b] for a in range(3) for b in range(3))
    cd = 0.37
    delta = np.full((n, n, n), np.trace(M) / cd)
    gd, gp = _grids(api, phi, delta, box, np.float64, "open")
    t = api.TidalTensor(gd, "fp64").build_method_a(gd, gp, cd)
    dirs = I.fov_directions((0.05, -0.03, 1.0), math.radians(20.0), math.radians(20.0), 7, 7)
    obs = (12.1, 11.8, 3.2)
    chis = 30.0
    for hi, lo in [(17.5, 0.0), (11.0, 4.5)]:
        out = api.trace(plan, t, [gpu_bundle(api, dirs, 7, 7, chis, hi, lo)], obs)
        assert bool((out.status == 0).all())
        qv = np.trace(M) - np.einsum("ri,ij,rj->r", dirs, M, dirs)
        gint = (chis * (hi ** 2 - lo ** 2) / 2 - (hi ** 3 - lo ** 3) / 3) / chis
        np.testing.assert_allclose(out.kappa.cpu().numpy(), qv * gint, rtol=0,
                                   atol=1e-11 * np.abs(qv * gint).max())


def test_method_a_segments_add_up(api, plan):
    import torch
    n, box = 32, 64.0
    phi, delta = _case(44, n, box)
    _, dirs = small_periodic_case(seed=44, n=n, box=box, nx=16, ny=16)
    gd, gp = _grids(api, phi, delta, box, np.float64)
    t = api.TidalTensor(gd, "fp64").build_method_a(gd, gp, 1e-4)
    obs = (0.0, 0.0, 0.0)
    chis = 120.0
    one = api.trace(plan, t, [gpu_bundle(api, dirs, 16, 16, chis, 110.0, 0.0)], obs)
    kap = torch.zeros(256, dtype=torch.float64, device="cuda")
    edges = np.linspace(110.0, 0.0, 12)
    for a, b in zip(edges[:-1], edges[1:]):
        api.trace(plan, t, [gpu_bundle(api, dirs, 16, 16, chis, a, b)], obs, kappa=kap)
    k1 = one.kappa.cpu().numpy()
    np.testing.assert_allclose(kap.cpu().numpy(), k1, rtol=0, atol=1e-12 * np.abs(k1).max())


def test_method_a_rejections(api, plan):
    from paper_1601_02012_amd import _abi as A
    n, box = 16, 32.0
    phi, delta = _case(45, n, box)
    gd, gp = _grids(api, phi, delta, box, np.float64)
    t = api.TidalTensor(gd, "fp64").build_method_a(gd, gp, 1e-4)
    _, dirs = small_periodic_case(seed=45, n=n, box=box, nx=8, ny=8)
    b = [gpu_bundle(api, dirs, 8, 8, 30.0, 30.0, 0.0)]
    for kw in ({"quantity": "gamma1"}, {"integral": "ngp"}):
        with pytest.raises(A.RRError) as e:
            api.trace(plan, t, b, (0.0, 0.0, 0.0), **kw)
        assert e.value.status == -2
    with pytest.raises(A.RRError):
        t.build(gp)
    tb = api.TidalTensor(gp, "fp64")
    with pytest.raises(A.RRError):
        tb.build_method_a(gd, gp, 1e-4)
