"""rr_trace_rays_noalloc (the allocation-free trace, for callers that cannot
allocate device memory) against rr_trace_rays on the same inputs: two calls
in a row, the second with a smaller input, each bitwise equal to the
plan-based trace in the same launch shape (same kernels), on a uniform grid
and on an octree, direct and persistent; more bundles than its fixed table
holds are refused before anything is enqueued."""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I
from tests._cases import gpu_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available()
    from paper_1601_02012_amd import api as A
    return A


def _bundles(api, specs):
    """specs: (center, fov_deg, nx, ny, chi_s, chi_hi, chi_lo); packed at offsets."""
    import torch
    out, off = [], 0
    for center, fov_deg, nx, ny, chi_s, hi, lo in specs:
        fov = math.radians(fov_deg)
        d = torch.as_tensor(I.fov_directions(center, fov, fov, nx, ny)).cuda()
        out.append(api.RayBundle(d, nx, ny, chi_s, hi, lo, off, center, fov, fov))
        off += nx * ny
    return out


def _compare(api, tens, bundles, obs, persistent):
    import torch
    nr = api.total_rays(bundles)
    fp32 = tens.precision == 1
    dt = torch.float32 if fp32 else torch.float64
    plan = api.Plan()
    ref = api.trace(plan, tens, bundles, obs, persistent=persistent, debug=True)
    kap = torch.full((nr,), 0.25, dtype=dt, device="cuda")
    kap.zero_()
    comp = torch.zeros(nr, dtype=torch.float32, device="cuda") if fp32 else None
    st = torch.full((nr,), -5, dtype=torch.int32, device="cuda")
    hsh = torch.zeros(nr, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(nr, dtype=torch.int64, device="cuda")
    out = api.trace_noalloc(tens, bundles, obs, kappa=kap, kappa_comp=comp, status=st,
                            persistent=persistent, hash=hsh, count=cnt)
    torch.cuda.synchronize()
    assert torch.equal(out.kappa, ref.kappa)
    if fp32:
        assert torch.equal(out.kappa_comp, ref.kappa_comp)
    assert torch.equal(out.status, ref.status)
    assert torch.equal(out.hash, ref.hash)
    assert torch.equal(out.count, ref.count)
    assert bool((out.count > 0).all())
    plan.close()


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_equals_plan_trace_uniform(api, prec, persistent):
    import torch
    rng = np.random.default_rng(77)
    n, box = 32, 64.0
    phi = I.poisson_phi(I.gaussian_field(n, box, rng, slope=-2.0), box)
    g = gpu_grid(api, phi, box, dtype=torch.float32 if prec == "fp32" else torch.float64)
    t = api.TidalTensor(g, prec).build()
    obs = (1.5, 2.25, 0.5)
    big = _bundles(api, [((0.1, 0.0, 1.0), 6.0, 37, 13, 95.0, 95.0, 3.0),
                         ((0.0, 0.3, 1.0), 3.0, 16, 16, 80.0, 60.0, 10.0),
                         ((-0.2, 0.1, 1.0), 9.0, 5, 21, 120.0, 100.0, 0.0)])
    small = _bundles(api, [((0.2, -0.1, 1.0), 4.0, 9, 7, 70.0, 70.0, 20.0)])
    _compare(api, t, big, obs, persistent)      # first call
    _compare(api, t, small, obs, persistent)    # second call, smaller input
    t.close()


@pytest.mark.parametrize("persistent", [0, 1])
def test_noalloc_equals_plan_trace_octree(api, persistent):
    import torch
    rng = np.random.default_rng(78)
    tree = I.random_octree(8, 2, 0.25, rng)
    box = 32.0
    phi = rng.standard_normal(tree.n_cells) * 1e-5
    grid = api.Grid(torch.as_tensor(phi.astype(np.float32)).cuda(), box, n_base=tree.n,
                    child_oct=torch.as_tensor(tree.child_oct).cuda(), max_level=tree.max_level)
    t = api.TidalTensor(grid, "fp32").build()
    obs = (0.3, 0.7, 0.1)
    big = _bundles(api, [((0.1, 0.2, 1.0), 8.0, 24, 17, 60.0, 60.0, 0.0),
                         ((0.3, 0.0, 1.0), 5.0, 8, 8, 50.0, 40.0, 5.0)])
    small = _bundles(api, [((0.0, 0.0, 1.0), 2.0, 3, 4, 30.0, 30.0, 0.0)])
    _compare(api, t, big, obs, persistent)
    _compare(api, t, small, obs, persistent)
    t.close()


def test_noalloc_refuses_more_bundles_than_its_table(api):
    import torch
    rng = np.random.default_rng(79)
    n, box = 16, 32.0
    phi = I.poisson_phi(I.gaussian_field(n, box, rng, slope=-2.0), box)
    t = api.TidalTensor(gpu_grid(api, phi, box, dtype=torch.float32), "fp32").build()
    d = torch.as_tensor(I.fov_directions((0, 0, 1.0), 0.05, 0.05, 1, 1)).cuda()
    bundles = [api.RayBundle(d, 1, 1, 20.0, 20.0, 0.0, k) for k in range(1025)]
    kap = torch.full((1025,), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(api.RRError) as e:
        api.trace_noalloc(t, bundles, (0.5, 0.5, 0.5), kappa=kap)
    assert e.value.status == -8 and "1024" in str(e.value)
    torch.cuda.synchronize()
    assert bool((kap == 7.0).all())
    out = api.trace_noalloc(t, bundles[:1024], (0.5, 0.5, 0.5), kappa=kap[:1024].clone().zero_())
    torch.cuda.synchronize()
    ref = api.trace(api.Plan(), t, bundles[:1024], (0.5, 0.5, 0.5), persistent=0)
    assert torch.equal(out.kappa, ref.kappa)
    t.close()
