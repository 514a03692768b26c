"""Vertex-box builds (rr_build_tidal_tensor_box) and the ray vertex box
(rr_rays_vertex_box): a box build equals the whole-grid build on its
vertices and leaves the others alone, and a light cone traced with one box
build per chi segment gives bit-identical kappa, compensation, crossing
hashes and counts to whole-grid builds, with stale values planted outside
every box."""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I
from tests._cases import gpu_bundle, gpu_grid, hashes_u64

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


def _box_mask(n, lo, size):
    idx = [np.zeros(n, bool) for _ in range(3)]
    for a in range(3):
        idx[a][(lo[a] + np.arange(size[a])) % n] = True
    # vertex records are [z][y][x]
    return idx[2][:, None, None] & idx[1][None, :, None] & idx[0][None, None, :]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_box_build_equals_whole_grid_build_inside_and_keeps_outside(api, prec):
    n, box = 40, 80.0
    rng = np.random.default_rng(11)
    dt = np.float64 if prec == "fp64" else np.float32
    phi_a = rng.standard_normal((n, n, n)).astype(dt)
    phi_b = rng.standard_normal((n, n, n)).astype(dt)
    lo, size = (-7, 30, 13), (21, 17, 33)      # wraps in x and y, ragged against the tiles
    ga, gb = gpu_grid(api, phi_a, box), gpu_grid(api, phi_b, box)
    fa = api.TidalTensor(ga, prec).build().to_torch().cpu().numpy().reshape(n, n, n, 6)
    fb = api.TidalTensor(gb, prec).build().to_torch().cpu().numpy().reshape(n, n, n, 6)
    t = api.TidalTensor(ga, prec).build()
    t.build_box(lo, size, grid=gb)
    got = t.to_torch().cpu().numpy().reshape(n, n, n, 6)
    m = _box_mask(n, lo, size)
    assert m.sum() == 21 * 17 * 33
    assert np.array_equal(got[m], fb[m])
    assert np.array_equal(got[~m], fa[~m])
    # the whole grid as a box is the whole-grid build
    t.build_box((0, 0, 0), (n, n, n), grid=ga)
    assert np.array_equal(t.to_torch().cpu().numpy().reshape(n, n, n, 6), fa)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_windowed_light_cone_is_bitwise_the_whole_grid_light_cone(api, plan, prec):
    import torch
    n, box = 48, 96.0
    rng = np.random.default_rng(12)
    dt = np.float64 if prec == "fp64" else np.float32
    phi0 = I.poisson_phi(I.gaussian_field(n, box, rng, slope=-2.0), box)
    nx = ny = 24
    fov = math.radians(6.0)
    dirs = I.fov_directions((0.2, 0.1, 1.0), fov, fov, nx, ny)
    obs = (3.3, -1.7, 0.4)
    chi_s = 300.0
    edges = np.linspace(chi_s, 0.0, 7)
    phis = [(phi0 * (1.0 + 0.1 * k)).astype(dt) for k in range(6)]
    grids = [gpu_grid(api, p, box) for p in phis]
    poison = gpu_grid(api, (1e3 * rng.standard_normal((n, n, n))).astype(dt), box)

    full = api.TidalTensor(grids[0], prec)
    win = api.TidalTensor(poison, prec).build()
    kf = torch.zeros(nx * ny, dtype=torch.float64 if prec == "fp64" else torch.float32,
                     device="cuda")
    kw = torch.zeros_like(kf)
    cf = torch.zeros(nx * ny, dtype=torch.float32, device="cuda") if prec == "fp32" else None
    cw = torch.zeros_like(cf) if cf is not None else None
    smaller = 0
    for k, (a, b) in enumerate(zip(edges[:-1], edges[1:])):
        bun = [gpu_bundle(api, dirs, nx, ny, chi_s, a, b)]
        full.build(grid=grids[k])
        rf = api.trace(plan, full, bun, obs, kappa=kf, kappa_comp=cf, debug=True)
        lo, size = plan.vertex_box(win, bun, obs)
        assert all(0 < s <= n for s in size)
        smaller += int(np.prod(size) < n ** 3)
        win.build_box(lo, size, grid=grids[k])
        rw = api.trace(plan, win, bun, obs, kappa=kw, kappa_comp=cw, debug=True)
        assert np.array_equal(hashes_u64(rw.hash), hashes_u64(rf.hash))
        assert np.array_equal(rw.count.cpu().numpy(), rf.count.cpu().numpy())
        assert bool((rw.status == 0).all())
    assert smaller >= 3
    assert np.array_equal(kw.cpu().numpy(), kf.cpu().numpy())
    if cf is not None:
        assert np.array_equal(cw.cpu().numpy(), cf.cpu().numpy())


def test_vertex_box_bounds_and_open_grid_clipping(api, plan):
    """The box contains the lattice cells at both ends of every ray, padded by
    the slab rule and the upper corner; on open grids it stays inside [0, n)."""
    n, box = 32, 32.0
    phi = np.zeros((n, n, n), np.float64)
    g = gpu_grid(api, phi, box, boundary="open")
    t = api.TidalTensor(g, "fp64")
    dirs = I.fov_directions((0.0, 0.0, 1.0), math.radians(20.0), math.radians(20.0), 8, 8)
    obs = (16.0, 16.0, 3.0)
    bun = [gpu_bundle(api, dirs, 8, 8, 20.0, 20.0, 1.0)]
    lo, size = plan.vertex_box(t, bun, obs)
    for a in range(3):
        p = np.concatenate([obs[a] + 20.0 * dirs[:, a], obs[a] + 1.0 * dirs[:, a]])
        c0, c1 = int(np.floor(p.min())), int(np.floor(p.max()))
        assert lo[a] <= max(c0 - 1, 0) and lo[a] + size[a] >= min(c1 + 2, n)
        assert 0 <= lo[a] and lo[a] + size[a] <= n
    from paper_1601_02012_amd import _abi as A
    with pytest.raises(A.RRError) as e:
        t.build_box((-1, 0, 0), (4, 4, 4))
    assert e.value.status == -6


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("lo", [(0, 0, 0), (64, 2, 5), (-3, 7, 9)])
def test_large_box_and_whole_grid_streaming_builds(api, oracle, lo, prec):
    """n = 128: the whole-grid build (the streaming configuration, 64x16x16
    columns; FP64 rows of records leave through LDS as contiguous 16-byte
    stores, rows that wrap or stop short per lane) matches the oracle, and
    boxes above 1/8 of the grid (the same configuration) -- with even, odd and
    wrapping origins -- equal it on their vertices and leave the others
    alone."""
    n, box = 128, 128.0
    dt = np.float64 if prec == "fp64" else np.float32
    rng = np.random.default_rng(13)
    phi = rng.standard_normal((n, n, n)).astype(dt)
    g = gpu_grid(api, phi, box)
    whole = api.TidalTensor(g, prec).build().to_torch().cpu().numpy().reshape(n, n, n, 6)
    ref = oracle.vertex_tensor(phi.astype(np.float64)).reshape(n, n, n, 6)
    tol = 1e-13 if prec == "fp64" else 2e-6
    np.testing.assert_allclose(whole, ref, rtol=0, atol=tol * np.abs(ref).max())
    size = (128, 100, 40)
    assert 8 * np.prod(size) > n ** 3
    poison = gpu_grid(api, (1e3 * rng.standard_normal((n, n, n))).astype(dt), box)
    t = api.TidalTensor(poison, prec).build()
    before = t.to_torch().cpu().numpy().reshape(n, n, n, 6)
    t.build_box(lo, size, grid=g)
    got = t.to_torch().cpu().numpy().reshape(n, n, n, 6)
    m = _box_mask(n, lo, size)
    assert np.array_equal(got[m], whole[m])
    assert np.array_equal(got[~m], before[~m])
