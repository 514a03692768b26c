"""GPU parity of the octree path (tensor build and march) against the oracle.

Bars: per-leaf corner tensors to 1e-12 (FP64) / 2e-6 (FP32) of the field's
scale; crossing lists bit-exact (per-ray hash and counts); kappa to 1e-11
(FP64) or within max(1e-5 |kappa|, 1e-7) (FP32-Kahan)."""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I
from tests._cases import hashes_u64, kappa_tolerance_ok

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available()
    from paper_1601_02012_amd import api as A
    return A


@pytest.fixture(scope="module")
def plan(api):
    return api.Plan()


def _otree(oracle, t):
    return oracle.Octree(t.n, t.child_oct, t.oct_parent, t.oct_level, t.oct_coord, t.max_level)


def _smooth_phi(t, box, rng, noise=0.05, amplitude=1e-4):
    """Smooth periodic potential plus level-scaled noise, with the amplitude
    of Phi/c^2 in cosmological units (kappa ~ 1e-3 - 1e-2) so that the
    tolerance max(1e-5 |kappa|, 1e-7) means what it does for real maps."""
    return amplitude * _unit_phi(t, box, rng, noise)


def _unit_phi(t, box, rng, noise):
    x = t.centres(box)
    k = 2 * np.pi / box * np.array([1.0, 2.0, 1.0])
    k2 = 2 * np.pi / box * np.array([-2.0, 1.0, 3.0])
    phi = np.sin(x @ k + 0.3) + 0.5 * np.cos(x @ k2 - 0.1)
    return phi + noise * rng.standard_normal(t.n_cells) * (0.5 ** (2 * t.cell_level))


def _gpu_octree_grid(api, t, phi, box, dtype):
    import torch
    vals = torch.as_tensor(phi.astype(dtype)).cuda()
    co = torch.as_tensor(t.child_oct).cuda()
    return api.Grid(vals, box, n_base=t.n, child_oct=co, max_level=t.max_level)


@pytest.fixture(scope="module")
def tree_case():
    rng = np.random.default_rng(31)
    t = I.random_octree(12, 3, 0.18, rng, region=(2.0, 10.0))
    box = 24.0
    phi = _smooth_phi(t, box, rng)
    return t, box, phi


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_octree_corner_tensor_matches_oracle(api, oracle, tree_case, prec, tol):
    t, box, phi = tree_case
    dt = np.float64 if prec == "fp64" else np.float32
    g = _gpu_octree_grid(api, t, phi, box, dt)
    tt = api.TidalTensor(g, prec).build()
    got = tt.to_torch().double().cpu().numpy().reshape(t.n_cells, 8, 6)
    ot = _otree(oracle, t)
    tc = oracle.centre_tensor_octree(ot, phi.astype(dt).astype(np.float64))
    ref = oracle.corner_tensor_octree(ot, tc)
    lv = t.leaves()
    # the corner values are in base-cell units; compare on the field's scale
    scale = np.abs(ref[lv]).max()
    np.testing.assert_allclose(got[lv], ref[lv], rtol=0, atol=tol * scale)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_octree_blocks_of_refined_cells_are_nan(api, tree_case, prec):
    """Every component of the corner block of a cell that is not a leaf is
    NaN and every leaf's block is finite: after a same-level face crossing
    the direct march reads the target's child link only when the target's
    corner value is NaN (a finite value shows a leaf)."""
    t, box, phi = tree_case
    dt = np.float64 if prec == "fp64" else np.float32
    tt = api.TidalTensor(_gpu_octree_grid(api, t, phi, box, dt), prec).build()
    got = tt.to_torch().double().cpu().numpy().reshape(t.n_cells, 8, 6)
    refined = t.child_oct >= 0
    assert refined.sum() > 0
    assert np.all(np.isnan(got[refined]))
    assert np.all(np.isfinite(got[~refined]))
    tt.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_octree_trace_matches_oracle(api, oracle, plan, tree_case, prec):
    import torch
    t, box, phi = tree_case
    dt = np.float64 if prec == "fp64" else np.float32
    g = _gpu_octree_grid(api, t, phi, box, dt)
    tt = api.TidalTensor(g, prec).build()
    fov = math.radians(50.0)
    nx, ny = 21, 13
    dirs = I.fov_directions((0.2, 0.1, 1.0), fov, fov * 0.6, nx, ny)
    obs = (11.7, 12.2, 3.1)
    chis, hi, lo = 60.0, 45.0, 0.2
    b = api.RayBundle(torch.as_tensor(dirs).cuda(), nx, ny, chis, hi, lo)
    out = api.trace(plan, tt, [b], obs, debug=True)
    ot = _otree(oracle, t)
    ref = oracle.trace_octree(ot, box, obs, dirs, chis, hi, lo, phi=phi.astype(dt).astype(np.float64))
    assert np.array_equal(out.count.cpu().numpy(), ref.ncross)
    assert np.array_equal(hashes_u64(out.hash), ref.hash)
    k = out.kappa.double().cpu().numpy()
    if prec == "fp64":
        np.testing.assert_allclose(k, ref.kappa, rtol=0, atol=1e-11 * np.abs(ref.kappa).max())
    else:
        ok, worst = kappa_tolerance_ok(k, ref.kappa)
        assert ok, worst
    # the rays cross refinement boundaries on several levels
    lg = oracle.trace_octree(ot, box, obs, dirs[::7], chis, hi, lo,
                             phi=phi.astype(dt).astype(np.float64), log_stride=4096)
    levels = set()
    for r in range(lg.ncross.shape[0]):
        levels |= set(t.cell_level[lg.log[r][: lg.ncross[r]]["cell"]].tolist())
    assert len(levels) >= 3


def test_fully_refined_octree_equals_uniform(api, plan):
    """GPU octree refined everywhere to level 1 == GPU uniform grid of 2n."""
    import torch
    n, L = 8, 16.0
    t = I.full_octree(n, 1)
    kk = 2 * np.pi / L * np.array([1.0, 2.0, 1.0])
    fn = lambda x: np.sin(x @ kk + 0.2) + 0.3 * np.cos(x @ (2 * kk[::-1]))
    phi_c = fn(t.centres(L))
    n2 = 2 * n
    c2 = (np.arange(n2) + 0.5) * (L / n2)
    zz, yy, xx = np.meshgrid(c2, c2, c2, indexing="ij")
    phi_u = fn(np.stack([xx, yy, zz], -1))
    go = _gpu_octree_grid(api, t, phi_c, L, np.float64)
    gu = api.Grid(torch.as_tensor(phi_u).cuda(), L)
    to = api.TidalTensor(go, "fp64").build()
    tu = api.TidalTensor(gu, "fp64").build()
    fov = math.radians(6.0)
    dirs = I.fov_directions((0.2, 0.1, 1.0), fov, fov, 8, 8)
    b = api.RayBundle(torch.as_tensor(dirs).cuda(), 8, 8, 40.0, 35.0, 0.0)
    ko = api.trace(plan, to, [b], (0, 0, 0), debug=True)
    ku = api.trace(plan, tu, [b], (0, 0, 0), debug=True)
    assert torch.equal(ko.count, ku.count)
    np.testing.assert_allclose(ko.kappa.cpu().numpy(), ku.kappa.cpu().numpy(), rtol=0,
                               atol=1e-11 * float(ku.kappa.abs().max()))


def test_quadratic_potential_refinement_invariant(api, plan):
    """Constant transverse Laplacian: kappa equals it times the kernel
    integral on a multi-level octree (FP32-Kahan within tolerance)."""
    import torch
    rng = np.random.default_rng(77)
    n, L = 16, 16.0
    t = I.random_octree(n, 3, 0.25, rng, region=(3.0, 13.0))
    M = rng.normal(size=(3, 3)); M = M + M.T
    cen = t.centres(L)
    phi = 0.5 * np.einsum("ci,ij,cj->c", cen, M, cen)
    g = _gpu_octree_grid(api, t, phi, L, np.float64)
    fov = math.radians(20.0)
    dirs = I.fov_directions((0.0, 0.0, 1.0), fov, fov, 9, 9)
    chis, hi, lo = 12.0, 9.0, 0.0
    b = api.RayBundle(torch.as_tensor(dirs).cuda(), 9, 9, chis, hi, lo)
    qv = np.trace(M) - np.einsum("ri,ij,rj->r", dirs, M, dirs)
    expect = qv * ((chis * (hi ** 2 - lo ** 2) / 2 - (hi ** 3 - lo ** 3) / 3) / chis)
    for prec in ("fp64", "fp32"):
        tt = api.TidalTensor(g, prec).build()
        k = api.trace(plan, tt, [b], (8.0, 8.0, 3.5)).kappa.double().cpu().numpy()
        if prec == "fp64":
            np.testing.assert_allclose(k, expect, rtol=1e-10)
        else:
            ok, worst = kappa_tolerance_ok(k, expect)
            assert ok, worst


def test_malformed_octrees_rejected(api):
    import torch
    t = I.build_octree(6, 1, lambda l, c: np.all(c == np.array([2, 2, 2]), axis=1))
    # not 2:1 balanced: refine one level-1 cell at the edge of the refined region
    child = np.concatenate([t.child_oct, np.full(8, -1, np.int32)])
    child[6 ** 3 + 0] = t.n_octs
    vals = torch.zeros(child.shape[0], dtype=torch.float64, device="cuda")
    g = api.Grid(vals, 6.0, n_base=6, child_oct=torch.as_tensor(child).cuda(), max_level=2)
    with pytest.raises(api.RRError) as e:
        api.TidalTensor(g, "fp64")
    assert e.value.status == -5
    # octs not in breadth-first order
    t2 = I.build_octree(6, 1, lambda l, c: (c[:, 0] == 1) & (c[:, 1] == 1) & (c[:, 2] <= 1))
    child2 = t2.child_oct.copy()
    a_, b_ = np.nonzero(child2 >= 0)[0][:2]
    child2[a_], child2[b_] = child2[b_], child2[a_]
    g2 = api.Grid(torch.zeros(child2.shape[0], dtype=torch.float64, device="cuda"), 6.0,
                  n_base=6, child_oct=torch.as_tensor(child2).cuda(), max_level=1)
    with pytest.raises(api.RRError) as e2:
        api.TidalTensor(g2, "fp64")
    assert e2.value.status == -5


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_refinement_across_the_periodic_faces(api, oracle, plan, prec):
    """Refined octs touching the box faces: corner tensors whose coarse
    neighbours sit across the periodic boundary, and rays that wrap."""
    import torch
    rng = np.random.default_rng(41)
    t = I.random_octree(8, 2, 0.3, rng)
    base = t.cell_coord >> t.cell_level[:, None].astype(np.int64)
    assert np.any(t.child_oct[(base == 0).any(axis=1) | (base == 7).any(axis=1)] >= 0)
    box = 16.0
    phi = _smooth_phi(t, box, rng)
    dt = np.float64 if prec == "fp64" else np.float32
    g = _gpu_octree_grid(api, t, phi, box, dt)
    tt = api.TidalTensor(g, prec).build()
    got = tt.to_torch().double().cpu().numpy().reshape(t.n_cells, 8, 6)
    ot = _otree(oracle, t)
    tc = oracle.centre_tensor_octree(ot, phi.astype(dt).astype(np.float64))
    ref = oracle.corner_tensor_octree(ot, tc)
    lv = t.leaves()
    tol = 1e-12 if prec == "fp64" else 2e-6
    np.testing.assert_allclose(got[lv], ref[lv], rtol=0, atol=tol * np.abs(ref[lv]).max())
    fov = math.radians(40.0)
    dirs = I.fov_directions((-0.3, 0.4, 1.0), fov, fov, 16, 16)
    obs = (0.3, 15.7, 0.1)
    b = api.RayBundle(torch.as_tensor(dirs).cuda(), 16, 16, 50.0, 40.0, 0.0)
    out = api.trace(plan, tt, [b], obs, debug=True)
    r = oracle.trace_octree(ot, box, obs, dirs, 50.0, 40.0, 0.0, tc=tc)
    assert np.array_equal(hashes_u64(out.hash), r.hash)
    k = out.kappa.double().cpu().numpy()
    if prec == "fp64":
        np.testing.assert_allclose(k, r.kappa, rtol=0, atol=1e-11 * np.abs(r.kappa).max())
    else:
        ok, worst = kappa_tolerance_ok(k, r.kappa)
        assert ok, worst


@pytest.mark.parametrize("quantity,q", [("gamma1", 1), ("gamma2", 2)])
def test_octree_shear_matches_oracle(api, oracle, plan, tree_case, quantity, q):
    import torch
    t, box, phi = tree_case
    g = _gpu_octree_grid(api, t, phi, box, np.float64)
    tt = api.TidalTensor(g, "fp64").build()
    fov = math.radians(40.0)
    nx, ny = 17, 11
    dirs = I.fov_directions((0.2, 0.1, 1.0), fov, fov * 0.6, nx, ny)
    obs = (11.7, 12.2, 3.1)
    chis, hi, lo = 60.0, 45.0, 0.2
    b = api.RayBundle(torch.as_tensor(dirs).cuda(), nx, ny, chis, hi, lo)
    out = api.trace(plan, tt, [b], obs, debug=True, quantity=quantity)
    ref = oracle.trace_octree(_otree(oracle, t), box, obs, dirs, chis, hi, lo, phi=phi,
                              quantity=q)
    assert np.array_equal(hashes_u64(out.hash), ref.hash)
    k = out.kappa.cpu().numpy()
    np.testing.assert_allclose(k, ref.kappa, rtol=0, atol=1e-11 * np.abs(ref.kappa).max())
