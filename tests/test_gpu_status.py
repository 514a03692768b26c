"""Per-ray outcomes of rr_trace_rays other than success, on the uniform grid
and through an octree: a direction that is not a finite unit vector is
skipped (RR_RAY_BAD_DIRECTION, its kappa left as given), a ray whose
integral is not finite (a NaN in the potential next to its path) reports
RR_RAY_NONFINITE, and a ray cut off by max_crossings reports RR_RAY_MAX_STEPS
with exactly that many pieces; the other rays of the same launch are
unaffected (bitwise equal to a launch without the bad ones)."""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I
from tests._cases import gpu_bundle, gpu_grid

pytestmark = pytest.mark.gpu

RAY_OK, RAY_MAX_STEPS, RAY_NONFINITE, RAY_BAD_DIRECTION = 0, 2, 3, 4


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1601_02012_amd import api as A
    return A


def _tensors(api, prec):
    from tests.test_gpu_octree import _gpu_octree_grid, _smooth_phi
    rng = np.random.default_rng(5)
    n = 16
    phi = 1e-5 * rng.normal(size=(n, n, n))
    dt = np.float64 if prec == "fp64" else np.float32
    tu = api.TidalTensor(gpu_grid(api, phi.astype(dt), float(n)), prec).build()
    tr = I.random_octree(8, 2, 0.3, rng, region=(1.0, 7.0))
    po = _smooth_phi(tr, 8.0, rng)
    to = api.TidalTensor(_gpu_octree_grid(api, tr, po, 8.0, dt), prec).build()
    return [("uniform", tu, phi, n), ("octree", to, None, 8)]


def _dirs(k):
    fov = math.radians(20.0)
    return I.fov_directions((0.3, 0.2, 1.0), fov, fov, k, 1)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bad_direction_and_max_crossings(api, prec):
    import torch
    plan = api.Plan()
    for kind, t, _, n in _tensors(api, prec):
        good = _dirs(6)
        bad = np.array([[0.0, 0.0, 2.0], [np.nan, 0.0, 1.0], [0.6, 0.6, 0.6]])
        dirs = np.concatenate([good, bad])
        obs = (1.5, 2.5, 0.5)
        fp32 = prec == "fp32"
        kap0 = torch.full((9,), 7.0, dtype=torch.float32 if fp32 else torch.float64,
                          device="cuda")
        out = api.trace(plan, t, [gpu_bundle(api, dirs, 9, 1, 30.0, 25.0, 1.0)], obs,
                        kappa=kap0.clone(), debug=True)
        st = out.status.cpu().numpy()
        assert np.all(st[:6] == RAY_OK), kind
        assert np.all(st[6:] == RAY_BAD_DIRECTION), kind
        assert np.all(out.kappa.cpu().numpy()[6:] == 7.0), kind
        ref = api.trace(plan, t, [gpu_bundle(api, good, 6, 1, 30.0, 25.0, 1.0)], obs,
                        kappa=kap0[:6].clone(), debug=True)
        assert torch.equal(out.kappa[:6], ref.kappa), kind
        # a crossing limit below the rays' counts
        lim = 5
        cut = api.trace(plan, t, [gpu_bundle(api, good, 6, 1, 30.0, 25.0, 1.0)], obs,
                        max_crossings=lim, debug=True)
        assert np.all(cut.status.cpu().numpy() == RAY_MAX_STEPS), kind
        assert np.all(cut.count.cpu().numpy() == lim), kind
        t.close()
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nonfinite_integral(api, prec):
    """A NaN planted in the uniform potential: the rays through its stencil
    report RR_RAY_NONFINITE, the rays far from it stay OK and bitwise equal
    to the same launch on the clean potential."""
    import torch
    n = 16
    rng = np.random.default_rng(6)
    phi = 1e-5 * rng.normal(size=(n, n, n))
    dt = np.float64 if prec == "fp64" else np.float32
    dirty = phi.copy()
    dirty[8, 8, 8] = np.nan                       # [z][y][x]
    t_clean = api.TidalTensor(gpu_grid(api, phi.astype(dt), float(n)), prec).build()
    t_dirty = api.TidalTensor(gpu_grid(api, dirty.astype(dt), float(n)), prec).build()
    # rays along +z through the NaN's column and far from it
    obs = (8.5, 8.5, 0.5)
    far = (2.5, 13.5, 0.5)
    d = np.array([[0.0, 0.0, 1.0]])
    plan = api.Plan()
    hit = api.trace(plan, t_dirty, [gpu_bundle(api, d, 1, 1, 15.0, 15.0, 0.0)], obs, debug=True)
    assert hit.status.cpu().numpy()[0] == RAY_NONFINITE
    a = api.trace(plan, t_dirty, [gpu_bundle(api, d, 1, 1, 15.0, 15.0, 0.0)], far, debug=True)
    b = api.trace(plan, t_clean, [gpu_bundle(api, d, 1, 1, 15.0, 15.0, 0.0)], far, debug=True)
    assert a.status.cpu().numpy()[0] == RAY_OK
    assert torch.equal(a.kappa, b.kappa)
    t_clean.close()
    t_dirty.close()
    plan.close()


def test_coordinate_range_rejected(api):
    """Lattice coordinates are 32-bit on the device: an observer or a window
    end beyond 2^29 base cells (2^25 for an octree, whose finest level is 16
    times finer) is rejected on the host before any launch."""
    plan = api.Plan()
    for kind, t, _, n in _tensors(api, "fp64"):
        lim = 2.0 ** (25 if kind == "octree" else 29)
        h0 = 1.0                                  # both test grids have box = n
        d = _dirs(2)
        ok = gpu_bundle(api, d, 2, 1, 30.0, 25.0, 1.0)
        api.trace(plan, t, [ok], (lim * 0.5 * h0, 0.5, 0.5))
        with pytest.raises(api.RRError):
            api.trace(plan, t, [ok], (lim * 2.0 * h0, 0.5, 0.5))
        far = gpu_bundle(api, d, 2, 1, 4.0 * lim, 3.0 * lim, 1.0)
        with pytest.raises(api.RRError):
            api.trace(plan, t, [far], (0.5, 0.5, 0.5))
        t.close()
    plan.close()
