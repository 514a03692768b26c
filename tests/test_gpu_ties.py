"""Seeded stress of the crossing rule's tie handling (Sec. III F): random
2:1-balanced octrees of two and three levels and uniform grids, observers on
lattice points of the finer levels (multiples of 1/4 base cell), directions
mixing exact axis, face-diagonal and body-diagonal ones with random ones,
windows ending on planes of the base lattice.  Every case against the FP64
oracle: crossing hashes and counts bit-exact, FP64 kappa to 1e-11 of the
map's scale."""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I
from tests._cases import gpu_bundle, gpu_grid, hashes_u64
from tests.test_oracle_degenerate import DEGENERATE_DIRS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1601_02012_amd import api as A
    return A


def _dirs(rng, k):
    rnd = rng.normal(size=(k, 3))
    rnd /= np.linalg.norm(rnd, axis=1)[:, None]
    return np.ascontiguousarray(np.concatenate([DEGENERATE_DIRS, rnd]))


def _compare(out, ref):
    assert np.all(out.status.cpu().numpy() == 0)
    assert np.array_equal(out.count.cpu().numpy(), ref.ncross)
    assert np.array_equal(hashes_u64(out.hash), ref.hash)
    k = out.kappa.cpu().numpy()
    np.testing.assert_allclose(k, ref.kappa, rtol=0, atol=1e-11 * np.abs(ref.kappa).max())


@pytest.mark.parametrize("seed", range(6))
def test_octree_ties(api, oracle, seed):
    from tests.test_gpu_octree import _gpu_octree_grid, _otree, _smooth_phi
    rng = np.random.default_rng(1000 + seed)
    levels = 2 + seed % 2
    tr = I.random_octree(8, levels, 0.35, rng, region=(0.0, 8.0))
    box = 8.0
    phi = _smooth_phi(tr, box, rng)
    t = api.TidalTensor(_gpu_octree_grid(api, tr, phi, box, np.float64), "fp64").build()
    ot = _otree(oracle, tr)
    tc = oracle.centre_tensor_octree(ot, phi)
    plan = api.Plan()
    dirs = _dirs(rng, 19)
    nd = dirs.shape[0]
    for _ in range(4):
        obs = tuple(float(v) for v in rng.integers(0, 32, size=3) * 0.25)
        hi = float(rng.integers(10, 30))
        lo = float(rng.integers(0, 4))
        gb = gpu_bundle(api, dirs, nd, 1, 40.0, hi, lo)
        out = api.trace(plan, t, [gb], obs, debug=True, max_crossings=100000)
        ref = oracle.trace_octree(ot, box, obs, dirs, 40.0, hi, lo, tc=tc)
        _compare(out, ref)
    plan.close()
    t.close()


@pytest.mark.parametrize("seed", range(3))
def test_uniform_ties(api, oracle, seed):
    rng = np.random.default_rng(2000 + seed)
    n = 8
    phi = 1e-5 * rng.normal(size=(n, n, n))
    t = api.TidalTensor(gpu_grid(api, phi, float(n)), "fp64").build()
    tv = oracle.vertex_tensor(phi)
    plan = api.Plan()
    dirs = _dirs(rng, 19)
    nd = dirs.shape[0]
    for _ in range(4):
        obs = tuple(float(v) for v in rng.integers(0, 32, size=3) * 0.25)
        hi = float(rng.integers(10, 30))
        lo = float(rng.integers(0, 4))
        gb = gpu_bundle(api, dirs, nd, 1, 40.0, hi, lo)
        out = api.trace(plan, t, [gb], obs, debug=True, max_crossings=100000)
        ref = oracle.trace_uniform(n, float(n), obs, dirs, 40.0, hi, lo, tv=tv)
        _compare(out, ref)
    plan.close()
    t.close()


@pytest.mark.parametrize("seed", range(3))
def test_octree_ties_split_march_bitwise(api, seed):
    """The same kind of cases with the march split into passes: kappa and
    status bitwise equal to one pass, FP64 and FP32-Kahan."""
    import torch
    from tests.test_gpu_octree import _gpu_octree_grid, _smooth_phi
    rng = np.random.default_rng(3000 + seed)
    tr = I.random_octree(8, 3, 0.35, rng, region=(0.0, 8.0))
    phi = _smooth_phi(tr, 8.0, rng)
    dirs = _dirs(rng, 19)
    nd = dirs.shape[0]
    obs = [tuple(float(v) for v in rng.integers(0, 32, size=3) * 0.25) for _ in range(3)]
    for prec, dt in (("fp64", np.float64), ("fp32", np.float32)):
        t = api.TidalTensor(_gpu_octree_grid(api, tr, phi, 8.0, dt), prec).build()
        for o in obs:
            res = []
            for passes in (1, 7):
                plan = api.Plan()
                gb = gpu_bundle(api, dirs, nd, 1, 40.0, 29.0, 1.0)
                plan.set_shape([gb], persistent=0, block=64, passes=passes)
                out = api.trace(plan, t, [gb], o, persistent=-1)
                torch.cuda.synchronize()
                res.append((out.kappa.cpu().numpy(), out.status.cpu().numpy()))
                plan.close()
            assert np.all(res[0][1] == 0)
            assert np.array_equal(res[0][0], res[1][0]), (prec, o)
        t.close()
