"""GPU parity on the degenerate cases of the crossing rule (Sec. III F):
rays along a lattice axis or in a lattice plane (a direction component of
exactly zero), rays through lattice edges and vertices (two or three planes
at one parameter), observers on lattice planes and vertices, windows ending
within rounding of a plane, and windows starting exactly on a plane; on a
uniform periodic grid (FP64 and FP32-Kahan) and through a refined octree.

Bars as everywhere: crossing hashes and counts bit-exact, FP64 kappa to 1e-11
of the map's scale, FP32-Kahan within max(1e-5 |kappa|, 1e-7) (potentials at
cosmological Phi/c^2 amplitudes)."""
import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I
from tests._cases import gpu_bundle, gpu_grid, hashes_u64, kappa_tolerance_ok
from tests.test_oracle_degenerate import DEGENERATE_DIRS, OBSERVERS, degenerate_case

pytestmark = pytest.mark.gpu

WINDOWS = [(29.0, 0.7), (17.0, 3.0)]


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1601_02012_amd import api as A
    return A


def _check(out, ref, prec):
    assert np.all(out.status.cpu().numpy() == 0)
    assert np.array_equal(out.count.cpu().numpy(), ref.ncross)
    assert np.array_equal(hashes_u64(out.hash), ref.hash)
    k = out.kappa.double().cpu().numpy()
    if prec == "fp64":
        np.testing.assert_allclose(k, ref.kappa, rtol=0, atol=1e-11 * np.abs(ref.kappa).max())
    else:
        ok, worst = kappa_tolerance_ok(k, ref.kappa)
        assert ok, worst


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_degenerate_rays_uniform(api, oracle, prec):
    n, phi = degenerate_case()
    phi = 1e-5 * phi
    if prec == "fp32":
        phi = phi.astype(np.float32)
    tv = oracle.vertex_tensor(phi.astype(np.float64))
    t = api.TidalTensor(gpu_grid(api, phi, float(n)), prec).build()
    plan = api.Plan()
    nd = len(DEGENERATE_DIRS)
    for obs in OBSERVERS:
        for hi, lo in WINDOWS:
            gb = gpu_bundle(api, DEGENERATE_DIRS, nd, 1, 40.0, hi, lo)
            out = api.trace(plan, t, [gb], obs, debug=True, max_crossings=100000)
            ref = oracle.trace_uniform(n, float(n), obs, DEGENERATE_DIRS, 40.0, hi, lo, tv=tv)
            _check(out, ref, prec)
    # windows that start exactly on a plane, one ray per bundle
    o = np.array([2.3, 4.1, 1.7])
    for d in DEGENERATE_DIRS[[0, 4, 5, 7, 10]]:
        a = int(np.argmax(np.abs(d)))
        plane = np.floor(o[a] + 20.0 * d[a])
        hi = float((plane - o[a]) * (1.0 / d[a]))
        gb = gpu_bundle(api, d[None, :], 1, 1, 40.0, hi, 0.5)
        out = api.trace(plan, t, [gb], tuple(o), debug=True, max_crossings=100000)
        ref = oracle.trace_uniform(n, float(n), o, d[None, :], 40.0, hi, 0.5, tv=tv)
        _check(out, ref, prec)
    plan.close()
    t.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_degenerate_rays_octree(api, oracle, prec):
    from tests.test_gpu_octree import _gpu_octree_grid, _otree, _smooth_phi
    rng = np.random.default_rng(41)
    tr = I.random_octree(8, 2, 0.3, rng, region=(1.0, 7.0))
    box = 8.0
    phi = _smooth_phi(tr, box, rng)
    dt = np.float64 if prec == "fp64" else np.float32
    t = api.TidalTensor(_gpu_octree_grid(api, tr, phi, box, dt), prec).build()
    ot = _otree(oracle, tr)
    tc = oracle.centre_tensor_octree(ot, phi.astype(dt).astype(np.float64))
    plan = api.Plan()
    nd = len(DEGENERATE_DIRS)
    for obs in OBSERVERS:
        for hi, lo in WINDOWS:
            gb = gpu_bundle(api, DEGENERATE_DIRS, nd, 1, 40.0, hi, lo)
            out = api.trace(plan, t, [gb], obs, debug=True, max_crossings=100000)
            ref = oracle.trace_octree(ot, box, obs, DEGENERATE_DIRS, 40.0, hi, lo, tc=tc)
            _check(out, ref, prec)
    plan.close()
    t.close()


def test_degenerate_rays_split_march_bitwise(api):
    """The same rays through the octree with the march split into passes
    (every ray stops on a face and resumes there, also after edge and vertex
    crossings into coarser leaves): bitwise the one-pass result."""
    import torch
    from tests.test_gpu_octree import _gpu_octree_grid, _smooth_phi
    rng = np.random.default_rng(41)
    tr = I.random_octree(8, 2, 0.3, rng, region=(1.0, 7.0))
    box = 8.0
    phi = _smooth_phi(tr, box, rng)
    nd = len(DEGENERATE_DIRS)
    for prec, dt in (("fp64", np.float64), ("fp32", np.float32)):
        t = api.TidalTensor(_gpu_octree_grid(api, tr, phi, box, dt), prec).build()
        for obs in OBSERVERS:
            res = []
            for passes in (1, 5):
                plan = api.Plan()
                gb = gpu_bundle(api, DEGENERATE_DIRS, nd, 1, 40.0, 29.0, 0.7)
                plan.set_shape([gb], persistent=0, block=64, passes=passes)
                out = api.trace(plan, t, [gb], obs, persistent=-1)
                torch.cuda.synchronize()
                res.append((out.kappa.cpu().numpy(), out.status.cpu().numpy()))
                plan.close()
            assert np.all(res[0][1] == 0)
            assert np.array_equal(res[0][0], res[1][0]), (prec, obs)
        t.close()


def test_degenerate_rays_many_sources(api, oracle):
    """The many-source walk (Eqs. Isources, Isources1) on the same rays, on
    the uniform grid and through the octree, with source distances on lattice
    planes of the axis-aligned rays and inside cells: cut crossing hashes and
    counts bit-exact per window, FP64 pieces and moments to 1e-11 of their
    scale."""
    from tests.test_gpu_octree import _gpu_octree_grid, _otree, _smooth_phi
    sources = np.array([29.0, 21.3, 17.0, 9.7, 4.0, 1.5])
    windows = [(29.0, 12.0), (12.0, 0.7)]
    nd = len(DEGENERATE_DIRS)
    n, phiu = degenerate_case()
    phiu = 1e-5 * phiu
    rng = np.random.default_rng(41)
    tr = I.random_octree(8, 2, 0.3, rng, region=(1.0, 7.0))
    phio = _smooth_phi(tr, 8.0, rng)
    ot = _otree(oracle, tr)
    cv = oracle.corner_tensor_octree(ot, oracle.centre_tensor_octree(ot, phio))
    tv = oracle.vertex_tensor(phiu)
    cases = [("uniform", api.TidalTensor(gpu_grid(api, phiu, float(n)), "fp64").build()),
             ("octree", api.TidalTensor(_gpu_octree_grid(api, tr, phio, 8.0, np.float64),
                                        "fp64").build())]
    plan = api.Plan()
    for kind, t in cases:
        for obs in OBSERVERS:
            state = None
            mom = pcs = None
            for hi, lo in windows:
                gb = gpu_bundle(api, DEGENERATE_DIRS, nd, 1, sources[0], hi, lo)
                state = api.trace_sources(plan, t, [gb], obs, sources, state=state, debug=True,
                                          max_crossings=100000)
                if kind == "uniform":
                    r = oracle.trace_uniform_sources(n, float(n), obs, DEGENERATE_DIRS, hi, lo,
                                                     sources, tv=tv, moments=mom, pieces=pcs)
                else:
                    r = oracle.trace_octree_sources(ot, 8.0, obs, DEGENERATE_DIRS, hi, lo,
                                                    sources, cv=cv, moments=mom, pieces=pcs)
                mom, pcs = r.moments, r.pieces
                assert np.all(state.status.cpu().numpy() == 0), (kind, obs)
                assert np.array_equal(state.count.cpu().numpy(), r.ncross), (kind, obs)
                assert np.array_equal(hashes_u64(state.hash), r.hash), (kind, obs)
            got_p = state.pieces.cpu().numpy()
            got_m = state.moments.cpu().numpy()
            for c in range(2):
                np.testing.assert_allclose(got_p[..., c], pcs[..., c], rtol=0,
                                           atol=1e-11 * np.abs(pcs[..., c]).max())
                np.testing.assert_allclose(got_m[:, c], mom[:, c], rtol=0,
                                           atol=1e-11 * np.abs(mom[:, c]).max())
        t.close()
    plan.close()


def test_degenerate_rays_method_a_and_isw(api, oracle):
    """Method A (with its surface terms at the window ends) and the ISW
    scalar on the same rays and observers, uniform grid, FP64: hashes and
    counts bit-exact, integrals to 1e-11 of the map's scale."""
    import torch
    n, phi = degenerate_case(seed=23)
    phi = 1e-5 * phi
    rng = np.random.default_rng(24)
    delta = rng.normal(size=(n, n, n))
    prev = 0.97 * phi
    box = float(n)
    cdelta = 3e-5
    gp = api.Grid(torch.as_tensor(phi).cuda(), box)
    gd = api.Grid(torch.as_tensor(delta).cuda(), box, field="delta")
    gprev = api.Grid(torch.as_tensor(prev).cuda(), box)
    gi = api.Grid(gp.values, box, field="phi_dot")
    ta = api.TidalTensor(gd, "fp64").build_method_a(gd, gp, cdelta)
    ti = api.TidalTensor(gi, "fp64").build_isw(gp, gprev, 2.0)
    fv = oracle.method_a_vertex_fields(phi, delta)
    qv = oracle.isw_vertex_field(phi, prev, 2.0)
    plan = api.Plan()
    nd = len(DEGENERATE_DIRS)
    for obs in OBSERVERS:
        for hi, lo in WINDOWS:
            gb = gpu_bundle(api, DEGENERATE_DIRS, nd, 1, 40.0, hi, lo)
            out = api.trace(plan, ta, [gb], obs, debug=True, max_crossings=100000)
            ref = oracle.trace_uniform_method_a(n, box, obs, DEGENERATE_DIRS, 40.0, hi, lo,
                                                delta_coeff=cdelta, fv=fv)
            _check(out, ref, "fp64")
            out = api.trace(plan, ti, [gb], obs, quantity="scalar", debug=True,
                            max_crossings=100000)
            ref = oracle.trace_uniform_isw(n, box, obs, DEGENERATE_DIRS, hi, lo, qv=qv)
            _check(out, ref, "fp64")
    plan.close()
    ta.close()
    ti.close()


def test_degenerate_rays_adjoint(api, oracle):
    """The adjoint's own walk on the same rays (uniform periodic FP32 grid):
    dL/dPhi within 1e-4 of the oracle gradient's scale, and the dot-product
    identity <A^T w, Phi> = <w, A Phi> against the forward trace."""
    import torch
    n, phi = degenerate_case(seed=25)
    phi = (1e-5 * phi).astype(np.float32)
    box = float(n)
    rng = np.random.default_rng(26)
    nd = len(DEGENERATE_DIRS)
    w = rng.standard_normal(nd).astype(np.float32)
    g = gpu_grid(api, phi, box)
    t = api.TidalTensor(g, "fp32").build()
    plan = api.Plan()
    for obs in OBSERVERS:
        for hi, lo in WINDOWS:
            gb = gpu_bundle(api, DEGENERATE_DIRS, nd, 1, 40.0, hi, lo)
            got = api.trace_adjoint(plan, t, g, [gb], obs,
                                    torch.as_tensor(w).cuda()).cpu().numpy()
            ref = oracle.trace_adjoint_uniform(n, box, obs, DEGENERATE_DIRS, 40.0, hi, lo,
                                               w.astype(np.float64))
            scale = np.abs(ref).max()
            np.testing.assert_allclose(got.reshape(-1), ref.reshape(-1), rtol=0,
                                       atol=1e-4 * scale)
            fwd = api.trace(plan, t.build(g), [gb], obs, persistent=0)
            lhs = float(np.dot(w.astype(np.float64), fwd.kappa.double().cpu().numpy()))
            rhs = float(np.sum(got.astype(np.float64) * phi.astype(np.float64)))
            assert lhs == pytest.approx(rhs, rel=1e-4, abs=1e-12)
    plan.close()
    t.close()
