"""A march split into resumable passes (rr_plan_set_shape / rr_plan_autotune
with passes > 1) stops every ray exactly on a face and resumes there: the
pieces and their order are those of one pass, so every output must be
bitwise equal to the one-pass march -- uniform and octree, FP32-Kahan and
FP64, direct and persistent launches, the many-source walk, Method A's
surface terms, the ISW scalar, and a replayed graph."""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I
from tests._cases import gpu_bundle, gpu_grid, small_periodic_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1601_02012_amd import api as A
    return A


def _bundles(api, dirs_a, dirs_b, chis, hi, lo):
    return [gpu_bundle(api, dirs_a, 37, 13, chis, hi, lo, 0),
            gpu_bundle(api, dirs_b, 9, 21, chis, hi * 0.8, lo, 37 * 13)]


def _dirs():
    fov = math.radians(9.0)
    d1 = I.fov_directions((0.15, -0.1, 1.0), fov, fov * 13 / 37, 37, 13)
    d2 = I.fov_directions((-0.3, 0.2, 1.0), fov / 2, fov / 2, 9, 21)
    return d1, d2


def _run(api, t, bundles, obs, shape, **kw):
    import torch
    plan = api.Plan()
    if shape is not None:
        plan.set_shape(bundles, **shape)
    nr = 37 * 13 + 9 * 21
    fp32 = t.precision == 1
    kap = torch.zeros(nr, dtype=torch.float32 if fp32 else torch.float64, device="cuda")
    comp = torch.zeros(nr, dtype=torch.float32, device="cuda") if fp32 else None
    st = torch.zeros(nr, dtype=torch.int32, device="cuda")
    out = api.trace(plan, t, bundles, obs, kappa=kap, kappa_comp=comp, status=st,
                    persistent=-1, **kw)
    torch.cuda.synchronize()
    plan.close()
    return (out.kappa.cpu().numpy(), None if comp is None else comp.cpu().numpy(),
            st.cpu().numpy())


SHAPES = [dict(persistent=0, block=256, passes=2), dict(persistent=0, block=64, passes=7),
          dict(persistent=1, waves_per_cu=16, passes=5)]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_uniform_passes_bitwise(api, prec):
    n, box = 32, 64.0
    phi, _ = small_periodic_case(seed=6, n=n, box=box)
    if prec == "fp32":
        phi = phi.astype(np.float32)
    t = api.TidalTensor(gpu_grid(api, phi, box), prec).build()
    d1, d2 = _dirs()
    b = _bundles(api, d1, d2, 300.0, 300.0, 2.5)
    ref = _run(api, t, b, (3.0, 1.0, 2.0), None)
    assert np.all(ref[2] == 0)
    for sh in SHAPES:
        got = _run(api, t, b, (3.0, 1.0, 2.0), sh)
        for x, y in zip(got, ref):
            assert (x is None and y is None) or np.array_equal(x, y), sh
    # shear and NGP records too
    got = _run(api, t, b, (3.0, 1.0, 2.0), SHAPES[1], quantity="gamma2")
    ref2 = _run(api, t, b, (3.0, 1.0, 2.0), None, quantity="gamma2")
    assert all(np.array_equal(x, y) for x, y in zip(got, ref2) if x is not None)
    tc = api.TidalTensor(gpu_grid(api, phi, box), prec).build_centres()
    got = _run(api, tc, b, (3.0, 1.0, 2.0), SHAPES[0], integral="ngp")
    ref3 = _run(api, tc, b, (3.0, 1.0, 2.0), None, integral="ngp")
    assert all(np.array_equal(x, y) for x, y in zip(got, ref3) if x is not None)
    t.close()
    tc.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_octree_passes_bitwise(api, prec):
    from tests.test_gpu_octree import _gpu_octree_grid, _smooth_phi
    rng = np.random.default_rng(77)
    tr = I.random_octree(12, 3, 0.2, rng, region=(2.0, 10.0))
    box = 24.0
    phi = _smooth_phi(tr, box, rng)
    dt = np.float64 if prec == "fp64" else np.float32
    t = api.TidalTensor(_gpu_octree_grid(api, tr, phi, box, dt), prec).build()
    d1, d2 = _dirs()
    b = _bundles(api, d1, d2, 90.0, 90.0, 0.3)
    ref = _run(api, t, b, (11.7, 12.2, 3.1), None)
    for sh in SHAPES:
        got = _run(api, t, b, (11.7, 12.2, 3.1), sh)
        for x, y in zip(got, ref):
            assert (x is None and y is None) or np.array_equal(x, y), sh
    t.close()


def test_sources_method_a_and_isw_passes_bitwise(api):
    import torch
    n, box = 32, 64.0
    phi, _ = small_periodic_case(seed=8, n=n, box=box)
    d1, d2 = _dirs()
    obs = (5.0, 4.0, 3.0)
    # many sources: moments and pieces
    t = api.TidalTensor(gpu_grid(api, phi.astype(np.float32), box), "fp32").build()
    src = [280.0, 190.3, 77.7, 12.0]
    outs = []
    for sh in (None, SHAPES[1], SHAPES[2]):
        plan = api.Plan()
        b = _bundles(api, d1, d2, 280.0, 280.0, 0.0)
        if sh is not None:
            plan.set_shape(b, **sh)
        s = api.trace_sources(plan, t, b, obs, src, persistent=-1)
        torch.cuda.synchronize()
        outs.append((s.moments.cpu().numpy(), s.pieces.cpu().numpy(), s.status.cpu().numpy()))
        plan.close()
    for o in outs[1:]:
        assert all(np.array_equal(x, y) for x, y in zip(o, outs[0]))
    t.close()
    # Method A: the surface term of the window start is added once
    rng = np.random.default_rng(5)
    delta = 0.1 * I.gaussian_field(n, box, rng, slope=-2.0)
    gp = api.Grid(torch.as_tensor(phi.astype(np.float32)).cuda(), box)
    gd = api.Grid(torch.as_tensor(delta.astype(np.float32)).cuda(), box, field="delta")
    ta = api.TidalTensor(gd, "fp32").build_method_a(gd, gp, 3e-5)
    b = _bundles(api, d1, d2, 300.0, 250.0, 20.0)
    ref = _run(api, ta, b, obs, None)
    got = _run(api, ta, b, obs, SHAPES[1])
    assert all(np.array_equal(x, y) for x, y in zip(got, ref) if x is not None)
    ta.close()
    # ISW scalar
    gprev = api.Grid(torch.as_tensor((0.97 * phi).astype(np.float32)).cuda(), box)
    gi = api.Grid(gp.values, box, field="phi_dot")
    ti = api.TidalTensor(gi, "fp32").build_isw(gp, gprev, 2.0)
    ref = _run(api, ti, b, obs, None, quantity="scalar")
    got = _run(api, ti, b, obs, SHAPES[0], quantity="scalar")
    assert all(np.array_equal(x, y) for x, y in zip(got, ref) if x is not None)
    ti.close()


def test_split_march_in_a_graph_replays(api):
    import torch
    n, box = 32, 64.0
    phi, _ = small_periodic_case(seed=9, n=n, box=box)
    t = api.TidalTensor(gpu_grid(api, phi.astype(np.float32), box), "fp32").build()
    d1, d2 = _dirs()
    b = _bundles(api, d1, d2, 200.0, 200.0, 0.0)
    obs = (1.0, 2.0, 3.0)
    ref = _run(api, t, b, obs, None)
    plan = api.Plan()
    plan.set_shape(b, persistent=1, waves_per_cu=8, passes=6)
    nr = 37 * 13 + 9 * 21
    kap = torch.zeros(nr, dtype=torch.float32, device="cuda")
    comp = torch.zeros(nr, dtype=torch.float32, device="cuda")
    st = torch.zeros(nr, dtype=torch.int32, device="cuda")
    gs = torch.cuda.Stream()
    with torch.cuda.stream(gs):
        api.trace(plan, t, b, obs, kappa=kap, kappa_comp=comp, status=st, persistent=-1)
        gs.synchronize()
        plan.graph_begin()
        api.trace(plan, t, b, obs, kappa=kap, kappa_comp=comp, status=st, persistent=-1)
        plan.graph_end()
    gs.synchronize()
    for _ in range(3):
        kap.zero_()
        comp.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(gs):
            plan.graph_launch()
        gs.synchronize()
        assert np.array_equal(kap.cpu().numpy(), ref[0])
        assert np.array_equal(comp.cpu().numpy(), ref[1])
        assert np.array_equal(st.cpu().numpy(), ref[2])
    plan.close()
    t.close()


def test_debug_outputs_keep_one_pass(api):
    """With crossing hashes requested the shape's passes are not used: the
    hashes cover the whole window."""
    n, box = 32, 64.0
    phi, _ = small_periodic_case(seed=10, n=n, box=box)
    t = api.TidalTensor(gpu_grid(api, phi, box), "fp64").build()
    d1, d2 = _dirs()
    b = _bundles(api, d1, d2, 150.0, 150.0, 0.0)
    p1, p2 = api.Plan(), api.Plan()
    p2.set_shape(b, passes=8)
    o1 = api.trace(p1, t, b, (0.5, 0.5, 0.5), debug=True, persistent=-1)
    o2 = api.trace(p2, t, b, (0.5, 0.5, 0.5), debug=True, persistent=-1)
    import torch
    assert torch.equal(o1.hash, o2.hash) and torch.equal(o1.count, o2.count)
    with pytest.raises(api.RRError):
        p2.set_shape(b, passes=0)
    p1.close()
    p2.close()
    t.close()


def test_octree_split_march_in_a_graph_replays(api):
    """The octree march, persistent and split into passes (the batched
    configuration's shape), captured in a HIP graph: every replay equals the
    eager result bit for bit, with the program's own work between replays."""
    import torch
    from tests.test_gpu_octree import _gpu_octree_grid, _smooth_phi
    rng = np.random.default_rng(78)
    tr = I.random_octree(12, 3, 0.2, rng, region=(2.0, 10.0))
    box = 24.0
    phi = _smooth_phi(tr, box, rng)
    t = api.TidalTensor(_gpu_octree_grid(api, tr, phi, box, np.float32), "fp32").build()
    d1, d2 = _dirs()
    b = _bundles(api, d1, d2, 90.0, 90.0, 0.3)
    obs = (11.7, 12.2, 3.1)
    ref = _run(api, t, b, obs, None)
    plan = api.Plan()
    plan.set_shape(b, persistent=1, waves_per_cu=16, passes=5)
    nr = 37 * 13 + 9 * 21
    kap = torch.zeros(nr, dtype=torch.float32, device="cuda")
    comp = torch.zeros(nr, dtype=torch.float32, device="cuda")
    st = torch.zeros(nr, dtype=torch.int32, device="cuda")
    gs = torch.cuda.Stream()
    with torch.cuda.stream(gs):
        api.trace(plan, t, b, obs, kappa=kap, kappa_comp=comp, status=st, persistent=-1)
        gs.synchronize()
        plan.graph_begin()
        api.trace(plan, t, b, obs, kappa=kap, kappa_comp=comp, status=st, persistent=-1)
        plan.graph_end()
    gs.synchronize()
    for _ in range(3):
        kap.zero_()
        comp.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(gs):
            plan.graph_launch()
        gs.synchronize()
        assert np.array_equal(kap.cpu().numpy(), ref[0])
        assert np.array_equal(comp.cpu().numpy(), ref[1])
        assert np.array_equal(st.cpu().numpy(), ref[2])
    plan.close()
    t.close()
