"""Full-size AMR and batched cases, checked on sampled rays and leaves.

The AMR octree is the 256^3-base, 4-level tree refined where a cell holds more
than 8 of 2^24 particles (NFW haloes on a lognormal background).  The GPU
builds its whole tensor and traces the whole 4096^2 map (and the 64 uneven
bundles of the batched case in one persistent launch); the oracle recomputes
sampled leaves' corner tensors and sampled rays one by one."""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I
from tests._cases import hashes_u64, kappa_tolerance_ok

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available()
    from paper_1601_02012_amd import api as A
    return A


@pytest.fixture(scope="module")
def amr(api, oracle):
    import torch
    case = I.config3()
    t = case.tree
    print(f"[amr] {t.n_cells} cells, {t.n_octs} octs, levels {np.bincount(t.cell_level)}",
          flush=True)
    phi32 = case.phi.astype(np.float32)
    ot = oracle.Octree(t.n, t.child_oct, t.oct_parent, t.oct_level, t.oct_coord, t.max_level)
    tc = oracle.centre_tensor_octree(ot, phi32.astype(np.float64))
    grid = api.Grid(torch.as_tensor(phi32).cuda(), case.box, n_base=t.n,
                    child_oct=torch.as_tensor(t.child_oct).cuda(), max_level=t.max_level)
    tens = api.TidalTensor(grid, "fp32").build()
    torch.cuda.synchronize()
    return case, ot, tc, grid, tens


def test_amr_corner_tensor_sampled_leaves(api, oracle, amr):
    case, ot, tc, grid, tens = amr
    t = case.tree
    rng = np.random.default_rng(3)
    lv = t.leaves()
    sel = []
    for level in range(t.max_level + 1):
        cand = lv[t.cell_level[lv] == level]
        if cand.size:
            sel.append(rng.choice(cand, size=min(400, cand.size), replace=False))
    sel = np.sort(np.concatenate(sel))
    ref = oracle.corner_tensor_octree_cells(ot, tc, sel)
    got = tens.to_torch().double().cpu().numpy().reshape(t.n_cells, 8, 6)[sel]
    scale = np.abs(ref).max()
    np.testing.assert_allclose(got, ref, rtol=0, atol=2e-6 * scale)


def test_amr_full_map_sampled_rays(api, oracle, amr):
    """4096^2 rays over 10x10 deg to z = 1 (FP32-Kahan, the benchmarked launch):
    every ray finishes, and 256 sampled rays match the oracle (crossing hashes
    bit-exact, kappa within tolerance)."""
    import torch
    case, ot, tc, grid, tens = amr
    b = I.config3_rays()
    plan = api.Plan()
    gb = api.RayBundle(torch.as_tensor(b.dirs).cuda(), b.nx, b.ny, b.chi_s, b.chi_hi, b.chi_lo)
    out = api.trace(plan, tens, [gb], case.observer, persistent=1)
    st = out.status.cpu().numpy()
    assert np.all(st == 0)
    k_all = out.kappa.double().cpu().numpy()
    assert np.all(np.isfinite(k_all))
    rng = np.random.default_rng(4)
    sel = np.sort(rng.choice(b.nx * b.ny, size=256, replace=False))
    ref = oracle.trace_octree(ot, case.box, case.observer, b.dirs[sel], b.chi_s, b.chi_hi,
                              b.chi_lo, tc=tc)
    ok, worst = kappa_tolerance_ok(k_all[sel], ref.kappa)
    assert ok, worst
    sb = api.RayBundle(torch.as_tensor(b.dirs[sel]).cuda(), len(sel), 1, b.chi_s, b.chi_hi,
                       b.chi_lo)
    dbg = api.trace(plan, tens, [sb], case.observer, debug=True)
    assert np.array_equal(hashes_u64(dbg.hash), ref.hash)
    assert np.array_equal(dbg.count.cpu().numpy(), ref.ncross)


def test_batched_bundles_persistent_and_graph(api, oracle, amr):
    """64 bundles of uneven size (256^2 .. 2048^2), source redshift and field
    of view through the AMR octree in one persistent launch fed by the device
    queue; replayed from a HIP graph; one 8x8 tile per bundle checked against
    the oracle."""
    import torch
    case, ot, tc, grid, tens = amr
    specs = I.config4_specs()
    plan = api.Plan()
    bundles, host_dirs, offset = [], [], 0
    for s in specs:
        b = I.bundle_from_spec(s)
        host_dirs.append(b.dirs)
        bundles.append(api.RayBundle(torch.as_tensor(b.dirs).cuda(), b.nx, b.ny, b.chi_s,
                                     b.chi_hi, b.chi_lo, offset))
        offset += b.nx * b.ny
    nr = offset
    print(f"[batched] {nr} rays in {len(specs)} bundles", flush=True)
    kap = torch.zeros(nr, dtype=torch.float32, device="cuda")
    comp = torch.zeros(nr, dtype=torch.float32, device="cuda")
    st = torch.zeros(nr, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        api.trace(plan, tens, bundles, case.observer, kappa=kap, kappa_comp=comp, status=st,
                  persistent=1)
        s.synchronize()
        eager = kap.clone()
        plan.graph_begin()
        api.trace(plan, tens, bundles, case.observer, kappa=kap, kappa_comp=comp, status=st,
                  persistent=1)
        plan.graph_end()
    for rep in range(2):
        kap.zero_()
        comp.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            plan.graph_launch()
        s.synchronize()
        assert torch.equal(kap, eager), rep
    assert bool((st == 0).all())
    # one tile (the centre 8x8 block) per bundle against the oracle
    k = eager.double().cpu().numpy()
    for s_, b, d in zip(specs, bundles, host_dirs):
        c0 = (b.nx // 2) & ~7
        idx = np.array([iy * b.nx + ix for iy in range(c0, c0 + 8) for ix in range(c0, c0 + 8)])
        ref = oracle.trace_octree(ot, case.box, case.observer, d[idx], b.chi_s, b.chi_hi,
                                  b.chi_lo, tc=tc)
        ok, worst = kappa_tolerance_ok(k[b.ray_offset + idx], ref.kappa)
        assert ok, (s_, worst)


@pytest.fixture(scope="module")
def lightcone():
    """The light cone to z = 1: 512^3 lognormal potential in a 1 Gpc/h box,
    scaled by s_k for each of the 20 segments, 2048^2 rays over 5x5 deg."""
    n, box, nray = 512, 1000.0, 2048
    _, phi0 = I.config2_fields(n, box)
    fov = math.radians(5.0)
    dirs = I.fov_directions((0.0, 0.0, 1.0), fov, fov, nray, nray)
    return n, box, nray, phi0, I.lightcone_segments(20), I.chi_of_z(1.0), dirs


def test_lightcone_full_size_sampled_rays(api, oracle, lightcone):
    """The light cone as it is timed: per segment an FP32 potential, the whole
    grid's tensor rebuilt, all 2048^2 rays in one one-wavefront-per-tile
    launch, FP32-Kahan.  Sampled rays (the map's corners, edge midpoints and
    centre, and 1500 at random) against the FP64 oracle over all 20 segments:
    every ray finishes, crossing hashes and counts bit-exact per segment (the
    same rays traced again with crossing hashes), kappa within tolerance."""
    import torch
    n, box, nray, phi0, segs, chi_s, dirs = lightcone
    obs = (0.0, 0.0, 0.0)
    nr = nray * nray
    m, h = nray - 1, nray // 2
    fixed = [0, m, m * nray, m * nray + m, h, h * nray, h * nray + m, m * nray + h,
             h * nray + h]
    rng = np.random.default_rng(2048)
    sel = np.unique(np.concatenate([fixed, rng.choice(nr, size=1500, replace=False)]))
    sdirs = np.ascontiguousarray(dirs[sel])
    phi0_d = torch.as_tensor(phi0, device="cuda")
    dirs_d = torch.as_tensor(dirs, device="cuda")
    sdirs_d = torch.as_tensor(sdirs, device="cuda")
    plan = api.Plan()
    kap = torch.zeros(nr, dtype=torch.float32, device="cuda")
    comp = torch.zeros(nr, dtype=torch.float32, device="cuda")
    st = torch.zeros(nr, dtype=torch.int32, device="cuda")
    t = None
    ref = np.zeros(len(sel))
    for k, (hi, lo, s) in enumerate(segs):
        phi = (phi0_d * s).to(torch.float32).contiguous()
        g = api.Grid(phi, box)
        if t is None:
            t = api.TidalTensor(g, "fp32")
        t.build(g)
        api.trace(plan, t, [api.RayBundle(dirs_d, nray, nray, chi_s, hi, lo)], obs, kappa=kap,
                  kappa_comp=comp, status=st, persistent=0)
        dbg = api.trace(plan, t, [api.RayBundle(sdirs_d, len(sel), 1, chi_s, hi, lo)], obs,
                        debug=True, persistent=0)
        tv = oracle.vertex_tensor(phi.double().cpu().numpy())
        r = oracle.trace_uniform(n, box, obs, sdirs, chi_s, hi, lo, tv=tv)
        del tv
        assert np.all(r.status == oracle.RAY_OK)
        assert np.array_equal(dbg.count.cpu().numpy(), r.ncross), k
        assert np.array_equal(hashes_u64(dbg.hash), r.hash), k
        ref += r.kappa
        print(f"[lightcone] segment {k}: {int(r.ncross.sum())} sampled crossings", flush=True)
    torch.cuda.synchronize()
    assert bool((st == 0).all())
    ok, worst = kappa_tolerance_ok(kap.double().cpu().numpy()[sel], ref)
    print(f"[lightcone] worst |err| / tol over {len(sel)} rays: {worst:.3g}", flush=True)
    assert ok, worst
    t.close()
    plan.close()


def test_adjoint_full_size_sampled_rays(api, oracle):
    """The adjoint case (256^3 FP32 potential, 1024^2 rays over 5x5 deg to
    chi_s = 256) in the timed launch: with dL/dkappa nonzero on 400 sampled
    rays only, dL/dPhi is those rays' gradient, which the oracle computes ray
    by ray (every cell within 1e-4 of the gradient's scale); with the full
    seeded weights the dot-product identity <A^T w, dPhi> = <w, A dPhi> holds
    on a random dPhi (kappa is linear in Phi)."""
    import torch
    case, w = I.config5()
    b = case.bundles[0]
    n, box = case.n, case.box
    nr = b.nx * b.ny
    g = api.Grid(torch.as_tensor(case.phi, device="cuda"), box)
    t = api.TidalTensor(g, "fp32").build()
    plan = api.Plan()
    gb = [api.RayBundle(torch.as_tensor(b.dirs, device="cuda"), b.nx, b.ny, b.chi_s, b.chi_hi,
                        b.chi_lo)]
    rng = np.random.default_rng(55)
    sel = np.sort(rng.choice(nr, size=400, replace=False))
    ws = np.zeros(nr, dtype=np.float32)
    ws[sel] = w[sel].astype(np.float32)
    got = api.trace_adjoint(plan, t, g, gb, case.observer,
                            torch.as_tensor(ws, device="cuda")).cpu().numpy()
    ref = oracle.trace_adjoint_uniform(n, box, case.observer, b.dirs[sel], b.chi_s, b.chi_hi,
                                       b.chi_lo, ws[sel].astype(np.float64))
    scale = np.abs(ref).max()
    assert scale > 0
    np.testing.assert_allclose(got.reshape(-1), ref.reshape(-1), rtol=0, atol=1e-4 * scale)
    # the dot-product identity with every ray weighted
    wt = torch.as_tensor(w.astype(np.float32), device="cuda")
    grad = api.trace_adjoint(plan, t, g, gb, case.observer, wt).double()
    dphi = torch.as_tensor(rng.standard_normal((n, n, n)).astype(np.float32) * 1e-5,
                           device="cuda")
    kd = api.trace(plan, t.build(api.Grid(dphi, box)), gb, case.observer,
                   persistent=0).kappa.double()
    lhs = float(torch.dot(wt.double(), kd).item())
    rhs = float(torch.sum(grad * dphi.double()).item())
    assert lhs == pytest.approx(rhs, rel=1e-4)
    t.close()
    plan.close()


def test_lightcone_fp64_tensor_above_4gib(api, oracle, lightcone):
    """The 512^3 light cone's farthest segment with an FP64 tensor (6.4 GB:
    the march addresses it with 64-bit offsets): sampled rays bit-exact in
    their crossings and within 1e-11 of the map's scale against the oracle."""
    import torch
    n, box, nray, phi0, segs, chi_s, dirs = lightcone
    hi, lo, s = segs[0]
    rng = np.random.default_rng(64)
    sel = np.sort(rng.choice(nray * nray, size=600, replace=False))
    sdirs = np.ascontiguousarray(dirs[sel])
    phi = (torch.as_tensor(phi0, device="cuda") * s).to(torch.float32).contiguous()
    t = api.TidalTensor(api.Grid(phi, box), "fp64").build()
    assert n ** 3 * 48 >= 1 << 32
    plan = api.Plan()
    out = api.trace(plan, t, [api.RayBundle(torch.as_tensor(sdirs, device="cuda"), len(sel), 1,
                                            chi_s, hi, lo)], (0.0, 0.0, 0.0), debug=True)
    tv = oracle.vertex_tensor(phi.double().cpu().numpy())
    ref = oracle.trace_uniform(n, box, (0.0, 0.0, 0.0), sdirs, chi_s, hi, lo, tv=tv)
    del tv
    assert np.all(out.status.cpu().numpy() == 0)
    assert np.array_equal(out.count.cpu().numpy(), ref.ncross)
    assert np.array_equal(hashes_u64(out.hash), ref.hash)
    k = out.kappa.cpu().numpy()
    np.testing.assert_allclose(k, ref.kappa, rtol=0, atol=1e-11 * np.abs(ref.kappa).max())
    t.close()
    plan.close()


def test_amr_fp64_corner_blocks_above_4gib(api, oracle, amr):
    """The AMR tree with FP64 corner blocks (20.6 M cells x 384 B = 7.9 GB,
    64-bit offsets in the octree march): 200 sampled rays of the 4096^2 map
    bit-exact in their crossings and within 1e-11 of the map's scale."""
    import torch
    case, ot, tc, grid, tens = amr
    assert case.tree.n_cells * 384 >= 1 << 32
    t64 = api.TidalTensor(grid, "fp64").build()
    b = I.config3_rays()
    rng = np.random.default_rng(65)
    sel = np.sort(rng.choice(b.nx * b.ny, size=200, replace=False))
    plan = api.Plan()
    sb = api.RayBundle(torch.as_tensor(b.dirs[sel]).cuda(), len(sel), 1, b.chi_s, b.chi_hi,
                       b.chi_lo)
    out = api.trace(plan, t64, [sb], case.observer, debug=True)
    ref = oracle.trace_octree(ot, case.box, case.observer, b.dirs[sel], b.chi_s, b.chi_hi,
                              b.chi_lo, tc=tc)
    assert np.all(out.status.cpu().numpy() == 0)
    assert np.array_equal(out.count.cpu().numpy(), ref.ncross)
    assert np.array_equal(hashes_u64(out.hash), ref.hash)
    k = out.kappa.cpu().numpy()
    np.testing.assert_allclose(k, ref.kappa, rtol=0, atol=1e-11 * np.abs(ref.kappa).max())
    t64.close()
    plan.close()
