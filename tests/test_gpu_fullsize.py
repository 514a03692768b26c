"""Full-size cases, checked on every ray or on sampled rays and leaves.

The light cone is the 512^3 lognormal potential of a 1 Gpc/h box over 20
segments to z = 1 with 2048^2 rays: Method B on every ray, the many-source,
Method A and ISW legs on a 1/64 subset of the map's tiles, each traced on the
GPU over the whole map in the launch configuration that is timed.

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


@pytest.fixture(scope="module")
def amr_corners(oracle, amr):
    """The oracle's corner tensors of every leaf (FP64, 8 x 6 per cell)."""
    case, ot, tc, grid, tens = amr
    cv = oracle.corner_tensor_octree(ot, tc)
    print(f"[amr] oracle corner tensors ready ({cv.nbytes / 1e9:.1f} GB)", flush=True)
    return cv


def tile_subset(nx, ny, every=64, phase=17):
    """Ray ids of a deterministic 1/every subset of a map's 8x8 tiles (tile ids
    t with t % every == phase % every, at least one tile): the oracle-traced
    subset of a map too large for the oracle in full."""
    tx, ty = (nx + 7) // 8, (ny + 7) // 8
    tiles = np.arange(tx * ty)
    pick = tiles[tiles % every == phase % min(every, tiles.size)]
    ids = []
    for t in pick:
        x0, y0 = (t % tx) * 8, (t // tx) * 8
        for iy in range(y0, min(y0 + 8, ny)):
            ids.extend(range(iy * nx + x0, iy * nx + min(x0 + 8, nx)))
    return np.asarray(ids, dtype=np.int64)


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


def test_amr_full_map_tile_subset(api, oracle, amr, amr_corners):
    """4096^2 rays over 10x10 deg to z = 1, FP32-Kahan, in the launch shape the
    benchmark's tuner picks for it (one wavefront per tile, 16 passes): every
    ray finishes; on a deterministic 1/64 subset of the 8x8 tiles (262 144
    rays, ~6.6e8 crossings) the crossing hashes and counts equal the oracle's
    bit for bit and kappa is within max(1e-5 |kappa|, 1e-7)."""
    import torch
    case, ot, tc, grid, tens = amr
    b = I.config3_rays()
    plan = api.Plan()
    gb = [api.RayBundle(torch.as_tensor(b.dirs).cuda(), b.nx, b.ny, b.chi_s, b.chi_hi,
                        b.chi_lo)]
    plan.set_shape(gb, persistent=0, block=256, passes=16)
    nr = b.nx * b.ny
    kap = torch.zeros(nr, dtype=torch.float32, device="cuda")
    comp = torch.zeros(nr, dtype=torch.float32, device="cuda")
    st = torch.zeros(nr, dtype=torch.int32, device="cuda")
    api.trace(plan, tens, gb, case.observer, kappa=kap, kappa_comp=comp, status=st,
              persistent=-1)
    assert bool((st == 0).all())
    k_all = kap.double().cpu().numpy()
    assert np.all(np.isfinite(k_all))
    dbg = api.trace(plan, tens, gb, case.observer, debug=True, persistent=0)
    h_all = hashes_u64(dbg.hash)
    c_all = dbg.count.cpu().numpy()
    sel = tile_subset(b.nx, b.ny)
    print(f"[amr] oracle on {sel.size} rays of the map", flush=True)
    ref = oracle.trace_octree(ot, case.box, case.observer, b.dirs[sel], b.chi_s, b.chi_hi,
                              b.chi_lo, cv=amr_corners)
    assert np.all(ref.status == oracle.RAY_OK)
    print(f"[amr] {int(ref.ncross.sum())} oracle crossings", flush=True)
    assert np.array_equal(c_all[sel], ref.ncross)
    assert np.array_equal(h_all[sel], ref.hash)
    ok, worst = kappa_tolerance_ok(k_all[sel], ref.kappa)
    print(f"[amr] worst |err| / tol over {sel.size} rays: {worst:.3g}", flush=True)
    assert ok, worst
    plan.close()


def test_batched_bundles_persistent_and_graph(api, oracle, amr, amr_corners):
    """64 bundles of uneven size (256^2 .. 2048^2), source redshift and field
    of view through the AMR octree in one persistent launch fed by the device
    queue, split into 16 passes and replayed from a HIP graph (replays equal
    the eager run bit for bit); on a deterministic 1/64 subset of every
    bundle's 8x8 tiles the crossing hashes and counts (from one persistent
    launch of all bundles with crossing hashes) equal the oracle's and kappa
    is within tolerance."""
    import torch
    case, ot, tc, grid, tens = amr
    specs = I.config4_specs()
    plan = api.Plan()
    bundles, host_dirs, offset = [], [], 0
    for s in specs:
        b = I.bundle_from_spec(s)
        host_dirs.append(b.dirs)
        bundles.append(api.RayBundle(torch.as_tensor(b.dirs).cuda(), b.nx, b.ny, b.chi_s,
                                     b.chi_hi, b.chi_lo, offset, b.center, b.fov_x, b.fov_y))
        offset += b.nx * b.ny
    nr = offset
    print(f"[batched] {nr} rays in {len(specs)} bundles", flush=True)
    plan.set_shape(bundles, persistent=1, waves_per_cu=16, passes=16)
    kap = torch.zeros(nr, dtype=torch.float32, device="cuda")
    comp = torch.zeros(nr, dtype=torch.float32, device="cuda")
    st = torch.zeros(nr, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        api.trace(plan, tens, bundles, case.observer, kappa=kap, kappa_comp=comp, status=st,
                  persistent=-1)
        s.synchronize()
        eager = kap.clone()
        plan.graph_begin()
        api.trace(plan, tens, bundles, case.observer, kappa=kap, kappa_comp=comp, status=st,
                  persistent=-1)
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
    dbg = api.trace(plan, tens, bundles, case.observer, debug=True, persistent=1)
    h_all = hashes_u64(dbg.hash)
    c_all = dbg.count.cpu().numpy()
    del dbg
    k = eager.double().cpu().numpy()
    total = 0
    for s_, b, d in zip(specs, bundles, host_dirs):
        idx = tile_subset(b.nx, b.ny)
        ref = oracle.trace_octree(ot, case.box, case.observer, d[idx], b.chi_s, b.chi_hi,
                                  b.chi_lo, cv=amr_corners)
        total += int(ref.ncross.sum())
        assert np.all(ref.status == oracle.RAY_OK), s_
        assert np.array_equal(c_all[b.ray_offset + idx], ref.ncross), s_
        assert np.array_equal(h_all[b.ray_offset + idx], ref.hash), s_
        ok, worst = kappa_tolerance_ok(k[b.ray_offset + idx], ref.kappa)
        assert ok, (s_, worst)
    print(f"[batched] {total} oracle crossings on the tile subsets", flush=True)
    plan.close()


# the many-source leg's source redshifts
LIGHTCONE_SOURCE_Z = [1.0, 0.9, 0.8, 0.7, 0.6, 0.5, 0.4, 0.3, 0.2, 0.1]


@pytest.fixture(scope="module")
def lightcone_fields():
    """(delta0, phi0) of the 512^3, 1 Gpc/h light cone (FP64)."""
    return I.config2_fields(512, 1000.0)


@pytest.fixture(scope="module")
def lightcone(lightcone_fields):
    """The light cone to z = 1: 512^3 lognormal potential in a 1 Gpc/h box,
    scaled by s_k for each of the 20 segments, 2048^2 rays over 5x5 deg."""
    n, box, nray = 512, 1000.0, 2048
    phi0 = lightcone_fields[1]
    fov = math.radians(5.0)
    dirs = I.fov_directions((0.0, 0.0, 1.0), fov, fov, nray, nray)
    return n, box, nray, phi0, I.lightcone_segments(20), I.chi_of_z(1.0), dirs


def test_lightcone_full_size_every_ray(api, oracle, lightcone):
    """The light cone as it is timed: per segment an FP32 potential, the whole
    grid's tensor rebuilt, all 2048^2 rays in one one-wavefront-per-tile
    launch, FP32-Kahan, kappa and its compensation carried over the 20
    segments.  Every ray against the FP64 oracle: in each of the 20 segments
    the crossing hashes and counts of all 4 194 304 rays equal the oracle's
    bit for bit (the rays traced again with crossing hashes), every ray
    finishes, and the final kappa of every ray is within
    max(1e-5 |kappa|, 1e-7).

    The same tensors also carry the many-source leg as it is timed: ten
    sources (z = 1.0, 0.9, ..., 0.1) in one walk over the 20 segments with
    FP32-Kahan moments, then kappa from the pieces.  On a 1/64 subset of the
    map's 8x8 tiles the walk's crossing hashes and counts of every segment
    equal the oracle's (its walk carrying moments and pieces over the
    segments the same way) and every source's kappa is within
    max(1e-5 |kappa|, 1e-7) of the oracle's."""
    import torch
    n, box, nray, phi0, segs, chi_s, dirs = lightcone
    obs = (0.0, 0.0, 0.0)
    nr = nray * nray
    phi0_d = torch.as_tensor(phi0, device="cuda")
    dirs_d = torch.as_tensor(dirs, device="cuda")
    plan = api.Plan()
    kap = torch.zeros(nr, dtype=torch.float32, device="cuda")
    comp = torch.zeros(nr, dtype=torch.float32, device="cuda")
    st = torch.zeros(nr, dtype=torch.int32, device="cuda")
    dk = torch.zeros(nr, dtype=torch.float32, device="cuda")
    dc = torch.zeros(nr, dtype=torch.float32, device="cuda")
    ds = torch.zeros(nr, dtype=torch.int32, device="cuda")
    t = None
    ref = np.zeros(nr)
    total = 0
    ids = tile_subset(nray, nray)
    sub = np.ascontiguousarray(dirs[ids])
    src = np.array([I.chi_of_z(z) for z in LIGHTCONE_SOURCE_Z])
    state = api.SourcesOutput(torch.zeros((nr, 4), dtype=torch.float32, device="cuda"),
                              torch.zeros((nr, src.size, 2), dtype=torch.float64, device="cuda"),
                              torch.zeros(nr, dtype=torch.int32, device="cuda"))
    dstate = mom = pcs = None
    for k, (hi, lo, s) in enumerate(segs):
        phi = (phi0_d * s).to(torch.float32).contiguous()
        g = api.Grid(phi, box)
        if t is None:
            t = api.TidalTensor(g, "fp32")
        t.build(g)
        bundle = [api.RayBundle(dirs_d, nray, nray, chi_s, hi, lo)]
        api.trace(plan, t, bundle, obs, kappa=kap, kappa_comp=comp, status=st, persistent=0)
        dbg = api.trace(plan, t, bundle, obs, kappa=dk, kappa_comp=dc, status=ds, debug=True,
                        persistent=0)
        h_gpu = hashes_u64(dbg.hash)
        c_gpu = dbg.count.cpu().numpy()
        tv = oracle.vertex_tensor(phi.double().cpu().numpy())
        r = oracle.trace_uniform(n, box, obs, dirs, chi_s, hi, lo, tv=tv)
        assert np.all(r.status == oracle.RAY_OK), k
        assert np.array_equal(c_gpu, r.ncross), k
        assert np.array_equal(h_gpu, r.hash), k
        ref += r.kappa
        total += int(r.ncross.sum())
        # the many-source walk through the same tensor
        api.trace_sources(plan, t, bundle, obs, src, state=state, persistent=0)
        dstate = api.trace_sources(plan, t, bundle, obs, src, state=dstate, debug=True,
                                   persistent=0)
        rs = oracle.trace_uniform_sources(n, box, obs, sub, hi, lo, src, tv=tv, moments=mom,
                                          pieces=pcs)
        del tv
        mom, pcs = rs.moments, rs.pieces
        assert np.all(rs.status == oracle.RAY_OK), k
        assert np.array_equal(dstate.count.cpu().numpy()[ids], rs.ncross), k
        assert np.array_equal(hashes_u64(dstate.hash)[ids], rs.hash), k
        print(f"[lightcone] segment {k}: {int(r.ncross.sum())} crossings, every ray's hash and "
              "count equal; the sampled rays' many-source walk too", flush=True)
    torch.cuda.synchronize()
    assert bool((st == 0).all())
    ok, worst = kappa_tolerance_ok(kap.double().cpu().numpy(), ref)
    print(f"[lightcone] {total} crossings; worst |err| / tol over {nr} rays: {worst:.3g}",
          flush=True)
    assert ok, worst
    assert bool((state.status == 0).all())
    kw = api.kappa_from_pieces(plan, t, src, state).cpu().numpy()[ids]
    kr = oracle.kappa_from_pieces(src, box, n, mom, pcs)
    worst = 0.0
    for j in range(src.size):
        ok, w = kappa_tolerance_ok(kw[:, j], kr[:, j])
        worst = max(worst, w)
        assert ok, (LIGHTCONE_SOURCE_Z[j], w)
    print(f"[lightcone] many sources: {ids.size} sampled rays x {src.size} sources; worst "
          f"|err| / tol {worst:.3g}", flush=True)
    t.close()
    plan.close()


def _lightcone_gpu(api, lightcone):
    import torch
    n, box, nray, phi0, segs, chi_s, dirs = lightcone
    nr = nray * nray
    dirs_d = torch.as_tensor(dirs, device="cuda")
    zeros = lambda dt: torch.zeros(nr, dtype=dt, device="cuda")
    return dirs_d, zeros, tile_subset(nray, nray)


def test_lightcone_method_a_full_size_tile_subset(api, oracle, lightcone, lightcone_fields):
    """Method A over the light cone as it is timed: per segment the vertex
    fields (c s_k delta, grad Phi_k) of the whole 512^3 grid rebuilt, all
    2048^2 rays in one one-wavefront-per-tile launch, kappa and its
    compensation carried over the 20 segments in FP32-Kahan.  On a 1/64
    subset of the map's 8x8 tiles the crossing hashes and counts of every
    segment equal the FP64 oracle's bit for bit and the final kappa is within
    max(1e-5 |kappa|, 1e-7)."""
    import torch
    n, box, nray, phi0, segs, chi_s, dirs = lightcone
    obs = (0.0, 0.0, 0.0)
    dirs_d, zeros, ids = _lightcone_gpu(api, lightcone)
    sub = np.ascontiguousarray(dirs[ids])
    d32 = lightcone_fields[0].astype(np.float32)
    d64 = d32.astype(np.float64)
    gd = api.Grid(torch.as_tensor(d32, device="cuda"), box, field="delta")
    t = api.TidalTensor(gd, "fp32")
    plan = api.Plan()
    kap, comp, st = zeros(torch.float32), zeros(torch.float32), zeros(torch.int32)
    c0 = I.poisson_coefficient()
    ref = np.zeros(ids.size)
    for k, (hi, lo, s) in enumerate(segs):
        phi = (phi0 * s).astype(np.float32)
        gp = api.Grid(torch.as_tensor(phi, device="cuda"), box)
        t.build_method_a(gd, gp, c0 * s)
        bundle = [api.RayBundle(dirs_d, nray, nray, chi_s, hi, lo)]
        api.trace(plan, t, bundle, obs, kappa=kap, kappa_comp=comp, status=st, persistent=0)
        dbg = api.trace(plan, t, bundle, obs, debug=True, persistent=0)
        r = oracle.trace_uniform_method_a(n, box, obs, sub, chi_s, hi, lo, delta_coeff=c0 * s,
                                          phi=phi.astype(np.float64), delta=d64)
        assert np.all(r.status == oracle.RAY_OK), k
        assert np.array_equal(dbg.count.cpu().numpy()[ids], r.ncross), k
        assert np.array_equal(hashes_u64(dbg.hash)[ids], r.hash), k
        ref += r.kappa
        del dbg, gp
    torch.cuda.synchronize()
    assert bool((st == 0).all())
    ok, worst = kappa_tolerance_ok(kap.double().cpu().numpy()[ids], ref)
    print(f"[method A] {ids.size} sampled rays: hashes and counts equal in all 20 segments; "
          f"worst |err| / tol {worst:.3g}", flush=True)
    assert ok, worst
    t.close()
    plan.close()


def test_lightcone_isw_full_size_tile_subset(api, oracle, lightcone):
    """The ISW leg as it is timed: per segment the vertex field of
    (Phi_k - Phi_k-1)/dt over the whole grid and all 2048^2 rays with the
    constant kernel 2 a_k / c, FP32-Kahan over the 20 segments.  On a 1/64
    tile subset the crossing hashes and counts of every segment equal the
    oracle's and the final map is within max(1e-5 |x|, 1e-5 rms): the map's
    rms is ~2e-6, so the kappa floor of 1e-7 (1e-5 of a kappa map's rms)
    becomes 1e-5 of this map's rms."""
    import torch
    n, box, nray, phi0, segs, chi_s, dirs = lightcone
    obs = (0.0, 0.0, 0.0)
    dirs_d, zeros, ids = _lightcone_gpu(api, lightcone)
    sub = np.ascontiguousarray(dirs[ids])
    steps = I.isw_steps(len(segs))
    plan = api.Plan()
    out, comp, st = zeros(torch.float32), zeros(torch.float32), zeros(torch.int32)
    ref = np.zeros(ids.size)
    # the potential one step before the first segment
    prev = (phi0 * segs[0][2]).astype(np.float32) * np.float32(steps[0][0] / steps[0][1])
    gprev = api.Grid(torch.as_tensor(prev, device="cuda"), box)
    t = None
    for k, (hi, lo, s) in enumerate(segs):
        curr = (phi0 * s).astype(np.float32)
        gcurr = api.Grid(torch.as_tensor(curr, device="cuda"), box)
        if t is None:
            t = api.TidalTensor(api.Grid(gcurr.values, box, field="phi_dot"), "fp32")
        t.build_isw(gcurr, gprev, steps[k][2])
        bundle = [api.RayBundle(dirs_d, nray, nray, chi_s, hi, lo)]
        api.trace(plan, t, bundle, obs, kappa=out, kappa_comp=comp, status=st,
                  quantity="scalar", kappa_scale=steps[k][3], persistent=0)
        dbg = api.trace(plan, t, bundle, obs, quantity="scalar", kappa_scale=steps[k][3],
                        debug=True, persistent=0)
        qv = oracle.isw_vertex_field(curr.astype(np.float64), prev.astype(np.float64),
                                     steps[k][2])
        r = oracle.trace_uniform_isw(n, box, obs, sub, hi, lo, qv=qv, scale=steps[k][3])
        del qv
        assert np.all(r.status == oracle.RAY_OK), k
        assert np.array_equal(dbg.count.cpu().numpy()[ids], r.ncross), k
        assert np.array_equal(hashes_u64(dbg.hash)[ids], r.hash), k
        ref += r.kappa
        prev, gprev = curr, gcurr
        del dbg
    torch.cuda.synchronize()
    assert bool((st == 0).all())
    rms = float(np.sqrt(np.mean(ref ** 2)))
    assert 1e-7 < rms < 1e-4, rms
    ok, worst = kappa_tolerance_ok(out.double().cpu().numpy()[ids], ref, abs_=1e-5 * rms)
    print(f"[isw] {ids.size} sampled rays, map rms {rms:.3g}: hashes and counts equal in all "
          f"20 segments; worst |err| / tol {worst:.3g}", flush=True)
    assert ok, worst
    t.close()
    plan.close()


def _rays_near_box(dirs, obs, lo, hi, chi_lo, chi_hi):
    """Rays of unit directions ``dirs`` from ``obs`` whose segment
    [chi_lo, chi_hi] meets the axis-aligned box [lo, hi) (cell units), and
    the parameter range over which each one is inside it (slab test)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / dirs
        t0 = (lo[None, :] - obs[None, :]) * inv
        t1 = (hi[None, :] - obs[None, :]) * inv
    tmin = np.where(np.isnan(t0), -np.inf, np.minimum(t0, t1))
    tmax = np.where(np.isnan(t1), np.inf, np.maximum(t0, t1))
    # an axis the ray does not move along: inside iff its coordinate is
    inside = (obs[None, :] >= lo[None, :]) & (obs[None, :] < hi[None, :])
    flat = dirs == 0.0
    tmin = np.where(flat, np.where(inside, -np.inf, np.inf), tmin)
    tmax = np.where(flat, np.where(inside, np.inf, -np.inf), tmax)
    enter = np.maximum(tmin.max(axis=1), chi_lo)
    leave = np.minimum(tmax.min(axis=1), chi_hi)
    hit = enter < leave
    return np.nonzero(hit)[0], enter[hit], leave[hit]


def test_adjoint_full_size(api, oracle):
    """The adjoint case as stated: 256^3 FP32 potential, 1024^2 rays over 5x5
    deg to chi_s = 256, L = sum(w kappa) with the full seeded w.
     * Forward: every ray's crossing hash and count equal the oracle's, kappa
       within tolerance (the timed launch shape).
     * dL/dPhi from rr_trace_rays_adjoint with every weight: every cell within
       1e-4 max|grad| of the oracle's gradient (FP64 transpose of the chain).
     * Central differences in the FP64 oracle on 32 cells sampled among those
       with a non-zero oracle gradient: kappa is linear in Phi (Born
       approximation, Eq. jacobian2) and additive over pieces of the line of
       sight (Eq. sumIc), so (L(Phi + eps e_c) - L(Phi - eps e_c)) / (2 eps)
       over the rays and chi range that pass within three cells of the
       stencil's reach (cells c-2..c+2 feed the corners of c's neighbours) is
       the derivative up to rounding, for any eps; it matches the oracle's
       gradient to 1e-4 relative and the GPU's to 1e-4 max|grad|."""
    import torch
    case, w = I.config5()
    b = case.bundles[0]
    n, box = case.n, case.box
    nr = b.nx * b.ny
    obs = np.asarray(case.observer, dtype=np.float64)
    g = api.Grid(torch.as_tensor(case.phi, device="cuda"), box)
    t = api.TidalTensor(g, "fp32").build()
    plan = api.Plan()
    gb = [api.RayBundle(torch.as_tensor(b.dirs, device="cuda"), b.nx, b.ny, b.chi_s, b.chi_hi,
                        b.chi_lo, 0, b.center, b.fov_x, b.fov_y)]
    phi64 = case.phi.astype(np.float64)
    fwd = api.trace(plan, t, gb, case.observer, persistent=0, debug=True)
    r = oracle.trace_uniform(n, box, case.observer, b.dirs, b.chi_s, b.chi_hi, b.chi_lo,
                             phi=phi64)
    assert np.all(r.status == oracle.RAY_OK)
    assert np.array_equal(fwd.count.cpu().numpy(), r.ncross)
    assert np.array_equal(hashes_u64(fwd.hash), r.hash)
    ok, worst = kappa_tolerance_ok(fwd.kappa.double().cpu().numpy(), r.kappa)
    assert ok, worst
    print(f"[adjoint] forward: {int(r.ncross.sum())} crossings, every hash equal", flush=True)
    wt = torch.as_tensor(w.astype(np.float32), device="cuda")
    got = api.trace_adjoint(plan, t, g, gb, case.observer, wt).double().cpu().numpy()
    ref = oracle.trace_adjoint_uniform(n, box, case.observer, b.dirs, b.chi_s, b.chi_hi,
                                       b.chi_lo, w.astype(np.float32).astype(np.float64))
    scale = np.abs(ref).max()
    assert scale > 0
    err = np.abs(got - ref).max()
    print(f"[adjoint] max |GPU - oracle| / max|grad| = {err / scale:.3g}", flush=True)
    assert err <= 1e-4 * scale
    # central differences on 32 cells (h0 = 1: cell units are box units here)
    h0 = box / n
    assert h0 == 1.0
    rng = np.random.default_rng(5005)
    nz = np.flatnonzero(np.abs(ref) > 1e-6 * scale)
    cells = rng.choice(nz, size=32, replace=False)
    w64 = w.astype(np.float32).astype(np.float64)
    eps = 1e-3
    for c in cells:
        cz, cy, cx = np.unravel_index(c, (n, n, n))
        fd = 0.0
        # periodic images of the reach box [c-3, c+4) that the cone can meet
        for sz in (-n, 0, n):
            for sy in (-n, 0, n):
                for sx in (-n, 0, n):
                    lo = np.array([cx - 3 + sx, cy - 3 + sy, cz - 3 + sz], dtype=np.float64)
                    hi = lo + 7.0
                    ids, t_in, t_out = _rays_near_box(b.dirs, obs, lo, hi, b.chi_lo, b.chi_hi)
                    if ids.size == 0:
                        continue
                    w_hi = min(b.chi_hi, float(t_out.max()) + 2.0)
                    w_lo = max(b.chi_lo, float(t_in.min()) - 2.0)
                    part = []
                    for sign in (1.0, -1.0):
                        pp = phi64.copy()
                        pp[cz, cy, cx] += sign * eps
                        rr = oracle.trace_uniform(n, box, case.observer, b.dirs[ids], b.chi_s,
                                                  w_hi, w_lo, phi=pp)
                        part.append(rr.kappa)
                    fd += float(np.dot(w64[ids], part[0] - part[1])) / (2.0 * eps)
        assert abs(fd - ref.flat[c]) <= 1e-4 * abs(ref.flat[c]), (c, fd, ref.flat[c])
        assert abs(fd - got.flat[c]) <= 1e-4 * scale, (c, fd, got.flat[c])
    print(f"[adjoint] central differences on {cells.size} cells agree", flush=True)
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
