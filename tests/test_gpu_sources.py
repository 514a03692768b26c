"""GPU parity of the many-source walk (Sec. VII, Eqs. Isources, Isources1)
against the FP64 oracle.

Bars: the cut crossing lists bit-exact (per-ray FNV-1a hash and count per
window); FP64 pieces and moments to 1e-11 of their scale; FP32-Kahan kappa of
every source within max(1e-5 |kappa|, 1e-7) of the oracle's single-source
trace for that source (the definition the walk must reproduce)."""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I
from tests._cases import gpu_bundle, gpu_grid, hashes_u64, kappa_tolerance_ok

pytestmark = pytest.mark.gpu

# c1 geometry (64^3, box 256, 128^2 rays over 2x2 deg from the corner); the
# sources include window boundaries (180, 100) and the far end of the walk
SOURCES = np.array([256.0, 211.7, 180.0, 150.3, 100.0, 63.9, 30.7, 5.5])
WINDOWS = [(256.0, 180.0), (180.0, 100.0), (100.0, 0.0)]


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1601_02012_amd import api as A
    return A


@pytest.fixture(scope="module")
def plan(api):
    return api.Plan()


@pytest.fixture(scope="module")
def c1():
    return I.config1()


def _walk_gpu(api, plan, t, c1, dirs, nx, ny, *, quantity="kappa", persistent=0):
    state = None
    hashes, counts = [], []
    for hi, lo in WINDOWS:
        gb = gpu_bundle(api, dirs, nx, ny, SOURCES[0], hi, lo)
        state = api.trace_sources(plan, t, [gb], c1.observer, SOURCES, state=state,
                                  quantity=quantity, persistent=persistent, debug=True)
        assert np.all(state.status.cpu().numpy() == 0)
        hashes.append(hashes_u64(state.hash))
        counts.append(state.count.cpu().numpy())
    return state, hashes, counts


def _walk_oracle(oracle, c1, dirs, tv, quantity=0):
    mom = pcs = None
    hashes, counts = [], []
    for hi, lo in WINDOWS:
        r = oracle.trace_uniform_sources(c1.n, c1.box, c1.observer, dirs, hi, lo, SOURCES, tv=tv,
                                         quantity=quantity, moments=mom, pieces=pcs)
        mom, pcs = r.moments, r.pieces
        hashes.append(r.hash)
        counts.append(r.ncross)
    return mom, pcs, hashes, counts


@pytest.mark.parametrize("quantity,q", [("kappa", 0), ("gamma1", 1)])
def test_fp64_pieces_and_cut_crossings_match_oracle(api, oracle, plan, c1, quantity, q):
    b = c1.bundles[0]
    t = api.TidalTensor(gpu_grid(api, c1.phi, c1.box), "fp64").build()
    st, gh, gc = _walk_gpu(api, plan, t, c1, b.dirs, b.nx, b.ny, quantity=quantity)
    tv = oracle.vertex_tensor(c1.phi)
    mom, pcs, oh, oc = _walk_oracle(oracle, c1, b.dirs, tv, q)
    for w in range(len(WINDOWS)):
        assert np.array_equal(gc[w], oc[w])
        assert np.array_equal(gh[w], oh[w])
    got_p = st.pieces.cpu().numpy()
    got_m = st.moments.cpu().numpy()
    for c in range(2):
        sc = np.abs(pcs[..., c]).max()
        np.testing.assert_allclose(got_p[..., c], pcs[..., c], rtol=0, atol=1e-11 * sc)
        np.testing.assert_allclose(got_m[:, c], mom[:, c], rtol=0,
                                   atol=1e-11 * np.abs(mom[:, c]).max())
    kap = api.kappa_from_pieces(plan, t, SOURCES, st).cpu().numpy()
    ref = oracle.kappa_from_pieces(SOURCES, c1.box, c1.n, mom, pcs)
    np.testing.assert_allclose(kap, ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    t.close()


def test_fp32_kahan_every_source_within_tolerance(api, oracle, plan, c1):
    """FP32 tensor and Kahan moments: kappa of each of the eight sources
    against the oracle's own trace from that source to the observer."""
    b = c1.bundles[0]
    phi32 = c1.phi.astype(np.float32)
    t = api.TidalTensor(gpu_grid(api, phi32, c1.box), "fp32").build()
    st, gh, gc = _walk_gpu(api, plan, t, c1, b.dirs, b.nx, b.ny)
    tv = oracle.vertex_tensor(phi32.astype(np.float64))
    _, _, oh, oc = _walk_oracle(oracle, c1, b.dirs, tv)
    for w in range(len(WINDOWS)):
        assert np.array_equal(gh[w], oh[w])
    kap = api.kappa_from_pieces(plan, t, SOURCES, st).cpu().numpy()
    worst = 0.0
    for j, cs in enumerate(SOURCES):
        ref = oracle.trace_uniform(c1.n, c1.box, c1.observer, b.dirs, cs, cs, 0.0, tv=tv)
        ok, w = kappa_tolerance_ok(kap[:, j], ref.kappa)
        worst = max(worst, w)
        assert ok, (cs, w)
    print(f"worst |err| / tol over sources: {worst:.3g}")
    t.close()


def test_bundles_offsets_persistent_and_direct_agree(api, oracle, plan, c1):
    """Two ragged bundles (several tiles and partial tiles) at offsets in the
    same arrays: persistent and one-wavefront-per-tile launches give the same
    bits, and the FP32 pieces follow the FP64 oracle."""
    import torch
    fov = math.radians(3.0)
    d1 = I.fov_directions((0.05, 0.02, 1.0), fov, fov * 13 / 37, 37, 13)
    d2 = I.fov_directions((-0.1, 0.07, 1.0), fov / 2, fov / 2, 9, 21)
    phi32 = c1.phi.astype(np.float32)
    t = api.TidalTensor(gpu_grid(api, phi32, c1.box), "fp32").build()
    outs = []
    for persistent in (0, 1):
        state = None
        for hi, lo in WINDOWS:
            gb = [gpu_bundle(api, d1, 37, 13, SOURCES[0], hi, lo, 0),
                  gpu_bundle(api, d2, 9, 21, SOURCES[0], hi, lo, 37 * 13)]
            state = api.trace_sources(plan, t, gb, c1.observer, SOURCES, state=state,
                                      persistent=persistent)
        torch.cuda.synchronize()
        outs.append((state.moments.cpu().numpy(), state.pieces.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    tv = oracle.vertex_tensor(phi32.astype(np.float64))
    dirs = np.concatenate([d1, d2])
    mom, pcs, _, _ = _walk_oracle(oracle, c1, dirs, tv)
    kap = api.kappa_from_pieces(plan, t, SOURCES, api.SourcesOutput(
        torch.as_tensor(outs[0][0]).cuda(), torch.as_tensor(outs[0][1]).cuda(), None)).cpu().numpy()
    ref = oracle.kappa_from_pieces(SOURCES, c1.box, c1.n, mom, pcs)
    ok, worst = kappa_tolerance_ok(kap, ref)
    assert ok, worst
    t.close()


def test_single_source_equals_plain_trace(api, oracle, plan, c1):
    """One source at the start of the walk: nothing is cut, the pieces stay
    as given, and kappa_from_pieces equals rr_trace_rays with that chi_s."""
    import torch
    b = c1.bundles[0]
    t = api.TidalTensor(gpu_grid(api, c1.phi, c1.box), "fp64").build()
    src = np.array([256.0])
    gb = gpu_bundle(api, b.dirs, b.nx, b.ny, 256.0, 256.0, 0.0)
    nr = b.nx * b.ny
    st = api.SourcesOutput(torch.zeros((nr, 2), dtype=torch.float64, device="cuda"),
                           torch.full((nr, 1, 2), 3.0, dtype=torch.float64, device="cuda"),
                           torch.zeros(nr, dtype=torch.int32, device="cuda"))
    st = api.trace_sources(plan, t, [gb], c1.observer, src, state=st, debug=True)
    plain = api.trace(plan, t, [gb], c1.observer, debug=True)
    assert np.array_equal(hashes_u64(st.hash), hashes_u64(plain.hash))
    assert torch.all(st.pieces == 3.0)
    st.pieces.zero_()
    kap = api.kappa_from_pieces(plan, t, src, st).cpu().numpy()[:, 0]
    ref = plain.kappa.cpu().numpy()
    np.testing.assert_allclose(kap, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    t.close()


def test_empty_bundle_and_rejected_arguments(api, plan, c1):
    import torch
    t = api.TidalTensor(gpu_grid(api, c1.phi.astype(np.float32), c1.box), "fp32").build()
    empty = api.RayBundle(torch.zeros((0, 3), dtype=torch.float64, device="cuda"), 0, 0,
                          256.0, 256.0, 0.0)
    st = api.trace_sources(plan, t, [empty], c1.observer, SOURCES)
    assert st.moments.shape[0] == 0
    b = c1.bundles[0]
    gb = gpu_bundle(api, b.dirs, b.nx, b.ny, 256.0, 256.0, 0.0)
    with pytest.raises(api.RRError):
        api.trace_sources(plan, t, [gb], c1.observer, [100.0, 200.0])     # not decreasing
    with pytest.raises(api.RRError):
        api.trace_sources(plan, t, [gb], c1.observer, [100.0, -1.0])
    with pytest.raises(api.RRError):
        api.trace_sources(plan, t, [gb], c1.observer, [float("nan")])
    t.close()
    tc = api.TidalTensor(gpu_grid(api, c1.phi.astype(np.float32), c1.box), "fp32").build_centres()
    with pytest.raises(api.RRError):
        api.trace_sources(plan, tc, [gb], c1.observer, SOURCES)           # NGP records
    tc.close()


# ---------------------------------------------------------------- octree --
@pytest.fixture(scope="module")
def tree_case():
    from tests.test_gpu_octree import _smooth_phi
    rng = np.random.default_rng(41)
    t = I.random_octree(12, 3, 0.2, rng, region=(2.0, 10.0))
    box = 24.0
    return t, box, _smooth_phi(t, box, rng)


OCT_SOURCES = np.array([60.0, 47.3, 31.05, 20.0, 8.8, 0.9])
OCT_WINDOWS = [(60.0, 20.0), (20.0, 0.0)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_octree_sources_match_oracle(api, oracle, plan, tree_case, prec):
    """Multi-level octree: cut crossing hashes bit-exact per window, FP64
    pieces to 1e-11 of their scale, FP32-Kahan kappa of every source within
    max(1e-5 |kappa|, 1e-7) of the oracle's single-source octree trace."""
    import torch
    from tests.test_gpu_octree import _gpu_octree_grid, _otree
    t, box, phi = tree_case
    dt = np.float64 if prec == "fp64" else np.float32
    tt = api.TidalTensor(_gpu_octree_grid(api, t, phi, box, dt), prec).build()
    fov = math.radians(50.0)
    nx, ny = 21, 13
    dirs = I.fov_directions((0.2, 0.1, 1.0), fov, fov * 0.6, nx, ny)
    obs = (11.7, 12.2, 3.1)
    ot = _otree(oracle, t)
    p64 = phi.astype(dt).astype(np.float64)
    cv = oracle.corner_tensor_octree(ot, oracle.centre_tensor_octree(ot, p64))
    state = None
    mom = pcs = None
    for hi, lo in OCT_WINDOWS:
        b = api.RayBundle(torch.as_tensor(dirs).cuda(), nx, ny, OCT_SOURCES[0], hi, lo)
        state = api.trace_sources(plan, tt, [b], obs, OCT_SOURCES, state=state, debug=True)
        r = oracle.trace_octree_sources(ot, box, obs, dirs, hi, lo, OCT_SOURCES, cv=cv,
                                        moments=mom, pieces=pcs)
        mom, pcs = r.moments, r.pieces
        assert np.all(state.status.cpu().numpy() == 0)
        assert np.array_equal(state.count.cpu().numpy(), r.ncross)
        assert np.array_equal(hashes_u64(state.hash), r.hash)
    kap = api.kappa_from_pieces(plan, tt, OCT_SOURCES, state).cpu().numpy()
    if prec == "fp64":
        got = state.pieces.cpu().numpy()
        for c in range(2):
            np.testing.assert_allclose(got[..., c], pcs[..., c], rtol=0,
                                       atol=1e-11 * np.abs(pcs[..., c]).max())
        ref = oracle.kappa_from_pieces(OCT_SOURCES, box, t.n, mom, pcs)
        np.testing.assert_allclose(kap, ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    else:
        for j, cs in enumerate(OCT_SOURCES):
            ref = oracle.trace_octree(ot, box, obs, dirs, cs, cs, 0.0, cv=cv)
            ok, worst = kappa_tolerance_ok(kap[:, j], ref.kappa)
            assert ok, (cs, worst)
    tt.close()
