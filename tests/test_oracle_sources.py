"""Pins of the oracle's many-source walk (Sec. VII, Eqs. Isources, Isources1).

The walk integrates A = int chi Q and B = int chi^2 Q once, stopping at every
source distance; kappa of each source follows from the pieces.  Pinned
against: Gauss quadrature of the trilinear field (the two cell integrals),
the single-source definition of kappa (Eq. kappa through Eq. Iclensing, the
oracle's independently pinned walk) for every source, the closed form of a
constant transverse Laplacian, the crossing count and window splitting.
"""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I
from tests._independent import GL5_W, GL5_X
from tests.test_oracle_octree import _otree

RNG = np.random.default_rng(20261203)


def _trilinear(Qv, u):
    q = np.zeros(u.shape[0])
    for v in range(8):
        ix, iy, iz = v & 1, (v >> 1) & 1, (v >> 2) & 1
        w = ((u[:, 0] if ix else 1 - u[:, 0]) * (u[:, 1] if iy else 1 - u[:, 1])
             * (u[:, 2] if iz else 1 - u[:, 2]))
        q += w * Qv[v]
    return q


def _periodic_case(seed, n=20, box=40.0, nx=9, ny=7, fov_deg=12.0):
    rng = np.random.default_rng(seed)
    phi = I.poisson_phi(I.gaussian_field(n, box, rng, slope=-2.0), box)
    fov = math.radians(fov_deg)
    dirs = I.fov_directions((0.2, -0.15, 1.0), fov, fov * ny / nx, nx, ny)
    return phi, dirs


def test_PS1_cell_moments_gauss(oracle):
    """int chi Q and int chi^2 Q over a piece of a cell, for random vertex
    values and cell sizes, against 5-point Gauss quadrature of the trilinear
    field evaluated point by point (exact: degree <= 5)."""
    for _ in range(40):
        h = float(RNG.choice([1.0, 0.5, 0.125]))
        p1 = RNG.integers(-5, 5, size=3) * h
        Qv = RNG.normal(size=8)
        d = RNG.normal(size=3); d /= np.linalg.norm(d)
        # entry and exit points strictly inside the cell
        a = p1 + h * RNG.uniform(0.05, 0.95, size=3)
        chiA = float(RNG.uniform(5.0, 60.0))
        L = h * float(RNG.uniform(0.01, 0.3))
        o = a - chiA * d
        chiB = chiA - L
        got = oracle.cell_moments(Qv, p1, h, d, o, chiA, chiB)
        chi = 0.5 * (chiA + chiB) + 0.5 * L * GL5_X
        u = (o[None, :] + chi[:, None] * d[None, :] - p1[None, :]) / h
        q = _trilinear(Qv, u)
        ea = 0.5 * L * np.sum(GL5_W * chi * q)
        eb = 0.5 * L * np.sum(GL5_W * chi * chi * q)
        assert got[0] == pytest.approx(ea, rel=1e-11, abs=1e-13 * abs(chiA * L))
        assert got[1] == pytest.approx(eb, rel=1e-11, abs=1e-13 * abs(chiA * chiA * L))


@pytest.mark.parametrize("seed,quantity", [(0, 0), (1, 0), (2, 1), (3, 2)])
def test_PS2_every_source_equals_its_own_trace(oracle, seed, quantity):
    """One walk from the farthest source gives, for every source, the kappa
    (or shear) of a separate trace with that chi_s (Eq. Isources)."""
    n, box = 20, 40.0
    phi, dirs = _periodic_case(seed, n, box)
    tv = oracle.vertex_tensor(phi)
    o = np.array([3.3, 17.1, 2.2])
    src = np.array([93.7, 71.05, 52.3, 30.9, 12.4, 3.1])
    r = oracle.trace_uniform_sources(n, box, o, dirs, src[0], 0.0, src, tv=tv,
                                     quantity=quantity, kappa_scale=1.7)
    assert np.all(r.status == oracle.RAY_OK)
    kap = oracle.kappa_from_pieces(src, box, n, r.moments, r.pieces)
    for j, cs in enumerate(src):
        ref = oracle.trace_uniform(n, box, o, dirs, cs, cs, 0.0, tv=tv, quantity=quantity,
                                   kappa_scale=1.7)
        scale = np.max(np.abs(ref.kappa))
        np.testing.assert_allclose(kap[:, j], ref.kappa, rtol=1e-10, atol=1e-12 * scale)
    # the walk cuts one cell per source (none of these distances is on a face)
    plain = oracle.trace_uniform(n, box, o, dirs, src[0], src[0], 0.0, tv=tv)
    assert np.array_equal(r.ncross, plain.ncross + len(src) - 1)


def test_PS3_constant_laplacian_closed_form(oracle):
    """Quadratic Phi (constant transverse Laplacian q per ray): each piece is
    q (chi_{j-1}^2 - chi_j^2) / 2 and q (chi_{j-1}^3 - chi_j^3) / 3, and kappa
    of source j is q chi_j^2 / 6."""
    n = 24
    idx = np.arange(n, dtype=np.float64) + 0.5
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    X = [x, y, z]
    M = RNG.normal(size=(3, 3)); M = M + M.T
    phi = sum(0.5 * M[a, b] * X[a] * X[b] for a in range(3) for b in range(3))
    o = np.array([11.5, 12.25, 3.0])
    d = RNG.normal(size=(12, 3)) * 0.08 + np.array([0.0, 0.0, 1.0])
    dirs = d / np.linalg.norm(d, axis=1)[:, None]
    src = np.array([17.5, 13.25, 9.0, 4.4, 1.3])
    hi = 18.0
    r = oracle.trace_uniform_sources(n, float(n), o, dirs, hi, 0.0, src, phi=phi,
                                     open_boundary=True)
    assert np.all(r.status == oracle.RAY_OK)
    qv = np.trace(M) - np.einsum("ri,ij,rj->r", dirs, M, dirs)
    prev = hi
    for j, cs in enumerate(src):
        np.testing.assert_allclose(r.pieces[:, j, 0], qv * (prev ** 2 - cs ** 2) / 2, rtol=1e-11)
        np.testing.assert_allclose(r.pieces[:, j, 1], qv * (prev ** 3 - cs ** 3) / 3, rtol=1e-11)
        prev = cs
    np.testing.assert_allclose(r.moments[:, 0], qv * prev ** 2 / 2, rtol=1e-11)
    np.testing.assert_allclose(r.moments[:, 1], qv * prev ** 3 / 3, rtol=1e-11)
    kap = oracle.kappa_from_pieces(src, float(n), n, r.moments, r.pieces)
    np.testing.assert_allclose(kap, qv[:, None] * src[None, :] ** 2 / 6, rtol=1e-10)


def test_PS4_windows_carry_the_state(oracle):
    """Tracing in several chi windows (one per N-body step), with the moments
    and pieces carried from window to window, gives the one-window result;
    a source on a window boundary is taken once, at the end of the window
    above it."""
    n, box = 20, 40.0
    phi, dirs = _periodic_case(7, n, box)
    tv = oracle.vertex_tensor(phi)
    o = np.array([1.0, 2.0, 3.0])
    src = np.array([80.0, 61.5, 40.0, 22.2, 9.0])
    one = oracle.trace_uniform_sources(n, box, o, dirs, 80.0, 0.0, src, tv=tv)
    cuts = [80.0, 61.5, 48.3, 40.0, 31.7, 5.0, 0.0]
    mom, pcs = None, None
    for hi, lo in zip(cuts[:-1], cuts[1:]):
        rr = oracle.trace_uniform_sources(n, box, o, dirs, hi, lo, src, tv=tv, moments=mom,
                                          pieces=pcs)
        mom, pcs = rr.moments, rr.pieces
    sa = np.max(np.abs(one.pieces[..., 0])); sb = np.max(np.abs(one.pieces[..., 1]))
    np.testing.assert_allclose(pcs[..., 0], one.pieces[..., 0], rtol=1e-11, atol=1e-13 * sa)
    np.testing.assert_allclose(pcs[..., 1], one.pieces[..., 1], rtol=1e-11, atol=1e-13 * sb)
    k1 = oracle.kappa_from_pieces(src, box, n, one.moments, one.pieces)
    k2 = oracle.kappa_from_pieces(src, box, n, mom, pcs)
    np.testing.assert_allclose(k2, k1, rtol=1e-10, atol=1e-12 * np.max(np.abs(k1)))


def test_PS5_sources_on_faces_and_window_ends(oracle):
    """Rays along +z from an observer on a lattice plane cross faces at
    integer chi: a source there cuts nothing; a source at chi_hi is not a stop
    of this window (its piece stays as given); one at chi_lo is."""
    n = 16
    phi, _ = _periodic_case(3, n, float(n))
    tv = oracle.vertex_tensor(phi)
    o = np.array([3.25, 5.5, 2.0])
    dirs = np.array([[0.0, 0.0, 1.0]])
    src = np.array([12.0, 9.0, 6.5, 4.0])
    sentinel = np.full((1, 4, 2), 7.0)
    r = oracle.trace_uniform_sources(n, float(n), o, dirs, 12.0, 4.0, src, tv=tv,
                                     pieces=sentinel)
    plain = oracle.trace_uniform(n, float(n), o, dirs, 12.0, 12.0, 4.0, tv=tv)
    assert r.ncross[0] == plain.ncross[0] + 1          # only 6.5 cuts a cell
    assert np.all(r.pieces[0, 0] == 7.0)               # chi_hi: not a stop here
    assert np.all(r.pieces[0, 1:] != 7.0)
    assert np.all(r.moments == 0.0)                    # 4.0 = chi_lo was the last stop
    # kappa of the 9.0 source from the pieces below it equals its own trace
    r2 = oracle.trace_uniform_sources(n, float(n), o, dirs, 4.0, 0.0, src, tv=tv,
                                      moments=r.moments, pieces=r.pieces)
    kap = oracle.kappa_from_pieces(src, float(n), n, r2.moments, r2.pieces)
    ref = oracle.trace_uniform(n, float(n), o, dirs, 9.0, 9.0, 0.0, tv=tv)
    assert kap[0, 1] == pytest.approx(ref.kappa[0], rel=1e-11, abs=1e-14)


@pytest.mark.parametrize("seed", [0, 1])
def test_PS6_octree_every_source_equals_its_own_trace(oracle, seed):
    """The same identity on a random multi-level octree (2:1 balanced)."""
    rng = np.random.default_rng(300 + seed)
    n, L = 16, 32.0
    t = I.random_octree(n, 3, 0.3, rng)
    ot = _otree(oracle, t)
    assert oracle.octree_check(ot) == 0
    phi = I.poisson_phi(I.gaussian_field(n, L, rng, slope=-2.0), L)
    cen = t.centres(L)
    # potential per cell: nearest base-cell value plus a smooth refined-scale term
    base = np.floor(cen / (L / n)).astype(np.int64) % n
    pc = phi[base[:, 2], base[:, 1], base[:, 0]] + 1e-4 * np.sin(cen @ np.array([0.7, -0.4, 0.9]))
    cv = oracle.corner_tensor_octree(ot, oracle.centre_tensor_octree(ot, pc))
    fov = math.radians(10.0)
    dirs = I.fov_directions((0.1, 0.2, 1.0), fov, fov, 6, 5)
    o = np.array([2.0, 7.5, 1.25])
    src = np.array([70.3, 44.4, 21.9, 6.05])
    r = oracle.trace_octree_sources(ot, L, o, dirs, src[0], 0.0, src, cv=cv)
    assert np.all(r.status == oracle.RAY_OK)
    kap = oracle.kappa_from_pieces(src, L, n, r.moments, r.pieces)
    for j, cs in enumerate(src):
        ref = oracle.trace_octree(ot, L, o, dirs, cs, cs, 0.0, cv=cv)
        np.testing.assert_allclose(kap[:, j], ref.kappa, rtol=1e-10,
                                   atol=1e-12 * np.max(np.abs(ref.kappa)))
    plain = oracle.trace_octree(ot, L, o, dirs, src[0], src[0], 0.0, cv=cv)
    assert np.array_equal(r.ncross, plain.ncross + len(src) - 1)
