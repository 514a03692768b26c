"""Pins of the Method A oracle (Eq. kappa2): the Poisson term delta_coeff g
delta, the gradient term (n . grad Phi) dg/dchi, and the per-step surface
term -[g n . grad Phi] (Eqs. 2nterm, 2dterm2), each checked against what the
mathematics fixes: integration by parts against Method B on a quadratic
potential, Gauss quadrature of the gradient kernel per cell, telescoping of
the surface terms, and second-order convergence of A - B for a sinusoid."""
import math

import numpy as np
import pytest

from tests._independent import GL5_W, GL5_X

RNG = np.random.default_rng(777)


def _grid_coords(n, h=1.0):
    idx = (np.arange(n, dtype=np.float64) + 0.5) * h
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    return x, y, z


def _dirs(k, spread):
    d = np.column_stack([RNG.uniform(-spread, spread, k), RNG.uniform(-spread, spread, k),
                         np.ones(k)])
    return d / np.linalg.norm(d, axis=1)[:, None]


def test_PA1_quadratic_potential_equals_method_b(oracle):
    """Phi = x^T M x / 2 with delta_coeff delta = tr M: central differences,
    vertex means and trilinear interpolation are exact for the linear gradient,
    and integrating the gradient term by parts leaves -n^T M n int g, so each
    step's Method A kappa (surface term included) is (tr M - n^T M n) int g --
    the Method B closed form -- on any chi window."""
    n = 24
    M = RNG.normal(size=(3, 3)); M = M + M.T
    x, y, z = _grid_coords(n)
    X = [x, y, z]
    phi = sum(0.5 * M[a, b] * X[a] * X[b] for a in range(3) for b in range(3))
    cd = 0.37
    delta = np.full((n, n, n), np.trace(M) / cd)
    o = np.array([12.1, 11.8, 3.2])
    dirs = _dirs(12, 0.25)
    chis = 30.0
    for hi, lo in [(17.5, 0.0), (11.0, 4.5), (17.5, 9.25)]:
        r = oracle.trace_uniform_method_a(n, float(n), o, dirs, chis, hi, lo, delta_coeff=cd,
                                          phi=phi, delta=delta, open_boundary=True)
        assert (r.status == 0).all()
        qv = np.trace(M) - np.einsum("ri,ij,rj->r", dirs, M, dirs)
        gint = (chis * (hi ** 2 - lo ** 2) / 2 - (hi ** 3 - lo ** 3) / 3) / chis
        np.testing.assert_allclose(r.kappa, qv * gint, rtol=0,
                                   atol=1e-11 * np.abs(qv * gint).max())
        # the walk is Method B's
        rb = oracle.trace_uniform(n, float(n), o, dirs, chis, hi, lo, phi=phi, open_boundary=True)
        assert np.array_equal(r.hash, rb.hash)


def test_PA2_gradient_kernel_cell_integral_equals_gauss(oracle):
    """The gradient term's cell integral (kernel 1 - 2 chi / chi_s against the
    cubic along the segment) equals 5-point Gauss quadrature (exact to degree 9)."""
    for _ in range(200):
        Q = RNG.normal(size=8)
        h = 2.0 ** -RNG.integers(0, 4)
        p1 = RNG.integers(-20, 20, size=3) * h
        d = RNG.normal(size=3); d /= np.linalg.norm(d)
        chis = RNG.uniform(30, 80)
        ua = RNG.uniform(0, 1, size=3)
        chiA = RNG.uniform(5, 25)
        o = p1 + ua * h - chiA * d
        tmax = min(((ua[a] if d[a] > 0 else 1 - ua[a]) * h / abs(d[a])) for a in range(3))
        chiB = chiA - RNG.uniform(0.05, 1.0) * tmax
        got = oracle.cell_integral_k(Q, p1, h, d, o, chis, chiA, chiB)
        mid, half = 0.5 * (chiA + chiB), 0.5 * (chiA - chiB)
        chi = mid + half * GL5_X
        u = (o[None] + chi[:, None] * d[None] - p1[None]) / h
        q = np.zeros_like(chi)
        for v in range(8):
            ix, iy, iz = v & 1, (v >> 1) & 1, (v >> 2) & 1
            q += Q[v] * (u[:, 0] if ix else 1 - u[:, 0]) * (u[:, 1] if iy else 1 - u[:, 1]) \
                * (u[:, 2] if iz else 1 - u[:, 2])
        ref = half * np.sum(GL5_W * (1.0 - 2.0 * chi / chis) * q)
        assert got == pytest.approx(ref, rel=1e-10, abs=1e-12 * np.abs(Q).max() * half)


def test_PA3_surface_terms_telescope(oracle):
    """A static field split into steps: the surface terms of the inner step
    boundaries cancel (the trilinear field is continuous), so the sum over
    steps is the one-step value; over [0, chi_s] the surface term vanishes
    (g = 0 at both ends), leaving the two integrals."""
    n = 16
    phi = RNG.normal(size=(n, n, n))
    delta = RNG.normal(size=(n, n, n))
    fv = oracle.method_a_vertex_fields(phi, delta)
    o = RNG.uniform(0, n, size=3)
    dirs = _dirs(9, 0.4)
    chis = 45.0
    cd = 0.8
    one = oracle.trace_uniform_method_a(n, float(n), o, dirs, chis, 37.0, 1.5, delta_coeff=cd,
                                        fv=fv)
    edges = np.linspace(37.0, 1.5, 11)
    tot = np.zeros(len(dirs))
    for a, b in zip(edges[:-1], edges[1:]):
        tot += oracle.trace_uniform_method_a(n, float(n), o, dirs, chis, a, b, delta_coeff=cd,
                                             fv=fv).kappa
    np.testing.assert_allclose(tot, one.kappa, rtol=0, atol=1e-11 * np.abs(one.kappa).max())
    # full window: no surface term -> equals the two integrals over [0, chi_s]
    full = oracle.trace_uniform_method_a(n, float(n), o, dirs, chis, chis, 0.0, delta_coeff=cd,
                                         fv=fv)
    halves = [oracle.trace_uniform_method_a(n, float(n), o, dirs, chis, a, b, delta_coeff=cd,
                                            fv=fv).kappa for a, b in [(chis, 20.0), (20.0, 0.0)]]
    np.testing.assert_allclose(halves[0] + halves[1], full.kappa, rtol=0,
                               atol=1e-11 * np.abs(full.kappa).max())


def test_PA4_method_a_converges_to_the_continuum(oracle):
    """Smooth periodic potential with delta_coeff delta = its exact Laplacian
    at the cell centres: Method A integrates the continuum kappa of Eq. kappa
    (Eq. kappa2 is Eq. kappa integrated by parts, the time-derivative term
    vanishing for a static field), at second order -- the error falls about 4x
    per halving of the cell size, and so does its distance to Method B.  The
    window is [0, chi_s], where the surface term vanishes: a surface term at an
    interior chi samples the field at one point, whose O(h^2) error changes
    sign with the point's place in its cell."""
    from scipy.integrate import quad
    L = 64.0
    A, p0 = 1.0, 0.3
    kk = 2 * np.pi * np.array([1.0, 1.0, 2.0]) / L
    o = np.array([10.3, 21.7, 5.1])
    d = np.array([0.2, -0.1, 1.0]); d /= np.linalg.norm(d)
    chis, hi, lo = 150.0, 150.0, 0.0
    kn = kk @ d
    qc = lambda c: -A * (kk @ kk - kn * kn) * np.sin(kk @ (o + c * d) + p0)
    ref = quad(lambda c: c * (chis - c) / chis * qc(c), lo, hi, limit=400, epsabs=0,
               epsrel=1e-13)[0]
    cd = 1.0
    errs, diffs = [], []
    for n in (64, 128, 256):
        h = L / n
        x, y, z = _grid_coords(n, h)
        phi = A * np.sin(kk[0] * x + kk[1] * y + kk[2] * z + p0)
        delta = -(kk @ kk) * phi / cd
        ra = oracle.trace_uniform_method_a(n, L, o, d[None], chis, hi, lo, delta_coeff=cd,
                                           phi=phi, delta=delta)
        rb = oracle.trace_uniform(n, L, o, d[None], chis, hi, lo, phi=phi)
        errs.append(abs(ra.kappa[0] - ref))
        diffs.append(abs(ra.kappa[0] - rb.kappa[0]))
    for e in (errs, diffs):
        ratios = [e[i] / e[i + 1] for i in range(2)]
        for rt in ratios:
            assert 3.0 < rt < 5.5, (errs, diffs)
