"""Pins of the oracle's ISW integrand (Sec. VII, Eq. I1 with Q = dPhi/dt).

Q per cell is (Phi_curr - Phi_prev) / dt, averaged to vertices and trilinear
in each cell; each ray adds scale * int Q dchi (box units).  Pinned against:
Gauss quadrature per cell, the closed form of a linear Q (the vertex mean and
the trilinear reconstruction are exact for it), a lattice sinusoid's vertex
values, and an independent brute-force walk.
"""
import numpy as np
import pytest

from tests._independent import GL5_W, GL5_X, crossings

RNG = np.random.default_rng(20261204)


def _trilinear(Qv, u):
    q = np.zeros(u.shape[0])
    for v in range(8):
        ix, iy, iz = v & 1, (v >> 1) & 1, (v >> 2) & 1
        w = ((u[:, 0] if ix else 1 - u[:, 0]) * (u[:, 1] if iy else 1 - u[:, 1])
             * (u[:, 2] if iz else 1 - u[:, 2]))
        q += w * Qv[v]
    return q


def test_PI1_cell_integral_gauss(oracle):
    for _ in range(60):
        h = float(RNG.choice([1.0, 0.25]))
        p1 = RNG.integers(-4, 4, size=3) * h
        Qv = RNG.normal(size=8)
        d = RNG.normal(size=3); d /= np.linalg.norm(d)
        a = p1 + h * RNG.uniform(0.05, 0.95, size=3)
        chiA = float(RNG.uniform(2.0, 40.0))
        L = h * float(RNG.uniform(0.01, 0.3))
        o = a - chiA * d
        got = oracle.cell_integral_one(Qv, p1, h, d, o, chiA, chiA - L)
        chi = chiA - 0.5 * L + 0.5 * L * GL5_X
        u = (o[None, :] + chi[:, None] * d[None, :] - p1[None, :]) / h
        ref = 0.5 * L * np.sum(GL5_W * _trilinear(Qv, u))
        assert got == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_PI2_linear_rate_closed_form(oracle):
    """(Phi_curr - Phi_prev) linear in position (open grid, box != n so the
    cell size enters): I = scale inv_dt int (a0 + g . (o + chi n)) dchi."""
    n, box = 24, 60.0
    h = box / n
    idx = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    a0, g = 0.37, RNG.normal(size=3) * 0.05
    prev = RNG.normal(size=(n, n, n))
    cur = prev + a0 + g[0] * x + g[1] * y + g[2] * z
    inv_dt, scale = 2.5, 0.8
    o = np.array([30.3, 29.1, 8.2])
    d = RNG.normal(size=(10, 3)) * 0.1 + np.array([0.0, 0.0, 1.0])
    dirs = d / np.linalg.norm(d, axis=1)[:, None]
    hi, lo = 38.0, 1.5
    r = oracle.trace_uniform_isw(n, box, o, dirs, hi, lo, phi_curr=cur, phi_prev=prev,
                                 inv_dt=inv_dt, open_boundary=True, scale=scale)
    assert np.all(r.status == oracle.RAY_OK)
    ref = scale * inv_dt * ((a0 + g @ o) * (hi - lo) + (dirs @ g) * (hi ** 2 - lo ** 2) / 2)
    np.testing.assert_allclose(r.kappa, ref, rtol=1e-11)


def test_PI3_sinusoid_vertex_values(oracle):
    """Lattice sinusoid: the mean of the eight cells around vertex v is
    A prod_a cos(k_a / 2) sin(k . v + p) (cell centres at v +- 1/2)."""
    n = 16
    kk = 2 * np.pi * np.array([1, -2, 3]) / n
    A, p = 1.3, 0.2
    c = np.arange(n) + 0.5
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    cur = A * np.sin(kk[0] * x + kk[1] * y + kk[2] * z + p)
    prev = np.zeros_like(cur)
    qv = oracle.isw_vertex_field(cur, prev, 3.0).reshape(n, n, n)
    v = np.arange(n, dtype=np.float64)
    z, y, x = np.meshgrid(v, v, v, indexing="ij")
    ref = 3.0 * A * np.prod(np.cos(kk / 2)) * np.sin(kk[0] * x + kk[1] * y + kk[2] * z + p)
    np.testing.assert_allclose(qv, ref, atol=1e-13)


def _brute(n, qv, o, d, hi, lo, h0):
    """Independent walk: every plane crossing by enumeration, the cell by
    floor, 5-point Gauss per piece of the trilinear vertex field."""
    qv = qv.reshape(n, n, n)
    pts = np.concatenate([[hi], crossings(o, d, lo, hi), [lo]])
    total = 0.0
    for a_, b_ in zip(pts[:-1], pts[1:]):
        mid = 0.5 * (a_ + b_)
        m = np.floor(o + mid * d).astype(np.int64)
        chi = mid + 0.5 * (a_ - b_) * GL5_X
        u = o[None, :] + chi[:, None] * d[None, :] - m[None, :]
        corner = [qv[(m[2] + ((v >> 2) & 1)) % n, (m[1] + ((v >> 1) & 1)) % n, (m[0] + (v & 1)) % n]
                  for v in range(8)]
        total += 0.5 * (a_ - b_) * np.sum(GL5_W * _trilinear(corner, u))
    return total * h0, len(pts) - 1


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_PI4_bruteforce_walk(oracle, seed):
    rng = np.random.default_rng(400 + seed)
    n, box = 12, 30.0
    h0 = box / n
    cur, prev = rng.normal(size=(2, n, n, n))
    qv = oracle.isw_vertex_field(cur, prev, 0.7)
    o = rng.uniform(0, box, size=3)
    d = rng.normal(size=(6, 3)); d /= np.linalg.norm(d, axis=1)[:, None]
    hi, lo = 47.0, 3.0
    r = oracle.trace_uniform_isw(n, box, o, d, hi, lo, qv=qv)
    for k in range(len(d)):
        ref, npieces = _brute(n, qv, o / h0, d[k], hi / h0, lo / h0, h0)
        assert r.ncross[k] == npieces
        assert r.kappa[k] == pytest.approx(ref, rel=1e-11, abs=1e-12)
