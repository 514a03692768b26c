"""P12: the oracle gradient dL/dPhi of L = sum(w * kappa).

kappa is linear in Phi (straight rays, Born approximation, Sec. IV A), so the
gradient is pinned by the dot-product identity <w, A phi> = <A^T w, phi> and
by central finite differences, which are exact up to rounding for any step."""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I


def _setup(seed=0, n=12, nr=6):
    rng = np.random.default_rng(seed)
    phi = rng.normal(size=(n, n, n))
    fov = math.radians(8.0)
    dirs = I.fov_directions((0.3, -0.2, 1.0), fov, fov, nr, nr)
    w = rng.normal(size=nr * nr)
    return rng, phi, dirs, w


def test_P12_dot_product_identity(oracle):
    rng, phi, dirs, w = _setup()
    n = phi.shape[0]
    o = np.array([1.3, 2.2, 0.4])
    chis, hi, lo = 40.0, 30.0, 2.0
    fwd = oracle.trace_uniform(n, float(n), o, dirs, chis, hi, lo, phi=phi, kappa_scale=0.7)
    g = oracle.trace_adjoint_uniform(n, float(n), o, dirs, chis, hi, lo, w, kappa_scale=0.7)
    lhs = float(w @ fwd.kappa)
    rhs = float(np.sum(g * phi))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_P12_finite_differences(oracle):
    rng, phi, dirs, w = _setup(seed=3)
    n = phi.shape[0]
    o = np.array([0.0, 0.0, 0.0])
    chis, hi, lo = 40.0, 33.0, 0.0
    g = oracle.trace_adjoint_uniform(n, float(n), o, dirs, chis, hi, lo, w)
    nz = np.argwhere(np.abs(g) > 1e-6 * np.abs(g).max())
    pick = nz[rng.choice(len(nz), size=12, replace=False)]
    for (k, j, i) in pick:
        vals = []
        for eps in (+0.37, -0.37):
            p = phi.copy()
            p[k, j, i] += eps
            vals.append(float(w @ oracle.trace_uniform(n, float(n), o, dirs, chis, hi, lo, phi=p).kappa))
        fd = (vals[0] - vals[1]) / 0.74
        assert fd == pytest.approx(g[k, j, i], rel=1e-8, abs=1e-10 * np.abs(g).max())
