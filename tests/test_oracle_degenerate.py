"""Pins of the oracle's walk on the degenerate cases of the crossing rule
(Sec. III F, Eqs. disttocross, rayposition): rays along a lattice axis or in
a lattice plane (a direction component exactly zero: that axis is never
crossed), rays through lattice edges and vertices (two or three planes at the
same parameter: every tied axis steps at once), observers on lattice planes
and vertices, and windows that start exactly on a plane (the point belongs to
the cell the ray moves into).  Against the independent enumerate-all-planes
tracer: crossing lists bit for bit, kappa to rounding."""
import math

import numpy as np
import pytest

from tests._independent import brute_trace, transverse_laplacian

S2, S3 = math.sqrt(0.5), math.sqrt(1.0 / 3.0)
DEGENERATE_DIRS = np.array([
    [1.0, 0.0, 0.0], [-1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, -1.0, 0.0],
    [0.0, 0.0, 1.0], [0.0, 0.0, -1.0],
    [S2, S2, 0.0], [S2, 0.0, -S2], [0.0, -S2, S2], [-S2, S2, 0.0],
    [S3, S3, S3], [-S3, S3, S3], [S3, -S3, -S3],
])
OBSERVERS = [(0.0, 0.0, 0.0), (3.0, 3.0, 0.5), (2.25, 5.0, 1.75), (2.3, 4.1, 1.7)]


def degenerate_case(seed=21, n=8):
    rng = np.random.default_rng(seed)
    return n, rng.normal(size=(n, n, n))


@pytest.mark.parametrize("obs", OBSERVERS)
def test_PD1_degenerate_rays_match_bruteforce(oracle, obs):
    n, phi = degenerate_case()
    tv = oracle.vertex_tensor(phi)
    o = np.array(obs)
    chis, hi, lo = 40.0, 29.0, 0.7
    r = oracle.trace_uniform(n, float(n), o, DEGENERATE_DIRS, chis, hi, lo, tv=tv, log_stride=512)
    assert np.all(r.status == oracle.RAY_OK)
    for k, d in enumerate(DEGENERATE_DIRS):
        kap, segs = brute_trace(n, tv, o, d, chis, hi, lo, log=True)
        got = [(int(s["cell"]), float(s["chi_a"]), float(s["chi_b"]))
               for s in r.log[k][: r.ncross[k]]]
        assert got == segs, (obs, d)
        scale = np.abs(transverse_laplacian(tv, d)).max() * chis * hi
        assert abs(r.kappa[k] - kap) < 1e-12 * scale


def test_PD2_window_starting_on_a_plane(oracle):
    """chi_hi equal to a plane's crossing parameter: the walk starts in the
    cell beyond that plane (the one the ray moves into) and the first piece
    is a full cell, for axis-aligned and diagonal rays alike."""
    n, phi = degenerate_case(seed=22)
    tv = oracle.vertex_tensor(phi)
    o = np.array([2.3, 4.1, 1.7])
    chis, lo = 40.0, 0.5
    for d in DEGENERATE_DIRS[[4, 5, 10]]:
        a = int(np.argmax(np.abs(d)))
        plane = np.floor(o[a] + 20.0 * d[a])
        hi = float((plane - o[a]) * (1.0 / d[a]))     # the crossing parameter of that plane
        r = oracle.trace_uniform(n, float(n), o, d[None, :], chis, hi, lo, tv=tv, log_stride=512)
        kap, segs = brute_trace(n, tv, o, d, chis, hi, lo, log=True)
        got = [(int(s["cell"]), float(s["chi_a"]), float(s["chi_b"]))
               for s in r.log[0][: r.ncross[0]]]
        assert got == segs
        # the first piece is in the cell below the plane along the motion
        # (chi decreasing: x_a decreases where n_a > 0)
        want = int(plane) - 1 if d[a] > 0 else int(plane)
        cell = got[0][0]
        assert (cell // n ** a) % n == want % n
        assert got[0][1] == hi and got[0][2] < hi
