"""Pin of the oracle's octree walk (Sec. III F on the levels of Sec. III A)
against a point-location walker written independently of it: at the start of
every piece the walker finds the leaf holding the ray by descending from the
base cell, applying the slab rule on every level (a point on a plane belongs
to the cell the ray moves into; an axis the ray does not move along keeps the
floor of its coordinate), and ends the piece at that leaf's first exit plane
or at chi_lo.  There is no neighbour stepping and no ascend / descend
bookkeeping, so a slip in the walk's level changes, ties or periodic wrap
shows up as a different crossing list, compared bit for bit."""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I
from tests.test_oracle_degenerate import DEGENERATE_DIRS


def _tplane(P, o, r):
    return (P - o) * r


def _slab0(o, d, r, chi):
    """Level-0 slab of one axis holding the ray at chi (slab rule)."""
    if d == 0.0:
        return int(math.floor(o))
    m = int(math.floor(o + chi * d))
    for _ in range(8):
        t_lo, t_hi = _tplane(float(m), o, r), _tplane(float(m + 1), o, r)
        t_exit, t_entry = (t_lo, t_hi) if d > 0 else (t_hi, t_lo)
        if not (t_exit < chi):
            m += -1 if d > 0 else 1
        elif not (chi <= t_entry):
            m += 1 if d > 0 else -1
        else:
            break
    return m


def point_location_walk(tr, o, d, hi, lo):
    n = tr.n
    nb = n ** 3
    r = [1.0 / d[a] if d[a] != 0.0 else 0.0 for a in range(3)]
    pieces = []
    chi = hi
    while True:
        m = [_slab0(o[a], d[a], r[a], chi) for a in range(3)]
        w = [mm % n for mm in m]
        cell = (w[2] * n + w[1]) * n + w[0]
        l = 0
        while tr.child_oct[cell] >= 0:
            k = int(tr.child_oct[cell])
            ch = 0
            for a in range(3):
                mid = 2 * m[a] + 1
                if d[a] == 0.0:
                    bit = int(math.ldexp(o[a], l + 1) >= mid)
                else:
                    t = _tplane(mid * math.ldexp(1.0, -(l + 1)), o[a], r[a])
                    bit = int(chi > t) if d[a] > 0 else int(chi <= t)
                m[a] = 2 * m[a] + bit
                ch |= bit << a
            cell = nb + 8 * k + ch
            l += 1
        chi_b = lo
        for a in range(3):
            if d[a] != 0.0:
                plane = m[a] if d[a] > 0 else m[a] + 1
                chi_b = max(chi_b, _tplane(plane * math.ldexp(1.0, -l), o[a], r[a]))
        pieces.append((cell, chi, chi_b))
        if chi_b == lo:
            return pieces
        chi = chi_b


def _otree(oracle, t):
    return oracle.Octree(t.n, t.child_oct, t.oct_parent, t.oct_level, t.oct_coord, t.max_level)


@pytest.mark.parametrize("seed,p", [(0, 0.08), (1, 0.15), (2, 0.25), (3, 0.15), (4, 0.35)])
def test_PO1_octree_walk_equals_point_location(oracle, seed, p):
    """Random trees with every level mix (mostly level-0 leaves to mostly
    level 1-4), degenerate and random rays, observers on 1/8-cell points."""
    rng = np.random.default_rng(600 + seed)
    tr = I.random_octree(8, 2 + seed % 3, p, rng, region=(0.0, 8.0))
    ot = _otree(oracle, tr)
    tc = oracle.centre_tensor_octree(ot, np.zeros(tr.n_cells))
    rnd = rng.normal(size=(8, 3))
    rnd /= np.linalg.norm(rnd, axis=1)[:, None]
    dirs = np.concatenate([DEGENERATE_DIRS, rnd])
    for _ in range(3):
        obs = rng.integers(0, 64, size=3) * 0.125
        hi = float(rng.integers(8, 20)) + 0.25 * float(rng.integers(0, 4))
        lo = 0.5 * float(rng.integers(0, 3))
        res = oracle.trace_octree(ot, 8.0, obs, dirs, 40.0, hi, lo, tc=tc, log_stride=4096)
        assert np.all(res.status == oracle.RAY_OK)
        for k, d in enumerate(dirs):
            got = [(int(s["cell"]), float(s["chi_a"]), float(s["chi_b"]))
                   for s in res.log[k][: res.ncross[k]]]
            assert got == point_location_walk(tr, obs, d, hi, lo), (seed, obs.tolist(), k)
