"""Independent checkers used to pin the oracle (test-side code only).

Nothing here calls the oracle's walk or its per-cell integral: the brute-force
tracer finds every plane crossing by enumerating planes, locates cells by
``floor`` and integrates g(chi) * Q(p(chi)) with 5-point Gauss-Legendre on
each piece, where Q is the trilinear interpolant of tr T - n^T T n.
"""
import numpy as np

GL5_X, GL5_W = np.polynomial.legendre.leggauss(5)


def transverse_laplacian(T, d):
    """tr T - n^T T n for T rows (xx, yy, zz, xy, xz, yz)."""
    T = np.asarray(T)
    nx, ny, nz = d
    tr = T[..., 0] + T[..., 1] + T[..., 2]
    ntn = (nx * nx * T[..., 0] + ny * ny * T[..., 1] + nz * nz * T[..., 2]
           + 2 * nx * ny * T[..., 3] + 2 * nx * nz * T[..., 4] + 2 * ny * nz * T[..., 5])
    return tr - ntn


def crossings(o, d, lo, hi):
    """All plane parameters t in (lo, hi) with t = (m - o_a) * (1/n_a)."""
    ts = []
    for a in range(3):
        if d[a] == 0.0:
            continue
        r = 1.0 / d[a]
        p_lo, p_hi = sorted((o[a] + lo * d[a], o[a] + hi * d[a]))
        ms = np.arange(np.floor(p_lo) - 1, np.ceil(p_hi) + 2, dtype=np.float64)
        t = (ms - o[a]) * r
        ts.append(t[(t > lo) & (t < hi)])
    ts = np.concatenate(ts) if ts else np.zeros(0)
    return np.unique(ts)[::-1]


def cell_of_piece(o, d, b, a):
    """Lattice cell holding the piece chi in [b, a] (b < a): per axis the
    cell whose two planes' parameters t = (m - o) * (1/n) bracket the piece,
    found from floor of the midpoint and corrected by those parameters (a
    piece narrower than the rounding of the position stays on its side of a
    plane).  An axis the ray does not move along keeps floor(o)."""
    mid = 0.5 * (a + b)
    m = np.floor(np.asarray(o) + mid * np.asarray(d)).astype(np.int64)
    for ax in range(3):
        if d[ax] == 0.0:
            m[ax] = int(np.floor(o[ax]))
            continue
        r = 1.0 / d[ax]
        for _ in range(4):
            t0 = (float(m[ax]) - o[ax]) * r
            t1 = (float(m[ax] + 1) - o[ax]) * r
            lo_t, hi_t = min(t0, t1), max(t0, t1)
            if b < lo_t:      # the piece lies at smaller parameters
                m[ax] += -1 if d[ax] > 0 else 1
            elif a > hi_t:    # ... at larger parameters
                m[ax] += 1 if d[ax] > 0 else -1
            else:
                break
    return m


def brute_trace(n, tv, o, d, chis, hi, lo, log=False):
    """kappa (and optionally the (cell, chi_a, chi_b) list) of one ray."""
    tv = np.asarray(tv).reshape(n, n, n, 6)
    Qv = transverse_laplacian(tv, d)               # [z][y][x]
    pts = np.concatenate([[hi], crossings(o, d, lo, hi), [lo]])
    total = 0.0
    segs = []
    for a_, b_ in zip(pts[:-1], pts[1:]):
        mid = 0.5 * (a_ + b_)
        m = cell_of_piece(o, d, b_, a_)
        half = 0.5 * (a_ - b_)
        chi = mid + half * GL5_X
        p = np.asarray(o)[None, :] + chi[:, None] * np.asarray(d)[None, :]
        u = p - m[None, :]
        q = np.zeros_like(chi)
        for v in range(8):
            ix, iy, iz = v & 1, (v >> 1) & 1, (v >> 2) & 1
            w = ((u[:, 0] if ix else 1 - u[:, 0]) * (u[:, 1] if iy else 1 - u[:, 1])
                 * (u[:, 2] if iz else 1 - u[:, 2]))
            q += w * Qv[(m[2] + iz) % n, (m[1] + iy) % n, (m[0] + ix) % n]
        g = chi * (chis - chi) / chis
        total += half * np.sum(GL5_W * g * q)
        if log:
            cell = ((m[2] % n) * n + (m[1] % n)) * n + (m[0] % n)
            segs.append((int(cell), float(a_), float(b_)))
    return (total, segs) if log else total
