"""Seeded synthetic inputs for the Method-B convergence path.

This module produces *inputs only*: cosmological distances, ray directions,
potential fields and AMR octrees.  It holds none of the ray-tracing
arithmetic (no tidal tensor, no vertex interpolation, no cell walk, no
per-cell integral), so both the HIP path and the FP64 oracle can consume its
arrays without sharing any of the method's code.

Paper references (RAY-RAMSES, arXiv:1601.02012):
  * ray angular grid: Sec. III E, Eq. (txty); ray ids: Eq. (rayid);
  * comoving distance chi(z) = c int dz/H(z): Sec. III B, below Eq. (raypos);
  * cosmology of the lensing runs (Omega_b, Omega_c, h): Sec. VI A;
  * Gaussian test potential: Sec. V, Eq. (gaussian);
  * Poisson relation used for delta -> Phi: Sec. IV D, Eq. (kappa2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------- cosmology --
C_OVER_H0 = 2997.92458          # c/H0 in Mpc/h
OMEGA_M = 0.049 + 0.267         # Sec. VI A: Omega_b0 + Omega_c0
OMEGA_L = 1.0 - OMEGA_M


def _E(z):
    return math.sqrt(OMEGA_M * (1.0 + z) ** 3 + OMEGA_L)


def _gl_nodes(n=64):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def _integrate(f, a, b, pieces=64, order=32):
    """Composite Gauss-Legendre quadrature in FP64 (smooth integrands)."""
    x, w = _gl_nodes(order)
    edges = np.linspace(a, b, pieces + 1)
    tot = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
        tot += half * sum(wi * f(mid + half * xi) for xi, wi in zip(x, w))
    return tot


def chi_of_z(z: float) -> float:
    """Comoving distance in Mpc/h for flat LCDM with Omega_m = 0.316."""
    if z <= 0.0:
        return 0.0
    return C_OVER_H0 * _integrate(lambda t: 1.0 / _E(t), 0.0, float(z), pieces=16, order=24)


def z_of_chi(chi: float) -> float:
    """Inverse of chi_of_z by bisection (FP64)."""
    lo, hi = 0.0, 20.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if chi_of_z(mid) < chi:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-15:
            break
    return 0.5 * (lo + hi)


def growth_D(a: float) -> float:
    """Linear growth D+(a) of flat LCDM (unnormalised integral form)."""
    if a <= 0.0:
        return 0.0
    H = lambda aa: math.sqrt(OMEGA_M / aa ** 3 + OMEGA_L)
    integral = _integrate(lambda aa: 1.0 / (aa * H(aa)) ** 3, 1e-8, a, pieces=32, order=24)
    return 2.5 * OMEGA_M * H(a) * integral


# --------------------------------------------------------------- directions --
def fov_angles(fov: float, n: int) -> np.ndarray:
    """Eq. (txty): theta_i = fov/(n-1) * (i-1) - fov/2, i = 1..n (radians).

    A single ray (n == 1) sits on the bundle axis."""
    if n == 1:
        return np.zeros(1)
    i = np.arange(1, n + 1, dtype=np.float64)
    return fov / (n - 1) * (i - 1.0) - fov / 2.0


def _basis(center):
    """Frame (e1, e2, e3) of a map centred on ``center`` (gnomonic reading of
    Eq. txty): e3 the unit centre, e1 = normalise(h x e3) with h = z^ unless
    e3 is within ~26 deg of the z axis (then h = x^), e2 = e3 x e1; on the z
    axis itself e1 = x^ and e2 = +-y^.  Plain float arithmetic in a fixed
    order (no dot-product library call), one rounding per operation."""
    c0, c1, c2 = (float(v) for v in center)
    r = math.sqrt((c0 * c0 + c1 * c1) + c2 * c2)
    e3 = (c0 / r, c1 / r, c2 / r)
    if e3[0] == 0.0 and e3[1] == 0.0:
        return (1.0, 0.0, 0.0), (0.0, -1.0 if e3[2] < 0.0 else 1.0, 0.0), e3
    h = (0.0, 0.0, 1.0) if abs(e3[2]) < 0.9 else (1.0, 0.0, 0.0)
    u = (h[1] * e3[2] - h[2] * e3[1], h[2] * e3[0] - h[0] * e3[2], h[0] * e3[1] - h[1] * e3[0])
    ru = math.sqrt((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2])
    e1 = (u[0] / ru, u[1] / ru, u[2] / ru)
    e2 = (e3[1] * e1[2] - e3[2] * e1[1], e3[2] * e1[0] - e3[0] * e1[2],
          e3[0] * e1[1] - e3[1] * e1[0])
    return e1, e2, e3


def fov_directions(center, fov_x: float, fov_y: float, nx: int, ny: int) -> np.ndarray:
    """Unit ray directions (observer -> source), shape (ny*nx, 3), FP64.

    Flat-sky gnomonic mapping of the Eq. (txty) angles about ``center``;
    row-major by ray id, ray id = iy*nx + ix (0-based Eq. (rayid)):
    d = (tan(theta_x) e1 + tan(theta_y) e2) + e3, n = d / sqrt((d_x^2 + d_y^2)
    + d_z^2), every operation rounded on its own, tan from the C library."""
    tx = np.array([math.tan(a) for a in fov_angles(fov_x, nx)])
    ty = np.array([math.tan(a) for a in fov_angles(fov_y, ny)])
    e1, e2, e3 = (np.array(v) for v in _basis(center))
    d = (tx[None, :, None] * e1[None, None, :] + ty[:, None, None] * e2[None, None, :]
         + e3[None, None, :])
    d = d.reshape(-1, 3)
    norm = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
    return np.ascontiguousarray(d / norm[:, None])


def rayid(ix, iy, nx):
    """0-based Eq. (rayid)."""
    return iy * nx + ix


def rayid_inverse(rid, nx):
    return rid % nx, rid // nx


# ------------------------------------------------------------------- fields --
def _kgrid(n: int, box: float):
    k1 = 2.0 * np.pi * np.fft.fftfreq(n, d=box / n)
    kz = 2.0 * np.pi * np.fft.rfftfreq(n, d=box / n)
    return k1, kz


def _k2(n, box):
    k1, kz = _kgrid(n, box)
    return (k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + kz[None, None, :] ** 2)


def gaussian_field(n: int, box: float, rng: np.random.Generator, slope: float = -2.0,
                   workers: int = -1) -> np.ndarray:
    """Zero-mean, unit-variance Gaussian field with P(k) ~ k^slope, [z][y][x]."""
    import scipy.fft as sfft
    w = rng.standard_normal((n, n, n))
    wk = sfft.rfftn(w, workers=workers)
    del w
    k2 = _k2(n, box)
    k2[0, 0, 0] = 1.0
    wk *= k2 ** (slope / 4.0)
    wk[0, 0, 0] = 0.0
    del k2
    g = sfft.irfftn(wk, s=(n, n, n), workers=workers)
    g -= g.mean()
    g /= g.std()
    return g


def lognormal_delta(n: int, box: float, rng: np.random.Generator, slope: float = -2.0,
                    sigma_g: float = 1.0) -> np.ndarray:
    g = gaussian_field(n, box, rng, slope) * sigma_g
    return np.exp(g - 0.5 * sigma_g ** 2) - 1.0


def poisson_phi(delta: np.ndarray, box: float, a: float = 1.0, workers: int = -1) -> np.ndarray:
    """Phi/c^2 from delta with the comoving Poisson relation (continuum k^2).

    nabla^2 (Phi/c^2) = (3/2) Omega_m (H0/c)^2 delta / a, as used in Eq. (kappa2)."""
    import scipy.fft as sfft
    n = delta.shape[0]
    dk = sfft.rfftn(delta, workers=workers)
    k2 = _k2(n, box)
    k2[0, 0, 0] = 1.0
    dk *= -1.5 * OMEGA_M / (C_OVER_H0 ** 2 * a) / k2
    dk[0, 0, 0] = 0.0
    return sfft.irfftn(dk, s=delta.shape, workers=workers)


def gaussian_potential(n: int, box: float, amp: float, sigma: float, center=None,
                       pad: int = 0) -> np.ndarray:
    """Eq. (gaussian) sampled at cell centres of an n^3 grid of side ``box``.

    With ``pad`` > 0 the grid is extended by ``pad`` ghost cells per side
    (same cell size); returns shape (n+2pad)^3 in [z][y][x] order."""
    h = box / n
    if center is None:
        center = (0.5 * box,) * 3
    idx = (np.arange(-pad, n + pad, dtype=np.float64) + 0.5) * h
    z = idx[:, None, None] - center[2]
    y = idx[None, :, None] - center[1]
    x = idx[None, None, :] - center[0]
    r2 = x * x + y * y + z * z
    return amp * np.exp(-r2 / (2.0 * sigma * sigma))


# ------------------------------------------------------------ configurations --
@dataclass
class Bundle:
    dirs: np.ndarray            # (n_rays, 3) FP64 unit vectors
    nx: int
    ny: int
    chi_s: float
    chi_hi: float
    chi_lo: float
    center: tuple = (0.0, 0.0, 1.0)
    fov_x: float = 0.0
    fov_y: float = 0.0


@dataclass
class UniformCase:
    name: str
    n: int
    box: float
    phi: np.ndarray             # [z][y][x]
    observer: tuple
    bundles: list
    segments: list = field(default_factory=list)   # list of (chi_hi, chi_lo, scale)
    open_boundary: bool = False


def seeds(config: int, n_streams: int = 4):
    ss = np.random.SeedSequence(1000 + config)
    return [np.random.default_rng(s) for s in ss.spawn(n_streams)]


def config1(n: int = 64, box: float = 256.0, nray: int = 128) -> UniformCase:
    """Plain FP64 case: 64^3 Gaussian delta with P ~ k^-2, box 256 Mpc/h,
    observer at the box corner, 128^2 rays over 2x2 deg, chi_s = 256 Mpc/h."""
    rf, *_ = seeds(1)
    delta = gaussian_field(n, box, rf, slope=-2.0)
    phi = poisson_phi(delta, box)
    fov = math.radians(2.0)
    d = fov_directions((0.0, 0.0, 1.0), fov, fov, nray, nray)
    b = Bundle(d, nray, nray, 256.0, 256.0, 0.0, (0.0, 0.0, 1.0), fov, fov)
    return UniformCase("c1", n, box, phi, (0.0, 0.0, 0.0), [b])


def lightcone_segments(n_seg: int = 20, a_src: float = 0.5):
    """Equal steps in the scale factor from a_src to 1: (chi_hi, chi_lo, s_k).

    s_k = [D(a)/a]/[D(1)/1] at the segment mid-point scales the potential of
    synthetic N-body step k (the potential is static within a step)."""
    a = np.linspace(a_src, 1.0, n_seg + 1)
    chis = [chi_of_z(1.0 / ai - 1.0) for ai in a]
    d1 = growth_D(1.0)
    out = []
    for k in range(n_seg):
        am = 0.5 * (a[k] + a[k + 1])
        out.append((chis[k], chis[k + 1], (growth_D(am) / am) / d1))
    return out


def cosmic_time(a: float) -> float:
    """Cosmic time at scale factor a in units of 1/H0 (flat LCDM)."""
    H = lambda aa: math.sqrt(OMEGA_M / aa ** 3 + OMEGA_L)
    return _integrate(lambda aa: 1.0 / (aa * H(aa)), 1e-8, a, pieces=32, order=24)


def isw_steps(n_seg: int = 20, a_src: float = 0.5):
    """Per light-cone segment of lightcone_segments: (s_prev, s_curr, inv_dt,
    scale) for the ISW integrand.  The potential of step k is s_k Phi0 at the
    segment's mid-point a_k; the previous step's sits one step earlier (for
    the first segment, at a_0 - da); inv_dt = 1 / (t(a_k) - t(a_k-1)) in H0
    units and scale = 2 a_k / (c/H0) per Mpc/h, so that
    scale * int (dPhi/dt) dchi = (2/c) int a dPhi/dt dchi, the ISW
    temperature shift of Phi/c^2 (dimensionless)."""
    a = np.linspace(a_src, 1.0, n_seg + 1)
    mids = 0.5 * (a[:-1] + a[1:])
    da = mids[1] - mids[0] if n_seg > 1 else 1.0 - a_src
    d1 = growth_D(1.0)
    s = lambda aa: (growth_D(aa) / aa) / d1
    out = []
    for k, am in enumerate(mids):
        ap = mids[k - 1] if k > 0 else am - da
        out.append((s(ap), s(am), 1.0 / (cosmic_time(am) - cosmic_time(ap)),
                    2.0 * am / C_OVER_H0))
    return out


def config2_phi0(n: int = 512, box: float = 1000.0) -> np.ndarray:
    return config2_fields(n, box)[1]


def config2_fields(n: int = 512, box: float = 1000.0):
    """(delta0, phi0) of the light cone: the lognormal density contrast (mean
    removed, the k = 0 mode the Poisson solve drops) and its Phi/c^2 at a = 1."""
    rf, *_ = seeds(2)
    delta = lognormal_delta(n, box, rf, slope=-2.0, sigma_g=1.0)
    phi = poisson_phi(delta, box)
    return delta - delta.mean(), phi


def poisson_coefficient(a: float = 1.0) -> float:
    """(3/2) Omega_m (H0/c)^2 / a in (Mpc/h)^-2: nabla^2 (Phi/c^2) = this x delta."""
    return 1.5 * OMEGA_M / (C_OVER_H0 ** 2 * a)


def config2(n: int = 512, box: float = 1000.0, nray: int = 2048, fov_deg: float = 5.0,
            n_seg: int = 20) -> UniformCase:
    """Light cone to z = 1 through a replicated 512^3 box of 1 Gpc/h,
    2048^2 rays over 5x5 deg, 20 chi-segments (one per synthetic step)."""
    phi0 = config2_phi0(n, box)
    chi_s = chi_of_z(1.0)
    fov = math.radians(fov_deg)
    d = fov_directions((0.0, 0.0, 1.0), fov, fov, nray, nray)
    b = Bundle(d, nray, nray, chi_s, chi_s, 0.0, (0.0, 0.0, 1.0), fov, fov)
    segs = lightcone_segments(n_seg)
    return UniformCase("c2", n, box, phi0, (0.0, 0.0, 0.0), [b], segs)


def config5(n: int = 256, box: float = 256.0, nray: int = 1024, fov_deg: float = 5.0):
    """Adjoint case: 256^3 FP32 Gaussian potential, 1024^2 rays over 5x5 deg,
    chi_s = 256, plus seeded loss weights w ~ N(0,1)."""
    rf, rw, *_ = seeds(5)
    delta = gaussian_field(n, box, rf, slope=-2.0)
    phi = poisson_phi(delta, box).astype(np.float32)
    fov = math.radians(fov_deg)
    d = fov_directions((0.0, 0.0, 1.0), fov, fov, nray, nray)
    b = Bundle(d, nray, nray, 256.0, 256.0, 0.0, (0.0, 0.0, 1.0), fov, fov)
    w = rw.standard_normal(nray * nray)
    return UniformCase("c5", n, box, phi, (0.0, 0.0, 0.0), [b]), w


# ------------------------------------------------------------------- octrees --
@dataclass
class OctreeInput:
    """Octree in the library layout: base cells 0..n^3-1 ([z][y][x]); oct k owns
    cells n^3 + 8k + (ix + 2iy + 4iz); octs in breadth-first order."""
    n: int
    max_level: int
    child_oct: np.ndarray       # int32 [n_cells]
    oct_parent: np.ndarray      # int64 [n_octs]
    oct_level: np.ndarray       # int32 [n_octs]
    oct_coord: np.ndarray       # int32 [n_octs, 3] level coords of child 0
    cell_level: np.ndarray      # int32 [n_cells]
    cell_coord: np.ndarray      # int64 [n_cells, 3] level coords

    @property
    def n_cells(self):
        return self.child_oct.shape[0]

    @property
    def n_octs(self):
        return self.oct_level.shape[0]

    def centres(self, box):
        """Cell-centre positions in box units, (n_cells, 3) as (x, y, z)."""
        h = (box / self.n) / (2.0 ** self.cell_level)
        return (self.cell_coord + 0.5) * h[:, None]

    def leaves(self):
        return np.nonzero(self.child_oct < 0)[0]


def _key(c, nl):
    c = np.mod(c, nl)
    return (c[..., 2] * nl + c[..., 1]) * nl + c[..., 0]


def _unkey(k, nl):
    return np.stack([k % nl, (k // nl) % nl, k // (nl * nl)], axis=-1)


_OFF27 = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)],
                  dtype=np.int64)
_CHILD = np.array([(c & 1, (c >> 1) & 1, (c >> 2) & 1) for c in range(8)], dtype=np.int64)


def build_octree(n: int, max_level: int, refine) -> OctreeInput:
    """Build a 2:1-balanced (faces, edges and corners) periodic octree.

    ``refine(level, coords)`` gets the level-l integer coords (m, 3) of existing
    cells and returns a boolean mask of those to refine (l < max_level)."""
    refined = []                                  # sorted keys per level
    exist = np.arange(n ** 3, dtype=np.int64)     # existing cell keys at level 0
    for l in range(max_level):
        nl = n << l
        mask = np.asarray(refine(l, _unkey(exist, nl)), dtype=bool)
        refined.append(np.unique(exist[mask]))
        kids = (2 * _unkey(refined[l], nl)[:, None, :] + _CHILD[None]).reshape(-1, 3)
        exist = np.unique(_key(kids, nl * 2))
    # 2:1 balance: a refined level-l cell needs its 26 neighbours (and itself)
    # to exist at level l, i.e. their parents refined at level l-1.
    for l in range(max_level - 1, 0, -1):
        if refined[l].size == 0:
            continue
        nl = n << l
        c = _unkey(refined[l], nl)
        nb = (c[:, None, :] + _OFF27[None]).reshape(-1, 3)
        parents = np.unique(_key(np.floor_divide(np.mod(nb, nl), 2), nl // 2))
        refined[l - 1] = np.union1d(refined[l - 1], parents)
    # the union may have created refined cells whose parent is not refined:
    # close upwards (a cell exists only if its parent is refined)
    for l in range(1, max_level):
        nl = n << l
        par = np.unique(_key(np.floor_divide(_unkey(refined[l], nl), 2), nl // 2))
        missing = np.setdiff1d(par, refined[l - 1])
        if missing.size:
            raise RuntimeError("balance closure failed")
    # breadth-first layout
    n_base = n ** 3
    cell_level = [np.zeros(n_base, np.int32)]
    cell_coord = [_unkey(np.arange(n_base, dtype=np.int64), n)]
    oct_parent, oct_level, oct_coord = [], [], []
    # cell index of each existing cell per level, as sorted (key, index) arrays
    lvl_keys = np.arange(n_base, dtype=np.int64)
    lvl_index = np.arange(n_base, dtype=np.int64)
    next_cell = n_base
    n_oct = 0
    child_oct_parts = []
    for l in range(max_level):
        nl = n << l
        r = refined[l]
        pos = np.searchsorted(lvl_keys, r)
        assert np.all(lvl_keys[pos] == r)
        pidx = lvl_index[pos]
        order = np.argsort(pidx)                  # BFS: parents in cell order
        pidx = pidx[order]
        pc = _unkey(r[order], nl)
        k = np.arange(n_oct, n_oct + pidx.size, dtype=np.int64)
        child_oct_parts.append((pidx, k))
        oct_parent.append(pidx)
        oct_level.append(np.full(pidx.size, l + 1, np.int32))
        oct_coord.append(2 * pc)
        kids = (2 * pc[:, None, :] + _CHILD[None]).reshape(-1, 3)
        kid_index = next_cell + np.arange(kids.shape[0], dtype=np.int64)
        cell_level.append(np.full(kids.shape[0], l + 1, np.int32))
        cell_coord.append(kids)
        kk = _key(kids, 2 * nl)
        srt = np.argsort(kk)
        lvl_keys, lvl_index = kk[srt], kid_index[srt]
        next_cell += kids.shape[0]
        n_oct += pidx.size
    child_oct = np.full(next_cell, -1, np.int32)
    for pidx, k in child_oct_parts:
        child_oct[pidx] = k.astype(np.int32)
    cat = lambda xs, dt, shape: (np.concatenate(xs).astype(dt) if xs else np.zeros(shape, dt))
    return OctreeInput(n, max_level, child_oct,
                       cat(oct_parent, np.int64, (0,)), cat(oct_level, np.int32, (0,)),
                       cat(oct_coord, np.int32, (0, 3)).reshape(-1, 3),
                       np.concatenate(cell_level).astype(np.int32),
                       np.concatenate(cell_coord).astype(np.int64))


def random_octree(n: int, max_level: int, p: float, rng: np.random.Generator,
                  region=None) -> OctreeInput:
    """Octree refined at random (probability p per cell and level), optionally
    only inside ``region`` = (lo, hi) in base-cell units."""
    def refine(l, c):
        m = rng.random(c.shape[0]) < p
        if region is not None:
            lo, hi = region
            x = (c + 0.5) / float(1 << l)
            m &= np.all((x >= lo) & (x < hi), axis=1)
        return m
    return build_octree(n, max_level, refine)


def full_octree(n: int, level: int) -> OctreeInput:
    """Every cell refined down to ``level`` (equivalent to a uniform n*2^level grid)."""
    return build_octree(n, level, lambda l, c: np.ones(c.shape[0], bool))


# ------------------------------------------------------------ AMR light cone --
RHO_CRIT = 2.77536627e11        # critical density, (Msun/h) / (Mpc/h)^3
G_NEWTON = 4.30091727e-9        # Mpc (km/s)^2 / Msun
C_KMS = 299792.458


def _nfw_f(c):
    return np.log1p(c) - c / (1.0 + c)


def _nfw_sample_x(u, c, iters=60):
    """Inverse of the NFW enclosed-mass profile m(x) = ln(1+x) - x/(1+x) on
    [0, c] (bisection, vectorised); u in [0, m(c)]."""
    lo = np.zeros_like(u)
    hi = np.full_like(u, c)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        below = _nfw_f(mid) < u
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return 0.5 * (lo + hi)


@dataclass
class HaloCatalogue:
    centres: np.ndarray     # (h, 3) Mpc/h
    m200: np.ndarray        # Msun/h
    r200: np.ndarray        # Mpc/h
    conc: float


def amr_particles(n: int = 256, box: float = 256.0, n_part: int = 1 << 24,
                  halo_frac: float = 0.3, conc: float = 5.0, seed_cfg: int = 3):
    """Particles of the AMR configuration: NFW haloes (masses log-uniform in
    [1e12, 1e15] Msun/h, concentration 5, radii truncated at R200) holding
    ``halo_frac`` of the particles, the rest multinomial-sampled from a
    lognormal density on the base grid.  Returns (positions, haloes, delta)."""
    rng_f, rng_h, rng_p, _ = seeds(seed_cfg)
    m_p = OMEGA_M * RHO_CRIT * (box / n) ** 3 * (n ** 3 / n_part)
    budget = halo_frac * n_part * m_p
    masses = []
    tot = 0.0
    while tot < budget:
        m = 10.0 ** rng_h.uniform(12.0, 15.0)
        if tot + m > budget:
            break
        masses.append(m)
        tot += m
    masses = np.array(masses)
    r200 = (3.0 * masses / (4.0 * np.pi * 200.0 * RHO_CRIT)) ** (1.0 / 3.0)
    centres = rng_h.uniform(0.0, box, size=(len(masses), 3))
    npart_h = np.maximum(np.round(masses / m_p).astype(np.int64), 1)
    pos = []
    fc = _nfw_f(conc)
    for c0, r2, k in zip(centres, r200, npart_h):
        x = _nfw_sample_x(rng_p.uniform(0.0, fc, size=k), conc)
        r = x * (r2 / conc)
        v = rng_p.normal(size=(k, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        pos.append(c0[None, :] + r[:, None] * v)
    n_halo = int(npart_h.sum())
    delta = lognormal_delta(n, box, rng_f, slope=-2.0, sigma_g=1.0)
    w = (1.0 + delta).ravel()
    counts = rng_p.multinomial(n_part - n_halo, w / w.sum())
    cells = np.repeat(np.arange(n ** 3, dtype=np.int64), counts)
    h = box / n
    base = np.stack([cells % n, (cells // n) % n, cells // (n * n)], -1).astype(np.float64)
    pos.append((base + rng_p.uniform(0.0, 1.0, size=base.shape)) * h)
    pos = np.mod(np.concatenate(pos), box)
    return pos, HaloCatalogue(centres, masses, r200, conc), delta


def amr_octree_from_particles(pos, n: int, box: float, max_level: int = 4,
                              threshold: int = 8) -> OctreeInput:
    """Refine every cell holding more than ``threshold`` particles, down to
    ``max_level``; then 2:1-balance over faces, edges and corners."""
    h = box / n

    def refine(l, coords):
        nl = n << l
        ip = np.floor(pos / (h / (1 << l))).astype(np.int64) % nl
        keys = (ip[:, 2] * nl + ip[:, 1]) * nl + ip[:, 0]
        uk, cnt = np.unique(keys, return_counts=True)
        ck = _key(coords, nl)
        idx = np.searchsorted(uk, ck)
        idx = np.minimum(idx, len(uk) - 1)
        found = uk[idx] == ck
        return found & (cnt[idx] > threshold)

    return build_octree(n, max_level, refine)


def _trilinear_periodic(field, pts_cells):
    """Trilinear interpolation of a periodic cell-centred field [z][y][x] at
    points given in cell units (cell centres at i + 0.5)."""
    n = field.shape[0]
    p = pts_cells - 0.5
    i0 = np.floor(p).astype(np.int64)
    f = p - i0
    out = np.zeros(p.shape[0])
    for dz in (0, 1):
        wz = f[:, 2] if dz else 1.0 - f[:, 2]
        for dy in (0, 1):
            wy = f[:, 1] if dy else 1.0 - f[:, 1]
            for dx in (0, 1):
                wx = f[:, 0] if dx else 1.0 - f[:, 0]
                out += wx * wy * wz * field[(i0[:, 2] + dz) % n, (i0[:, 1] + dy) % n,
                                            (i0[:, 0] + dx) % n]
    return out


def amr_potential(t: OctreeInput, box: float, haloes: HaloCatalogue, delta) -> np.ndarray:
    """Phi/c^2 at every cell centre (leaf and refined cells): the Poisson
    potential of the lognormal background interpolated to the centre, plus a
    truncated NFW potential per halo inside 2 R200 (shifted to zero there)."""
    n = t.n
    h = box / n
    phi_bg = poisson_phi(delta, box)
    cen = t.centres(box)
    phi = _trilinear_periodic(phi_bg, cen / h)
    # cells grouped by base cell for the halo neighbourhood queries
    base = (t.cell_coord >> t.cell_level[:, None].astype(np.int64))
    bkey = (base[:, 2] * n + base[:, 1]) * n + base[:, 0]
    order = np.argsort(bkey, kind="stable")
    sk = bkey[order]
    starts = np.searchsorted(sk, np.arange(n ** 3 + 1))
    c = haloes.conc
    fc = _nfw_f(c)
    for c0, m, r2 in zip(haloes.centres, haloes.m200, haloes.r200):
        rs = r2 / c
        rt = 2.0 * r2
        amp = G_NEWTON * m / fc / C_KMS ** 2
        phi_t = -amp * np.log1p(rt / rs) / rt
        lo = np.floor((c0 - rt) / h).astype(np.int64)
        hi = np.floor((c0 + rt) / h).astype(np.int64)
        rng_ax = [np.arange(lo[a], hi[a] + 1) % n for a in range(3)]
        bz, by, bx = np.meshgrid(rng_ax[2], rng_ax[1], rng_ax[0], indexing="ij")
        bk = ((bz * n + by) * n + bx).ravel()
        segs = [order[starts[b]:starts[b + 1]] for b in bk]
        cells = np.concatenate(segs) if segs else np.zeros(0, np.int64)
        dvec = cen[cells] - c0[None, :]
        dvec -= box * np.round(dvec / box)
        r = np.sqrt(np.sum(dvec * dvec, axis=1))
        inside = r < rt
        rr = np.maximum(r[inside], 1e-6 * rs)
        phi[cells[inside]] += -amp * np.log1p(rr / rs) / rr - phi_t
    return phi


@dataclass
class AmrCase:
    tree: OctreeInput
    box: float
    phi: np.ndarray
    haloes: HaloCatalogue
    observer: tuple = (0.0, 0.0, 0.0)


def config3(n: int = 256, box: float = 256.0, n_part: int = 1 << 24, max_level: int = 4):
    """AMR octree: 256^3 base grid, refinement where a cell holds > 8 of 2^24
    particles (NFW haloes on a lognormal background), up to 4 levels."""
    pos, haloes, delta = amr_particles(n, box, n_part)
    t = amr_octree_from_particles(pos, n, box, max_level)
    del pos
    phi = amr_potential(t, box, haloes, delta)
    return AmrCase(t, box, phi, haloes)


def config3_rays(nray: int = 4096, fov_deg: float = 10.0):
    fov = math.radians(fov_deg)
    chi_s = chi_of_z(1.0)
    d = fov_directions((0.0, 0.0, 1.0), fov, fov, nray, nray)
    return Bundle(d, nray, nray, chi_s, chi_s, 0.0, (0.0, 0.0, 1.0), fov, fov)


@dataclass
class BundleSpec:
    side: int
    z_s: float
    chi_s: float
    fov: float
    center: tuple


def config4_specs(n_bundles: int = 64):
    """64 bundles: side 8*round(32*2^U) with U ~ U[0, 3] (256..2048 rays per
    side), z_s ~ U[0.5, 2], square field of view ~ U[1, 10] deg, centre
    directions uniform on the sphere."""
    _, _, _, rb = seeds(4)
    out = []
    for _ in range(n_bundles):
        side = int(8 * round(32 * 2.0 ** rb.uniform(0.0, 3.0)))
        zs = float(rb.uniform(0.5, 2.0))
        fov = math.radians(float(rb.uniform(1.0, 10.0)))
        v = rb.normal(size=3)
        v /= np.linalg.norm(v)
        out.append(BundleSpec(side, zs, chi_of_z(zs), fov, tuple(v)))
    return out


def bundle_from_spec(s: BundleSpec) -> Bundle:
    d = fov_directions(s.center, s.fov, s.fov, s.side, s.side)
    return Bundle(d, s.side, s.side, s.chi_s, s.chi_s, 0.0, s.center, s.fov, s.fov)
