"""Octree pins of the FP64 oracle (Sec. III H, Sec. IV C of the paper)."""
import math

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I


def _otree(oracle, t):
    return oracle.Octree(t.n, t.child_oct, t.oct_parent, t.oct_level, t.oct_coord, t.max_level)


# --------------------------------------------------------------------- P8 --
@pytest.mark.parametrize("dim,nc,nfv,ac,af", [
    (2, 2, [2, 2], 1 / 3, [1 / 6, 1 / 6]),            # vertex V3 of the 2D figure
    (2, 3, [3], 4 / 15, [1 / 5]),                     # V4
    (2, 1, [2, 1, 2], 4 / 9, [2 / 9, 1 / 9, 2 / 9]),  # V5
    (3, 7, [7], 8 / 63, [1 / 9]),                     # 7 coarse + 1 fine (Eq. rhoV_1)
    (3, 4, [4, 4, 4, 4], 1 / 6, [1 / 12] * 4),        # flat 3D interface
])
def test_P8_weight_examples(oracle, dim, nc, nfv, ac, af):
    """Worked weights of Eqs. (alphaconst), (alphaconst2), (alphac3d), (alphaf3d);
    each set sums to one."""
    a_c, a_f = oracle.vertex_weights(dim, nc, nfv)
    assert a_c == pytest.approx(ac, rel=1e-15)
    np.testing.assert_allclose(a_f, af, rtol=1e-15)
    assert nc * a_c + a_f.sum() == pytest.approx(1.0, rel=1e-15)


def test_P8_seven_coarse_one_fine_in_a_tree(oracle):
    """One refined base cell: its outer corner is shared by 7 coarse leaves and
    1 fine leaf with N_fv = 7, so the vertex gets 8/63 per coarse centre and
    1/9 for the fine one (the 3D example in Sec. III H)."""
    n = 4
    target = (1, 1, 1)
    t = I.build_octree(n, 1, lambda l, c: np.all(c == np.array(target), axis=1))
    ot = _otree(oracle, t)
    rng = np.random.default_rng(5)
    tc = rng.normal(size=(t.n_cells, 6))
    cv = oracle.corner_tensor_octree(ot, tc)
    base = lambda i, j, k: (k * n + j) * n + i
    # fine child at the (0,0,0) corner of the refined cell: vertex (1,1,1) of the base lattice
    fine = n ** 3 + 0
    coarse = [base(1 - dx, 1 - dy, 1 - dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)
              if (dx, dy, dz) != (0, 0, 0)]
    expect = 8 / 63 * tc[coarse].sum(0) + 1 / 9 * tc[fine]
    np.testing.assert_allclose(cv[fine, 0], expect, rtol=1e-13)
    # a mid-edge hanging vertex of the coarse neighbour: fine child 1 (ix=1) at
    # its (1,0,0)... its lower-x/lower-y/lower-z corner at level-1 (3,2,2) lies
    # on the base edge between (1,1,1)+(0.5,0,0); value = mean of the two ends
    v_end0 = cv[fine, 0]
    # the other end (2,1,1) on the base lattice is the corner (1,0,0) of child 1
    v_end1 = cv[n ** 3 + 1, 1]
    np.testing.assert_allclose(cv[n ** 3 + 1, 0], 0.5 * (v_end0 + v_end1), rtol=1e-13)


# --------------------------------------------------------------------- P7 --
@pytest.mark.parametrize("seed,levels,p", [(0, 2, 0.2), (1, 3, 0.15), (2, 4, 0.08), (3, 3, 0.5)])
def test_P7_vertex_interpolation_conserves_mass(oracle, seed, levels, p):
    """Sec. III H: the total 'mass' from cell centres equals the total from the
    vertex reconstruction, on random 2:1-balanced octrees."""
    rng = np.random.default_rng(seed)
    t = I.random_octree(6, levels, p, rng)
    ot = _otree(oracle, t)
    assert oracle.octree_check(ot) == 0
    phi = rng.normal(size=t.n_cells)
    tc = oracle.centre_tensor_octree(ot, phi)
    cv = oracle.corner_tensor_octree(ot, tc)
    lv = t.leaves()
    vol = (0.5 ** t.cell_level[lv]) ** 3
    m_centre = (vol[:, None] * tc[lv]).sum(0)
    m_vertex = (vol[:, None] * cv[lv].mean(axis=1)).sum(0)
    np.testing.assert_allclose(m_vertex, m_centre, rtol=1e-12, atol=1e-12 * np.abs(tc).max())


def test_octree_check_detects_unbalance(oracle):
    n = 6
    t = I.build_octree(n, 1, lambda l, c: np.all(c == np.array([2, 2, 2]), axis=1))
    ot = _otree(oracle, t)
    assert oracle.octree_check(ot) == 0
    # hand-made level-2 refinement inside one level-1 cell at the edge of the
    # refined region: refine a level-1 cell whose 26 neighbours do not all exist
    child = t.child_oct.copy()
    n_cells = t.n_cells
    new_child = np.concatenate([child, np.full(8, -1, np.int32)])
    k_new = t.n_octs
    new_child[n ** 3 + 0] = k_new
    ot2 = oracle.Octree(n, new_child, np.append(t.oct_parent, n ** 3),
                        np.append(t.oct_level, 2), np.vstack([t.oct_coord, 2 * t.oct_coord[0]]), 2)
    assert oracle.octree_check(ot2) > 0
    assert n_cells + 8 == new_child.shape[0]


# -------------------------------------------------------------------- P10 --
def test_P10_fully_refined_octree_equals_uniform(oracle):
    """An octree refined everywhere to level 1 traces exactly like the uniform
    grid of twice the resolution: the same crossing parameters (up to the
    exact factor 2 of the unit change) and the same kappa."""
    n = 8
    L = 16.0
    t = I.full_octree(n, 1)
    ot = _otree(oracle, t)
    rng = np.random.default_rng(10)
    kk = 2 * np.pi / L * np.array([1.0, 2.0, 1.0])
    cen = t.centres(L)
    phi_cells = np.sin(cen @ kk + 0.2) + 0.3 * np.cos(cen @ (2 * kk[::-1]))
    n2 = 2 * n
    c2 = (np.arange(n2) + 0.5) * (L / n2)
    zz, yy, xx = np.meshgrid(c2, c2, c2, indexing="ij")
    pts = np.stack([xx, yy, zz], -1)
    phi_u = np.sin(pts @ kk + 0.2) + 0.3 * np.cos(pts @ (2 * kk[::-1]))
    fov = math.radians(6.0)
    dirs = I.fov_directions((0.2, 0.1, 1.0), fov, fov, 6, 6)
    o = np.array([0.0, 0.0, 0.0])
    chis, hi, lo = 40.0, 35.0, 0.0
    ro = oracle.trace_octree(ot, L, o, dirs, chis, hi, lo, phi=phi_cells, log_stride=512)
    ru = oracle.trace_uniform(n2, L, o, dirs, chis, hi, lo, phi=phi_u, log_stride=512)
    np.testing.assert_array_equal(ro.ncross, ru.ncross)
    for k in range(len(dirs)):
        a = ro.log[k][: ro.ncross[k]]
        b = ru.log[k][: ru.ncross[k]]
        assert np.array_equal(2.0 * a["chi_a"], b["chi_a"])
        assert np.array_equal(2.0 * a["chi_b"], b["chi_b"])
    np.testing.assert_allclose(ro.kappa, ru.kappa, rtol=1e-11, atol=1e-13 * np.abs(ru.kappa).max())


# --------------------------------------------------------------- P2 octree --
@pytest.mark.parametrize("seed", [0, 1])
def test_P2_quadratic_on_octree_refinement_invariant(oracle, seed):
    """Constant transverse Laplacian on a random multi-level octree: kappa is
    that constant times the kernel integral, independent of the refinement."""
    rng = np.random.default_rng(100 + seed)
    n = 16
    L = 16.0
    t = I.random_octree(n, 3, 0.25, rng, region=(3.0, 13.0))
    ot = _otree(oracle, t)
    assert oracle.octree_check(ot) == 0
    M = rng.normal(size=(3, 3)); M = M + M.T
    cen = t.centres(L)
    phi = 0.5 * np.einsum("ci,ij,cj->c", cen, M, cen)
    o = np.array([8.0, 8.0, 3.5])
    fov = math.radians(20.0)
    dirs = I.fov_directions((0.0, 0.0, 1.0), fov, fov, 7, 7)
    chis, hi, lo = 12.0, 9.0, 0.0          # stays inside [2.5, 13.5]^3: no wrap of the stencil
    r = oracle.trace_octree(ot, L, o, dirs, chis, hi, lo, phi=phi, log_stride=1024)
    levels = set()
    for k in range(len(dirs)):
        levels |= set(t.cell_level[r.log[k][: r.ncross[k]]["cell"]].tolist())
    assert len(levels) >= 3                  # the rays do cross refinement boundaries
    qv = np.trace(M) - np.einsum("ri,ij,rj->r", dirs, M, dirs)
    expect = qv * ((chis * (hi ** 2 - lo ** 2) / 2 - (hi ** 3 - lo ** 3) / 3) / chis)
    np.testing.assert_allclose(r.kappa, expect, rtol=1e-11)


@pytest.mark.parametrize("seed", [0, 1])
def test_P2_quadratic_ngp_on_octree(oracle, seed):
    """Eq. (Iclensing_ngp) on a multi-level octree: a quadratic potential has
    the same exact centre tensor in every leaf, so the nearest-grid-point
    kappa is the constant times the kernel integral, and the walk (crossing
    hashes) is the one of the trilinear integral."""
    rng = np.random.default_rng(300 + seed)
    n, L = 16, 16.0
    t = I.random_octree(n, 3, 0.25, rng, region=(3.0, 13.0))
    ot = _otree(oracle, t)
    M = rng.normal(size=(3, 3)); M = M + M.T
    cen = t.centres(L)
    phi = 0.5 * np.einsum("ci,ij,cj->c", cen, M, cen)
    o = np.array([8.0, 8.0, 3.5])
    fov = math.radians(20.0)
    dirs = I.fov_directions((0.0, 0.0, 1.0), fov, fov, 7, 7)
    chis, hi, lo = 12.0, 9.0, 0.0
    r = oracle.trace_octree(ot, L, o, dirs, chis, hi, lo, phi=phi, ngp=True)
    rt = oracle.trace_octree(ot, L, o, dirs, chis, hi, lo, phi=phi)
    assert np.array_equal(r.hash, rt.hash)
    qv = np.trace(M) - np.einsum("ri,ij,rj->r", dirs, M, dirs)
    expect = qv * ((chis * (hi ** 2 - lo ** 2) / 2 - (hi ** 3 - lo ** 3) / 3) / chis)
    # per-cell closed forms cancel: rounding is relative to the map's scale
    np.testing.assert_allclose(r.kappa, expect, rtol=0, atol=1e-12 * np.abs(expect).max())


def test_P2_quadratic_shear_on_octree(oracle):
    """Constant tensor on a multi-level octree: gamma1 and gamma2 are the
    projections on e_theta, e_phi (Eqs. gamma1, gamma2, Eq. n1n2 read without
    its 1/sin(theta)) times the kernel integral, whatever the refinement."""
    rng = np.random.default_rng(320)
    n, L = 16, 16.0
    t = I.random_octree(n, 3, 0.25, rng, region=(3.0, 13.0))
    ot = _otree(oracle, t)
    M = rng.normal(size=(3, 3)); M = M + M.T
    cen = t.centres(L)
    phi = 0.5 * np.einsum("ci,ij,cj->c", cen, M, cen)
    o = np.array([8.0, 8.0, 3.5])
    fov = math.radians(20.0)
    dirs = I.fov_directions((0.1, 0.0, 1.0), fov, fov, 7, 7)
    chis, hi, lo = 12.0, 9.0, 0.0
    gint = (chis * (hi ** 2 - lo ** 2) / 2 - (hi ** 3 - lo ** 3) / 3) / chis
    th = np.arccos(dirs[:, 2])
    ph = np.arctan2(dirs[:, 1], dirs[:, 0])
    et = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], 1)
    ep = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], 1)
    quad = lambda u, v: np.einsum("ri,ij,rj->r", u, M, v)
    g1 = oracle.trace_octree(ot, L, o, dirs, chis, hi, lo, phi=phi, quantity=oracle.Q_GAMMA1)
    g2 = oracle.trace_octree(ot, L, o, dirs, chis, hi, lo, phi=phi, quantity=oracle.Q_GAMMA2)
    e1 = (quad(ep, ep) - quad(et, et)) * gint
    e2 = 2 * quad(ep, et) * gint
    np.testing.assert_allclose(g1.kappa, e1, rtol=0, atol=1e-11 * np.abs(e1).max())
    np.testing.assert_allclose(g2.kappa, e2, rtol=0, atol=1e-11 * np.abs(e2).max())


def test_P8_face_centre_hanging_vertex(oracle):
    """A vertex in the middle of a coarse face takes the mean of the face's
    four coarse corner values (Sec. III H, text after Eq. rhoV_1)."""
    n = 4
    t = I.build_octree(n, 1, lambda l, c: np.all(c == np.array([1, 1, 1]), axis=1))
    ot = _otree(oracle, t)
    rng = np.random.default_rng(6)
    tc = rng.normal(size=(t.n_cells, 6))
    cv = oracle.corner_tensor_octree(ot, tc)
    # child 0 (level-1 coords (2,2,2)) has corner 3 = (3,3,2): the centre of the
    # refined cell's lower-z face, i.e. of the upper face of coarse cell (1,1,0)
    base = lambda i, j, k: (k * n + j) * n + i
    corner_val = lambda cell, v: cv[cell, v]
    c0 = base(1, 1, 0)
    face = [corner_val(c0, v) for v in (4, 5, 6, 7)]      # upper-z face of the coarse cell
    np.testing.assert_allclose(cv[n ** 3 + 0, 3], np.mean(face, axis=0), rtol=1e-13)


@pytest.mark.parametrize("seed", [0, 1])
def test_P17_cubic_potential_exact_centre_tensor_on_octree(oracle, seed):
    """Cubic Phi on a multi-level octree: the level-l stencil is exact for
    cubics, and the coarse-level fallback (trilinear 3/4-1/4 interpolation of
    a linear tensor field) is exact too, so every interior cell's centre
    tensor equals the analytic Hessian at its centre (Sec. IV C, option 2)."""
    rng = np.random.default_rng(200 + seed)
    n, L = 12, 12.0
    t = I.random_octree(n, 3, 0.3, rng, region=(3.0, 9.0))
    ot = _otree(oracle, t)
    M = rng.normal(size=(3, 3)); M = M + M.T
    Ct = rng.normal(size=(3, 3, 3)) * 0.1
    C = sum(np.transpose(Ct, p) for p in [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]) / 6
    x = t.centres(L)
    phi = 0.5 * np.einsum("ci,ij,cj->c", x, M, x) + np.einsum("abc,ia,ib,ic->i", C, x, x, x) / 6
    tc = oracle.centre_tensor_octree(ot, phi)
    H = M[None] + np.einsum("abc,ic->iab", C, x)
    ref = np.stack([H[:, 0, 0], H[:, 1, 1], H[:, 2, 2], H[:, 0, 1], H[:, 0, 2], H[:, 1, 2]], -1)
    h = (L / n) / (2.0 ** t.cell_level)
    # interior: the cell and its stencil (plus the coarse fallback cells) stay away from the faces
    inside = np.all((x > 2.5 * (L / n)) & (x < L - 2.5 * (L / n)), axis=1)
    fallback_cells = 0
    for lvl in range(1, t.max_level + 1):
        sel = inside & (t.cell_level == lvl)
        np.testing.assert_allclose(tc[sel], ref[sel], rtol=0, atol=1e-9 * np.abs(ref).max())
        # cells of this level with a face neighbour missing at their level take the fallback
        nl = n << lvl
        key = lambda c: (c[:, 2] * nl + c[:, 1]) * nl + c[:, 0]
        have = set(key(t.cell_coord[t.cell_level == lvl]).tolist())
        cc = t.cell_coord[sel]
        for a in range(3):
            for s_ in (-1, 1):
                nb_ = cc.copy()
                nb_[:, a] += s_
                fallback_cells += sum(k not in have for k in key(nb_).tolist())
    np.testing.assert_allclose(tc[inside & (t.cell_level == 0)], ref[inside & (t.cell_level == 0)],
                               rtol=0, atol=1e-9 * np.abs(ref).max())
    assert fallback_cells > 0
