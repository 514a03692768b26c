"""ctypes front end of the FP64 CPU oracle (``liboracle_rro.so``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg load this module.  The product path (the HIP library and its
Python binding) never imports it.

All arrays are numpy; FP32 inputs are widened exactly to FP64.  Distances are
in box units (e.g. Mpc/h); the C code converts to base-grid units.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle_rro.so")
SOURCES = ["rro_uniform.c", "rro_adjoint.c", "rro_octree.c", "rro_method_a.c",
           "rro_sources.c", "rro_isw.c"]

RAY_OK, RAY_OUT_OF_DOMAIN, RAY_MAX_STEPS = 0, 1, 2
Q_KAPPA, Q_GAMMA1, Q_GAMMA2 = 0, 1, 2


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-Wall", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class Segment(C.Structure):
    _fields_ = [("cell", C.c_int64), ("chi_a", C.c_double), ("chi_b", C.c_double)]


SEG_DTYPE = np.dtype([("cell", np.int64), ("chi_a", np.float64), ("chi_b", np.float64)])


class _Octree(C.Structure):
    _fields_ = [("n", C.c_int32), ("max_level", C.c_int32), ("n_octs", C.c_int64),
                ("child_oct", C.c_void_p), ("oct_parent", C.c_void_p),
                ("oct_level", C.c_void_p), ("oct_coord", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.rro_centre_tensor_uniform.argtypes = [i32, i32, dbl, vp, vp]
        L.rro_vertex_tensor_uniform.argtypes = [i32, vp, vp]
        L.rro_trace_uniform.argtypes = [i32, i32, dbl, vp, i64, vp, vp, vp, vp, dbl, i32, i32,
                                        vp, vp, i64, i32, vp, vp, vp, vp, vp, i64]
        L.rro_trace_uniform.restype = i32
        L.rro_trace_adjoint_uniform.argtypes = [i32, dbl, vp, i64, vp, vp, vp, vp, dbl, vp,
                                                i32, vp]
        L.rro_trace_adjoint_uniform.restype = i32
        L.rro_octree_check.argtypes = [vp]
        L.rro_octree_check.restype = i32
        L.rro_centre_tensor_octree.argtypes = [vp, vp, vp]
        L.rro_corner_tensor_octree.argtypes = [vp, vp, vp]
        L.rro_corner_tensor_octree_cells.argtypes = [vp, vp, i64, vp, vp]
        L.rro_vertex_weights.argtypes = [i32, i32, i32, vp, vp, vp]
        L.rro_trace_octree.argtypes = [vp, dbl, vp, i64, vp, vp, vp, vp, dbl, i32, vp, vp, i32,
                                       i64, i32, vp, vp, vp, vp, vp, i64]
        L.rro_trace_octree.restype = i32
        L.rro_cell_integral.argtypes = [vp, vp, dbl, vp, vp, dbl, dbl, dbl]
        L.rro_cell_integral.restype = dbl
        L.rro_cell_integral_k.argtypes = [vp, vp, dbl, vp, vp, dbl, dbl, dbl]
        L.rro_cell_integral_k.restype = dbl
        L.rro_method_a_vertex_fields.argtypes = [i32, i32, dbl, vp, vp, vp]
        L.rro_trace_uniform_method_a.argtypes = [i32, i32, dbl, vp, i64, vp, vp, vp, vp, dbl, dbl,
                                                 vp, i64, i32, vp, vp, vp, vp]
        L.rro_trace_uniform_method_a.restype = i32
        L.rro_trace_uniform_sources.argtypes = [i32, i32, dbl, vp, i64, vp, vp, vp, i32, vp,
                                                dbl, i32, vp, i64, i32, vp, vp, vp, vp, vp]
        L.rro_trace_uniform_sources.restype = i32
        L.rro_trace_octree_sources.argtypes = [vp, dbl, vp, i64, vp, vp, vp, i32, vp, dbl, i32,
                                               vp, i64, i32, vp, vp, vp, vp, vp]
        L.rro_trace_octree_sources.restype = i32
        L.rro_kappa_from_pieces.argtypes = [i64, i32, vp, dbl, i32, vp, vp, vp]
        L.rro_cell_moments.argtypes = [vp, vp, dbl, vp, vp, dbl, dbl, vp]
        L.rro_isw_vertex_field.argtypes = [i32, i32, vp, vp, dbl, vp]
        L.rro_trace_uniform_isw.argtypes = [i32, i32, dbl, vp, i64, vp, vp, vp, dbl, vp, i64,
                                            i32, vp, vp, vp, vp]
        L.rro_trace_uniform_isw.restype = i32
        L.rro_cell_integral_one.argtypes = [vp, vp, dbl, vp, vp, dbl, dbl]
        L.rro_cell_integral_one.restype = dbl
        L.rro_projection.argtypes = [vp, vp, i32]
        L.rro_projection.restype = dbl
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------- uniform --
def centre_tensor(phi, open_boundary=False, h=1.0):
    """Eq. (tidalexample) at every cell centre; returns (n^3, 6)."""
    phi = _f64(phi)
    n = phi.shape[0]
    tc = np.empty((n ** 3, 6))
    lib().rro_centre_tensor_uniform(n, int(open_boundary), h, _p(phi), _p(tc))
    return tc


def vertex_tensor(phi, open_boundary=False):
    """Centre tensor averaged to vertices (grid units, h = 1); returns (n^3, 6)."""
    phi = _f64(phi)
    n = phi.shape[0]
    tc = centre_tensor(phi, open_boundary)
    tv = np.empty_like(tc)
    lib().rro_vertex_tensor_uniform(n, _p(tc), _p(tv))
    return tv


def _per_ray(v, n):
    v = np.asarray(v, dtype=np.float64)
    if v.ndim == 0:
        v = np.full(n, float(v))
    return np.ascontiguousarray(v)


@dataclass
class TraceResult:
    kappa: np.ndarray
    hash: np.ndarray
    ncross: np.ndarray
    status: np.ndarray
    log: np.ndarray | None = None


def trace_uniform(n, box, observer, dirs, chi_s, chi_hi, chi_lo, *, tv=None, tc=None,
                  phi=None, open_boundary=False, kappa_scale=1.0, quantity=Q_KAPPA,
                  ngp=False, max_steps=1 << 40, threads=0, log_stride=0) -> TraceResult:
    """Trace rays (FP64).  Give ``tv`` (vertex tensor) / ``tc`` (centre tensor,
    for NGP) or ``phi`` to have them computed here."""
    dirs = _f64(dirs).reshape(-1, 3)
    nr = dirs.shape[0]
    if phi is not None:
        if ngp:
            tc = centre_tensor(phi, open_boundary)
        else:
            tv = vertex_tensor(phi, open_boundary)
    obs = _f64(observer)
    cs, ch, cl = _per_ray(chi_s, nr), _per_ray(chi_hi, nr), _per_ray(chi_lo, nr)
    kappa = np.zeros(nr)
    hsh = np.zeros(nr, dtype=np.uint64)
    ncr = np.zeros(nr, dtype=np.int64)
    st = np.zeros(nr, dtype=np.int32)
    log = np.zeros((nr, log_stride), dtype=SEG_DTYPE) if log_stride else None
    tv_ = _f64(tv) if tv is not None else None
    tc_ = _f64(tc) if tc is not None else None
    lib().rro_trace_uniform(n, int(open_boundary), float(box), _p(obs), nr, _p(dirs), _p(cs),
                            _p(ch), _p(cl), float(kappa_scale), quantity, int(ngp), _p(tv_),
                            _p(tc_), int(max_steps), int(threads), _p(kappa), _p(hsh),
                            _p(ncr), _p(st), _p(log), int(log_stride))
    return TraceResult(kappa, hsh, ncr, st, log)


def method_a_vertex_fields(phi, delta, open_boundary=False, h=1.0):
    """Method A vertex fields (Eq. kappa2): per vertex (delta, dPhi/dx, dPhi/dy,
    dPhi/dz), central differences and the eight-cell mean; returns (n^3, 4)."""
    phi = _f64(phi)
    delta = _f64(delta)
    n = phi.shape[0]
    fv = np.empty((n ** 3, 4))
    lib().rro_method_a_vertex_fields(n, int(open_boundary), h, _p(phi), _p(delta), _p(fv))
    return fv


def trace_uniform_method_a(n, box, observer, dirs, chi_s, chi_hi, chi_lo, *, delta_coeff,
                           fv=None, phi=None, delta=None, open_boundary=False, kappa_scale=1.0,
                           max_steps=1 << 40, threads=0) -> TraceResult:
    """Method A kappa (FP64): delta_coeff g delta + (n . grad Phi) dg/dchi and
    the step's surface term; ``fv`` from method_a_vertex_fields, or ``phi`` and
    ``delta`` to compute it here."""
    dirs = _f64(dirs).reshape(-1, 3)
    nr = dirs.shape[0]
    if fv is None:
        fv = method_a_vertex_fields(phi, delta, open_boundary)
    kappa = np.zeros(nr)
    hsh = np.zeros(nr, dtype=np.uint64)
    ncr = np.zeros(nr, dtype=np.int64)
    st = np.zeros(nr, dtype=np.int32)
    lib().rro_trace_uniform_method_a(n, int(open_boundary), float(box), _p(_f64(observer)), nr,
                                     _p(dirs), _p(_per_ray(chi_s, nr)), _p(_per_ray(chi_hi, nr)),
                                     _p(_per_ray(chi_lo, nr)), float(kappa_scale),
                                     float(delta_coeff), _p(_f64(fv)), int(max_steps),
                                     int(threads), _p(kappa), _p(hsh), _p(ncr), _p(st))
    return TraceResult(kappa, hsh, ncr, st, None)


def cell_integral_k(Q, p1, h, direction, o, chis, chiA, chiB):
    """One cell of the Method A gradient term (kernel 1 - 2 chi / chi_s)."""
    return lib().rro_cell_integral_k(_p(_f64(Q)), _p(_f64(p1)), float(h), _p(_f64(direction)),
                                     _p(_f64(o)), float(chis), float(chiA), float(chiB))


@dataclass
class SourcesResult:
    moments: np.ndarray      # (n_rays, 2): int chi Q, int chi^2 Q left after the last stop
    pieces: np.ndarray       # (n_rays, n_src, 2): handed out at each source
    hash: np.ndarray
    ncross: np.ndarray
    status: np.ndarray


def _sources_io(nr, n_src, chi_src, moments, pieces):
    src = _f64(chi_src).reshape(-1)
    assert src.shape[0] == n_src
    mom = np.zeros((nr, 2)) if moments is None else np.array(moments, dtype=np.float64)
    pcs = np.zeros((nr, n_src, 2)) if pieces is None else np.array(pieces, dtype=np.float64)
    return src, np.ascontiguousarray(mom), np.ascontiguousarray(pcs)


def trace_uniform_sources(n, box, observer, dirs, chi_hi, chi_lo, chi_src, *, tv=None, phi=None,
                          open_boundary=False, kappa_scale=1.0, quantity=Q_KAPPA,
                          moments=None, pieces=None, max_steps=1 << 40,
                          threads=0) -> SourcesResult:
    """One walk for many source distances (Eqs. Isources, Isources1), FP64.
    ``moments`` / ``pieces`` carry the state of earlier chi windows."""
    dirs = _f64(dirs).reshape(-1, 3)
    nr = dirs.shape[0]
    if tv is None:
        tv = vertex_tensor(phi, open_boundary)
    src, mom, pcs = _sources_io(nr, len(np.atleast_1d(chi_src)), chi_src, moments, pieces)
    hsh = np.zeros(nr, dtype=np.uint64)
    ncr = np.zeros(nr, dtype=np.int64)
    st = np.zeros(nr, dtype=np.int32)
    lib().rro_trace_uniform_sources(n, int(open_boundary), float(box), _p(_f64(observer)), nr,
                                    _p(dirs), _p(_per_ray(chi_hi, nr)), _p(_per_ray(chi_lo, nr)),
                                    src.shape[0], _p(src), float(kappa_scale), int(quantity),
                                    _p(_f64(tv)), int(max_steps), int(threads), _p(mom), _p(pcs),
                                    _p(hsh), _p(ncr), _p(st))
    return SourcesResult(mom, pcs, hsh, ncr, st)


def cell_moments(Q, p1, h, direction, o, chi_a, chi_b):
    """(int chi Q, int chi^2 Q) over one cell's piece [chi_b, chi_a] (grid units)."""
    out = np.zeros(2)
    lib().rro_cell_moments(_p(_f64(Q)), _p(_f64(p1)), float(h), _p(_f64(direction)),
                           _p(_f64(o)), float(chi_a), float(chi_b), _p(out))
    return out


def kappa_from_pieces(chi_src, box, n_base, moments, pieces):
    """kappa (n_rays, n_src) of every source after the walk reached the observer."""
    src = _f64(chi_src).reshape(-1)
    mom = _f64(moments).reshape(-1, 2)
    pcs = _f64(pieces).reshape(mom.shape[0], src.shape[0], 2)
    out = np.zeros((mom.shape[0], src.shape[0]))
    lib().rro_kappa_from_pieces(mom.shape[0], src.shape[0], _p(src), float(box), int(n_base),
                                _p(mom), _p(pcs), _p(out))
    return out


def isw_vertex_field(phi_curr, phi_prev, inv_dt, open_boundary=False):
    """Vertex values of (phi_curr - phi_prev) * inv_dt (eight-cell mean); (n^3,)."""
    pc = _f64(phi_curr)
    pp = _f64(phi_prev)
    n = pc.shape[0]
    qv = np.empty(n ** 3)
    lib().rro_isw_vertex_field(n, int(open_boundary), _p(pc), _p(pp), float(inv_dt), _p(qv))
    return qv


def trace_uniform_isw(n, box, observer, dirs, chi_hi, chi_lo, *, qv=None, phi_curr=None,
                      phi_prev=None, inv_dt=1.0, open_boundary=False, scale=1.0,
                      max_steps=1 << 40, threads=0) -> TraceResult:
    """ISW integral scale * int Q dchi (box units) per ray, FP64; ``qv`` from
    isw_vertex_field, or the two potentials to compute it here."""
    dirs = _f64(dirs).reshape(-1, 3)
    nr = dirs.shape[0]
    if qv is None:
        qv = isw_vertex_field(phi_curr, phi_prev, inv_dt, open_boundary)
    out = np.zeros(nr)
    hsh = np.zeros(nr, dtype=np.uint64)
    ncr = np.zeros(nr, dtype=np.int64)
    st = np.zeros(nr, dtype=np.int32)
    lib().rro_trace_uniform_isw(n, int(open_boundary), float(box), _p(_f64(observer)), nr,
                                _p(dirs), _p(_per_ray(chi_hi, nr)), _p(_per_ray(chi_lo, nr)),
                                float(scale), _p(_f64(qv)), int(max_steps), int(threads),
                                _p(out), _p(hsh), _p(ncr), _p(st))
    return TraceResult(out, hsh, ncr, st, None)


def cell_integral_one(Q, p1, h, direction, o, chi_a, chi_b):
    """int Q dchi over one cell's piece (grid units)."""
    return lib().rro_cell_integral_one(_p(_f64(Q)), _p(_f64(p1)), float(h), _p(_f64(direction)),
                                       _p(_f64(o)), float(chi_a), float(chi_b))


def trace_adjoint_uniform(n, box, observer, dirs, chi_s, chi_hi, chi_lo, dl_dkappa,
                          kappa_scale=1.0, threads=0):
    dirs = _f64(dirs).reshape(-1, 3)
    nr = dirs.shape[0]
    out = np.zeros(n ** 3)
    w = _f64(dl_dkappa)
    lib().rro_trace_adjoint_uniform(n, float(box), _p(_f64(observer)), nr, _p(dirs),
                                    _p(_per_ray(chi_s, nr)), _p(_per_ray(chi_hi, nr)),
                                    _p(_per_ray(chi_lo, nr)), float(kappa_scale), _p(w),
                                    int(threads), _p(out))
    return out.reshape(n, n, n)


def cell_integral(Q, p1, h, direction, o, chis, chi_a, chi_b):
    """Eq. (Iclensing) for one cell (grid units)."""
    return lib().rro_cell_integral(_p(_f64(Q)), _p(_f64(p1)), float(h), _p(_f64(direction)),
                                   _p(_f64(o)), float(chis), float(chi_a), float(chi_b))


def projection(direction, T, quantity=Q_KAPPA):
    """Integrand projection of a tensor T = (xx, yy, zz, xy, xz, yz)."""
    return lib().rro_projection(_p(_f64(direction)), _p(_f64(T)), int(quantity))


# ---------------------------------------------------------------------- octree --
class Octree:
    """Host octree: base n^3 cells, then 8 cells per oct in BFS order."""

    def __init__(self, n, child_oct, oct_parent, oct_level, oct_coord, max_level):
        self.n = int(n)
        self.child_oct = np.ascontiguousarray(child_oct, dtype=np.int32)
        self.oct_parent = np.ascontiguousarray(oct_parent, dtype=np.int64)
        self.oct_level = np.ascontiguousarray(oct_level, dtype=np.int32)
        self.oct_coord = np.ascontiguousarray(oct_coord, dtype=np.int32).reshape(-1, 3)
        self.max_level = int(max_level)
        self.n_octs = int(self.oct_level.shape[0])
        self._c = _Octree(self.n, self.max_level, self.n_octs, _p(self.child_oct),
                          _p(self.oct_parent), _p(self.oct_level), _p(self.oct_coord))

    @property
    def n_cells(self):
        return self.n ** 3 + 8 * self.n_octs

    def ref(self):
        return C.byref(self._c)


def octree_check(t: Octree) -> int:
    return int(lib().rro_octree_check(t.ref()))


def centre_tensor_octree(t: Octree, phi):
    phi = _f64(phi)
    assert phi.shape[0] == t.n_cells
    tc = np.empty((t.n_cells, 6))
    lib().rro_centre_tensor_octree(t.ref(), _p(phi), _p(tc))
    return tc


def corner_tensor_octree(t: Octree, tc):
    cv = np.empty((t.n_cells, 8, 6))
    lib().rro_corner_tensor_octree(t.ref(), _p(_f64(tc)), _p(cv))
    return cv


def corner_tensor_octree_cells(t: Octree, tc, cells):
    """Corner tensors (n, 8, 6) of the listed leaf cells only."""
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    cv = np.empty((cells.shape[0], 8, 6))
    lib().rro_corner_tensor_octree_cells(t.ref(), _p(_f64(tc)), cells.shape[0], _p(cells), _p(cv))
    return cv


def vertex_weights(dim, n_coarse, n_fv):
    n_fv = np.ascontiguousarray(n_fv, dtype=np.int32)
    ac = C.c_double()
    af = np.zeros(len(n_fv))
    lib().rro_vertex_weights(dim, n_coarse, len(n_fv), _p(n_fv), C.byref(ac), _p(af))
    return ac.value, af


def trace_octree(t: Octree, box, observer, dirs, chi_s, chi_hi, chi_lo, *, cv=None, tc=None,
                 phi=None, kappa_scale=1.0, quantity=Q_KAPPA, ngp=False, max_steps=1 << 40,
                 threads=0, log_stride=0) -> TraceResult:
    """Trace rays through the octree (FP64).  ``ngp`` integrates each leaf's
    centre tensor (Eq. Iclensing_ngp) instead of its corner reconstruction."""
    dirs = _f64(dirs).reshape(-1, 3)
    nr = dirs.shape[0]
    if (cv is None or ngp) and tc is None:
        tc = centre_tensor_octree(t, phi)
    if ngp:
        cv = None
    kappa = np.zeros(nr)
    hsh = np.zeros(nr, dtype=np.uint64)
    ncr = np.zeros(nr, dtype=np.int64)
    st = np.zeros(nr, dtype=np.int32)
    log = np.zeros((nr, log_stride), dtype=SEG_DTYPE) if log_stride else None
    cv_ = _f64(cv) if cv is not None else None
    tc_ = _f64(tc) if tc is not None else None
    lib().rro_trace_octree(t.ref(), float(box), _p(_f64(observer)), nr, _p(dirs),
                           _p(_per_ray(chi_s, nr)), _p(_per_ray(chi_hi, nr)),
                           _p(_per_ray(chi_lo, nr)), float(kappa_scale), int(quantity),
                           _p(cv_), _p(tc_), int(bool(ngp)), int(max_steps), int(threads), _p(kappa), _p(hsh),
                           _p(ncr), _p(st),
                           _p(log), int(log_stride))
    return TraceResult(kappa, hsh, ncr, st, log)


def trace_octree_sources(t: Octree, box, observer, dirs, chi_hi, chi_lo, chi_src, *, cv=None,
                         phi=None, kappa_scale=1.0, quantity=Q_KAPPA, moments=None, pieces=None,
                         max_steps=1 << 40, threads=0) -> SourcesResult:
    """The many-source walk through the octree (FP64); ``cv`` per-leaf corner
    tensors, or ``phi`` to compute them here."""
    dirs = _f64(dirs).reshape(-1, 3)
    nr = dirs.shape[0]
    if cv is None:
        cv = corner_tensor_octree(t, centre_tensor_octree(t, phi))
    src, mom, pcs = _sources_io(nr, len(np.atleast_1d(chi_src)), chi_src, moments, pieces)
    hsh = np.zeros(nr, dtype=np.uint64)
    ncr = np.zeros(nr, dtype=np.int64)
    st = np.zeros(nr, dtype=np.int32)
    lib().rro_trace_octree_sources(t.ref(), float(box), _p(_f64(observer)), nr, _p(dirs),
                                   _p(_per_ray(chi_hi, nr)), _p(_per_ray(chi_lo, nr)),
                                   src.shape[0], _p(src), float(kappa_scale), int(quantity),
                                   _p(_f64(cv)), int(max_steps), int(threads), _p(mom), _p(pcs),
                                   _p(hsh), _p(ncr), _p(st))
    return SourcesResult(mom, pcs, hsh, ncr, st)
