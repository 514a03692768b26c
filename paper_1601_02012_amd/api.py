"""Python binding of librayramses (argument marshalling only).

Every step of the ray-tracing path runs in the HIP kernels of the library;
PyTorch supplies device memory and the current HIP stream.  Names follow the
C ABI in include/rayramses.h.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _abi as A
from ._abi import RRError  # noqa: F401  (re-export)

PREC = {"fp64": A.PREC_FP64, "fp32": A.PREC_FP32_KAHAN, "fp32_kahan": A.PREC_FP32_KAHAN}
QUANTITY = {"kappa": A.Q_KAPPA, "gamma1": A.Q_GAMMA1, "gamma2": A.Q_GAMMA2,
            "scalar": A.Q_SCALAR}

_lib = A.lib()   # fail loudly at import if the HIP library is missing


def _stream(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def _prec(p):
    return PREC[p] if isinstance(p, str) else int(p)


def _check_buffer(t: Optional[torch.Tensor], name: str, dtype: torch.dtype, min_numel: int,
                  exact: bool = False) -> None:
    """Reject a caller-supplied buffer before any launch: wrong dtype, not
    contiguous, or fewer elements than the kernels index (ValueError)."""
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    n = t.numel()
    if (n != min_numel) if exact else (n < min_numel):
        raise ValueError(f"{name} holds {n} elements, needs "
                         f"{'exactly' if exact else 'at least'} {min_numel}")


def fov_directions(center, fov_x: float, fov_y: float, nx: int, ny: int) -> np.ndarray:
    """rr_fov_directions: (ny*nx, 3) FP64 unit directions of a flat-sky map
    (Eq. txty angles, gnomonic about ``center``; ray id = iy*nx + ix).  Runs
    on the host; copy the result to the device for a RayBundle."""
    c = (C.c_double * 3)(*[float(v) for v in center])
    out = np.empty((int(nx) * int(ny), 3), dtype=np.float64)
    A.check("rr_fov_directions",
            _lib.rr_fov_directions(c, float(fov_x), float(fov_y), int(nx), int(ny),
                                   out.ctypes.data_as(C.c_void_p)))
    return out


class Grid:
    """A potential field on a uniform grid or a 2:1 octree (device tensors).

    values: uniform -> (n, n, n) [z][y][x]; octree -> (n_cells,) one per cell.
    child_oct: octree only, int32 (n_cells,)."""

    def __init__(self, values: torch.Tensor, box: float, *, n_base: Optional[int] = None,
                 boundary: str = "periodic", child_oct: Optional[torch.Tensor] = None,
                 max_level: int = 0, field: str = "phi"):
        if values.dtype not in (torch.float32, torch.float64):
            raise TypeError("values must be float32 or float64")
        self.values = values.contiguous()
        self.box = float(box)
        self.octree = child_oct is not None
        self.child_oct = child_oct.contiguous() if child_oct is not None else None
        if self.octree:
            if n_base is None:
                raise ValueError("octree grids need n_base")
            self.n = int(n_base)
        else:
            self.n = int(values.shape[0]) if n_base is None else int(n_base)
        self.boundary = A.BOUNDARY_OPEN if boundary == "open" else A.BOUNDARY_PERIODIC
        self.max_level = int(max_level)
        fields = {"phi": A.FIELD_PHI, "delta": A.FIELD_DELTA, "phi_dot": A.FIELD_PHI_DOT}
        if field not in fields:
            raise ValueError("field is 'phi' (potential), 'delta' (density contrast) or "
                             "'phi_dot' (the potential's rate of change, ISW)")
        self.field = fields[field]

    def desc(self) -> A.FieldDesc:
        d = A.FieldDesc()
        d.kind = A.GRID_OCTREE if self.octree else A.GRID_UNIFORM
        d.field = self.field
        d.boundary = self.boundary
        d.dtype = A.F32 if self.values.dtype == torch.float32 else A.F64
        d.n_base = self.n
        d.max_level = self.max_level
        d.box_size = self.box
        d.values = _ptr(self.values)
        d.child_oct = _ptr(self.child_oct)
        d.n_cells = int(self.values.numel()) if self.octree else 0
        return d


class TidalTensor:
    """Library-owned vertex tensor of a grid (rr_tensor)."""

    def __init__(self, grid: Grid, precision="fp32"):
        self.grid = grid
        self.precision = _prec(precision)
        h = C.c_void_p()
        d = grid.desc()
        A.check("rr_tensor_create", _lib.rr_tensor_create(C.byref(d), self.precision, C.byref(h)))
        self.handle = h

    def build(self, grid: Optional[Grid] = None, stream=None) -> "TidalTensor":
        g = grid if grid is not None else self.grid
        self.grid = g
        d = g.desc()
        A.check("rr_build_tidal_tensor",
                _lib.rr_build_tidal_tensor(self.handle, C.byref(d), _stream(stream)))
        return self

    def build_method_a(self, delta: Grid, phi: Grid, delta_coeff: float,
                       stream=None) -> "TidalTensor":
        """rr_build_method_a_fields: (delta_coeff delta, grad phi) vertex fields of a
        tensor created from a density grid (Method A, Eq. kappa2)."""
        dd, dp = delta.desc(), phi.desc()
        A.check("rr_build_method_a_fields",
                _lib.rr_build_method_a_fields(self.handle, C.byref(dd), C.byref(dp),
                                              float(delta_coeff), _stream(stream)))
        return self

    def build_isw(self, phi_curr: Grid, phi_prev: Grid, inv_dt: float,
                  stream=None) -> "TidalTensor":
        """rr_build_isw_field: vertex values of (phi_curr - phi_prev) * inv_dt for a
        tensor created from a 'phi_dot' grid (ISW integrand, trace with
        quantity="scalar")."""
        dc, dp = phi_curr.desc(), phi_prev.desc()
        A.check("rr_build_isw_field",
                _lib.rr_build_isw_field(self.handle, C.byref(dc), C.byref(dp), float(inv_dt),
                                        _stream(stream)))
        return self

    def build_centres(self, grid: Optional[Grid] = None, stream=None) -> "TidalTensor":
        """rr_build_tidal_tensor_centres: cell-centre records for the NGP integral."""
        g = grid if grid is not None else self.grid
        self.grid = g
        d = g.desc()
        A.check("rr_build_tidal_tensor_centres",
                _lib.rr_build_tidal_tensor_centres(self.handle, C.byref(d), _stream(stream)))
        return self

    def build_box(self, lo, size, grid: Optional[Grid] = None, stream=None) -> "TidalTensor":
        """rr_build_tidal_tensor_box: rebuild only the vertices of the periodic box."""
        g = grid if grid is not None else self.grid
        self.grid = g
        d = g.desc()
        lo_a = (C.c_int32 * 3)(*[int(x) for x in lo])
        sz_a = (C.c_int32 * 3)(*[int(x) for x in size])
        A.check("rr_build_tidal_tensor_box",
                _lib.rr_build_tidal_tensor_box(self.handle, C.byref(d), lo_a, sz_a,
                                               _stream(stream)))
        return self

    def layout(self):
        p = C.c_void_p()
        n = C.c_int64()
        rb = C.c_int32()
        pr = C.c_int32()
        A.check("rr_tensor_layout", _lib.rr_tensor_layout(self.handle, C.byref(p), C.byref(n),
                                                          C.byref(rb), C.byref(pr)))
        return p.value, n.value, rb.value, pr.value

    def to_torch(self) -> torch.Tensor:
        """Copy of the records as a (n_records, record_words) device tensor."""
        ptr, n, rb, pr = self.layout()
        dt = torch.float32 if pr == A.PREC_FP32_KAHAN else torch.float64
        words = rb // (4 if dt == torch.float32 else 8)
        out = torch.empty((n, words), dtype=dt, device="cuda")
        _memcpy_d2d(out.data_ptr(), ptr, n * rb)
        return out

    def close(self):
        if getattr(self, "handle", None):
            _lib.rr_tensor_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip = None


def _memcpy_d2d(dst: int, src: int, nbytes: int):
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        _hip.hipMemcpyAsync.restype = C.c_int
    err = _hip.hipMemcpyAsync(C.c_void_p(dst), C.c_void_p(src), C.c_size_t(nbytes), 3,
                              _stream())
    if err != 0:
        raise RuntimeError(f"hipMemcpyAsync failed ({err})")


class Plan:
    """Work queue, bundle-table cache and captured graph (rr_plan)."""

    def __init__(self):
        h = C.c_void_p()
        A.check("rr_plan_create", _lib.rr_plan_create(C.byref(h)))
        self.handle = h

    def autotune(self, tensor: "TidalTensor", bundles, observer, *, kappa_scale=1.0,
                 quantity="kappa", stream=None):
        """rr_plan_autotune: pick the fastest launch shape for these bundles."""
        tp = _params(observer, tensor.precision, quantity, kappa_scale, -1)
        arr = _bundle_array(bundles)
        A.check("rr_plan_autotune", _lib.rr_plan_autotune(self.handle, tensor.handle, C.byref(tp),
                                                          arr, len(bundles), _stream(stream)))
        pers, blk, wpc, pas, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_float()
        A.check("rr_plan_tuned_shape",
                _lib.rr_plan_tuned_shape(self.handle, arr, len(bundles), C.byref(pers),
                                         C.byref(blk), C.byref(wpc), C.byref(pas), C.byref(ms)))
        return {"persistent": pers.value, "block": blk.value, "waves_per_cu": wpc.value,
                "passes": pas.value, "ms": ms.value}

    def set_shape(self, bundles, *, persistent=0, block=256, waves_per_cu=16, passes=1):
        """rr_plan_set_shape: the launch shape calls with persistent=-1 use for
        these bundles (passes > 1: the march split into resumable passes)."""
        arr = _bundle_array(bundles)
        A.check("rr_plan_set_shape",
                _lib.rr_plan_set_shape(self.handle, arr, len(bundles), int(persistent),
                                       int(block), int(waves_per_cu), int(passes)))

    def vertex_box(self, tensor: "TidalTensor", bundles, observer, stream=None):
        """rr_rays_vertex_box: (lo, size) of the vertices these bundles' rays read."""
        tp = _params(observer, tensor.precision)
        arr = _bundle_array(bundles)
        lo = (C.c_int32 * 3)()
        size = (C.c_int32 * 3)()
        A.check("rr_rays_vertex_box",
                _lib.rr_rays_vertex_box(self.handle, tensor.handle, C.byref(tp), arr, len(bundles),
                                        lo, size, _stream(stream)))
        return tuple(lo), tuple(size)

    def graph_begin(self, stream=None):
        A.check("rr_graph_begin", _lib.rr_graph_begin(self.handle, _stream(stream)))

    def graph_end(self, stream=None):
        A.check("rr_graph_end", _lib.rr_graph_end(self.handle, _stream(stream)))

    def graph_launch(self, stream=None):
        A.check("rr_graph_launch", _lib.rr_graph_launch(self.handle, _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            _lib.rr_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class RayBundle:
    """Rays of one nx-by-ny map (device FP64 unit directions, ray id = iy*nx+ix).
    ``center_dir``, ``fov_x`` and ``fov_y`` optionally record the field of view
    the directions were made from (checked by the library)."""
    dirs: torch.Tensor
    nx: int
    ny: int
    chi_s: float
    chi_hi: float
    chi_lo: float
    ray_offset: int = 0
    center_dir: Optional[tuple] = None
    fov_x: float = 0.0
    fov_y: float = 0.0

    @property
    def n_rays(self):
        return self.nx * self.ny

    def window(self, chi_hi: float, chi_lo: float) -> "RayBundle":
        return RayBundle(self.dirs, self.nx, self.ny, self.chi_s, chi_hi, chi_lo, self.ray_offset,
                         self.center_dir, self.fov_x, self.fov_y)


def _bundle_array(bundles: Sequence[RayBundle]):
    arr = (A.Bundle * max(1, len(bundles)))()
    for i, b in enumerate(bundles):
        if b.n_rays:
            if b.dirs.dtype != torch.float64 or b.dirs.shape[-1] != 3:
                raise TypeError("bundle directions must be float64 (n, 3)")
            if b.dirs.numel() != 3 * b.n_rays:
                raise ValueError("bundle directions do not match nx*ny")
        arr[i].ray_offset = b.ray_offset
        arr[i].n_rays = b.n_rays
        arr[i].dir = _ptr(b.dirs) if b.n_rays else None
        arr[i].nx = b.nx
        arr[i].ny = b.ny
        arr[i].chi_s = b.chi_s
        arr[i].chi_hi = b.chi_hi
        arr[i].chi_lo = b.chi_lo
        if b.center_dir is not None:
            c = [float(v) for v in b.center_dir]
            r = math.sqrt((c[0] * c[0] + c[1] * c[1]) + c[2] * c[2])
            for k in range(3):
                arr[i].center_dir[k] = c[k] / r if r > 0.0 else c[k]
            arr[i].fov_x = float(b.fov_x)
            arr[i].fov_y = float(b.fov_y)
    return arr


def _params(observer, precision, quantity="kappa", kappa_scale=1.0, persistent=-1,
            max_crossings=0, hash=None, count=None, log=None, log_stride=0, integral="trilinear"):
    tp = A.TraceParams()
    for k in range(3):
        tp.observer[k] = float(observer[k])
    tp.kappa_scale = float(kappa_scale)
    tp.precision = precision
    tp.quantity = QUANTITY[quantity] if isinstance(quantity, str) else int(quantity)
    tp.integral = A.INTEGRAL_NGP if integral == "ngp" else A.INTEGRAL_TRILINEAR
    tp.persistent = int(persistent)
    tp.max_crossings = int(max_crossings)
    tp.crossing_hash = _ptr(hash)
    tp.crossing_count = _ptr(count)
    tp.crossing_log = _ptr(log)
    tp.log_stride = int(log_stride)
    return tp


LOG_DTYPE = np.dtype([("cell", np.int64), ("chi_a", np.float64), ("chi_b", np.float64)])


@dataclass
class TraceOutput:
    kappa: torch.Tensor
    kappa_comp: Optional[torch.Tensor]
    status: Optional[torch.Tensor]
    hash: Optional[torch.Tensor] = None
    count: Optional[torch.Tensor] = None
    log: Optional[torch.Tensor] = None


def total_rays(bundles: Sequence[RayBundle]) -> int:
    return max([b.ray_offset + b.n_rays for b in bundles] + [0])


def trace(plan: Plan, tensor: TidalTensor, bundles: Sequence[RayBundle], observer, *,
          kappa: Optional[torch.Tensor] = None, kappa_comp: Optional[torch.Tensor] = None,
          status: Optional[torch.Tensor] = None, kappa_scale: float = 1.0, quantity="kappa",
          persistent: int = -1, max_crossings: int = 0, debug: bool = False,
          log_stride: int = 0, integral: str = "trilinear", stream=None) -> TraceOutput:
    """rr_trace_rays: add each ray's integral to ``kappa`` (allocated if None).
    ``integral``: "trilinear" (vertex tensor) or "ngp" (cell-centre tensor)."""
    nr = total_rays(bundles)
    fp32 = tensor.precision == A.PREC_FP32_KAHAN
    dev = "cuda"
    _check_buffer(kappa, "kappa", torch.float32 if fp32 else torch.float64, nr)
    _check_buffer(kappa_comp, "kappa_comp", torch.float32, nr)
    _check_buffer(status, "status", torch.int32, nr)
    if kappa_comp is not None and not fp32:
        raise ValueError("kappa_comp is only used by the FP32-Kahan precision")
    if kappa is None:
        kappa = torch.zeros(nr, dtype=torch.float32 if fp32 else torch.float64, device=dev)
    if kappa_comp is None and fp32:
        kappa_comp = torch.zeros(nr, dtype=torch.float32, device=dev)
    if status is None:
        status = torch.zeros(nr, dtype=torch.int32, device=dev)
    hsh = cnt = log = None
    if debug:
        hsh = torch.zeros(nr, dtype=torch.int64, device=dev)
        cnt = torch.zeros(nr, dtype=torch.int64, device=dev)
    if log_stride:
        log = torch.zeros((nr, log_stride, 3), dtype=torch.float64, device=dev)
    tp = _params(observer, tensor.precision, quantity, kappa_scale, persistent, max_crossings,
                 hsh, cnt, log, log_stride, integral)
    arr = _bundle_array(bundles)
    A.check("rr_trace_rays",
            _lib.rr_trace_rays(plan.handle, tensor.handle, C.byref(tp), arr, len(bundles),
                               _ptr(kappa), _ptr(kappa_comp) if fp32 else None, _ptr(status),
                               _stream(stream)))
    return TraceOutput(kappa, kappa_comp, status, hsh, cnt, log)


def trace_noalloc(tensor: TidalTensor, bundles: Sequence[RayBundle], observer, *,
                  kappa: torch.Tensor, kappa_comp: Optional[torch.Tensor] = None,
                  status: Optional[torch.Tensor] = None, kappa_scale: float = 1.0,
                  quantity="kappa", persistent: int = 0, max_crossings: int = 0,
                  hash: Optional[torch.Tensor] = None, count: Optional[torch.Tensor] = None,
                  integral: str = "trilinear", stream=None) -> TraceOutput:
    """rr_trace_rays_noalloc: rr_trace_rays without a plan and without any
    device allocation (the caller passes every output buffer)."""
    nr = total_rays(bundles)
    fp32 = tensor.precision == A.PREC_FP32_KAHAN
    if kappa is None:
        raise ValueError("trace_noalloc needs the caller's kappa buffer")
    _check_buffer(kappa, "kappa", torch.float32 if fp32 else torch.float64, nr)
    _check_buffer(kappa_comp, "kappa_comp", torch.float32, nr)
    _check_buffer(status, "status", torch.int32, nr)
    _check_buffer(hash, "hash", torch.int64, nr)
    _check_buffer(count, "count", torch.int64, nr)
    if kappa_comp is not None and not fp32:
        raise ValueError("kappa_comp is only used by the FP32-Kahan precision")
    tp = _params(observer, tensor.precision, quantity, kappa_scale, persistent, max_crossings,
                 hash, count, None, 0, integral)
    arr = _bundle_array(bundles)
    A.check("rr_trace_rays_noalloc",
            _lib.rr_trace_rays_noalloc(tensor.handle, C.byref(tp), arr, len(bundles),
                                       _ptr(kappa), _ptr(kappa_comp), _ptr(status),
                                       _stream(stream)))
    return TraceOutput(kappa, kappa_comp, status, hash, count)


class SourcesOutput:
    """State of the many-source walk: per-ray moments (FP32 Kahan pairs
    {A, A_comp, B, B_comp} or FP64 {A, B}), pieces (n_rays, n_src, 2) FP64,
    status and optional debug outputs."""

    def __init__(self, moments, pieces, status, hash=None, count=None):
        self.moments, self.pieces, self.status = moments, pieces, status
        self.hash, self.count = hash, count


def _src_array(chi_src):
    src = np.ascontiguousarray(np.asarray(chi_src, dtype=np.float64).reshape(-1))
    return src, src.ctypes.data_as(C.POINTER(C.c_double))


def trace_sources(plan: Plan, tensor: TidalTensor, bundles: Sequence[RayBundle], observer,
                  chi_src, *, state: Optional[SourcesOutput] = None, kappa_scale: float = 1.0,
                  quantity="kappa", persistent: int = -1, max_crossings: int = 0,
                  debug: bool = False, stream=None) -> SourcesOutput:
    """rr_trace_rays_sources: one walk for every source distance in ``chi_src``
    (decreasing).  Pass the previous window's ``state`` to continue it."""
    nr = total_rays(bundles)
    fp32 = tensor.precision == A.PREC_FP32_KAHAN
    dev = "cuda"
    src, src_p = _src_array(chi_src)
    if state is not None:
        _check_buffer(state.moments, "state.moments", torch.float32 if fp32 else torch.float64,
                      nr * (4 if fp32 else 2))
        _check_buffer(state.pieces, "state.pieces", torch.float64, nr * len(src) * 2)
        _check_buffer(state.status, "state.status", torch.int32, nr)
        if state.pieces.dim() != 3 or state.pieces.shape[1:] != (len(src), 2):
            raise ValueError("state.pieces must have shape (n_rays, n_src, 2)")
    if state is None:
        mom = torch.zeros((nr, 4) if fp32 else (nr, 2),
                          dtype=torch.float32 if fp32 else torch.float64, device=dev)
        pcs = torch.zeros((nr, len(src), 2), dtype=torch.float64, device=dev)
        state = SourcesOutput(mom, pcs, torch.zeros(nr, dtype=torch.int32, device=dev))
    hsh = cnt = None
    if debug:
        hsh = torch.zeros(nr, dtype=torch.int64, device=dev)
        cnt = torch.zeros(nr, dtype=torch.int64, device=dev)
    tp = _params(observer, tensor.precision, quantity, kappa_scale, persistent, max_crossings,
                 hsh, cnt, None, 0)
    arr = _bundle_array(bundles)
    A.check("rr_trace_rays_sources",
            _lib.rr_trace_rays_sources(plan.handle, tensor.handle, C.byref(tp), arr, len(bundles),
                                       src_p, len(src), _ptr(state.moments), _ptr(state.pieces),
                                       _ptr(state.status), _stream(stream)))
    return SourcesOutput(state.moments, state.pieces, state.status, hsh, cnt)


def kappa_from_pieces(plan: Plan, tensor: TidalTensor, chi_src, state: SourcesOutput,
                      stream=None) -> torch.Tensor:
    """rr_kappa_from_pieces: (n_rays, n_src) FP64 kappa of every source."""
    src, src_p = _src_array(chi_src)
    nr = state.moments.shape[0]
    fp32 = tensor.precision == A.PREC_FP32_KAHAN
    _check_buffer(state.moments, "state.moments", torch.float32 if fp32 else torch.float64,
                  nr * (4 if fp32 else 2), exact=True)
    _check_buffer(state.pieces, "state.pieces", torch.float64, nr * len(src) * 2)
    out = torch.empty((nr, len(src)), dtype=torch.float64, device=state.moments.device)
    A.check("rr_kappa_from_pieces",
            _lib.rr_kappa_from_pieces(plan.handle, tensor.handle, src_p, len(src), nr,
                                      _ptr(state.moments), _ptr(state.pieces), _ptr(out),
                                      _stream(stream)))
    return out


def log_to_numpy(log: torch.Tensor) -> np.ndarray:
    """Convert a crossing log tensor (n, stride, 3 x 8 bytes) to records."""
    return log.cpu().numpy().view(LOG_DTYPE).reshape(log.shape[0], log.shape[1])


def trace_adjoint(plan: Plan, tensor: TidalTensor, grid: Grid, bundles: Sequence[RayBundle],
                  observer, dl_dkappa: torch.Tensor, *, dl_dphi: Optional[torch.Tensor] = None,
                  kappa_scale: float = 1.0, stream=None) -> torch.Tensor:
    """rr_trace_rays_adjoint: dL/dPhi (added to ``dl_dphi``, allocated if None)."""
    nr = total_rays(bundles)
    if not isinstance(dl_dkappa, torch.Tensor) or dl_dkappa.numel() < nr:
        raise ValueError(f"dl_dkappa must be a tensor of at least {nr} elements")
    _check_buffer(dl_dphi, "dl_dphi", torch.float32, grid.n ** 3, exact=True)
    if dl_dphi is None:
        dl_dphi = torch.zeros_like(grid.values, dtype=torch.float32)
    tp = _params(observer, tensor.precision, "kappa", kappa_scale, 0)
    arr = _bundle_array(bundles)
    d = grid.desc()
    w = dl_dkappa.to(torch.float32).contiguous()
    A.check("rr_trace_rays_adjoint",
            _lib.rr_trace_rays_adjoint(plan.handle, tensor.handle, C.byref(d), C.byref(tp), arr,
                                       len(bundles), _ptr(w), _ptr(dl_dphi), _stream(stream)))
    return dl_dphi


class Geometry:
    """Non-differentiable ray geometry for :class:`RayTraceKappa`."""

    def __init__(self, box: float, observer, bundles: Sequence[RayBundle], *,
                 kappa_scale: float = 1.0, plan: Optional[Plan] = None):
        self.box = float(box)
        self.observer = tuple(float(x) for x in observer)
        self.bundles = list(bundles)
        self.kappa_scale = kappa_scale
        self.plan = plan or Plan()
        self._tensor = None

    def tensor_for(self, grid: Grid) -> TidalTensor:
        if self._tensor is None or self._tensor.grid.n != grid.n:
            self._tensor = TidalTensor(grid, "fp32")
        return self._tensor


class RayTraceKappa(torch.autograd.Function):
    """kappa = A(phi) on a uniform periodic FP32 grid, with the hand-written
    adjoint (rr_trace_rays_adjoint) as backward."""

    @staticmethod
    def forward(ctx, phi: torch.Tensor, geometry: Geometry):
        grid = Grid(phi.detach().to(torch.float32).contiguous(), geometry.box)
        t = geometry.tensor_for(grid)
        t.build(grid)
        out = trace(geometry.plan, t, geometry.bundles, geometry.observer,
                    kappa_scale=geometry.kappa_scale, persistent=0)
        ctx.geometry = geometry
        ctx.grid = grid
        return out.kappa.clone()

    @staticmethod
    def backward(ctx, grad_kappa: torch.Tensor):
        g = ctx.geometry
        t = g.tensor_for(ctx.grid)
        dphi = trace_adjoint(g.plan, t, ctx.grid, g.bundles, g.observer,
                             grad_kappa.contiguous(), kappa_scale=g.kappa_scale)
        return dphi, None
