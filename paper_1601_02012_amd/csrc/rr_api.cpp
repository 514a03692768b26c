// rr_api.cpp -- host side of the C ABI declared in include/rayramses.h:
// argument validation, tensor and plan objects, bundle-table upload cache,
// launch configuration and HIP graph capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "rr_internal.hpp"
#include "rr_octree.hpp"

namespace {

thread_local std::string g_err;

rr_status fail(rr_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

rr_status hip_fail(hipError_t e, const char* what) {
  return fail(RR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

namespace rr {
rr_status fov_fail(rr_status s, const char* what) { return fail(s, "%s", what); }
}  // namespace rr

namespace {

#define RR_HIP(call, what)                   \
  do {                                       \
    hipError_t _e = (call);                  \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

}  // namespace

struct rr_tensor_s {
  int32_t kind = RR_GRID_UNIFORM;
  int32_t precision = RR_PREC_FP32_KAHAN;
  int32_t boundary = RR_BOUNDARY_PERIODIC;
  int32_t n = 0;
  int32_t dtype = RR_F32;
  double box = 0.0;
  void* data = nullptr;        // uniform: vertex records; octree: per-leaf corner blocks
  int64_t n_records = 0;
  int32_t record_bytes = 0;
  void* grad = nullptr;        // adjoint workspace (allocated on first use)
  int32_t content = 0;         // uniform records: 0 unbuilt, 1 vertex tensors, 2 cell centres,
                               // 3 Method A vertex fields
  int32_t method_a = 0;        // created from a density field: (c delta, grad Phi) records
  int32_t isw = 0;             // created from a rate field: one scalar per vertex
  std::unique_ptr<rr::OctreeTensor> oct;
};

namespace {

struct CachedTable {
  std::vector<rr_bundle> key;
  int32_t n = 0;
  double box = 0.0;
  int32_t persistent_order = 0;
  rr::DevBundle* dev = nullptr;
  int64_t n_tiles = 0;
  uint64_t last_use = 0;       // plan clock at the last call that used it
  hipEvent_t used = nullptr;   // recorded after the last launch that read it
  bool captured = false;       // used by the capture in progress
  bool in_graph = false;       // read by the plan's instantiated graph
};

// Tables a plan keeps before it releases the least recently used one.
constexpr size_t kMaxTables = 256;

// A source-distance list (many-source walk) on the device, base-cell units.
struct CachedSources {
  std::vector<double> key;   // as given, box units
  double h0 = 0.0;
  double* dev = nullptr;
};

// Launch shape chosen by rr_plan_autotune for one bundle set.
struct TunedShape {
  std::vector<rr_bundle> key;
  int32_t persistent = 0;
  int32_t block = 256;
  int32_t waves_per_cu = 16;
  int32_t passes = 1;
  float ms = 0.0f;
};

}  // namespace

struct rr_plan_s {
  unsigned long long* queue = nullptr;   // eight work counters (one per XCD); bytes 64.. hold ray bounds
  std::vector<CachedTable> tables;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int cu_count = 0;
  int waves_per_cu = 0;      // persistent occupancy target (default)
  int prefer_persistent = 0; // default when the caller passes persistent = -1
  int device = 0;
  std::vector<TunedShape> tuned;
  std::vector<CachedSources> sources;
  double* resume = nullptr;   // per ray: where the next pass of a split march starts
  int64_t resume_cap = 0;
  uint64_t clock = 0;         // counts get_table calls (least-recently-used order)
};

namespace {

bool finite3(const double* v) {
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

rr_status validate_field(const rr_field_desc* f) {
  if (!f) return fail(RR_ERR_INVALID_ARG, "field descriptor is NULL");
  if (f->kind != RR_GRID_UNIFORM && f->kind != RR_GRID_OCTREE)
    return fail(RR_ERR_INVALID_ARG, "unknown grid kind %d", f->kind);
  if (f->field != RR_FIELD_PHI && f->field != RR_FIELD_DELTA && f->field != RR_FIELD_PHI_DOT)
    return fail(RR_ERR_INVALID_ARG, "unknown field kind %d", f->field);
  if (f->field == RR_FIELD_DELTA && f->kind != RR_GRID_UNIFORM)
    return fail(RR_ERR_UNSUPPORTED, "Method A (density fields) is implemented for uniform grids");
  if (f->field == RR_FIELD_PHI_DOT && f->kind != RR_GRID_UNIFORM)
    return fail(RR_ERR_UNSUPPORTED, "the ISW integrand is implemented for uniform grids");
  if (f->dtype != RR_F32 && f->dtype != RR_F64)
    return fail(RR_ERR_INVALID_ARG, "unknown dtype %d", f->dtype);
  if (f->boundary != RR_BOUNDARY_PERIODIC && f->boundary != RR_BOUNDARY_OPEN)
    return fail(RR_ERR_INVALID_ARG, "unknown boundary %d", f->boundary);
  if (f->n_base < 4 || f->n_base > 4096)
    return fail(RR_ERR_INVALID_ARG, "n_base %d outside [4, 4096]", f->n_base);
  if (f->boundary == RR_BOUNDARY_OPEN && f->n_base < 6)
    return fail(RR_ERR_DOMAIN, "open grid needs n_base >= 6 (two stencil layers per side)");
  if (!(f->box_size > 0.0) || !std::isfinite(f->box_size))
    return fail(RR_ERR_INVALID_ARG, "box_size must be positive and finite");
  if (!f->values) return fail(RR_ERR_INVALID_ARG, "values is NULL");
  if (f->kind == RR_GRID_OCTREE) {
    if (f->boundary != RR_BOUNDARY_PERIODIC)
      return fail(RR_ERR_UNSUPPORTED, "octree fields must be periodic");
    if (!f->child_oct) return fail(RR_ERR_INVALID_ARG, "octree child_oct is NULL");
    const int64_t nb = (int64_t)f->n_base * f->n_base * f->n_base;
    if (f->n_cells < nb || (f->n_cells - nb) % 8 != 0)
      return fail(RR_ERR_OCTREE, "n_cells must be n_base^3 + 8 * n_octs");
    if (f->max_level < 0 || f->max_level > rr::kMaxLevel)
      return fail(RR_ERR_INVALID_ARG, "max_level %d outside [0, %d]", f->max_level, rr::kMaxLevel);
  } else if (f->max_level != 0) {
    return fail(RR_ERR_INVALID_ARG, "uniform grids have max_level 0");
  }
  return RR_OK;
}

}  // namespace

extern "C" {

const char* rr_last_error(void) { return g_err.c_str(); }
int32_t rr_version(void) { return 10100; }

rr_status rr_tensor_create(const rr_field_desc* f, rr_precision p, rr_tensor* out) {
  if (!out) return fail(RR_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  rr_status st = validate_field(f);
  if (st != RR_OK) return st;
  if (p != RR_PREC_FP64 && p != RR_PREC_FP32_KAHAN)
    return fail(RR_ERR_INVALID_ARG, "unknown precision %d", (int)p);
  std::unique_ptr<rr_tensor_s> t(new rr_tensor_s);
  t->kind = f->kind;
  t->precision = p;
  t->boundary = f->boundary;
  t->n = f->n_base;
  t->dtype = f->dtype;
  t->box = f->box_size;
  if (f->kind == RR_GRID_UNIFORM) {
    const int64_t nv = (int64_t)f->n_base * f->n_base * f->n_base;
    t->method_a = f->field == RR_FIELD_DELTA;
    t->isw = f->field == RR_FIELD_PHI_DOT;
    t->record_bytes = (t->method_a ? 4 : (t->isw ? 1 : 6)) * (p == RR_PREC_FP32_KAHAN ? 4 : 8);
    t->n_records = nv;
    hipError_t e = hipMalloc(&t->data, (size_t)nv * t->record_bytes);
    if (e != hipSuccess) return fail(RR_ERR_OOM, "vertex tensor: %s", hipGetErrorString(e));
  } else {
    std::string msg;
    t->oct.reset(rr::OctreeTensor::create(f, p, &st, &msg));
    if (!t->oct) return fail(st, "%s", msg.c_str());
    t->data = t->oct->corners;
    t->n_records = t->oct->n_cells;
    t->record_bytes = t->oct->corner_record_bytes;
  }
  *out = t.release();
  return RR_OK;
}

rr_status rr_tensor_destroy(rr_tensor t) {
  if (!t) return RR_OK;
  if (t->kind == RR_GRID_UNIFORM && t->data) (void)hipFree(t->data);
  if (t->grad) (void)hipFree(t->grad);
  delete t;
  return RR_OK;
}

rr_status rr_tensor_layout(rr_tensor t, const void** data, int64_t* n_records,
                           int32_t* record_bytes, int32_t* precision) {
  if (!t) return fail(RR_ERR_INVALID_ARG, "tensor is NULL");
  if (data) *data = t->data;
  if (n_records) *n_records = t->n_records;
  if (record_bytes) *record_bytes = t->record_bytes;
  if (precision) *precision = t->precision;
  return RR_OK;
}

rr_status rr_build_tidal_tensor(rr_tensor t, const rr_field_desc* f, rr_stream s) {
  if (!t) return fail(RR_ERR_INVALID_ARG, "tensor is NULL");
  if (t->method_a || t->isw || (f && f->field != RR_FIELD_PHI))
    return fail(RR_ERR_INVALID_ARG, "tidal tensors are built from potentials (Method A: "
                                    "rr_build_method_a_fields; ISW: rr_build_isw_field)");
  rr_status st = validate_field(f);
  if (st != RR_OK) return st;
  if (f->kind != t->kind || f->n_base != t->n || f->boundary != t->boundary)
    return fail(RR_ERR_INVALID_ARG, "field does not match the grid the tensor was created for");
  if (f->kind == RR_GRID_UNIFORM) {
    const int lo[3] = {0, 0, 0}, size[3] = {f->n_base, f->n_base, f->n_base};
    RR_HIP(rr::launch_vertex_tensor_uniform(t->precision, f->dtype, f->n_base,
                                            f->boundary == RR_BOUNDARY_OPEN, lo, size, f->values,
                                            t->data, (hipStream_t)s),
           "vertex tensor launch");
    t->content = 1;
    return RR_OK;
  }
  if (f->n_cells != t->oct->n_cells || f->child_oct != t->oct->child_oct_dev)
    return fail(RR_ERR_INVALID_ARG, "octree does not match the one the tensor was created for");
  RR_HIP(t->oct->build(f->values, f->dtype, (hipStream_t)s), "octree tensor launch");
  return RR_OK;
}

rr_status rr_build_tidal_tensor_box(rr_tensor t, const rr_field_desc* f, const int32_t lo[3],
                                     const int32_t size[3], rr_stream s) {
  if (!t) return fail(RR_ERR_INVALID_ARG, "tensor is NULL");
  if (t->method_a || t->isw || (f && f->field != RR_FIELD_PHI))
    return fail(RR_ERR_INVALID_ARG, "tidal tensors are built from potentials");
  if (!lo || !size) return fail(RR_ERR_INVALID_ARG, "box pointers are NULL");
  rr_status st = validate_field(f);
  if (st != RR_OK) return st;
  if (f->kind != RR_GRID_UNIFORM || t->kind != RR_GRID_UNIFORM)
    return fail(RR_ERR_UNSUPPORTED, "box builds are for uniform grids");
  if (f->n_base != t->n || f->boundary != t->boundary)
    return fail(RR_ERR_INVALID_ARG, "field does not match the grid the tensor was created for");
  const int n = f->n_base;
  for (int a = 0; a < 3; ++a) {
    if (size[a] < 0 || size[a] > n)
      return fail(RR_ERR_INVALID_ARG, "box size %d on axis %d outside [0, %d]", size[a], a, n);
    if (std::abs((int64_t)lo[a]) > (1ll << 30))
      return fail(RR_ERR_INVALID_ARG, "box origin %d on axis %d is too far out", lo[a], a);
    if (f->boundary == RR_BOUNDARY_OPEN && (lo[a] < 0 || lo[a] + size[a] > n))
      return fail(RR_ERR_DOMAIN, "open grids take boxes inside [0, n)");
  }
  if (t->content == 2)
    return fail(RR_ERR_INVALID_ARG, "the tensor holds cell-centre records: rebuild it whole");
  RR_HIP(rr::launch_vertex_tensor_uniform(t->precision, f->dtype, n,
                                          f->boundary == RR_BOUNDARY_OPEN, lo, size, f->values,
                                          t->data, (hipStream_t)s),
         "vertex tensor launch");
  t->content = 1;
  return RR_OK;
}

rr_status rr_build_tidal_tensor_centres(rr_tensor t, const rr_field_desc* f, rr_stream s) {
  if (!t) return fail(RR_ERR_INVALID_ARG, "tensor is NULL");
  if (t->method_a || t->isw || (f && f->field != RR_FIELD_PHI))
    return fail(RR_ERR_INVALID_ARG, "tidal tensors are built from potentials");
  rr_status st = validate_field(f);
  if (st != RR_OK) return st;
  if (f->kind != t->kind || f->n_base != t->n || f->boundary != t->boundary)
    return fail(RR_ERR_INVALID_ARG, "field does not match the grid the tensor was created for");
  if (f->kind == RR_GRID_OCTREE) return rr_build_tidal_tensor(t, f, s);   // keeps both
  RR_HIP(rr::launch_centre_tensor_uniform(t->precision, f->dtype, f->n_base,
                                          f->boundary == RR_BOUNDARY_OPEN, f->values, t->data,
                                          (hipStream_t)s),
         "centre tensor launch");
  t->content = 2;
  return RR_OK;
}

rr_status rr_build_isw_field(rr_tensor t, const rr_field_desc* phi_curr,
                             const rr_field_desc* phi_prev, double inv_dt, rr_stream s) {
  if (!t) return fail(RR_ERR_INVALID_ARG, "tensor is NULL");
  if (!t->isw)
    return fail(RR_ERR_INVALID_ARG, "the tensor was not created for the ISW integrand "
                                    "(field RR_FIELD_PHI_DOT)");
  for (const rr_field_desc* f : {phi_curr, phi_prev}) {
    rr_status st = validate_field(f);
    if (st != RR_OK) return st;
    if (f->field != RR_FIELD_PHI) return fail(RR_ERR_INVALID_ARG, "need two potentials");
    if (f->kind != RR_GRID_UNIFORM || f->n_base != t->n || f->boundary != t->boundary ||
        f->box_size != t->box)
      return fail(RR_ERR_INVALID_ARG, "field does not match the grid the tensor was created for");
  }
  if (phi_curr->dtype != phi_prev->dtype)
    return fail(RR_ERR_INVALID_ARG, "the two potentials must share a dtype");
  if (!std::isfinite(inv_dt)) return fail(RR_ERR_NONFINITE, "inv_dt is not finite");
  RR_HIP(rr::launch_isw_vertex_field(t->precision, phi_curr->dtype, t->n,
                                     t->boundary == RR_BOUNDARY_OPEN, phi_curr->values,
                                     phi_prev->values, inv_dt, t->data, (hipStream_t)s),
         "ISW field launch");
  t->content = 4;
  return RR_OK;
}

rr_status rr_build_method_a_fields(rr_tensor t, const rr_field_desc* delta,
                                   const rr_field_desc* phi, double delta_coeff, rr_stream s) {
  if (!t) return fail(RR_ERR_INVALID_ARG, "tensor is NULL");
  if (!t->method_a)
    return fail(RR_ERR_INVALID_ARG, "the tensor was created from a potential (Method B)");
  rr_status st = validate_field(delta);
  if (st != RR_OK) return st;
  st = validate_field(phi);
  if (st != RR_OK) return st;
  if (delta->field != RR_FIELD_DELTA || phi->field != RR_FIELD_PHI)
    return fail(RR_ERR_INVALID_ARG, "need a density field and a potential");
  for (const rr_field_desc* f : {delta, phi})
    if (f->kind != RR_GRID_UNIFORM || f->n_base != t->n || f->boundary != t->boundary ||
        f->box_size != t->box)
      return fail(RR_ERR_INVALID_ARG, "field does not match the grid the tensor was created for");
  if (delta->dtype != phi->dtype)
    return fail(RR_ERR_INVALID_ARG, "density and potential must share a dtype");
  if (!std::isfinite(delta_coeff)) return fail(RR_ERR_NONFINITE, "delta_coeff is not finite");
  const double h0 = t->box / (double)t->n;
  RR_HIP(rr::launch_method_a_vertex_fields(t->precision, phi->dtype, t->n,
                                           t->boundary == RR_BOUNDARY_OPEN, delta->values,
                                           phi->values, delta_coeff * h0 * h0, t->data,
                                           (hipStream_t)s),
         "Method A fields launch");
  t->content = 3;
  return RR_OK;
}

rr_status rr_plan_create(rr_plan* p) {
  if (!p) return fail(RR_ERR_INVALID_ARG, "plan out-pointer is NULL");
  *p = nullptr;
  std::unique_ptr<rr_plan_s> q(new rr_plan_s);
  RR_HIP(hipGetDevice(&q->device), "hipGetDevice");
  hipDeviceProp_t prop;
  RR_HIP(hipGetDeviceProperties(&prop, q->device), "hipGetDeviceProperties");
  q->cu_count = prop.multiProcessorCount;
  q->waves_per_cu = 16;
  hipError_t e = hipMalloc((void**)&q->queue, 256);
  if (e != hipSuccess) return fail(RR_ERR_OOM, "queue: %s", hipGetErrorString(e));
  RR_HIP(hipMemset(q->queue, 0, 256), "queue init");
  *p = q.release();
  return RR_OK;
}

rr_status rr_plan_destroy(rr_plan p) {
  if (!p) return RR_OK;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  for (auto& c : p->tables) {
    if (c.used) (void)hipEventSynchronize(c.used);
    if (c.dev) (void)hipFree(c.dev);
    if (c.used) (void)hipEventDestroy(c.used);
  }
  for (auto& c : p->sources)
    if (c.dev) (void)hipFree(c.dev);
  if (p->resume) (void)hipFree(p->resume);
  if (p->queue) (void)hipFree(p->queue);
  delete p;
  return RR_OK;
}

namespace {

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return false;
  return cs != hipStreamCaptureStatusNone;
}

// The field-of-view record of a bundle (Sec. III E, Eq. txty): all zero =
// not recorded; otherwise a finite unit centre, angles in [0, pi), and a
// positive angle on every axis that holds more than one ray.
rr_status validate_fov(const rr_bundle& x, int32_t i) {
  const double* c = x.center_dir;
  if (c[0] == 0.0 && c[1] == 0.0 && c[2] == 0.0 && x.fov_x == 0.0 && x.fov_y == 0.0)
    return RR_OK;
  if (!finite3(c) || !std::isfinite(x.fov_x) || !std::isfinite(x.fov_y))
    return fail(RR_ERR_NONFINITE, "bundle %d: field-of-view record is not finite", i);
  const double c2 = (c[0] * c[0] + c[1] * c[1]) + c[2] * c[2];
  if (!(std::fabs(c2 - 1.0) <= 1e-9))
    return fail(RR_ERR_INVALID_ARG, "bundle %d: center_dir is not a unit vector", i);
  if (!(x.fov_x >= 0.0 && x.fov_x < M_PI) || !(x.fov_y >= 0.0 && x.fov_y < M_PI))
    return fail(RR_ERR_INVALID_ARG, "bundle %d: fields of view must lie in [0, pi)", i);
  if ((x.nx > 1 && !(x.fov_x > 0.0)) || (x.ny > 1 && !(x.fov_y > 0.0)))
    return fail(RR_ERR_INVALID_ARG,
                "bundle %d: a %d x %d map needs a positive fov on every axis with several rays",
                i, x.nx, x.ny);
  return RR_OK;
}

rr_status validate_trace(rr_tensor t, const rr_trace_params* tp, const rr_bundle* b, int32_t nb) {
  rr_status st = RR_OK;
  if (!t) return fail(RR_ERR_INVALID_ARG, "tensor is NULL");
  if (!tp) return fail(RR_ERR_INVALID_ARG, "trace params are NULL");
  if (nb < 0 || (nb > 0 && !b)) return fail(RR_ERR_INVALID_ARG, "bad bundle array");
  if (tp->precision != t->precision)
    return fail(RR_ERR_INVALID_ARG, "trace precision %d differs from the tensor's %d",
                tp->precision, t->precision);
  if (tp->quantity < RR_Q_KAPPA || tp->quantity > RR_Q_SCALAR)
    return fail(RR_ERR_INVALID_ARG, "unknown quantity %d", tp->quantity);
  if (tp->integral != RR_INTEGRAL_TRILINEAR && tp->integral != RR_INTEGRAL_NGP)
    return fail(RR_ERR_INVALID_ARG, "unknown integral %d", tp->integral);
  if (t->isw) {
    if (tp->quantity != RR_Q_SCALAR || tp->integral != RR_INTEGRAL_TRILINEAR)
      return fail(RR_ERR_INVALID_ARG,
                  "an ISW tensor is traced with RR_Q_SCALAR and the trilinear integral");
    if (t->content != 0 && t->content != 4)
      return fail(RR_ERR_INVALID_ARG, "the ISW tensor holds no ISW field");
  } else if (tp->quantity == RR_Q_SCALAR) {
    return fail(RR_ERR_INVALID_ARG, "RR_Q_SCALAR needs an ISW tensor (rr_build_isw_field)");
  } else if (t->method_a) {
    if (tp->quantity != RR_Q_KAPPA || tp->integral != RR_INTEGRAL_TRILINEAR)
      return fail(RR_ERR_UNSUPPORTED, "Method A gives kappa with the trilinear integral only");
  } else if (t->kind == RR_GRID_UNIFORM && t->content != 0 &&
             t->content != (tp->integral == RR_INTEGRAL_NGP ? 2 : 1))
    return fail(RR_ERR_INVALID_ARG,
                tp->integral == RR_INTEGRAL_NGP
                    ? "the NGP integral reads cell-centre records (rr_build_tidal_tensor_centres)"
                    : "the trilinear integral reads vertex records (rr_build_tidal_tensor)");
  if (!finite3(tp->observer)) return fail(RR_ERR_NONFINITE, "observer is not finite");
  const double h0 = t->box / (double)t->n;
  // lattice coordinates are 32-bit on the device, at the finest level of an
  // octree 2^kMaxLevel times the base-cell ones: keeping the observer and the
  // far end of every window within 2^(29 - L) base cells of the origin keeps
  // every coordinate below 2^30
  const int L = t->kind == RR_GRID_OCTREE ? rr::kMaxLevel : 0;
  const double cell_cap = (double)(1 << (29 - L));
  for (int k = 0; k < 3; ++k)
    if (std::fabs(tp->observer[k] / h0) > cell_cap)
      return fail(RR_ERR_INVALID_ARG, "observer is more than 2^%d cells from the origin", 29 - L);
  if (!std::isfinite(tp->kappa_scale)) return fail(RR_ERR_NONFINITE, "kappa_scale not finite");
  if (tp->log_stride < 0 || (tp->crossing_log && tp->log_stride == 0))
    return fail(RR_ERR_INVALID_ARG, "crossing_log needs log_stride > 0");
  for (int32_t i = 0; i < nb; ++i) {
    const rr_bundle& x = b[i];
    if (x.n_rays < 0 || x.ray_offset < 0)
      return fail(RR_ERR_INVALID_ARG, "bundle %d: negative size or offset", i);
    if (x.n_rays == 0) continue;
    if (!x.dir) return fail(RR_ERR_INVALID_ARG, "bundle %d: dir is NULL", i);
    if (x.nx <= 0 || x.ny <= 0 || (int64_t)x.nx * x.ny != x.n_rays)
      return fail(RR_ERR_INVALID_ARG, "bundle %d: nx*ny (%d*%d) != n_rays (%lld)", i, x.nx, x.ny,
                  (long long)x.n_rays);
    if (!std::isfinite(x.chi_s) || !std::isfinite(x.chi_hi) || !std::isfinite(x.chi_lo))
      return fail(RR_ERR_NONFINITE, "bundle %d: chi values must be finite", i);
    st = validate_fov(x, i);
    if (st != RR_OK) return st;
    if (!(x.chi_s > 0.0)) return fail(RR_ERR_INVALID_ARG, "bundle %d: chi_s must be > 0", i);
    if (!(0.0 <= x.chi_lo && x.chi_lo < x.chi_hi && x.chi_hi <= x.chi_s))
      return fail(RR_ERR_INVALID_ARG,
                  "bundle %d: need 0 <= chi_lo < chi_hi <= chi_s (got %g, %g, %g)", i, x.chi_lo,
                  x.chi_hi, x.chi_s);
    // a unit ray crosses at most sqrt(3) * window * 2^level planes (+3 at the ends)
    const double span = (x.chi_hi - x.chi_lo) / h0 * std::sqrt(3.0) * (double)(1 << L);
    if (x.chi_hi / h0 > cell_cap || span > (double)(1 << 30))
      return fail(RR_ERR_INVALID_ARG, "bundle %d: chi window reaches more than 2^%d cells", i,
                  29 - L);
  }
  return RR_OK;
}

// Launch order of the bundles: as given, or (persistent launches)
// longest-processing-time first, the chi window setting the steps per ray.
// A stable insertion sort on the caller's index array (no allocation).
void launch_order(const rr_bundle* b, int32_t nb, int persistent, int32_t* order) {
  for (int32_t i = 0; i < nb; ++i) order[i] = i;
  if (!persistent) return;
  for (int32_t i = 1; i < nb; ++i) {
    const int32_t v = order[i];
    const double len = b[v].chi_hi - b[v].chi_lo;
    int32_t j = i - 1;
    for (; j >= 0 && (b[order[j]].chi_hi - b[order[j]].chi_lo) < len; --j) order[j + 1] = order[j];
    order[j + 1] = v;
  }
}

// One bundle-table entry in base-cell units; returns the tile count after it.
int64_t table_entry(rr_tensor t, const rr_bundle& x, int64_t tiles, rr::DevBundle* d) {
  const double h0 = t->box / (double)t->n;
  d->dir = x.dir;
  d->ray_offset = x.ray_offset;
  d->n_rays = x.n_rays;
  d->nx = x.n_rays ? x.nx : 0;
  d->ny = x.n_rays ? x.ny : 0;
  d->tiles_x = (d->nx + 7) / 8;
  d->tiles_y = (d->ny + 7) / 8;
  d->tile_begin = tiles;
  d->chi_s = x.chi_s / h0;
  d->chi_hi = x.chi_hi / h0;
  d->chi_lo = x.chi_lo / h0;
  return tiles + (int64_t)d->tiles_x * d->tiles_y;
}

// Release the least recently used bundle table that no graph reads, after
// the last launch that read it has finished.
rr_status evict_table(rr_plan p) {
  auto victim = p->tables.end();
  for (auto it = p->tables.begin(); it != p->tables.end(); ++it)
    if (!it->in_graph && !it->captured &&
        (victim == p->tables.end() || it->last_use < victim->last_use))
      victim = it;
  if (victim == p->tables.end())
    return fail(RR_ERR_CAPACITY, "all %zu bundle tables of the plan are held by its graph",
                p->tables.size());
  RR_HIP(hipEventSynchronize(victim->used), "bundle table release (wait)");
  RR_HIP(hipFree(victim->dev), "bundle table release");
  (void)hipEventDestroy(victim->used);
  p->tables.erase(victim);
  return RR_OK;
}

// After the launches of a call: the table's event marks its last reader
// (inside a capture the graph holds the table instead).
rr_status table_used(CachedTable* c, hipStream_t s) {
  if (!capturing(s)) RR_HIP(hipEventRecord(c->used, s), "bundle table event");
  return RR_OK;
}

// Find or upload the device bundle table for (bundles, grid unit).
rr_status get_table(rr_plan p, rr_tensor t, const rr_bundle* b, int32_t nb, int persistent,
                    hipStream_t s, CachedTable** out) {
  const bool cap = capturing(s);
  for (auto& c : p->tables) {
    if (c.n == t->n && c.box == t->box && c.persistent_order == persistent &&
        (int32_t)c.key.size() == nb &&
        (nb == 0 || std::memcmp(c.key.data(), b, sizeof(rr_bundle) * nb) == 0)) {
      c.last_use = ++p->clock;
      c.captured |= cap;
      *out = &c;
      return RR_OK;
    }
  }
  if (cap)
    return fail(RR_ERR_CAPACITY,
                "bundle table not uploaded before graph capture: run the call once first");
  if (p->tables.size() >= kMaxTables) {
    rr_status st = evict_table(p);
    if (st != RR_OK) return st;
  }
  std::vector<int32_t> order(nb);
  launch_order(b, nb, persistent, order.data());
  std::vector<rr::DevBundle> host(std::max(nb, 1));
  int64_t tiles = 0;
  for (int32_t k = 0; k < nb; ++k) tiles = table_entry(t, b[order[k]], tiles, &host[k]);
  CachedTable c;
  c.key.assign(b, b + nb);
  c.n = t->n;
  c.box = t->box;
  c.persistent_order = persistent;
  c.n_tiles = tiles;
  c.last_use = ++p->clock;
  RR_HIP(hipEventCreateWithFlags(&c.used, hipEventDisableTiming), "bundle table event");
  hipError_t e = hipMalloc((void**)&c.dev, sizeof(rr::DevBundle) * host.size());
  if (e != hipSuccess) {
    (void)hipEventDestroy(c.used);
    return fail(RR_ERR_OOM, "bundle table: %s", hipGetErrorString(e));
  }
  e = hipMemcpy(c.dev, host.data(), sizeof(rr::DevBundle) * host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(c.dev);
    (void)hipEventDestroy(c.used);
    return hip_fail(e, "bundle table upload");
  }
  p->tables.push_back(std::move(c));
  *out = &p->tables.back();
  return RR_OK;
}

constexpr int32_t kMaxSources = 4096;

rr_status validate_sources(const double* chi_src, int32_t n_src) {
  if (!chi_src) return fail(RR_ERR_INVALID_ARG, "chi_src is NULL");
  if (n_src < 1 || n_src > kMaxSources)
    return fail(RR_ERR_INVALID_ARG, "n_src %d outside [1, %d]", n_src, kMaxSources);
  for (int32_t j = 0; j < n_src; ++j) {
    if (!std::isfinite(chi_src[j])) return fail(RR_ERR_NONFINITE, "chi_src[%d] is not finite", j);
    if (!(chi_src[j] > 0.0)) return fail(RR_ERR_INVALID_ARG, "chi_src[%d] must be > 0", j);
    if (j > 0 && !(chi_src[j] < chi_src[j - 1]))
      return fail(RR_ERR_INVALID_ARG, "chi_src must be strictly decreasing (index %d)", j);
  }
  return RR_OK;
}

// Find or upload the device copy of a source list in the tensor's cell units.
rr_status get_sources(rr_plan p, rr_tensor t, const double* chi_src, int32_t n_src,
                      hipStream_t s, const double** out) {
  const double h0 = t->box / (double)t->n;
  for (auto& c : p->sources) {
    if (c.h0 == h0 && (int32_t)c.key.size() == n_src &&
        std::memcmp(c.key.data(), chi_src, sizeof(double) * n_src) == 0) {
      *out = c.dev;
      return RR_OK;
    }
  }
  if (capturing(s))
    return fail(RR_ERR_CAPACITY,
                "source list not uploaded before graph capture: run the call once first");
  if (p->sources.size() >= 64) return fail(RR_ERR_CAPACITY, "plan holds 64 source lists already");
  CachedSources c;
  c.key.assign(chi_src, chi_src + n_src);
  c.h0 = h0;
  std::vector<double> host(n_src);
  for (int32_t j = 0; j < n_src; ++j) host[j] = chi_src[j] / h0;
  hipError_t e = hipMalloc((void**)&c.dev, sizeof(double) * n_src);
  if (e != hipSuccess) return fail(RR_ERR_OOM, "source list: %s", hipGetErrorString(e));
  e = hipMemcpy(c.dev, host.data(), sizeof(double) * n_src, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(c.dev);
    return hip_fail(e, "source list upload");
  }
  p->sources.push_back(std::move(c));
  *out = p->sources.back().dev;
  return RR_OK;
}

}  // namespace

}  // extern "C"

namespace {

rr_status launch_trace(rr_plan p, rr_tensor t, const rr_trace_params* tp, const rr_bundle* bundles,
                       int32_t n_bundles, void* kappa, float* kappa_comp, int32_t* ray_status,
                       hipStream_t hs, int persistent, int block, int waves_per_cu,
                       const double* src = nullptr, int32_t n_src = 0, double* pieces = nullptr,
                       int passes = 1);

const TunedShape* find_tuned(rr_plan p, const rr_bundle* b, int32_t nb) {
  for (const auto& x : p->tuned)
    if ((int32_t)x.key.size() == nb &&
        (nb == 0 || std::memcmp(x.key.data(), b, sizeof(rr_bundle) * nb) == 0))
      return &x;
  return nullptr;
}

}  // namespace

extern "C" {

rr_status rr_trace_rays(rr_plan p, rr_tensor t, const rr_trace_params* tp, const rr_bundle* bundles,
                        int32_t n_bundles, void* kappa, float* kappa_comp, int32_t* ray_status,
                        rr_stream s) {
  if (!p) return fail(RR_ERR_INVALID_ARG, "plan is NULL");
  rr_status st = validate_trace(t, tp, bundles, n_bundles);
  if (st != RR_OK) return st;
  if (!kappa) return fail(RR_ERR_INVALID_ARG, "kappa is NULL");
  if (kappa_comp && t->precision != RR_PREC_FP32_KAHAN)
    return fail(RR_ERR_INVALID_ARG, "kappa_comp is only used by FP32_KAHAN");
  const hipStream_t hs = (hipStream_t)s;
  int persistent = tp->persistent < 0 ? p->prefer_persistent : (tp->persistent ? 1 : 0);
  int block = 256, waves_per_cu = p->waves_per_cu, passes = 1;
  if (tp->persistent < 0) {
    if (const TunedShape* ts = find_tuned(p, bundles, n_bundles)) {
      persistent = ts->persistent;
      block = ts->block;
      waves_per_cu = ts->waves_per_cu;
      passes = ts->passes;
    }
  }
  return launch_trace(p, t, tp, bundles, n_bundles, kappa, kappa_comp, ray_status, hs, persistent,
                      block, waves_per_cu, nullptr, 0, nullptr, passes);
}

rr_status rr_trace_rays_sources(rr_plan p, rr_tensor t, const rr_trace_params* tp,
                                const rr_bundle* bundles, int32_t n_bundles,
                                const double* chi_src, int32_t n_src, void* moments,
                                double* pieces, int32_t* ray_status, rr_stream s) {
  if (!p) return fail(RR_ERR_INVALID_ARG, "plan is NULL");
  rr_status st = validate_trace(t, tp, bundles, n_bundles);
  if (st != RR_OK) return st;
  st = validate_sources(chi_src, n_src);
  if (st != RR_OK) return st;
  bool any_rays = false;
  for (int32_t i = 0; i < n_bundles; ++i) any_rays |= bundles[i].n_rays > 0;
  if (any_rays && !moments) return fail(RR_ERR_INVALID_ARG, "moments is NULL");
  if (any_rays && !pieces) return fail(RR_ERR_INVALID_ARG, "pieces is NULL");
  if (t->method_a || t->isw || tp->integral != RR_INTEGRAL_TRILINEAR)
    return fail(RR_ERR_UNSUPPORTED,
                "the many-source walk integrates the tidal tensor with the trilinear integral");
  const hipStream_t hs = (hipStream_t)s;
  const double* src = nullptr;
  st = get_sources(p, t, chi_src, n_src, hs, &src);
  if (st != RR_OK) return st;
  int persistent = tp->persistent < 0 ? p->prefer_persistent : (tp->persistent ? 1 : 0);
  int block = 256, waves_per_cu = p->waves_per_cu, passes = 1;
  if (tp->persistent < 0) {
    if (const TunedShape* ts = find_tuned(p, bundles, n_bundles)) {
      persistent = ts->persistent;
      block = ts->block;
      waves_per_cu = ts->waves_per_cu;
      passes = ts->passes;
    }
  }
  return launch_trace(p, t, tp, bundles, n_bundles, moments, nullptr, ray_status, hs, persistent,
                      block, waves_per_cu, src, n_src, pieces, passes);
}

rr_status rr_kappa_from_pieces(rr_plan p, rr_tensor t, const double* chi_src, int32_t n_src,
                               int64_t n_rays, const void* moments, const double* pieces,
                               double* kappa, rr_stream s) {
  if (!p) return fail(RR_ERR_INVALID_ARG, "plan is NULL");
  if (!t) return fail(RR_ERR_INVALID_ARG, "tensor is NULL");
  rr_status st = validate_sources(chi_src, n_src);
  if (st != RR_OK) return st;
  if (n_rays < 0) return fail(RR_ERR_INVALID_ARG, "n_rays is negative");
  if (n_rays == 0) return RR_OK;
  if (!moments || !pieces || !kappa)
    return fail(RR_ERR_INVALID_ARG, "moments, pieces and kappa must be non-NULL");
  const hipStream_t hs = (hipStream_t)s;
  const double* src = nullptr;
  st = get_sources(p, t, chi_src, n_src, hs, &src);
  if (st != RR_OK) return st;
  RR_HIP(rr::launch_kappa_from_pieces(t->precision, moments, pieces, src, n_src, n_rays, kappa,
                                      hs),
         "kappa from pieces launch");
  return RR_OK;
}

rr_status rr_rays_vertex_box(rr_plan p, rr_tensor t, const rr_trace_params* tp,
                             const rr_bundle* bundles, int32_t n_bundles, int32_t lo[3],
                             int32_t size[3], rr_stream s) {
  if (!p) return fail(RR_ERR_INVALID_ARG, "plan is NULL");
  if (!lo || !size) return fail(RR_ERR_INVALID_ARG, "box pointers are NULL");
  rr_status st = validate_trace(t, tp, bundles, n_bundles);
  if (st != RR_OK) return st;
  if (t->kind != RR_GRID_UNIFORM) return fail(RR_ERR_UNSUPPORTED, "box builds are for uniform grids");
  const hipStream_t hs = (hipStream_t)s;
  if (capturing(hs)) return fail(RR_ERR_CAPACITY, "the ray box is computed outside captures");
  CachedTable* tab = nullptr;
  st = get_table(p, t, bundles, n_bundles, 0, hs, &tab);
  if (st != RR_OK) return st;
  int* dev = reinterpret_cast<int*>(reinterpret_cast<char*>(p->queue) + 64);
  int host[6] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN};
  RR_HIP(hipMemcpyAsync(dev, host, sizeof(host), hipMemcpyHostToDevice, hs), "bounds init");
  rr::TraceArgs a{};
  a.bundles = tab->dev;
  a.n_bundles = n_bundles;
  a.n_tiles = tab->n_tiles;
  const double h0 = t->box / (double)t->n;
  for (int k = 0; k < 3; ++k) a.o[k] = tp->observer[k] / h0;
  a.n = t->n;
  RR_HIP(rr::launch_ray_bounds(a, dev, hs), "ray bounds launch");
  st = table_used(tab, hs);
  if (st != RR_OK) return st;
  RR_HIP(hipMemcpyAsync(host, dev, sizeof(host), hipMemcpyDeviceToHost, hs), "bounds read");
  RR_HIP(hipStreamSynchronize(hs), "bounds sync");
  const int n = t->n;
  for (int k = 0; k < 3; ++k) {
    if (host[k] > host[3 + k]) {   // no traced ray
      lo[k] = 0;
      size[k] = 0;
      continue;
    }
    // cells of the walk: one slab beyond the end points either way (the slab
    // rule at a plane); vertices: their lower and upper corners, plus one
    // layer of margin
    const int64_t a0 = (int64_t)host[k] - 2, a1 = (int64_t)host[3 + k] + 3;   // [a0, a1)
    if (a1 - a0 >= n || t->boundary == RR_BOUNDARY_OPEN) {
      const int64_t c0 = t->boundary == RR_BOUNDARY_OPEN ? std::max<int64_t>(a0, 0) : 0;
      const int64_t c1 = t->boundary == RR_BOUNDARY_OPEN ? std::min<int64_t>(a1, n) : n;
      lo[k] = (int32_t)c0;
      size[k] = (int32_t)std::max<int64_t>(c1 - c0, 0);
    } else {
      lo[k] = (int32_t)a0;
      size[k] = (int32_t)(a1 - a0);
    }
  }
  return RR_OK;
}

rr_status rr_plan_autotune(rr_plan p, rr_tensor t, const rr_trace_params* tp,
                           const rr_bundle* bundles, int32_t n_bundles, rr_stream s) {
  if (!p) return fail(RR_ERR_INVALID_ARG, "plan is NULL");
  rr_status st = validate_trace(t, tp, bundles, n_bundles);
  if (st != RR_OK) return st;
  const hipStream_t hs = (hipStream_t)s;
  if (capturing(hs)) return fail(RR_ERR_CAPACITY, "autotuning cannot run inside a capture");
  int64_t nr = 0;
  for (int32_t i = 0; i < n_bundles; ++i)
    nr = std::max<int64_t>(nr, bundles[i].ray_offset + bundles[i].n_rays);
  if (nr == 0) return RR_OK;
  const size_t kb = (size_t)nr * (t->precision == RR_PREC_FP32_KAHAN ? 4 : 8);
  void *kap = nullptr, *comp = nullptr, *stat = nullptr;
  hipError_t e = hipMalloc(&kap, kb);
  if (e == hipSuccess) e = hipMalloc(&comp, (size_t)nr * 4);
  if (e == hipSuccess) e = hipMalloc(&stat, (size_t)nr * 4);
  if (e != hipSuccess) {
    if (kap) (void)hipFree(kap);
    if (comp) (void)hipFree(comp);
    return fail(RR_ERR_OOM, "autotune scratch: %s", hipGetErrorString(e));
  }
  rr_trace_params q = *tp;
  q.crossing_hash = nullptr;
  q.crossing_count = nullptr;
  q.crossing_log = nullptr;
  q.log_stride = 0;
  struct Cand { int persistent, block, waves, passes; };
  const Cand cands[] = {{0, 256, 0, 1},   {0, 64, 0, 1},    {1, 256, 8, 1},  {1, 256, 16, 1},
                        {1, 256, 32, 1},  {0, 256, 0, 4},   {0, 256, 0, 16}, {0, 64, 0, 16},
                        {1, 256, 16, 16}, {0, 256, 0, 32},  {1, 256, 16, 32}, {0, 256, 0, 64},
                        {1, 256, 16, 64}};
  hipEvent_t e0, e1;
  RR_HIP(hipEventCreate(&e0), "event");
  RR_HIP(hipEventCreate(&e1), "event");
  TunedShape best;
  best.key.assign(bundles, bundles + n_bundles);
  best.ms = 1e30f;
  for (const Cand& c : cands) {
    float ms_best = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {   // first run also uploads the bundle table
      RR_HIP(hipEventRecord(e0, hs), "event record");
      st = launch_trace(p, t, &q, bundles, n_bundles, kap, (float*)comp, (int32_t*)stat, hs,
                        c.persistent, c.block, c.waves ? c.waves : p->waves_per_cu, nullptr, 0,
                        nullptr, c.passes);
      if (st != RR_OK) break;
      RR_HIP(hipEventRecord(e1, hs), "event record");
      RR_HIP(hipEventSynchronize(e1), "event sync");
      float ms = 0.0f;
      RR_HIP(hipEventElapsedTime(&ms, e0, e1), "event time");
      if (rep > 0) ms_best = std::min(ms_best, ms);
    }
    if (st != RR_OK) break;
    if (ms_best < best.ms) {
      best.ms = ms_best;
      best.persistent = c.persistent;
      best.block = c.block;
      best.waves_per_cu = c.waves ? c.waves : p->waves_per_cu;
      best.passes = c.passes;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(kap);
  (void)hipFree(comp);
  (void)hipFree(stat);
  if (st != RR_OK) return st;
  for (auto& x : p->tuned)
    if (x.key.size() == best.key.size() &&
        std::memcmp(x.key.data(), best.key.data(), sizeof(rr_bundle) * x.key.size()) == 0) {
      x = best;
      return RR_OK;
    }
  p->tuned.push_back(best);
  return RR_OK;
}

rr_status rr_plan_set_shape(rr_plan p, const rr_bundle* bundles, int32_t n_bundles,
                            int32_t persistent, int32_t block, int32_t waves_per_cu,
                            int32_t passes) {
  if (!p) return fail(RR_ERR_INVALID_ARG, "plan is NULL");
  if (n_bundles < 0 || (n_bundles > 0 && !bundles))
    return fail(RR_ERR_INVALID_ARG, "bad bundle array");
  if (persistent != 0 && persistent != 1)
    return fail(RR_ERR_INVALID_ARG, "persistent must be 0 or 1");
  if (block != 64 && block != 256) return fail(RR_ERR_INVALID_ARG, "block must be 64 or 256");
  if (waves_per_cu < 1 || waves_per_cu > 32)
    return fail(RR_ERR_INVALID_ARG, "waves_per_cu outside [1, 32]");
  if (passes < 1 || passes > 64) return fail(RR_ERR_INVALID_ARG, "passes outside [1, 64]");
  TunedShape ts;
  ts.key.assign(bundles, bundles + n_bundles);
  ts.persistent = persistent;
  ts.block = persistent ? 256 : block;
  ts.waves_per_cu = waves_per_cu;
  ts.passes = passes;
  ts.ms = 0.0f;
  for (auto& x : p->tuned)
    if (x.key.size() == ts.key.size() &&
        (ts.key.empty() ||
         std::memcmp(x.key.data(), ts.key.data(), sizeof(rr_bundle) * x.key.size()) == 0)) {
      x = ts;
      return RR_OK;
    }
  p->tuned.push_back(ts);
  return RR_OK;
}

rr_status rr_plan_tuned_shape(rr_plan p, const rr_bundle* bundles, int32_t n_bundles,
                              int32_t* persistent, int32_t* block, int32_t* waves_per_cu,
                              int32_t* passes, float* ms) {
  if (!p) return fail(RR_ERR_INVALID_ARG, "plan is NULL");
  const TunedShape* ts = find_tuned(p, bundles, n_bundles);
  if (!ts) return fail(RR_ERR_INVALID_ARG, "no tuned shape for this bundle set");
  if (persistent) *persistent = ts->persistent;
  if (block) *block = ts->block;
  if (waves_per_cu) *waves_per_cu = ts->waves_per_cu;
  if (passes) *passes = ts->passes;
  if (ms) *ms = ts->ms;
  return RR_OK;
}

}  // extern "C"

namespace {

// Everything a march launch takes from the tensor, the trace parameters and
// the outputs (the bundle table, queue and pass state are set by the caller).
void march_args(rr_tensor t, const rr_trace_params* tp, void* kappa, float* kappa_comp,
                int32_t* ray_status, rr::TraceArgs* a) {
  const double h0 = t->box / (double)t->n;
  for (int k = 0; k < 3; ++k) a->o[k] = tp->observer[k] / h0;
  a->kappa_scale = tp->kappa_scale;
  a->n = t->n;
  a->open = t->boundary == RR_BOUNDARY_OPEN;
  a->quantity = tp->quantity;
  a->integral = tp->integral;
  a->mode = t->method_a ? 2 : (tp->integral == RR_INTEGRAL_NGP ? 1 : 0);
  if (t->isw) {
    // int Q dchi~ in base-cell units times h0: the integral in box units
    a->mode = 4;
    a->kappa_scale = tp->kappa_scale * h0;
  }
  a->max_crossings = tp->max_crossings;
  a->kappa = kappa;
  a->kappa_comp = kappa_comp;
  a->status = ray_status;
  a->hash = tp->crossing_hash;
  a->count = tp->crossing_count;
  a->log = tp->crossing_log;
  a->log_stride = tp->log_stride;
  a->pause_chi = -INFINITY;
}

rr_status launch_trace(rr_plan p, rr_tensor t, const rr_trace_params* tp, const rr_bundle* bundles,
                       int32_t n_bundles, void* kappa, float* kappa_comp, int32_t* ray_status,
                       hipStream_t hs, int persistent, int block, int waves_per_cu,
                       const double* src, int32_t n_src, double* pieces, int passes) {
  rr_status st;
  CachedTable* tab = nullptr;
  st = get_table(p, t, bundles, n_bundles, persistent, hs, &tab);
  if (st != RR_OK) return st;
  if (tab->n_tiles == 0) return RR_OK;

  rr::TraceArgs a{};
  march_args(t, tp, kappa, kappa_comp, ray_status, &a);
  a.bundles = tab->dev;
  a.n_bundles = n_bundles;
  a.n_tiles = tab->n_tiles;
  const double h0 = t->box / (double)t->n;
  if (src) {
    a.mode = 3;
    a.src = src;
    a.n_src = n_src;
    a.pieces = pieces;
  }
  a.queue = p->queue;
  const int grid_waves = p->cu_count * waves_per_cu;
  // A long window can be marched in passes: each pass stops every ray on the
  // first face at or below the pass's chi boundary and the next pass resumes
  // on that face (the same pieces in the same order: the results are
  // unchanged).  Rays that drift apart in a long march (one lane through a
  // refined halo, its neighbours past it) start each pass side by side again.
  // Only without debug outputs or a crossing limit, and with the Kahan state
  // kept in memory between passes.
  const bool debug = tp->crossing_hash || tp->crossing_count || tp->crossing_log;
  if (passes > 1 && (debug || tp->max_crossings > 0 ||
                     (t->precision == RR_PREC_FP32_KAHAN && !kappa_comp && !src)))
    passes = 1;
  double chi_top = 0.0, chi_bot = INFINITY;
  if (passes > 1) {
    int64_t nr = 0;
    for (int32_t i = 0; i < n_bundles; ++i) {
      if (bundles[i].n_rays == 0) continue;
      nr = std::max<int64_t>(nr, bundles[i].ray_offset + bundles[i].n_rays);
      chi_top = std::max(chi_top, bundles[i].chi_hi / h0);
      chi_bot = std::min(chi_bot, bundles[i].chi_lo / h0);
    }
    if (nr > p->resume_cap) {
      if (capturing(hs))
        return fail(RR_ERR_CAPACITY, "split march not prepared before graph capture: run the "
                                     "call once first");
      if (p->resume) (void)hipFree(p->resume);
      p->resume = nullptr;
      p->resume_cap = 0;
      hipError_t e = hipMalloc((void**)&p->resume, sizeof(double) * (size_t)nr);
      if (e != hipSuccess) return fail(RR_ERR_OOM, "pass state: %s", hipGetErrorString(e));
      p->resume_cap = nr;
    }
    RR_HIP(rr::launch_fill(p->resume, nr, INFINITY, hs), "pass state init");
    a.resume = p->resume;
  }
  for (int pass = 0; pass < passes; ++pass) {
    // pass boundaries at equal steps in chi over the bundles' windows; every
    // lane of a wave restarts from the same boundary, so neighbouring rays
    // stay in step (and share their cells' records) through the window
    if (passes > 1)
      a.pause_chi = pass == passes - 1 ? -INFINITY
                                       : chi_top - (chi_top - chi_bot) * (pass + 1) / passes;
    if (persistent) RR_HIP(rr::launch_queue_reset(p->queue, hs), "queue reset");
    if (t->kind == RR_GRID_UNIFORM) {
      RR_HIP(rr::launch_march_uniform(t->precision, t->data, a, persistent, block, grid_waves,
                                      hs),
             "march launch");
    } else {
      RR_HIP(t->oct->march(a, persistent, grid_waves, hs), "octree march launch");
    }
  }
  return table_used(tab, hs);
}

}  // namespace

extern "C" {

rr_status rr_trace_rays_adjoint(rr_plan p, rr_tensor t, const rr_field_desc* f,
                                const rr_trace_params* tp, const rr_bundle* bundles,
                                int32_t n_bundles, const float* dl_dkappa, float* dl_dphi,
                                rr_stream s) {
  if (!p) return fail(RR_ERR_INVALID_ARG, "plan is NULL");
  rr_status st = validate_trace(t, tp, bundles, n_bundles);
  if (st != RR_OK) return st;
  st = validate_field(f);
  if (st != RR_OK) return st;
  if (t->kind != RR_GRID_UNIFORM || f->kind != RR_GRID_UNIFORM)
    return fail(RR_ERR_UNSUPPORTED, "the adjoint is implemented for uniform grids only");
  if (t->boundary != RR_BOUNDARY_PERIODIC)
    return fail(RR_ERR_UNSUPPORTED, "the adjoint is implemented for periodic grids only");
  if (t->precision != RR_PREC_FP32_KAHAN || f->dtype != RR_F32)
    return fail(RR_ERR_UNSUPPORTED, "the adjoint takes an FP32 field and an FP32 tensor");
  if (tp->quantity != RR_Q_KAPPA || tp->integral != RR_INTEGRAL_TRILINEAR || t->method_a ||
      t->isw)
    return fail(RR_ERR_UNSUPPORTED,
                "the adjoint is implemented for Method B kappa with the trilinear integral");
  if (f->field != RR_FIELD_PHI) return fail(RR_ERR_INVALID_ARG, "the adjoint needs a potential");
  if (f->n_base != t->n) return fail(RR_ERR_INVALID_ARG, "field and tensor grids differ");
  if (!dl_dkappa || !dl_dphi) return fail(RR_ERR_INVALID_ARG, "gradient pointers are NULL");
  const hipStream_t hs = (hipStream_t)s;
  CachedTable* tab = nullptr;
  st = get_table(p, t, bundles, n_bundles, 0, hs, &tab);
  if (st != RR_OK) return st;
  const int64_t nv = (int64_t)t->n * t->n * t->n;
  if (!t->grad) {
    if (capturing(hs)) return fail(RR_ERR_CAPACITY, "first adjoint call inside a capture");
    hipError_t e = hipMalloc(&t->grad, (size_t)nv * 8 * sizeof(float));
    if (e != hipSuccess) return fail(RR_ERR_OOM, "adjoint workspace: %s", hipGetErrorString(e));
  }
  rr::TraceArgs a{};
  a.bundles = tab->dev;
  a.n_bundles = n_bundles;
  a.n_tiles = tab->n_tiles;
  const double h0 = t->box / (double)t->n;
  for (int k = 0; k < 3; ++k) a.o[k] = tp->observer[k] / h0;
  a.kappa_scale = tp->kappa_scale;
  a.n = t->n;
  a.open = 0;
  a.quantity = RR_Q_KAPPA;
  a.max_crossings = tp->max_crossings;
  RR_HIP(rr::launch_adjoint_uniform(a, dl_dkappa, (float*)t->grad, dl_dphi, hs), "adjoint launch");
  return table_used(tab, hs);
}

rr_status rr_graph_begin(rr_plan p, rr_stream s) {
  if (!p) return fail(RR_ERR_INVALID_ARG, "plan is NULL");
  if (!s) return fail(RR_ERR_INVALID_ARG, "graph capture needs a non-default stream");
  if (capturing((hipStream_t)s)) return fail(RR_ERR_CAPACITY, "stream is already capturing");
  for (auto& c : p->tables) c.captured = false;
  RR_HIP(hipStreamBeginCapture((hipStream_t)s, hipStreamCaptureModeThreadLocal), "begin capture");
  return RR_OK;
}

rr_status rr_graph_end(rr_plan p, rr_stream s) {
  if (!p) return fail(RR_ERR_INVALID_ARG, "plan is NULL");
  hipGraph_t g = nullptr;
  RR_HIP(hipStreamEndCapture((hipStream_t)s, &g), "end capture");
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = g;
  // the new graph holds exactly the tables its capture used
  for (auto& c : p->tables) {
    c.in_graph = c.captured;
    c.captured = false;
  }
  RR_HIP(hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0), "graph instantiate");
  return RR_OK;
}

rr_status rr_graph_launch(rr_plan p, rr_stream s) {
  if (!p) return fail(RR_ERR_INVALID_ARG, "plan is NULL");
  if (!p->exec) return fail(RR_ERR_INVALID_ARG, "no graph captured on this plan");
  RR_HIP(hipGraphLaunch(p->exec, (hipStream_t)s), "graph launch");
  // the graph's tables are released only after this replay has finished
  for (auto& c : p->tables)
    if (c.in_graph) RR_HIP(hipEventRecord(c.used, (hipStream_t)s), "bundle table event");
  return RR_OK;
}

}  // extern "C"

extern "C" {

rr_status rr_trace_rays_noalloc(rr_tensor t, const rr_trace_params* tp, const rr_bundle* bundles,
                                int32_t n_bundles, void* kappa, float* kappa_comp,
                                int32_t* ray_status, rr_stream s) {
  rr_status st = validate_trace(t, tp, bundles, n_bundles);
  if (st != RR_OK) return st;
  if (!kappa) return fail(RR_ERR_INVALID_ARG, "kappa is NULL");
  if (kappa_comp && t->precision != RR_PREC_FP32_KAHAN)
    return fail(RR_ERR_INVALID_ARG, "kappa_comp is only used by FP32_KAHAN");
  if (n_bundles > rr::kNoallocMaxBundles)
    return fail(RR_ERR_CAPACITY,
                "rr_trace_rays_noalloc takes at most %d bundles (its fixed device table); got %d",
                rr::kNoallocMaxBundles, n_bundles);
  const hipStream_t hs = (hipStream_t)s;
  void* queue = nullptr;
  rr::DevBundle* table = nullptr;
  RR_HIP(rr::noalloc_scratch(&queue, &table), "scratch array address");
  const int persistent = tp->persistent > 0 ? 1 : 0;
  // the table goes to the scratch array in chunks built on the stack
  int32_t order[rr::kNoallocMaxBundles];
  launch_order(bundles, n_bundles, persistent, order);
  constexpr int kChunk = 48;
  rr::DevBundle chunk[kChunk];
  int64_t tiles = 0;
  for (int32_t k = 0; k < n_bundles; k += kChunk) {
    const int m = std::min<int32_t>(kChunk, n_bundles - k);
    for (int i = 0; i < m; ++i) tiles = table_entry(t, bundles[order[k + i]], tiles, &chunk[i]);
    RR_HIP(rr::launch_put_bundles(table + k, chunk, m, hs), "bundle table launch");
  }
  if (tiles == 0) return RR_OK;
  rr::TraceArgs a{};
  march_args(t, tp, kappa, kappa_comp, ray_status, &a);
  a.bundles = table;
  a.n_bundles = n_bundles;
  a.n_tiles = tiles;
  a.queue = static_cast<unsigned long long*>(queue);
  int dev = 0, cus = 0;
  RR_HIP(hipGetDevice(&dev), "hipGetDevice");
  RR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
  const int grid_waves = cus * 16;
  if (persistent) RR_HIP(rr::launch_queue_reset(a.queue, hs), "queue reset");
  if (t->kind == RR_GRID_UNIFORM) {
    RR_HIP(rr::launch_march_uniform(t->precision, t->data, a, persistent, 256, grid_waves, hs),
           "march launch");
  } else {
    RR_HIP(t->oct->march(a, persistent, grid_waves, hs), "octree march launch");
  }
  return RR_OK;
}

}  // extern "C"
