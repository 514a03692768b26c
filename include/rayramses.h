/*
 * rayramses.h -- C ABI of the MI355X (gfx950) Method-B weak-lensing ray tracer.
 *
 * The library integrates, along straight rays from a source at comoving
 * distance chi_s to an observer, the convergence
 *     kappa = int g(chi_s, chi) [tr T - n^T T n] dchi,  g = chi (chi_s - chi) / chi_s,
 * where T = d_a d_b Phi is the tidal tensor of the potential (RAY-RAMSES,
 * arXiv:1601.02012, Sec. IV A Eq. (kappa), Sec. IV B Eqs. (Iclensing),
 * (n1n1), (n2n2), Sec. IV C Eq. (tidalexample)).  The integral is split into
 * one piece per crossed cell (Eqs. (sumIc), (Ic)); inside a cell the integrand
 * is the trilinear reconstruction from the cell's eight vertex values
 * (Eq. trilinear_int), and the vertex values are interpolated from cell
 * centres (Sec. III H; Eqs. (alphac3d), (alphaf3d) at refinement boundaries).
 *
 * Conventions shared by every entry point
 *  - Pointers named "device" are HIP device pointers owned by the caller; the
 *    library never frees them.  "host" pointers are read before the call
 *    returns.  Opaque handles (rr_tensor, rr_plan) are owned by the library and
 *    released by their destroy call.
 *  - Calls taking a stream are asynchronous on it (NULL = the default stream)
 *    and allocate nothing once the plan has seen the bundle set (see
 *    rr_trace_rays).  Argument errors are detected on the host before any
 *    launch: the call returns a negative rr_status and rr_last_error() gives a
 *    message; nothing is enqueued.  Per-ray run-time conditions are reported
 *    in the optional ray_status array, never by aborting.
 *  - Lengths (box size, observer, chi values) share one unit, e.g. Mpc/h.
 *    Internally they are converted to base-cell units with the FP64 divisions
 *    h0 = L / n_base, o~ = o / h0, chi~ = chi / h0; a level-l cell has size
 *    2^-l.  kappa is unchanged by that rescaling.  Pass Phi already divided by
 *    c^2 (or set kappa_scale) -- the 1/c^2 of Eq. (kappa).
 *  - Arrays of cells are [z][y][x] with x fastest.  Tensor components are
 *    ordered xx, yy, zz, xy, xz, yz.
 *  - Crossing rule (the paper's Eq. (disttocross) picks the face reached
 *    first; ties and the ownership of points on faces are not stated there):
 *    with t_a(P) = (P - o~_a) * (1 / n_a) evaluated in FP64 without
 *    contraction, a ray is in slab m of axis a when t_exit < chi <= t_entry;
 *    the exit point is chi_B = max(chi_lo, t_exit,x, t_exit,y, t_exit,z), and
 *    every axis whose exit parameter equals chi_B is stepped together, so no
 *    zero-length piece is ever produced.
 */
#ifndef RAYRAMSES_H
#define RAYRAMSES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A hipStream_t. */
typedef struct ihipStream_t* rr_stream;

typedef enum {
  RR_OK = 0,
  RR_ERR_INVALID_ARG = -1,   /* null pointer, bad size, chi window not 0 <= lo < hi <= chi_s, ... */
  RR_ERR_UNSUPPORTED = -2,   /* valid request the library does not implement */
  RR_ERR_OOM = -3,           /* device allocation failed (only in create / first-use calls) */
  RR_ERR_HIP = -4,           /* a HIP runtime call failed; message holds hipGetErrorString */
  RR_ERR_OCTREE = -5,        /* octree malformed or not 2:1 balanced over faces, edges, corners */
  RR_ERR_DOMAIN = -6,        /* open-boundary grid too small for the stencil */
  RR_ERR_NONFINITE = -7,     /* non-finite observer / direction / chi */
  RR_ERR_CAPACITY = -8,      /* graph or bundle cache full, or capture in a state that forbids the call */
} rr_status;

typedef enum { RR_GRID_UNIFORM = 0, RR_GRID_OCTREE = 1 } rr_grid_kind;
/* RR_FIELD_PHI: the potential (Method B, Eq. kappa; also Method A's gradient
 * term).  RR_FIELD_DELTA: the density contrast of Method A's Poisson term
 * (Eq. kappa2), uniform grids only; a tensor created from it holds Method A
 * vertex fields (rr_build_method_a_fields).  RR_FIELD_PHI_DOT: the rate of
 * change of the potential for the ISW integrand (Sec. VII), uniform grids
 * only; a tensor created from it holds one scalar per vertex
 * (rr_build_isw_field); values are not read at creation. */
typedef enum { RR_FIELD_PHI = 0, RR_FIELD_DELTA = 1, RR_FIELD_PHI_DOT = 2 } rr_field_kind;
/* PERIODIC: the grid is one period of a replicated box (the paper's tiled
 * boxes, Sec. III B, with one realization).  OPEN: no wrap; cells on the two
 * outer layers only feed stencils, and a ray entering a cell outside
 * [2, n-3]^3 stops with RR_RAY_OUT_OF_DOMAIN. */
typedef enum { RR_BOUNDARY_PERIODIC = 0, RR_BOUNDARY_OPEN = 1 } rr_boundary;
/* FP64: tensor, vertex values and per-cell integrals in double.
 * FP32_KAHAN: tensor and per-cell integrals in float, kappa accumulated with
 * Kahan compensation; crossing parameters and chi bookkeeping stay FP64. */
typedef enum { RR_PREC_FP64 = 0, RR_PREC_FP32_KAHAN = 1 } rr_precision;
typedef enum { RR_F32 = 0, RR_F64 = 1 } rr_dtype;
/* Integrand: kappa (Eq. kappa), gamma_1 (Eq. gamma1), gamma_2 (Eq. gamma2 with
 * the mixed projection e_phi^T T e_theta); RR_Q_SCALAR: the vertex scalar of
 * an ISW tensor integrated with a constant kernel (the only quantity such a
 * tensor takes). */
typedef enum { RR_Q_KAPPA = 0, RR_Q_GAMMA1 = 1, RR_Q_GAMMA2 = 2, RR_Q_SCALAR = 3 } rr_quantity;
/* Per-cell integral: trilinear vertex reconstruction (Eq. Iclensing, the
 * tensor holds vertex records: rr_build_tidal_tensor) or the
 * nearest-grid-point value of the cell centre times the integrated kernel
 * (Eq. Iclensing_ngp, the tensor holds cell-centre records:
 * rr_build_tidal_tensor_centres; octree tensors keep both). */
typedef enum { RR_INTEGRAL_TRILINEAR = 0, RR_INTEGRAL_NGP = 1 } rr_integral;

/* Per-ray status written to ray_status. */
enum {
  RR_RAY_OK = 0,
  RR_RAY_OUT_OF_DOMAIN = 1,  /* open grid: left [2, n-3]^3 */
  RR_RAY_MAX_STEPS = 2,      /* hit rr_trace_params.max_crossings */
  RR_RAY_NONFINITE = 3,      /* the accumulated value is NaN or Inf */
  RR_RAY_BAD_DIRECTION = 4,  /* direction not finite or | |n|^2 - 1 | > 1e-9: ray skipped */
};

/* Description of one potential field (paper Sec. III A: a domain-level grid of
 * n_base^3 cells, refined into octs of 8 cells each, 2:1 balanced). */
typedef struct {
  int32_t kind;          /* rr_grid_kind */
  int32_t field;         /* rr_field_kind */
  int32_t boundary;      /* rr_boundary; octrees must be PERIODIC */
  int32_t dtype;         /* rr_dtype of values */
  int32_t n_base;        /* base cells per side, >= 4 (open: >= 6) */
  int32_t max_level;     /* octree: deepest level present (0..4); uniform: 0 */
  double box_size;       /* L: side of the base grid */
  /* device.  Uniform: n_base^3 values, [z][y][x].  Octree: one value per cell,
   * leaf and refined cells alike: base cells 0..n_base^3-1, then oct k owns
   * cells n_base^3 + 8k + (ix + 2 iy + 4 iz); octs in breadth-first order
   * (all octs of level l before those of level l+1, each level ordered by
   * parent cell index). */
  const void* values;
  const int32_t* child_oct;  /* device, octree: n_cells entries, oct index or -1 */
  int64_t n_cells;           /* octree: n_base^3 + 8 * n_octs */
} rr_field_desc;

typedef struct rr_tensor_s* rr_tensor;
typedef struct rr_plan_s* rr_plan;

/* Allocate the vertex-tensor storage for a field of this shape and precision.
 * Uniform: one 6-component tensor per vertex (vertex (i,j,k) is the lower
 * corner of cell (i,j,k)).  Octree: the child_oct array is copied to the host
 * once to lay out levels and to check 2:1 balance (RR_ERR_OCTREE otherwise);
 * the tensor keeps the device child_oct pointer, which must stay valid while
 * the tensor is used (its structure must not change); for every leaf below
 * level 0 the number of its corners that touch a leaf one level coarser
 * (N_fv of Eqs. alphac3d, alphaf3d) is counted once here, on the device.
 * Synchronous (waits for that count on the null stream); allocates device
 * memory. */
rr_status rr_tensor_create(const rr_field_desc* f, rr_precision p, rr_tensor* out);
rr_status rr_tensor_destroy(rr_tensor t);

/* Tidal tensor at cell centres by central finite differences (Eq.
 * tidalexample, cell size of the cell's own level) and its interpolation to
 * cell vertices (Sec. III H).  Octree cells whose stencil is incomplete at
 * their level take the trilinear interpolation of the coarser level's
 * component (Sec. IV C, second approach).  f must describe the same grid as
 * at rr_tensor_create; values may change between calls (one call per N-body
 * step).  Asynchronous on s; no allocation. */
rr_status rr_build_tidal_tensor(rr_tensor t, const rr_field_desc* f, rr_stream s);

/* Method A (Sec. IV D, Eq. kappa2): kappa from the density contrast and the
 * potential's gradient instead of the tidal tensor.  The tensor is created
 * from a density descriptor (field RR_FIELD_DELTA, uniform grids only) and
 * holds per vertex (delta_coeff delta, dPhi/dx, dPhi/dy, dPhi/dz): cell
 * values of delta, gradients by central differences, both averaged over the
 * eight incident cells (Sec. III H).  delta_coeff multiplies delta into the
 * Laplacian of phi's units, in 1 / length^2 of the box unit (for phi = Phi/c^2:
 * 3/2 Omega_m (H0/c)^2 / a).  rr_trace_rays then adds, per ray and chi
 * segment, int g delta_coeff delta + int (n . grad phi) dg/dchi (kernel
 * 1 - 2 chi / chi_s) and the segment's surface term -[g n . grad phi] from
 * chi_lo to chi_hi (Eqs. 2nterm, 2dterm2); the term with the time derivative
 * of the potential is left out, as in the paper.  Kappa and the trilinear
 * integral only (RR_ERR_UNSUPPORTED otherwise); delta and phi share the grid
 * and dtype of the tensor.  Asynchronous on s; no allocation. */
rr_status rr_build_method_a_fields(rr_tensor t, const rr_field_desc* delta,
                                   const rr_field_desc* phi, double delta_coeff, rr_stream s);

/* ISW integrand (Sec. VII: Eq. I1 with Q the time derivative of the
 * potential, by finite differences between N-body steps).  The tensor is
 * created from a descriptor with field RR_FIELD_PHI_DOT (uniform grids) and
 * holds per vertex the mean over its eight cells of
 * (phi_curr - phi_prev) * inv_dt (Sec. III H); open grids leave the vertices
 * on the lower faces NaN.  rr_trace_rays with quantity RR_Q_SCALAR and the
 * trilinear integral then adds kappa_scale * int Q dchi (chi in the box's
 * length unit) per ray over its window: the paper gives no kernel K for this
 * case, so it is the constant kappa_scale of the step (e.g. 2 a / c in the
 * units of inv_dt).  phi_curr and phi_prev share the grid, boundary and
 * dtype of the tensor.  Asynchronous on s; no allocation. */
rr_status rr_build_isw_field(rr_tensor t, const rr_field_desc* phi_curr,
                             const rr_field_desc* phi_prev, double inv_dt, rr_stream s);

/* Cell-centre tidal tensor (Eq. tidalexample, the cell's own level) for the
 * nearest-grid-point integral (Eq. Iclensing_ngp): uniform tensors then hold
 * one record per cell (cell i at record i, same 6-component layout) instead
 * of vertex records, and trace with RR_INTEGRAL_NGP; tracing them with the
 * trilinear integral returns RR_ERR_INVALID_ARG, and vice versa.  Open grids
 * leave the outer cell layer NaN.  Octree tensors always hold both (this call
 * is rr_build_tidal_tensor).  Asynchronous on s; no allocation. */
rr_status rr_build_tidal_tensor_centres(rr_tensor t, const rr_field_desc* f, rr_stream s);

/* The same tensor, built only on the vertices of the periodic box
 * [lo, lo + size) (vertex lattice indices; lo may lie outside [0, n) and the
 * box wraps; 0 <= size[a] <= n).  Vertices outside the box keep the values
 * of earlier builds.  The rays of one N-body step only read the vertices
 * around their chi segment (rr_rays_vertex_box), and the tensor work can be
 * limited to them (Sec. III H: the interpolation is worth doing only where
 * rays need it).  Uniform grids only (RR_ERR_UNSUPPORTED otherwise); open
 * grids take boxes inside [0, n) (RR_ERR_DOMAIN).  Asynchronous on s; no
 * allocation. */
rr_status rr_build_tidal_tensor_box(rr_tensor t, const rr_field_desc* f, const int32_t lo[3],
                                    const int32_t size[3], rr_stream s);

/* Device layout of a built tensor, for inspection.  Uniform: *data holds
 * n_base^3 records of `stride` bytes, components first (float or double by
 * precision).  Octree: n_cells records of 8 corners x 6 components
 * (corner v = ix + 2 iy + 4 iz), meaningful for leaf cells. */
rr_status rr_tensor_layout(rr_tensor t, const void** data, int64_t* n_records,
                           int32_t* record_bytes, int32_t* precision);

/* A bundle of rays sharing a source distance and a chi window: the rays of a
 * flat-sky map of nx by ny directions (Sec. III E, Eqs. txty, rayid: ray id =
 * iy*nx + ix).  Each wavefront of the march holds an 8 x 8 tile of the map.
 * The directions are always passed explicitly; center_dir, fov_x and fov_y
 * record the field of view they were made from (rr_fov_directions) and are
 * checked on the host: all three zero means "not recorded"; otherwise
 * center_dir must be a finite unit vector (| |c|^2 - 1 | <= 1e-9), each fov
 * must lie in [0, pi), and an axis with more than one ray needs a positive
 * fov (RR_ERR_INVALID_ARG, or RR_ERR_NONFINITE for non-finite values). */
typedef struct {
  int64_t ray_offset;    /* index of this bundle's first ray in the output arrays */
  int64_t n_rays;        /* nx * ny; 0 is allowed (empty bundle) */
  const double* dir;     /* device: n_rays x 3 FP64 unit vectors, observer -> source */
  int32_t nx, ny;
  double chi_s;          /* source distance (defines g) */
  double chi_hi, chi_lo; /* this call's chi window, 0 <= chi_lo < chi_hi <= chi_s */
  double center_dir[3];  /* unit vector of the map centre (e3 of rr_fov_directions) */
  double fov_x, fov_y;   /* opening angles Upsilon_x, Upsilon_y of Eq. txty, radians */
} rr_bundle;

/* Ray directions of an nx by ny flat-sky map (Sec. III E).  Host only, FP64,
 * no GPU call: fills dir_host[3 * (iy * nx + ix) + a] (0-based Eq. rayid).
 * The angles follow Eq. txty, theta_i = fov / (N - 1) * (i - 1) - fov / 2 for
 * i = 1..N (a single ray, N = 1, sits on the axis: theta = 0).  The paper
 * does not say how (theta_x, theta_y) become a direction; the mapping here is
 * the gnomonic one about the map centre: with e3 = center_dir / |center_dir|,
 * e1 = normalise(h x e3) where h = z^ if |e3_z| < 0.9 else x^ (e1 = x^ and
 * e2 = +-y^ when e3 lies on the z axis), e2 = e3 x e1,
 *     d = (tan(theta_x) e1 + tan(theta_y) e2) + e3,  n = d / |d|,
 * evaluated in that order with separate roundings (no fused multiply-add),
 * |d| = sqrt((d_x^2 + d_y^2) + d_z^2), tan from the C library.  The same
 * bits come from any caller that evaluates the formula in the same order.
 *  center_dir host, 3 doubles, finite and non-zero (normalised here).
 *  fov_x, fov_y in [0, pi) radians; positive when the axis has nx (ny) > 1.
 *  nx, ny       1 .. 65536 each.
 *  dir_host     host, caller-owned, nx * ny * 3 doubles, written.
 * Returns RR_ERR_INVALID_ARG (NULL pointer, bad size or angle) or
 * RR_ERR_NONFINITE; nothing is written then. */
rr_status rr_fov_directions(const double center_dir[3], double fov_x, double fov_y, int32_t nx,
                            int32_t ny, double* dir_host);

typedef struct {
  double observer[3];        /* observer position in the periodic box; it and every
                              window's chi_hi must lie within 2^29 base cells of the
                              origin (octrees: 2^25), else RR_ERR_INVALID_ARG */
  double kappa_scale;        /* multiplies every per-cell integral */
  int32_t precision;         /* rr_precision, must equal the tensor's */
  int32_t quantity;          /* rr_quantity */
  int32_t integral;          /* rr_integral */
  int32_t persistent;        /* 0: one wavefront per tile; 1: persistent
                                workgroups pulling tiles from a device queue;
                                -1: let the plan's tuner choose */
  int64_t max_crossings;     /* per ray per call; <= 0 means no limit */
  /* Optional debug outputs (device, NULL to skip), indexed like kappa:
   * crossing_hash: FNV-1a (64 bit) over the little-endian bytes of every
   *   piece (int64 cell id, IEEE bits of chi_A~, IEEE bits of chi_B~), chi in
   *   base-cell units; the uniform cell id is (z*n + y)*n + x after wrapping,
   *   the octree id is the leaf's cell index;
   * crossing_count: number of pieces;
   * crossing_log: up to log_stride records {int64 cell, double chi_A, double
   *   chi_B} per ray at crossing_log + 24 * log_stride * ray. */
  uint64_t* crossing_hash;
  int64_t* crossing_count;
  void* crossing_log;
  int64_t log_stride;
} rr_trace_params;

/* A plan owns the work queue, the device copies of bundle tables, tuning
 * results and captured graphs.  Not thread-safe: one host thread per plan.
 * A plan serves one stream at a time: its queue counter and split-march
 * resume points are shared by every launch it makes, so calls on different
 * streams must be ordered by the caller (an event or a synchronisation
 * between them); the same holds for rr_trace_rays_adjoint on one tensor
 * (its workspace).  Bundle tables (one per distinct bundle array, chi
 * windows included) are cached up to 256; beyond that the least recently
 * used table that the captured graph does not reference is released, after
 * waiting for the last launch that read it. */
rr_status rr_plan_create(rr_plan* p);
rr_status rr_plan_destroy(rr_plan p);

/* Integrate every ray of every bundle through the tensor (Eqs. sumIc, Ic,
 * Iclensing) and ADD kappa_scale * sum of pieces to kappa[ray_offset + i].
 *  kappa      device: FP32 (FP32_KAHAN) or FP64 (FP64) per ray, in/out.
 *  kappa_comp device FP32 per ray, in/out Kahan compensation (FP32_KAHAN
 *             only; NULL = start from zero and drop it at the end).  Passing
 *             the same kappa/kappa_comp to consecutive chi segments makes the
 *             multi-segment result equal the single-segment one to rounding.
 *  ray_status device int32 per ray, optional, written (not accumulated).
 * The start cell of a segment is located from chi_hi by the slab rule, so a
 * ray's state between segments is just (kappa, kappa_comp).  The first call
 * with a new bundle table uploads it (synchronously, outside graph capture);
 * later calls with an identical table allocate and copy nothing. */
rr_status rr_trace_rays(rr_plan p, rr_tensor t, const rr_trace_params* tp,
                        const rr_bundle* bundles /* host */, int32_t n_bundles, void* kappa,
                        float* kappa_comp, int32_t* ray_status, rr_stream s);

/* Many source distances in one walk (Sec. VII, Eqs. Isources, Isources1).
 * The lensing kernel g = chi (chi_s - chi) / chi_s splits into chi and
 * chi^2 / chi_s, so the walk integrates A = int chi Q and B = int chi^2 Q
 * (Q the quantity of tp, trilinear reconstruction from the vertex tensor or
 * the octree's per-leaf corners) without a source distance, and stops at
 * each of a list of them:
 *  chi_src    host, n_src (1..4096) source distances in the length unit of
 *             the field, strictly decreasing.  A call stops at the sources
 *             with chi_lo <= chi_src[j] < chi_hi of its bundle window; a
 *             source inside a cell cuts that cell into two pieces (each is
 *             hashed and counted like a crossing).
 *  moments    device, per ray, in/out: the two integrals accumulated since
 *             the last stop, times kappa_scale, in base-cell units.
 *             FP32_KAHAN: 4 floats {A, A_comp, B, B_comp} (Kahan pairs);
 *             FP64: 2 doubles {A, B}.  Start from zeros.
 *  pieces     device, n_rays x n_src x 2 doubles: at the stop of source j
 *             the walk writes the pair accumulated since the previous stop
 *             (for FP32_KAHAN, sum minus compensation in FP64) and restarts
 *             the moments from zero; entries of sources not met are left as
 *             they are.
 *  ray_status as in rr_trace_rays.
 * Each bundle's chi_s is not used beyond the window check (give the
 * farthest source).  Traced over consecutive windows down to chi_lo = 0,
 * rr_kappa_from_pieces then gives kappa (or the shear) of every source.
 * moments and pieces may be NULL when no bundle has rays.
 * Debug outputs as in tp.  The source list is uploaded on first use
 * (synchronously, outside graph capture) and kept by the plan.  NGP and
 * Method A return RR_ERR_UNSUPPORTED. */
rr_status rr_trace_rays_sources(rr_plan p, rr_tensor t, const rr_trace_params* tp,
                                const rr_bundle* bundles, int32_t n_bundles,
                                const double* chi_src, int32_t n_src, void* moments,
                                double* pieces, int32_t* ray_status, rr_stream s);

/* kappa (FP64, n_rays x n_src, ray-major) of every source once the walk of
 * rr_trace_rays_sources has reached the observer: A and B below source j
 * are the moments left after the last stop plus the pieces of the sources
 * nearer than j (Eq. Isources1), and kappa_j = A_j - B_j / chi_src[j]
 * (Eq. Isources).  Sums in FP64; n_rays counts every ray of the arrays.
 * Asynchronous on s; the source list is uploaded like rr_trace_rays_sources. */
rr_status rr_kappa_from_pieces(rr_plan p, rr_tensor t, const double* chi_src, int32_t n_src,
                               int64_t n_rays, const void* moments, const double* pieces,
                               double* kappa, rr_stream s);

/* The vertex box (lo, size as taken by rr_build_tidal_tensor_box) that
 * contains every vertex the rays of these bundles read between their chi_lo
 * and chi_hi: the lattice bounds of the rays' end points, widened by the
 * slab rule and the cells' upper corners, clipped to the whole axis (or, on
 * open grids, to [0, n)).  An empty bundle set gives size 0.  Runs a small
 * reduction kernel on s and waits for it (synchronous; not inside a
 * capture); uploads the bundle table like rr_trace_rays.  Uniform grids
 * only. */
rr_status rr_rays_vertex_box(rr_plan p, rr_tensor t, const rr_trace_params* tp,
                             const rr_bundle* bundles, int32_t n_bundles, int32_t lo[3],
                             int32_t size[3], rr_stream s);

/* Tune the launch shape for this bundle set: times one-wavefront-per-tile
 * launches (64- and 256-thread workgroups) and persistent workgroups fed by
 * the device queue (8, 16 or 32 wavefronts per compute unit), each as one
 * pass over the chi window or split into 4 to 64 passes, on scratch outputs,
 * and remembers the fastest for the bundle set; later rr_trace_rays /
 * rr_trace_rays_sources calls with tp->persistent = -1 and the same bundles
 * use it.  A split march cuts the bundles' chi range into equal steps: a pass
 * stops every ray on the first face at or below its boundary and the next
 * pass resumes on that face, so rays that drift apart in a long march (one
 * through a refined halo, its neighbours past it) start each pass side by
 * side again; the pieces and their order do not change, and neither do the
 * results.  Passes are used only without debug outputs and
 * max_crossings, and (FP32_KAHAN) with kappa_comp given; the plan keeps one
 * double per ray for the resume points (allocated on first use, outside
 * graph capture).  Synchronous; allocates and frees scratch buffers; never
 * called inside a capture. */
rr_status rr_plan_autotune(rr_plan p, rr_tensor t, const rr_trace_params* tp,
                           const rr_bundle* bundles, int32_t n_bundles, rr_stream s);
/* Pin the launch shape that calls with tp->persistent = -1 use for this
 * bundle set, as rr_plan_autotune would record it: persistent 0 or 1, block
 * 64 or 256 (one-wavefront-per-tile launches), waves_per_cu 1..32
 * (persistent launches), passes 1..64 (split march, see rr_plan_autotune).
 * Host only; replaces an earlier choice for the same bundles. */
rr_status rr_plan_set_shape(rr_plan p, const rr_bundle* bundles, int32_t n_bundles,
                            int32_t persistent, int32_t block, int32_t waves_per_cu,
                            int32_t passes);

/* The shape chosen by rr_plan_autotune for a bundle set (and its time in ms);
 * passes = 1 for an unsplit march. */
rr_status rr_plan_tuned_shape(rr_plan p, const rr_bundle* bundles, int32_t n_bundles,
                              int32_t* persistent, int32_t* block, int32_t* waves_per_cu,
                              int32_t* passes, float* ms);

/* Gradient of L = sum_r w_r kappa_r with respect to the potential values of
 * a uniform periodic FP32 field: ADDS dL/dPhi to dl_dphi (device, n_base^3
 * FP32, same layout as f->values).  kappa is linear in Phi (straight rays,
 * Born approximation, Sec. IV A), and the result is the exact transpose of
 * the forward chain (per-cell integral, vertex mean, finite differences),
 * accumulated with FP32 atomics (order-dependent rounding).  The first call
 * on a tensor allocates a workspace of 8 FP32 values per vertex (32 B x n^3),
 * kept with the tensor until rr_tensor_destroy; the tensor's own values are
 * not modified.  Needs the FP32 Kahan precision, a periodic uniform field and
 * RR_Q_KAPPA; anything else returns RR_ERR_UNSUPPORTED. */
rr_status rr_trace_rays_adjoint(rr_plan p, rr_tensor t, const rr_field_desc* f,
                                const rr_trace_params* tp, const rr_bundle* bundles,
                                int32_t n_bundles, const float* dl_dkappa, float* dl_dphi,
                                rr_stream s);

/* rr_trace_rays for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments and results as rr_trace_rays, without a plan: the bundle
 * table and the persistent queue counter live in a fixed device array of the
 * library (72.5 KiB per GPU, held until the process ends; its address is
 * resolved once per device), written by kernels on s before the march.
 * Tiles go to the wavefronts in the same order as rr_trace_rays (bundles as
 * given, or longest chi window first for persistent launches; Z order of
 * the 8 x 8 tiles within a bundle; persistent launches use one counter per
 * chiplet).
 *  - n_bundles <= 1024, else RR_ERR_CAPACITY (nothing enqueued).
 *  - tp->persistent: 1 = persistent workgroups (16 wavefronts per compute
 *    unit) fed by the queue counter; 0 or -1 = one wavefront per 8x8 tile
 *    (256-thread workgroups).  The march is never split into passes.
 *  - No hipMalloc, hipFree or other allocating call; host memory is the
 *    stack only.
 *  - Every call on one GPU shares that GPU's array, which keeps the last
 *    call's table: calls on one stream are ordered, but calls that overlap
 *    on one GPU (other streams or host threads) race and must be ordered by
 *    the caller. */
rr_status rr_trace_rays_noalloc(rr_tensor t, const rr_trace_params* tp,
                                const rr_bundle* bundles /* host */, int32_t n_bundles,
                                void* kappa, float* kappa_comp, int32_t* ray_status, rr_stream s);

/* Capture every library call enqueued on s between begin and end into one
 * HIP graph owned by the plan (replaces any previous one), then replay it
 * with rr_graph_launch.  Bundle tables must have been uploaded before begin.
 * The graph holds kernel nodes only (queue counters are reset by a kernel). */
rr_status rr_graph_begin(rr_plan p, rr_stream s);
rr_status rr_graph_end(rr_plan p, rr_stream s);
rr_status rr_graph_launch(rr_plan p, rr_stream s);

/* Message of the last failed call on this host thread ("" if none). */
const char* rr_last_error(void);
/* Library version: major * 10000 + minor * 100 + patch. */
int32_t rr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RAYRAMSES_H */
