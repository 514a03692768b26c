/*
 * rro.h -- plain FP64 CPU oracle for the RAY-RAMSES Method-B convergence path.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP path; only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no source, header or generated table with the HIP
 * library, and the HIP library never calls it.
 *
 * Everything is double precision, built with -O2 -fno-fast-math
 * -ffp-contract=off, and follows the paper (RAY-RAMSES, arXiv:1601.02012)
 * step by step:
 *   centre tidal tensor      Sec. IV C, Eq. (tidalexample)
 *   AMR fallback             Sec. IV C (option 2: interpolate coarse d_a d_b Phi)
 *   vertex interpolation     Sec. III H (regular average), Eqs. (alphac3d),
 *                            (alphaf3d), hanging vertices (text after Eq. rhoV_1)
 *   ray walk                 Sec. III F 1, Eqs. (rayposition)-(disttocross)
 *   trilinear reconstruction Eqs. (trilinear_int), (trilinear_coef), (Deltas)
 *   d_N coefficients         App. B, Eq. (dns)
 *   per-cell lensing integral Eq. (Iclensing); NGP variant Eq. (Iclensing_ngp)
 *   kappa integrand          Eqs. (n1n1), (n2n2); shear Eqs. (gamma1), (gamma2), (n1n2)
 *   many source distances    Sec. VII, Eqs. (Isources), (Isources1)
 *   ISW integrand            Sec. VII, Eq. (I1) with Q = dPhi/dt
 *
 * Units: lengths are converted to base-grid units, h0 = L / n_base,
 * o~ = o / h0, chi~ = chi / h0; a level-l cell has size 2^-l.  kappa is
 * unit-free under this rescaling.
 *
 * Tensor component order everywhere: xx, yy, zz, xy, xz, yz.
 */
#ifndef RRO_H
#define RRO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { RRO_RAY_OK = 0, RRO_RAY_OUT_OF_DOMAIN = 1, RRO_RAY_MAX_STEPS = 2 };
enum { RRO_Q_KAPPA = 0, RRO_Q_GAMMA1 = 1, RRO_Q_GAMMA2 = 2 };

typedef struct {
  int64_t cell;      /* linear cell id (wrapped) */
  double chi_a;      /* entry chi (grid units), chi_a > chi_b */
  double chi_b;
} rro_segment;

/* ---- uniform grid -------------------------------------------------------- */
/* Centre tensor by Eq. (tidalexample) on an n^3 grid of cell size h ([z][y][x]).
 * open != 0: cells on the outer layer get NaN (their stencil leaves the grid). */
void rro_centre_tensor_uniform(int32_t n, int32_t open, double h, const double* phi,
                               double* tc /* n^3 x 6 */);
/* Vertex (i,j,k) = mean of the centre tensors of cells {i-1,i}x{j-1,j}x{k-1,k}
 * (periodic); NaN propagates for open grids. */
void rro_vertex_tensor_uniform(int32_t n, const double* tc, double* tv /* n^3 x 6 */);

/* Trace rays through the vertex tensor of a uniform grid.
 * dir: n_rays x 3 unit vectors (observer -> source); chi_* per ray in box units.
 * quantity: RRO_Q_KAPPA / RRO_Q_GAMMA1 / RRO_Q_GAMMA2.  ngp != 0 uses the
 * cell-centre tensor tc with Eq. (Iclensing_ngp) instead of tv.
 * Outputs (each optional, may be NULL): kappa, hash (FNV-1a 64 over every
 * segment's (int64 cell, bits chi_a, bits chi_b)), ncross, status, log. */
int32_t rro_trace_uniform(int32_t n, int32_t open, double box, const double* observer,
                          int64_t n_rays, const double* dir, const double* chi_s,
                          const double* chi_hi, const double* chi_lo, double kappa_scale,
                          int32_t quantity, int32_t ngp, const double* tv, const double* tc,
                          int64_t max_steps, int32_t n_threads,
                          double* kappa, uint64_t* hash, int64_t* ncross, int32_t* status,
                          rro_segment* log, int64_t log_stride);

/* One cell of Eq. (Iclensing) from the eight vertex values Q (paper's P_1..P_8),
 * lower corner p1, size h; dir/o/chis/chiA/chiB in grid units. */
double rro_cell_integral(const double* Q, const double* p1, double h, const double* dir,
                         const double* o, double chis, double chiA, double chiB);
/* The projection of T used as the integrand (Eqs. n1n1, n2n2, n1n2). */
double rro_projection(const double* dir, const double* T, int32_t quantity);

/* Method A (Eq. kappa2, Sec. IV D): vertex fields (delta, grad Phi) from
 * the cell values (central differences of spacing h, mean of the eight
 * incident cells); fv: n^3 x 4. */
void rro_method_a_vertex_fields(int32_t n, int32_t open, double h, const double* phi,
                                const double* delta, double* fv);
/* Trace with the Method A integrand: delta_coeff * g * delta (delta_coeff in
 * 1 / length^2 of the box unit, e.g. 3/2 Omega_m (H0/c)^2 / a) plus
 * (n . grad Phi) dg/dchi, and the step's surface term -[g n . grad Phi]
 * between chi_lo and chi_hi (Eqs. 2nterm, 2dterm2).  Kappa only. */
int32_t rro_trace_uniform_method_a(int32_t n, int32_t open, double box, const double* observer,
                                   int64_t n_rays, const double* dir, const double* chi_s,
                                   const double* chi_hi, const double* chi_lo,
                                   double kappa_scale, double delta_coeff, const double* fv,
                                   int64_t max_steps, int32_t n_threads, double* kappa,
                                   uint64_t* hash, int64_t* ncross, int32_t* status);
/* One cell of the gradient term: int (1 - 2 chi / chi_s) Q dchi over the
 * segment, Q trilinear from its eight vertex values (as rro_cell_integral). */
double rro_cell_integral_k(const double* Q, const double* p1, double h, const double* dir,
                           const double* o, double chis, double chiA, double chiB);

/* Many source distances in one walk (Sec. VII, Eqs. Isources, Isources1).
 * chi_src: n_src source distances (box units), strictly decreasing.  Per ray
 * the walk integrates kappa_scale * int chi Q and kappa_scale * int chi^2 Q
 * (grid units) into moments[2 r + 0..1] (in/out), stops at every chi_src[j]
 * with chi_lo <= chi_src[j] < chi_hi (a cell holding it is cut into two
 * pieces, each hashed and counted), writes the accumulated pair to
 * pieces[(r n_src + j) 2 + 0..1] and restarts it from zero.  Other pieces
 * are left as they are.  quantity as for rro_trace_uniform. */
int32_t rro_trace_uniform_sources(int32_t n, int32_t open, double box, const double* observer,
                                  int64_t n_rays, const double* dir, const double* chi_hi,
                                  const double* chi_lo, int32_t n_src, const double* chi_src,
                                  double kappa_scale, int32_t quantity, const double* tv,
                                  int64_t max_steps, int32_t n_threads, double* moments,
                                  double* pieces, uint64_t* hash, int64_t* ncross,
                                  int32_t* status);
/* One cell of the two integrals: out[0] = int chi Q, out[1] = int chi^2 Q
 * over [chi_B, chi_A] (arguments as rro_cell_integral). */
void rro_cell_moments(const double* Q, const double* p1, double h, const double* dir,
                      const double* o, double chiA, double chiB, double* out);
/* kappa[r n_src + j] of every source once the walk has reached the observer
 * (moments then hold what lies below the nearest source). */
void rro_kappa_from_pieces(int64_t n_rays, int32_t n_src, const double* chi_src, double box,
                           int32_t n_base, const double* moments, const double* pieces,
                           double* kappa);

/* ISW integrand (Sec. VII; Eq. I1 with Q = dPhi/dt): vertex values of
 * (phi_curr - phi_prev) * inv_dt (mean of the eight incident cells), then
 * out = scale * int Q dchi per ray over [chi_lo, chi_hi] (box units; the
 * kernel is the constant scale within a step). */
void rro_isw_vertex_field(int32_t n, int32_t open, const double* phi_curr,
                          const double* phi_prev, double inv_dt, double* qv /* n^3 */);
int32_t rro_trace_uniform_isw(int32_t n, int32_t open, double box, const double* observer,
                              int64_t n_rays, const double* dir, const double* chi_hi,
                              const double* chi_lo, double scale, const double* qv,
                              int64_t max_steps, int32_t n_threads, double* out, uint64_t* hash,
                              int64_t* ncross, int32_t* status);
/* int Q dchi over one cell's piece [chi_B, chi_A] (grid units). */
double rro_cell_integral_one(const double* Q, const double* p1, double h, const double* dir,
                             const double* o, double chiA, double chiB);

/* Adjoint of kappa = A(Phi) for a uniform grid: dL/dPhi += A^T (dL/dkappa).
 * Explicit transpose of: per-cell integral -> vertex average -> FD stencil. */
int32_t rro_trace_adjoint_uniform(int32_t n, double box, const double* observer,
                                  int64_t n_rays, const double* dir, const double* chi_s,
                                  const double* chi_hi, const double* chi_lo,
                                  double kappa_scale, const double* dl_dkappa,
                                  int32_t n_threads, double* dl_dphi /* n^3 */);

/* ---- octree --------------------------------------------------------------- */
/* Cells: base cells 0..n^3-1 ([z][y][x]), then oct k holds cells
 * n^3 + 8k + (ix + 2 iy + 4 iz).  child_oct[c] = k or -1.  Octs are in
 * breadth-first order.  oct_level[k] = level of its cells (1..max_level). */
typedef struct {
  int32_t n;
  int32_t max_level;
  int64_t n_octs;
  const int32_t* child_oct;   /* n_cells */
  const int64_t* oct_parent;  /* n_octs: parent cell */
  const int32_t* oct_level;   /* n_octs */
  const int32_t* oct_coord;   /* n_octs x 3: level-l integer coords of the oct's ix=iy=iz=0 cell */
} rro_octree;

/* Check 2:1 balance over faces, edges and corners.  Returns 0 if balanced. */
int32_t rro_octree_check(const rro_octree* t);
/* Centre tensor per cell (leaf and internal) with the level-l stencil where
 * all stencil cells exist at level l, else trilinear interpolation of the
 * coarser level's component (recursive). */
void rro_centre_tensor_octree(const rro_octree* t, const double* phi, double* tc /* n_cells x 6 */);
/* Corner tensors of every leaf: cv[c*48 + v*6 + comp], v = ix + 2 iy + 4 iz.
 * Regular / boundary (Eqs. alphac3d, alphaf3d) / hanging vertices. */
void rro_corner_tensor_octree(const rro_octree* t, const double* tc, double* cv /* n_cells x 48 */);
/* The same for a list of leaf cells only (cv: n_sel x 48). */
void rro_corner_tensor_octree_cells(const rro_octree* t, const double* tc, int64_t n_sel,
                                    const int64_t* cells, double* cv);
/* 3D mass-redistribution weights: alpha_coarse and alpha_fine for one vertex,
 * for dimension dim (2: Eqs. alphaconst/alphaconst2, 3: Eqs. alphac3d/alphaf3d). */
void rro_vertex_weights(int32_t dim, int32_t n_coarse, int32_t n_fine, const int32_t* n_fv,
                        double* alpha_coarse, double* alpha_fine /* n_fine */);
/* Trace through an octree.  cv: per-leaf corner tensors from
 * rro_corner_tensor_octree, or NULL to evaluate each visited leaf's corners
 * on the fly from the centre tensor tc.  ngp != 0 integrates the leaf's own
 * centre tensor tc with Eq. (Iclensing_ngp) instead.  quantity as for
 * rro_trace_uniform. */
int32_t rro_trace_octree(const rro_octree* t, double box, const double* observer,
                         int64_t n_rays, const double* dir, const double* chi_s,
                         const double* chi_hi, const double* chi_lo, double kappa_scale,
                         int32_t quantity, const double* cv, const double* tc, int32_t ngp,
                         int64_t max_steps,
                         int32_t n_threads, double* kappa, uint64_t* hash, int64_t* ncross,
                         int32_t* status, rro_segment* log, int64_t log_stride);
/* The many-source walk through the octree (per-leaf corner tensors cv). */
int32_t rro_trace_octree_sources(const rro_octree* t, double box, const double* observer,
                                 int64_t n_rays, const double* dir, const double* chi_hi,
                                 const double* chi_lo, int32_t n_src, const double* chi_src,
                                 double kappa_scale, int32_t quantity, const double* cv,
                                 int64_t max_steps, int32_t n_threads, double* moments,
                                 double* pieces, uint64_t* hash, int64_t* ncross,
                                 int32_t* status);

#ifdef __cplusplus
}
#endif
#endif
