/*
 * rro_octree.c -- FP64 oracle for 2:1-balanced AMR octrees.
 * TEST INFRASTRUCTURE ONLY (see rro.h).
 *
 * Readings of the paper taken here:
 *  - tidal tensor at a level-l cell: Eq. (tidalexample) with the level's cell
 *    size when every stencil cell exists at level l; otherwise that component
 *    is interpolated trilinearly from the eight level-(l-1) centres around the
 *    cell centre (weights 3/4, 1/4 per axis), Sec. IV C "second approach";
 *  - vertices (Sec. III H): all incident leaves on one level -> mean of their
 *    centre values; vertex in the middle of a coarse edge / face -> mean of
 *    the 2 / 4 coarse corner vertices; otherwise the mass-redistribution
 *    weights of Eqs. (alphac3d) and (alphaf3d), where N_fv,j counts the
 *    vertices of fine leaf j that touch at least one coarse leaf;
 *  - walk: the uniform rules on the current leaf's level; entering a refined
 *    neighbour takes the child next to the crossed face on the crossed axes
 *    and the slab rule on the others.
 */
#include "rro.h"
#include "rro_common.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static inline int64_t fdiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}
static inline int64_t fmod64(int64_t a, int64_t b) { return a - fdiv(a, b) * b; }

typedef struct {
  int64_t cell;
  int32_t level;
} loc_t;

/* Cell at level l with (unwrapped) level-l coords I, or the leaf that covers
 * it if the tree stops above level l.  .level < l means "does not exist at l". */
static loc_t descend(const rro_octree* t, int32_t l, const int64_t* I) {
  const int64_t n = t->n;
  int64_t b[3];
  for (int a = 0; a < 3; ++a) b[a] = fmod64(fdiv(I[a], (int64_t)1 << l), n);
  loc_t r;
  r.cell = (b[2] * n + b[1]) * n + b[0];
  r.level = 0;
  const int64_t nbase = n * n * n;
  for (int32_t lev = 1; lev <= l; ++lev) {
    const int32_t k = t->child_oct[r.cell];
    if (k < 0) return r;
    int child = 0;
    for (int a = 0; a < 3; ++a) {
      const int64_t bit = fmod64(fdiv(I[a], (int64_t)1 << (l - lev)), 2);
      child |= (int)bit << a;
    }
    r.cell = nbase + 8 * (int64_t)k + child;
    r.level = lev;
  }
  return r;
}

/* level and level coords of any cell */
static void cell_info(const rro_octree* t, int64_t c, int32_t* level, int64_t* I) {
  const int64_t n = t->n, nbase = n * n * n;
  if (c < nbase) {
    *level = 0;
    I[0] = c % n;
    I[1] = (c / n) % n;
    I[2] = c / (n * n);
    return;
  }
  const int64_t k = (c - nbase) / 8;
  const int child = (int)((c - nbase) % 8);
  *level = t->oct_level[k];
  for (int a = 0; a < 3; ++a) I[a] = t->oct_coord[3 * k + a] + ((child >> a) & 1);
}

static int64_t n_cells_of(const rro_octree* t) {
  return (int64_t)t->n * t->n * t->n + 8 * t->n_octs;
}

int32_t rro_octree_check(const rro_octree* t) {
  const int64_t nc = n_cells_of(t);
  int32_t bad = 0;
  /* every refined cell at level l needs all 26 neighbours present at level l */
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : bad)
  for (int64_t c = 0; c < nc; ++c) {
    if (t->child_oct[c] < 0) continue;
    int32_t l;
    int64_t I[3];
    cell_info(t, c, &l, I);
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int64_t J[3] = {I[0] + dx, I[1] + dy, I[2] + dz};
          if (descend(t, l, J).level != l) bad += 1;
        }
  }
  return bad;
}

/* ------------------------------------------------------------ centre tensor */
static const int stencil_xyz[6][4][3] = {
    /* placeholders for the mixed components: (+,+), (-,-), (+,-), (-,+) */
    {{0}}, {{0}}, {{0}},
    {{1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}},
    {{1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1}},
    {{0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}},
};

static int fd_component(const rro_octree* t, const double* phi, int32_t l, const int64_t* I,
                        int comp, double* out) {
  const double h = ldexp(1.0, -l);
  const double h2 = h * h;
  if (comp < 3) {
    int64_t Jm[3] = {I[0], I[1], I[2]}, Jp[3] = {I[0], I[1], I[2]};
    Jm[comp] -= 1;
    Jp[comp] += 1;
    const loc_t a = descend(t, l, Jm), b = descend(t, l, Jp), c = descend(t, l, I);
    if (a.level != l || b.level != l) return 0;
    *out = (phi[a.cell] - 2.0 * phi[c.cell] + phi[b.cell]) / h2;
    return 1;
  }
  double v[4];
  for (int s = 0; s < 4; ++s) {
    const int64_t J[3] = {I[0] + stencil_xyz[comp][s][0], I[1] + stencil_xyz[comp][s][1],
                          I[2] + stencil_xyz[comp][s][2]};
    const loc_t a = descend(t, l, J);
    if (a.level != l) return 0;
    v[s] = phi[a.cell];
  }
  *out = (v[0] + v[1] - v[2] - v[3]) / (4.0 * h2);
  return 1;
}

void rro_centre_tensor_octree(const rro_octree* t, const double* phi, double* tc) {
  const int64_t nc = n_cells_of(t);
  for (int32_t lev = 0; lev <= t->max_level; ++lev) {
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t c = 0; c < nc; ++c) {
      int32_t l;
      int64_t I[3];
      cell_info(t, c, &l, I);
      if (l != lev) continue;
      for (int comp = 0; comp < 6; ++comp) {
        double v;
        if (fd_component(t, phi, l, I, comp, &v)) {
          tc[6 * c + comp] = v;
          continue;
        }
        /* trilinear interpolation of the level-(l-1) component */
        int64_t P[3], off[3];
        for (int a = 0; a < 3; ++a) {
          P[a] = fdiv(I[a], 2);
          off[a] = (fmod64(I[a], 2) == 1) ? 1 : -1;
        }
        double acc = 0.0;
        for (int s = 0; s < 8; ++s) {
          int64_t J[3];
          double w = 1.0;
          for (int a = 0; a < 3; ++a) {
            const int use_nb = (s >> a) & 1;
            J[a] = P[a] + (use_nb ? off[a] : 0);
            w *= use_nb ? 0.25 : 0.75;
          }
          const loc_t q = descend(t, l - 1, J);
          acc += w * tc[6 * q.cell + comp];
        }
        tc[6 * c + comp] = acc;
      }
    }
  }
}

/* ----------------------------------------------------------- vertex weights */
void rro_vertex_weights(int32_t dim, int32_t n_coarse, int32_t n_fine, const int32_t* n_fv,
                        double* alpha_coarse, double* alpha_fine) {
  const double f = (dim == 2) ? 0.25 : 0.125;
  double s = 0.0;
  for (int j = 0; j < n_fine; ++j) s += n_fv[j];
  const double ac = 1.0 / (n_coarse + f * s);
  *alpha_coarse = ac;
  for (int j = 0; j < n_fine; ++j) alpha_fine[j] = f * n_fv[j] * ac;
}

/* Leaf that covers the octant o (bits 0/1 per axis: below/above) around the
 * level-lv lattice point V. */
static loc_t octant_leaf(const rro_octree* t, int32_t lv, const int64_t* V, int o) {
  int64_t J[3];
  for (int a = 0; a < 3; ++a) J[a] = V[a] - 1 + ((o >> a) & 1);
  loc_t q = descend(t, lv, J);
  if (q.level < lv) return q;                 /* coarser leaf */
  int32_t l = lv;
  while (t->child_oct[q.cell] >= 0) {         /* finer: child next to V */
    const int32_t k = t->child_oct[q.cell];
    int child = 0;
    for (int a = 0; a < 3; ++a) child |= (1 - ((o >> a) & 1)) << a;
    q.cell = (int64_t)t->n * t->n * t->n + 8 * (int64_t)k + child;
    q.level = ++l;
  }
  return q;
}

static int touches_level(const rro_octree* t, int32_t lv, const int64_t* V, int32_t level) {
  for (int o = 0; o < 8; ++o)
    if (octant_leaf(t, lv, V, o).level == level) return 1;
  return 0;
}

/* Tensor at the level-lv lattice point V (a corner of at least one leaf). */
static void vertex_value(const rro_octree* t, const double* tc, int32_t lv, const int64_t* V,
                         double* out) {
  loc_t leaf[8];
  int32_t lc = 1 << 30, lf = -1;
  for (int o = 0; o < 8; ++o) {
    leaf[o] = octant_leaf(t, lv, V, o);
    if (leaf[o].level < lc) lc = leaf[o].level;
    if (leaf[o].level > lf) lf = leaf[o].level;
  }
  for (int c = 0; c < 6; ++c) out[c] = 0.0;
  /* is V on the lattice of the coarsest incident level? */
  const int64_t s = (int64_t)1 << (lv - lc);
  int frac[3], nfrac = 0;
  for (int a = 0; a < 3; ++a) {
    frac[a] = fmod64(V[a], s) != 0;
    nfrac += frac[a];
  }
  if (nfrac > 0) {
    /* hanging: mid-edge (2 corners) or face centre (4 corners) of a coarse leaf */
    int cnt = 0;
    for (int sel = 0; sel < 8; ++sel) {
      int skip = 0;
      int64_t W[3];
      for (int a = 0; a < 3; ++a) {
        const int bit = (sel >> a) & 1;
        if (!frac[a] && bit) skip = 1;
        W[a] = frac[a] ? (fdiv(V[a], s) + bit) : fdiv(V[a], s);
      }
      if (skip) continue;
      double w[6];
      vertex_value(t, tc, lc, W, w);
      for (int c = 0; c < 6; ++c) out[c] += w[c];
      ++cnt;
    }
    for (int c = 0; c < 6; ++c) out[c] /= (double)cnt;
    return;
  }
  if (lc == lf) {
    /* regular: mean of the eight same-level centre values */
    for (int o = 0; o < 8; ++o)
      for (int c = 0; c < 6; ++c) out[c] += tc[6 * leaf[o].cell + c];
    for (int c = 0; c < 6; ++c) out[c] /= 8.0;
    return;
  }
  /* boundary vertex: Eqs. (alphac3d), (alphaf3d) */
  int32_t n_coarse = 0, n_fine = 0, nfv[8];
  int64_t fine_cell[8];
  for (int o = 0; o < 8; ++o) {
    if (leaf[o].level == lc) {
      ++n_coarse;
      continue;
    }
    /* fine leaf j: count its corners that touch a coarse leaf */
    int32_t lj;
    int64_t Ij[3];
    cell_info(t, leaf[o].cell, &lj, Ij);
    int32_t cntv = 0;
    for (int v = 0; v < 8; ++v) {
      const int64_t W[3] = {Ij[0] + (v & 1), Ij[1] + ((v >> 1) & 1), Ij[2] + ((v >> 2) & 1)};
      cntv += touches_level(t, lj, W, lc);
    }
    nfv[n_fine] = cntv;
    fine_cell[n_fine] = leaf[o].cell;
    ++n_fine;
  }
  double ac, af[8];
  rro_vertex_weights(3, n_coarse, n_fine, nfv, &ac, af);
  for (int o = 0; o < 8; ++o)
    if (leaf[o].level == lc)
      for (int c = 0; c < 6; ++c) out[c] += ac * tc[6 * leaf[o].cell + c];
  for (int j = 0; j < n_fine; ++j)
    for (int c = 0; c < 6; ++c) out[c] += af[j] * tc[6 * fine_cell[j] + c];
}

static void leaf_corners(const rro_octree* t, const double* tc, int64_t c, double cv[8][6]) {
  int32_t l;
  int64_t I[3];
  cell_info(t, c, &l, I);
  for (int v = 0; v < 8; ++v) {
    const int64_t V[3] = {I[0] + (v & 1), I[1] + ((v >> 1) & 1), I[2] + ((v >> 2) & 1)};
    vertex_value(t, tc, l, V, cv[v]);
  }
}

void rro_corner_tensor_octree(const rro_octree* t, const double* tc, double* cv) {
  const int64_t nc = n_cells_of(t);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t c = 0; c < nc; ++c) {
    double* out = cv + 48 * c;
    if (t->child_oct[c] >= 0) {
      for (int i = 0; i < 48; ++i) out[i] = NAN;
      continue;
    }
    double tmp[8][6];
    leaf_corners(t, tc, c, tmp);
    memcpy(out, tmp, sizeof(tmp));
  }
}

void rro_corner_tensor_octree_cells(const rro_octree* t, const double* tc, int64_t n_sel,
                                    const int64_t* cells, double* cv /* n_sel x 48 */) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t s = 0; s < n_sel; ++s) {
    double tmp[8][6];
    leaf_corners(t, tc, cells[s], tmp);
    memcpy(cv + 48 * s, tmp, sizeof(tmp));
  }
}

/* ------------------------------------------------------------------- tracing */
/* child bit on axis a when moving from level l slab m to level l+1 at chi */
static int slab_child(const rro_ray* ray, int a, int64_t m, int32_t l, double chi) {
  const double hl1 = ldexp(1.0, -(l + 1));
  const int64_t mid = 2 * m + 1;
  if (ray->n[a] == 0.0) return (ray->o[a] / hl1) >= (double)mid;
  const double tm = rro_tplane(ray, a, (double)mid * hl1);
  return ray->n[a] > 0.0 ? (chi > tm) : (chi <= tm);
}

int32_t rro_trace_octree(const rro_octree* t, double box, const double* observer,
                         int64_t n_rays, const double* dir, const double* chi_s,
                         const double* chi_hi, const double* chi_lo, double kappa_scale,
                         int32_t quantity, const double* cv, const double* tc, int32_t ngp,
                         int64_t max_steps,
                         int32_t n_threads, double* kappa, uint64_t* hash, int64_t* ncross,
                         int32_t* status, rro_segment* log, int64_t log_stride) {
  const double h0 = box / (double)t->n;
  double o[3];
  for (int a = 0; a < 3; ++a) o[a] = observer[a] / h0;
  if (n_threads > 0) rro_set_threads(n_threads);
  const int64_t nbase = (int64_t)t->n * t->n * t->n;

#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < n_rays; ++r) {
    rro_ray ray;
    rro_ray_init(&ray, dir + 3 * r, o, chi_s[r] / h0, quantity);
    const double lo = chi_lo[r] / h0;
    double chiA = chi_hi[r] / h0;
    int64_t m[3];
    for (int a = 0; a < 3; ++a) m[a] = rro_start_slab(&ray, a, chiA, 1.0);
    loc_t cur = descend(t, 0, m);
    int32_t l = 0;
    while (t->child_oct[cur.cell] >= 0) {
      int child = 0;
      for (int a = 0; a < 3; ++a) {
        const int bit = slab_child(&ray, a, m[a], l, chiA);
        m[a] = 2 * m[a] + bit;
        child |= bit << a;
      }
      cur.cell = nbase + 8 * (int64_t)t->child_oct[cur.cell] + child;
      ++l;
    }

    double sum = 0.0;
    uint64_t hv = RRO_FNV_OFFSET;
    int64_t count = 0;
    int32_t st = RRO_RAY_OK;
    for (;;) {
      if (count >= max_steps) {
        st = RRO_RAY_MAX_STEPS;
        break;
      }
      const double hl = ldexp(1.0, -l);
      int step[3];
      const double chiB = rro_exit(&ray, m, hl, chiA, lo, step);
      if (ngp) {
        /* Eq. (Iclensing_ngp): the leaf's own centre tensor */
        sum += rro_integral_ngp(&ray, tc + 6 * cur.cell, chiA, chiB);
      } else {
        double corner[8][6];
        if (cv) {
          memcpy(corner, cv + 48 * cur.cell, sizeof(corner));
        } else {
          leaf_corners(t, tc, cur.cell, corner);
        }
        const double p1[3] = {(double)m[0] * hl, (double)m[1] * hl, (double)m[2] * hl};
        sum += rro_integral_trilinear(&ray, corner, p1, hl, chiA, chiB);
      }
      if (log && count < log_stride) {
        rro_segment* s = log + r * log_stride + count;
        s->cell = cur.cell;
        s->chi_a = chiA;
        s->chi_b = chiB;
      }
      hv = rro_fnv_segment(hv, cur.cell, chiA, chiB);
      ++count;
      if (chiB == lo) break;
      for (int a = 0; a < 3; ++a)
        if (step[a]) m[a] += (ray.n[a] > 0.0) ? -1 : 1;
      chiA = chiB;
      /* locate the leaf that holds the ray just past the crossed face(s) */
      loc_t q = descend(t, l, m);
      if (q.level < l) {
        for (int a = 0; a < 3; ++a) m[a] = fdiv(m[a], (int64_t)1 << (l - q.level));
        l = q.level;
      }
      while (t->child_oct[q.cell] >= 0) {
        int child = 0;
        for (int a = 0; a < 3; ++a) {
          int bit;
          if (step[a])
            bit = ray.n[a] > 0.0 ? 1 : 0;
          else
            bit = slab_child(&ray, a, m[a], l, chiA);
          m[a] = 2 * m[a] + bit;
          child |= bit << a;
        }
        q.cell = nbase + 8 * (int64_t)t->child_oct[q.cell] + child;
        ++l;
      }
      cur = q;
    }
    if (kappa) kappa[r] = kappa_scale * sum;
    if (hash) hash[r] = hv;
    if (ncross) ncross[r] = count;
    if (status) status[r] = st;
  }
  return 0;
}

/* The many-source walk (Eqs. Isources, Isources1; see rro_sources.c) through
 * the octree: the same descent and ascent as rro_trace_octree, with the walk
 * also stopping at every source distance in [chi_lo, chi_hi). */
int32_t rro_trace_octree_sources(const rro_octree* t, double box, const double* observer,
                                 int64_t n_rays, const double* dir, const double* chi_hi,
                                 const double* chi_lo, int32_t n_src, const double* chi_src,
                                 double kappa_scale, int32_t quantity, const double* cv,
                                 int64_t max_steps, int32_t n_threads, double* moments,
                                 double* pieces, uint64_t* hash, int64_t* ncross,
                                 int32_t* status) {
  const double h0 = box / (double)t->n;
  double o[3];
  for (int a = 0; a < 3; ++a) o[a] = observer[a] / h0;
  double* src = (double*)malloc(sizeof(double) * (size_t)(n_src > 0 ? n_src : 1));
  for (int32_t j = 0; j < n_src; ++j) src[j] = chi_src[j] / h0;
  if (n_threads > 0) rro_set_threads(n_threads);
  const int64_t nbase = (int64_t)t->n * t->n * t->n;

#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < n_rays; ++r) {
    rro_ray ray;
    rro_ray_init(&ray, dir + 3 * r, o, 1.0, quantity);
    const double lo = chi_lo[r] / h0;
    double chiA = chi_hi[r] / h0;
    int64_t m[3];
    for (int a = 0; a < 3; ++a) m[a] = rro_start_slab(&ray, a, chiA, 1.0);
    loc_t cur = descend(t, 0, m);
    int32_t l = 0;
    while (t->child_oct[cur.cell] >= 0) {
      int child = 0;
      for (int a = 0; a < 3; ++a) {
        const int bit = slab_child(&ray, a, m[a], l, chiA);
        m[a] = 2 * m[a] + bit;
        child |= bit << a;
      }
      cur.cell = nbase + 8 * (int64_t)t->child_oct[cur.cell] + child;
      ++l;
    }
    int32_t jn = 0;
    while (jn < n_src && !(src[jn] < chiA)) ++jn;

    double A = moments[2 * r + 0], B = moments[2 * r + 1];
    uint64_t hv = RRO_FNV_OFFSET;
    int64_t count = 0;
    int32_t st = RRO_RAY_OK;
    for (;;) {
      if (count >= max_steps) {
        st = RRO_RAY_MAX_STEPS;
        break;
      }
      const double hl = ldexp(1.0, -l);
      const double stop = (jn < n_src && src[jn] >= lo) ? src[jn] : lo;
      int step[3];
      const double chiB = rro_exit(&ray, m, hl, chiA, stop, step);
      double corner[8][6];
      memcpy(corner, cv + 48 * cur.cell, sizeof(corner));
      double Q[9];
      Q[0] = 0.0;
      for (int i = 1; i <= 8; ++i) Q[i] = rro_quantity(&ray, corner[i - 1]);
      const double p1[3] = {(double)m[0] * hl, (double)m[1] * hl, (double)m[2] * hl};
      double ma, mb;
      rro_moments_trilinear_q(&ray, Q, p1, hl, chiA, chiB, &ma, &mb);
      A += kappa_scale * ma;
      B += kappa_scale * mb;
      hv = rro_fnv_segment(hv, cur.cell, chiA, chiB);
      ++count;
      if (jn < n_src && src[jn] == chiB) {
        pieces[(r * n_src + jn) * 2 + 0] = A;
        pieces[(r * n_src + jn) * 2 + 1] = B;
        A = 0.0;
        B = 0.0;
        ++jn;
      }
      if (chiB == lo) break;
      int any = 0;
      for (int a = 0; a < 3; ++a) any |= step[a];
      chiA = chiB;
      if (!any) continue;   /* stopped at a source inside the leaf */
      for (int a = 0; a < 3; ++a)
        if (step[a]) m[a] += (ray.n[a] > 0.0) ? -1 : 1;
      loc_t q = descend(t, l, m);
      if (q.level < l) {
        for (int a = 0; a < 3; ++a) m[a] = fdiv(m[a], (int64_t)1 << (l - q.level));
        l = q.level;
      }
      while (t->child_oct[q.cell] >= 0) {
        int child = 0;
        for (int a = 0; a < 3; ++a) {
          int bit;
          if (step[a])
            bit = ray.n[a] > 0.0 ? 1 : 0;
          else
            bit = slab_child(&ray, a, m[a], l, chiA);
          m[a] = 2 * m[a] + bit;
          child |= bit << a;
        }
        q.cell = nbase + 8 * (int64_t)t->child_oct[q.cell] + child;
        ++l;
      }
      cur = q;
    }
    moments[2 * r + 0] = A;
    moments[2 * r + 1] = B;
    if (hash) hash[r] = hv;
    if (ncross) ncross[r] = count;
    if (status) status[r] = st;
  }
  free(src);
  return 0;
}
