/*
 * rro_uniform.c -- FP64 oracle, uniform periodic (or open) grid.
 * TEST INFRASTRUCTURE ONLY (see rro.h).  Plain loops, no blocking, no fusion.
 */
#include "rro.h"
#include "rro_common.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static inline int64_t wrap(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

static inline int64_t lin(int64_t i, int64_t j, int64_t k, int64_t n) {
  return (wrap(k, n) * n + wrap(j, n)) * n + wrap(i, n);
}

/* Eq. (tidalexample) and its analogues for the other components. */
void rro_centre_tensor_uniform(int32_t n, int32_t open, double h, const double* phi, double* tc) {
  const double h2 = h * h;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) {
        double* out = tc + 6 * lin(i, j, k, n);
        if (open && (i < 1 || j < 1 || k < 1 || i > n - 2 || j > n - 2 || k > n - 2)) {
          for (int c = 0; c < 6; ++c) out[c] = NAN;
          continue;
        }
#define P(di, dj, dk) phi[lin(i + (di), j + (dj), k + (dk), n)]
        out[0] = (P(-1, 0, 0) - 2.0 * P(0, 0, 0) + P(1, 0, 0)) / h2;
        out[1] = (P(0, -1, 0) - 2.0 * P(0, 0, 0) + P(0, 1, 0)) / h2;
        out[2] = (P(0, 0, -1) - 2.0 * P(0, 0, 0) + P(0, 0, 1)) / h2;
        out[3] = (P(1, 1, 0) + P(-1, -1, 0) - P(1, -1, 0) - P(-1, 1, 0)) / (4.0 * h2);
        out[4] = (P(1, 0, 1) + P(-1, 0, -1) - P(1, 0, -1) - P(-1, 0, 1)) / (4.0 * h2);
        out[5] = (P(0, 1, 1) + P(0, -1, -1) - P(0, 1, -1) - P(0, -1, 1)) / (4.0 * h2);
#undef P
      }
}

/* Sec. III H: a vertex shared by eight cells of one level takes the mean of
 * the eight centre values.  Vertex (i,j,k) sits at the lower corner of cell
 * (i,j,k). */
void rro_vertex_tensor_uniform(int32_t n, const double* tc, double* tv) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) {
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int dz = -1; dz <= 0; ++dz)
          for (int dy = -1; dy <= 0; ++dy)
            for (int dx = -1; dx <= 0; ++dx) {
              const double* t = tc + 6 * lin(i + dx, j + dy, k + dz, n);
              for (int c = 0; c < 6; ++c) acc[c] += t[c];
            }
        double* out = tv + 6 * lin(i, j, k, n);
        for (int c = 0; c < 6; ++c) out[c] = acc[c] / 8.0;
      }
}

int32_t rro_trace_uniform(int32_t n, int32_t open, double box, const double* observer,
                          int64_t n_rays, const double* dir, const double* chi_s,
                          const double* chi_hi, const double* chi_lo, double kappa_scale,
                          int32_t quantity, int32_t ngp, const double* tv, const double* tc,
                          int64_t max_steps, int32_t n_threads,
                          double* kappa, uint64_t* hash, int64_t* ncross, int32_t* status,
                          rro_segment* log, int64_t log_stride) {
  const double h0 = box / (double)n;
  double o[3];
  for (int a = 0; a < 3; ++a) o[a] = observer[a] / h0;
  if (n_threads > 0) rro_set_threads(n_threads);

#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < n_rays; ++r) {
    rro_ray ray;
    rro_ray_init(&ray, dir + 3 * r, o, chi_s[r] / h0, quantity);
    const double lo = chi_lo[r] / h0;
    double chiA = chi_hi[r] / h0;
    int64_t m[3];
    for (int a = 0; a < 3; ++a) m[a] = rro_start_slab(&ray, a, chiA, 1.0);

    double sum = 0.0;
    uint64_t hv = RRO_FNV_OFFSET;
    int64_t count = 0;
    int32_t st = RRO_RAY_OK;
    for (;;) {
      if (open && (m[0] < 2 || m[1] < 2 || m[2] < 2 || m[0] > n - 3 || m[1] > n - 3 ||
                   m[2] > n - 3)) {
        st = RRO_RAY_OUT_OF_DOMAIN;
        break;
      }
      if (count >= max_steps) {
        st = RRO_RAY_MAX_STEPS;
        break;
      }
      int step[3];
      const double chiB = rro_exit(&ray, m, 1.0, chiA, lo, step);
      const int64_t cell = lin(m[0], m[1], m[2], n);
      double ic;
      if (ngp) {
        ic = rro_integral_ngp(&ray, tc + 6 * cell, chiA, chiB);
      } else {
        double tcorner[8][6];
        for (int v = 0; v < 8; ++v) {
          const double* t = tv + 6 * lin(m[0] + (v & 1), m[1] + ((v >> 1) & 1),
                                         m[2] + ((v >> 2) & 1), n);
          for (int c = 0; c < 6; ++c) tcorner[v][c] = t[c];
        }
        const double p1[3] = {(double)m[0], (double)m[1], (double)m[2]};
        ic = rro_integral_trilinear(&ray, tcorner, p1, 1.0, chiA, chiB);
      }
      sum += ic;
      if (log && count < log_stride) {
        rro_segment* s = log + r * log_stride + count;
        s->cell = cell;
        s->chi_a = chiA;
        s->chi_b = chiB;
      }
      hv = rro_fnv_segment(hv, cell, chiA, chiB);
      ++count;
      if (chiB == lo) break;
      for (int a = 0; a < 3; ++a)
        if (step[a]) m[a] += (ray.n[a] > 0.0) ? -1 : 1;
      chiA = chiB;
    }
    if (kappa) kappa[r] = kappa_scale * sum;
    if (hash) hash[r] = hv;
    if (ncross) ncross[r] = count;
    if (status) status[r] = st;
  }
  return 0;
}

/* Single-cell entry points used by the oracle's own pins. */
double rro_cell_integral(const double* Q /* 8 vertex values */, const double* p1, double h,
                         const double* dir, const double* o, double chis, double chiA,
                         double chiB) {
  rro_ray ray;
  rro_ray_init(&ray, dir, o, chis, RRO_Q_KAPPA);
  double q[9];
  q[0] = 0.0;
  for (int i = 0; i < 8; ++i) q[i + 1] = Q[i];
  return rro_integral_trilinear_q(&ray, q, p1, h, chiA, chiB);
}

double rro_projection(const double* dir, const double* T, int32_t quantity) {
  const double o[3] = {0, 0, 0};
  rro_ray ray;
  rro_ray_init(&ray, dir, o, 1.0, quantity);
  return rro_quantity(&ray, T);
}
