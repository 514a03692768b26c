/*
 * rro_method_a.c -- FP64 oracle of Method A (Sec. IV D, Eq. kappa2) on a
 * uniform periodic (or open) grid.
 * TEST INFRASTRUCTURE ONLY (see rro.h).  Plain loops, no blocking, no fusion.
 *
 * Per N-body step (chi segment [chi_lo, chi_hi], fields static within it):
 *   c^2 kappa += delta_coeff int g delta dchi            (Poisson term, Q = delta)
 *              + int (n . grad Phi) dg/dchi dchi         (K = 1 - 2 chi / chi_s)
 *              - [g n . grad Phi] evaluated from chi_lo to chi_hi
 *                                                        (surface term, Eq. 2nterm)
 * The term with the time derivative of the potential is dropped, as in the
 * paper.  delta and grad Phi are interpolated to vertices like the tidal
 * tensor (Sec. III H) and trilinearly inside cells.
 */
#include "rro.h"
#include "rro_common.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static inline int64_t wrap_a(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

static inline int64_t lin_a(int64_t i, int64_t j, int64_t k, int64_t n) {
  return (wrap_a(k, n) * n + wrap_a(j, n)) * n + wrap_a(i, n);
}

/* Cell centres: delta as given, grad Phi by central differences of spacing h
 * (the force RAMSES computes); vertices: the mean of the eight incident cells.
 * fv[4 v + 0] = delta, fv[4 v + 1..3] = d Phi / dx, dy, dz.  Open grids: the
 * gradient needs one neighbour per side, the vertex mean one more cell, so
 * vertex layers 0, 1 and n - 1 are NaN. */
void rro_method_a_vertex_fields(int32_t n, int32_t open, double h, const double* phi,
                                const double* delta, double* fv) {
  double* fc = (double*)malloc(sizeof(double) * 4 * (size_t)n * n * n);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) {
        double* out = fc + 4 * lin_a(i, j, k, n);
        out[0] = delta[lin_a(i, j, k, n)];
        out[1] = (phi[lin_a(i + 1, j, k, n)] - phi[lin_a(i - 1, j, k, n)]) / (2.0 * h);
        out[2] = (phi[lin_a(i, j + 1, k, n)] - phi[lin_a(i, j - 1, k, n)]) / (2.0 * h);
        out[3] = (phi[lin_a(i, j, k + 1, n)] - phi[lin_a(i, j, k - 1, n)]) / (2.0 * h);
      }
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) {
        double* out = fv + 4 * lin_a(i, j, k, n);
        if (open && (i < 2 || j < 2 || k < 2 || i > n - 2 || j > n - 2 || k > n - 2)) {
          for (int c = 0; c < 4; ++c) out[c] = NAN;
          continue;
        }
        double acc[4] = {0, 0, 0, 0};
        for (int dz = -1; dz <= 0; ++dz)
          for (int dy = -1; dy <= 0; ++dy)
            for (int dx = -1; dx <= 0; ++dx) {
              const double* c = fc + 4 * lin_a(i + dx, j + dy, k + dz, n);
              for (int u = 0; u < 4; ++u) acc[u] += c[u];
            }
        for (int u = 0; u < 4; ++u) out[u] = acc[u] / 8.0;
      }
  free(fc);
}

/* The cubic Q(chi_A + s) = sum_N d_N s^(N-1) of a trilinear field along the
 * segment (App. B, Eq. dns; Q[1..8] the values at the paper's P_i). */
static void rro_segment_poly(const rro_ray* ray, const double* Q, const double* p1, double h,
                             double chiA, double* d) {
  double al[9];
  al[1] = Q[1];
  al[2] = Q[2] - Q[1];
  al[3] = Q[3] - Q[1];
  al[4] = Q[5] - Q[1];
  al[5] = Q[4] - Q[3] - Q[2] + Q[1];
  al[6] = Q[7] - Q[5] - Q[3] + Q[1];
  al[7] = Q[6] - Q[5] - Q[2] + Q[1];
  al[8] = Q[8] - Q[7] - Q[6] - Q[4] + Q[2] + Q[5] + Q[3] - Q[1];
  const double a = ray->o[0] + chiA * ray->n[0] - p1[0];
  const double b = ray->o[1] + chiA * ray->n[1] - p1[1];
  const double c = ray->o[2] + chiA * ray->n[2] - p1[2];
  const double sx = ray->n[0], sy = ray->n[1], sz = ray->n[2];
  const double h2 = h * h, h3 = h * h * h;
  d[1] = al[1] + (al[2] * a + al[3] * b + al[4] * c) / h +
         (al[5] * a * b + al[6] * b * c + al[7] * a * c) / h2 + al[8] * a * b * c / h3;
  d[2] = (al[2] * sx + al[3] * sy + al[4] * sz) / h +
         ((al[6] * c + al[5] * a) * sy + (al[7] * c + al[5] * b) * sx +
          (al[7] * a + al[6] * b) * sz) / h2 +
         (al[8] * b * c * sx + al[8] * a * b * sz + al[8] * a * c * sy) / h3;
  d[3] = (al[5] * sx * sy + al[7] * sx * sz + al[6] * sy * sz) / h2 +
         (al[8] * a * sy * sz + al[8] * b * sx * sz + al[8] * c * sx * sy) / h3;
  d[4] = al[8] / h3 * (sx * sy * sz);
}

/* int_{chi_B}^{chi_A} (1 - 2 chi / chi_s) Q dchi: the kernel of the gradient
 * term integrated against the cubic, the analogue of Eq. (Iclensing) with
 * K = dg/dchi (R = chi_B - chi_A). */
double rro_integral_trilinear_k(const rro_ray* ray, const double* Q, const double* p1, double h,
                                double chiA, double chiB) {
  double d[5];
  rro_segment_poly(ray, Q, p1, h, chiA, d);
  const double chis = ray->chis;
  const double R = chiB - chiA;
  double sum = 0.0, RN = 1.0;
  for (int N = 1; N <= 4; ++N) {
    RN *= R;
    sum += d[N] * ((2.0 * chiA - chis) * RN / N + 2.0 * RN * R / (N + 1));
  }
  return sum / chis;
}

/* The trilinear value at chi_A + s. */
static double rro_segment_value(const rro_ray* ray, const double* Q, const double* p1, double h,
                                double chiA, double s) {
  double d[5];
  rro_segment_poly(ray, Q, p1, h, chiA, d);
  return d[1] + s * (d[2] + s * (d[3] + s * d[4]));
}

static inline double rro_g(double chi, double chis) { return chi * (chis - chi) / chis; }

int32_t rro_trace_uniform_method_a(int32_t n, int32_t open, double box, const double* observer,
                                   int64_t n_rays, const double* dir, const double* chi_s,
                                   const double* chi_hi, const double* chi_lo,
                                   double kappa_scale, double delta_coeff, const double* fv,
                                   int64_t max_steps, int32_t n_threads, double* kappa,
                                   uint64_t* hash, int64_t* ncross, int32_t* status) {
  const double h0 = box / (double)n;
  double o[3];
  for (int a = 0; a < 3; ++a) o[a] = observer[a] / h0;
  /* delta_coeff is per length^2 of the box unit: base-cell units multiply by h0^2 */
  const double cd = delta_coeff * h0 * h0;
  if (n_threads > 0) rro_set_threads(n_threads);

#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < n_rays; ++r) {
    rro_ray ray;
    rro_ray_init(&ray, dir + 3 * r, o, chi_s[r] / h0, RRO_Q_KAPPA);
    const double lo = chi_lo[r] / h0;
    const double hi = chi_hi[r] / h0;
    double chiA = hi;
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
      const int64_t cell = lin_a(m[0], m[1], m[2], n);
      double Qd[9], Qg[9];
      Qd[0] = Qg[0] = 0.0;
      for (int v = 0; v < 8; ++v) {
        const double* f = fv + 4 * lin_a(m[0] + (v & 1), m[1] + ((v >> 1) & 1),
                                         m[2] + ((v >> 2) & 1), n);
        Qd[v + 1] = cd * f[0];
        Qg[v + 1] = ray.n[0] * f[1] + ray.n[1] * f[2] + ray.n[2] * f[3];
      }
      const double p1[3] = {(double)m[0], (double)m[1], (double)m[2]};
      sum += rro_integral_trilinear_q(&ray, Qd, p1, 1.0, chiA, chiB);
      sum += rro_integral_trilinear_k(&ray, Qg, p1, 1.0, chiA, chiB);
      /* surface term of this step, Eq. (2nterm): -g n.grad Phi at chi_hi, +at chi_lo */
      if (count == 0) sum -= rro_g(hi, ray.chis) * rro_segment_value(&ray, Qg, p1, 1.0, chiA, 0.0);
      if (chiB == lo)
        sum += rro_g(lo, ray.chis) * rro_segment_value(&ray, Qg, p1, 1.0, chiA, chiB - chiA);
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

/* Single-cell entry points for the pins: the K-kernel integral and the
 * trilinear value along a segment. */
double rro_cell_integral_k(const double* Q /* 8 vertex values */, const double* p1, double h,
                           const double* dir, const double* o, double chis, double chiA,
                           double chiB) {
  rro_ray ray;
  rro_ray_init(&ray, dir, o, chis, RRO_Q_KAPPA);
  double Qp[9];
  Qp[0] = 0.0;
  for (int i = 0; i < 8; ++i) Qp[i + 1] = Q[i];
  return rro_integral_trilinear_k(&ray, Qp, p1, h, chiA, chiB);
}
