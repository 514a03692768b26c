/*
 * rro_adjoint.c -- FP64 oracle for dL/dPhi of kappa on a uniform periodic grid.
 * TEST INFRASTRUCTURE ONLY (see rro.h).
 *
 * kappa is linear in Phi (straight rays, Born approximation, Sec. IV A,
 * Eq. jacobian2), so the gradient is the transpose of the forward chain
 *   Phi --(Eq. tidalexample)--> centre tensor --(vertex mean, Sec. III H)-->
 *   vertex tensor --(Eqs. n1n1+n2n2, trilinear_coef, dns, Iclensing)--> kappa.
 * Each transpose is written as the explicit scatter form of its forward map.
 * The per-cell derivative dI_c/dQ_v is the forward closed form evaluated on
 * the unit vector e_v (exact because I_c is linear in the vertex values).
 */
#include "rro.h"
#include "rro_common.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static inline int64_t wrapi(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}
static inline int64_t lini(int64_t i, int64_t j, int64_t k, int64_t n) {
  return (wrapi(k, n) * n + wrapi(j, n)) * n + wrapi(i, n);
}

int32_t rro_trace_adjoint_uniform(int32_t n, double box, const double* observer,
                                  int64_t n_rays, const double* dir, const double* chi_s,
                                  const double* chi_hi, const double* chi_lo,
                                  double kappa_scale, const double* dl_dkappa,
                                  int32_t n_threads, double* dl_dphi) {
  const int64_t nc = (int64_t)n * n * n;
  const double h0 = box / (double)n;
  double o[3];
  for (int a = 0; a < 3; ++a) o[a] = observer[a] / h0;
  if (n_threads > 0) rro_set_threads(n_threads);

  double* lam = (double*)calloc((size_t)nc * 6, sizeof(double)); /* dL/d(vertex tensor) */
  double* gc = (double*)calloc((size_t)nc * 6, sizeof(double));  /* dL/d(centre tensor) */
  if (!lam || !gc) {
    free(lam);
    free(gc);
    return -1;
  }

  /* 1. transpose of the per-ray sum of per-cell integrals */
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < n_rays; ++r) {
    const double w = dl_dkappa[r] * kappa_scale;
    if (w == 0.0) continue;
    rro_ray ray;
    rro_ray_init(&ray, dir + 3 * r, o, chi_s[r] / h0, RRO_Q_KAPPA);
    /* dQ/dT_ab for this ray's direction: the projection on unit tensors */
    double dq[6];
    for (int c = 0; c < 6; ++c) {
      double e[6] = {0, 0, 0, 0, 0, 0};
      e[c] = 1.0;
      dq[c] = rro_quantity(&ray, e);
    }
    const double lo = chi_lo[r] / h0;
    double chiA = chi_hi[r] / h0;
    int64_t m[3];
    for (int a = 0; a < 3; ++a) m[a] = rro_start_slab(&ray, a, chiA, 1.0);
    for (;;) {
      int step[3];
      const double chiB = rro_exit(&ray, m, 1.0, chiA, lo, step);
      const double p1[3] = {(double)m[0], (double)m[1], (double)m[2]};
      for (int v = 0; v < 8; ++v) {
        double q[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        q[v + 1] = 1.0;
        const double dIdQ = rro_integral_trilinear_q(&ray, q, p1, 1.0, chiA, chiB);
        const int64_t vid =
            lini(m[0] + (v & 1), m[1] + ((v >> 1) & 1), m[2] + ((v >> 2) & 1), n);
        for (int c = 0; c < 6; ++c) {
#pragma omp atomic
          lam[6 * vid + c] += w * dIdQ * dq[c];
        }
      }
      if (chiB == lo) break;
      for (int a = 0; a < 3; ++a)
        if (step[a]) m[a] += (ray.n[a] > 0.0) ? -1 : 1;
      chiA = chiB;
    }
  }

  /* 2. transpose of the vertex mean: every vertex returns 1/8 to each of its
   *    eight cells */
  for (int64_t k = 0; k < n; ++k)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) {
        const double* l = lam + 6 * lini(i, j, k, n);
        for (int dz = -1; dz <= 0; ++dz)
          for (int dy = -1; dy <= 0; ++dy)
            for (int dx = -1; dx <= 0; ++dx) {
              double* g = gc + 6 * lini(i + dx, j + dy, k + dz, n);
              for (int c = 0; c < 6; ++c) g[c] += l[c] / 8.0;
            }
      }

  /* 3. transpose of the finite-difference stencil (h = 1 grid units) */
  for (int64_t k = 0; k < n; ++k)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) {
        const double* g = gc + 6 * lini(i, j, k, n);
#define ADD(di, dj, dk, v) dl_dphi[lini(i + (di), j + (dj), k + (dk), n)] += (v)
        ADD(-1, 0, 0, g[0]);
        ADD(0, 0, 0, -2.0 * g[0]);
        ADD(1, 0, 0, g[0]);
        ADD(0, -1, 0, g[1]);
        ADD(0, 0, 0, -2.0 * g[1]);
        ADD(0, 1, 0, g[1]);
        ADD(0, 0, -1, g[2]);
        ADD(0, 0, 0, -2.0 * g[2]);
        ADD(0, 0, 1, g[2]);
        ADD(1, 1, 0, g[3] / 4.0);
        ADD(-1, -1, 0, g[3] / 4.0);
        ADD(1, -1, 0, -g[3] / 4.0);
        ADD(-1, 1, 0, -g[3] / 4.0);
        ADD(1, 0, 1, g[4] / 4.0);
        ADD(-1, 0, -1, g[4] / 4.0);
        ADD(1, 0, -1, -g[4] / 4.0);
        ADD(-1, 0, 1, -g[4] / 4.0);
        ADD(0, 1, 1, g[5] / 4.0);
        ADD(0, -1, -1, g[5] / 4.0);
        ADD(0, 1, -1, -g[5] / 4.0);
        ADD(0, -1, 1, -g[5] / 4.0);
#undef ADD
      }
  free(lam);
  free(gc);
  return 0;
}
