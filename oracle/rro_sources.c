/*
 * rro_sources.c -- FP64 oracle of the many-source-distance walk (Sec. VII,
 * Eqs. Isources, Isources1) on a uniform periodic (or open) grid.
 * TEST INFRASTRUCTURE ONLY (see rro.h).  Plain loops, no blocking, no fusion.
 *
 * The lensing kernel g = chi (chi_s - chi) / chi_s splits into chi and
 * chi^2 / chi_s, so one walk from the farthest source towards the observer
 * can integrate A = int chi Q and B = int chi^2 Q without fixing chi_s.  The
 * walk stops at every source distance chi_s,j it passes (a cell holding one
 * is cut there into two pieces) and hands out the integrals accumulated
 * since the previous stop (the pieces between consecutive sources); kappa of
 * source j then follows from the pieces below chi_s,j (rro.h:
 * rro_kappa_from_pieces).
 */
#include "rro.h"
#include "rro_common.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static inline int64_t wrap_s(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

static inline int64_t lin_s(int64_t i, int64_t j, int64_t k, int64_t n) {
  return (wrap_s(k, n) * n + wrap_s(j, n)) * n + wrap_s(i, n);
}

int32_t rro_trace_uniform_sources(int32_t n, int32_t open, double box, const double* observer,
                                  int64_t n_rays, const double* dir, const double* chi_hi,
                                  const double* chi_lo, int32_t n_src, const double* chi_src,
                                  double kappa_scale, int32_t quantity, const double* tv,
                                  int64_t max_steps, int32_t n_threads, double* moments,
                                  double* pieces, uint64_t* hash, int64_t* ncross,
                                  int32_t* status) {
  const double h0 = box / (double)n;
  double o[3];
  for (int a = 0; a < 3; ++a) o[a] = observer[a] / h0;
  double* src = (double*)malloc(sizeof(double) * (size_t)(n_src > 0 ? n_src : 1));
  for (int32_t j = 0; j < n_src; ++j) src[j] = chi_src[j] / h0;
  if (n_threads > 0) rro_set_threads(n_threads);

#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < n_rays; ++r) {
    rro_ray ray;
    /* chi_s does not enter the walk: the two moments carry no source distance */
    rro_ray_init(&ray, dir + 3 * r, o, 1.0, quantity);
    const double lo = chi_lo[r] / h0;
    double chiA = chi_hi[r] / h0;
    int64_t m[3];
    for (int a = 0; a < 3; ++a) m[a] = rro_start_slab(&ray, a, chiA, 1.0);
    /* the sources this call stops at: chi_lo <= chi_s,j < chi_hi */
    int32_t jn = 0;
    while (jn < n_src && !(src[jn] < chiA)) ++jn;

    double A = moments[2 * r + 0], B = moments[2 * r + 1];
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
      /* the next stop: a source distance inside the window, else chi_lo */
      const double stop = (jn < n_src && src[jn] >= lo) ? src[jn] : lo;
      int step[3];
      const double chiB = rro_exit(&ray, m, 1.0, chiA, stop, step);
      const int64_t cell = lin_s(m[0], m[1], m[2], n);
      double tcorner[8][6];
      for (int v = 0; v < 8; ++v) {
        const double* t = tv + 6 * lin_s(m[0] + (v & 1), m[1] + ((v >> 1) & 1),
                                         m[2] + ((v >> 2) & 1), n);
        for (int c = 0; c < 6; ++c) tcorner[v][c] = t[c];
      }
      double Q[9];
      Q[0] = 0.0;
      for (int i = 1; i <= 8; ++i) Q[i] = rro_quantity(&ray, tcorner[i - 1]);
      const double p1[3] = {(double)m[0], (double)m[1], (double)m[2]};
      double ma, mb;
      rro_moments_trilinear_q(&ray, Q, p1, 1.0, chiA, chiB, &ma, &mb);
      A += kappa_scale * ma;
      B += kappa_scale * mb;
      hv = rro_fnv_segment(hv, cell, chiA, chiB);
      ++count;
      if (jn < n_src && src[jn] == chiB) {
        /* Eq. (Isources1): hand out what was accumulated since the last stop */
        pieces[(r * n_src + jn) * 2 + 0] = A;
        pieces[(r * n_src + jn) * 2 + 1] = B;
        A = 0.0;
        B = 0.0;
        ++jn;
      }
      if (chiB == lo) break;
      /* a stop inside the cell (no face at chi_B) continues in the same cell */
      for (int a = 0; a < 3; ++a)
        if (step[a]) m[a] += (ray.n[a] > 0.0) ? -1 : 1;
      chiA = chiB;
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

/* kappa of every source once the walk has reached the observer.  With
 * P_j = (A, B) piece handed out at source j (from the previous stop down to
 * chi_s,j) and (A_0, B_0) the integrals left below the nearest source:
 * Eq. (Isources) for the farthest source uses the whole of A and B below it,
 *   A(chi_s,0) = A_0 + sum_{i >= 1} A_i,
 * and Eq. (Isources1) takes each nearer source by removing the piece above it:
 *   A(chi_s,j) = A(chi_s,j-1) - A_j   (the same for B),
 *   kappa_j = A(chi_s,j) - B(chi_s,j) / chi_s,j   (grid units). */
void rro_kappa_from_pieces(int64_t n_rays, int32_t n_src, const double* chi_src, double box,
                           int32_t n_base, const double* moments, const double* pieces,
                           double* kappa) {
  const double h0 = box / (double)n_base;
  for (int64_t r = 0; r < n_rays; ++r) {
    double A = moments[2 * r + 0], B = moments[2 * r + 1];
    for (int32_t i = 1; i < n_src; ++i) {
      A += pieces[(r * n_src + i) * 2 + 0];
      B += pieces[(r * n_src + i) * 2 + 1];
    }
    for (int32_t j = 0; j < n_src; ++j) {
      if (j > 0) {
        A -= pieces[(r * n_src + j) * 2 + 0];
        B -= pieces[(r * n_src + j) * 2 + 1];
      }
      kappa[r * n_src + j] = A - B / (chi_src[j] / h0);
    }
  }
}

/* Single-cell entry point for the pins: out[0] = int chi Q, out[1] = int
 * chi^2 Q over [chi_B, chi_A] of the trilinear field with vertex values Q. */
void rro_cell_moments(const double* Q /* 8 vertex values */, const double* p1, double h,
                      const double* dir, const double* o, double chiA, double chiB,
                      double* out) {
  rro_ray ray;
  rro_ray_init(&ray, dir, o, 1.0, RRO_Q_KAPPA);
  double q[9];
  q[0] = 0.0;
  for (int i = 0; i < 8; ++i) q[i + 1] = Q[i];
  rro_moments_trilinear_q(&ray, q, p1, h, chiA, chiB, &out[0], &out[1]);
}
