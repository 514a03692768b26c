/*
 * rro_isw.c -- FP64 oracle of the ISW integrand (Sec. VII, "ISW
 * simulations"; Eq. I1 with Q the time derivative of the potential) on a
 * uniform periodic (or open) grid.
 * TEST INFRASTRUCTURE ONLY (see rro.h).  Plain loops, no blocking, no fusion.
 *
 * Per N-body step the cell value of Q is the finite difference
 * (Phi_curr - Phi_prev) / dt of the potentials of the current and the
 * previous step; vertices take the mean of their eight cells (Sec. III H)
 * and Q is trilinear inside a cell (Eq. trilinear_int).  The paper gives no
 * kernel K for this case: it is taken constant within a step, the caller's
 * scale factor, so each cell adds scale * int Q dchi over its piece (Eq. Ic
 * with K = 1), from the same cubic along the ray as Eq. (Iclensing).
 */
#include "rro.h"
#include "rro_common.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static inline int64_t wrap_i(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

static inline int64_t lin_i(int64_t i, int64_t j, int64_t k, int64_t n) {
  return (wrap_i(k, n) * n + wrap_i(j, n)) * n + wrap_i(i, n);
}

/* Vertex (i,j,k) = mean over cells {i-1,i} x {j-1,j} x {k-1,k} of
 * (phi_curr - phi_prev) * inv_dt.  Open grids: vertices on the lower faces
 * (index 0 on any axis) have no cell below and are NaN. */
void rro_isw_vertex_field(int32_t n, int32_t open, const double* phi_curr,
                          const double* phi_prev, double inv_dt, double* qv) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) {
        double* out = qv + lin_i(i, j, k, n);
        if (open && (i < 1 || j < 1 || k < 1)) {
          *out = NAN;
          continue;
        }
        double acc = 0.0;
        for (int dz = -1; dz <= 0; ++dz)
          for (int dy = -1; dy <= 0; ++dy)
            for (int dx = -1; dx <= 0; ++dx) {
              const int64_t c = lin_i(i + dx, j + dy, k + dz, n);
              acc += (phi_curr[c] - phi_prev[c]) * inv_dt;
            }
        *out = acc / 8.0;
      }
}

/* int_{chi_B}^{chi_A} Q dchi of the trilinear field: with chi = chi_A + s and
 * R = chi_B - chi_A, -sum_N d_N R^N / N (App. B, Eq. dns). */
static double rro_integral_trilinear_one(const rro_ray* ray, const double* Q, const double* p1,
                                         double h, double chiA, double chiB) {
  double d[5];
  rro_dn(ray, Q, p1, h, chiA, d);
  const double R = chiB - chiA;
  double sum = 0.0, RN = 1.0;
  for (int N = 1; N <= 4; ++N) {
    RN *= R;
    sum += d[N] * RN / N;
  }
  return -sum;
}

int32_t rro_trace_uniform_isw(int32_t n, int32_t open, double box, const double* observer,
                              int64_t n_rays, const double* dir, const double* chi_hi,
                              const double* chi_lo, double scale, const double* qv,
                              int64_t max_steps, int32_t n_threads, double* out, uint64_t* hash,
                              int64_t* ncross, int32_t* status) {
  const double h0 = box / (double)n;
  double o[3];
  for (int a = 0; a < 3; ++a) o[a] = observer[a] / h0;
  if (n_threads > 0) rro_set_threads(n_threads);

#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < n_rays; ++r) {
    rro_ray ray;
    rro_ray_init(&ray, dir + 3 * r, o, 1.0, RRO_Q_KAPPA);
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
      const int64_t cell = lin_i(m[0], m[1], m[2], n);
      double Q[9];
      Q[0] = 0.0;
      for (int v = 0; v < 8; ++v)
        Q[v + 1] = qv[lin_i(m[0] + (v & 1), m[1] + ((v >> 1) & 1), m[2] + ((v >> 2) & 1), n)];
      const double p1[3] = {(double)m[0], (double)m[1], (double)m[2]};
      /* lengths in base-cell units: int Q dchi~ times h0 gives box units */
      sum += rro_integral_trilinear_one(&ray, Q, p1, 1.0, chiA, chiB) * h0;
      hv = rro_fnv_segment(hv, cell, chiA, chiB);
      ++count;
      if (chiB == lo) break;
      for (int a = 0; a < 3; ++a)
        if (step[a]) m[a] += (ray.n[a] > 0.0) ? -1 : 1;
      chiA = chiB;
    }
    if (out) out[r] = scale * sum;
    if (hash) hash[r] = hv;
    if (ncross) ncross[r] = count;
    if (status) status[r] = st;
  }
  return 0;
}

/* Single-cell entry point for the pins (grid units, no h0 factor). */
double rro_cell_integral_one(const double* Q /* 8 vertex values */, const double* p1, double h,
                             const double* dir, const double* o, double chiA, double chiB) {
  rro_ray ray;
  rro_ray_init(&ray, dir, o, 1.0, RRO_Q_KAPPA);
  double q[9];
  q[0] = 0.0;
  for (int i = 0; i < 8; ++i) q[i + 1] = Q[i];
  return rro_integral_trilinear_one(&ray, q, p1, h, chiA, chiB);
}
