/*
 * rro_common.h -- per-ray helpers shared by the oracle's uniform and octree
 * tracers.  TEST INFRASTRUCTURE ONLY (see rro.h).
 */
#ifndef RRO_COMMON_H
#define RRO_COMMON_H
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define RRO_FNV_OFFSET 0xcbf29ce484222325ULL
#define RRO_FNV_PRIME 0x100000001b3ULL

static inline void rro_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* FNV-1a (64 bit) over the little-endian bytes of (cell, bits(chi_a), bits(chi_b)). */
static inline uint64_t rro_fnv_bytes(uint64_t h, uint64_t word) {
  for (int b = 0; b < 8; ++b) {
    h ^= (word >> (8 * b)) & 0xffu;
    h *= RRO_FNV_PRIME;
  }
  return h;
}
static inline uint64_t rro_fnv_segment(uint64_t h, int64_t cell, double a, double b) {
  uint64_t ua, ub;
  memcpy(&ua, &a, 8);
  memcpy(&ub, &b, 8);
  h = rro_fnv_bytes(h, (uint64_t)cell);
  h = rro_fnv_bytes(h, ua);
  h = rro_fnv_bytes(h, ub);
  return h;
}

typedef struct {
  double n[3];    /* (sin t cos p, sin t sin p, cos t): Eq. (rayposition) */
  double r[3];    /* 1/n_a, used for every plane crossing parameter */
  double o[3];    /* observer, grid units */
  double chis;    /* source distance, grid units */
  double st, ct, sp, cp;  /* sin/cos of theta and phi */
  int quantity;
} rro_ray;

static inline void rro_ray_init(rro_ray* ray, const double* d, const double* o, double chis,
                                int quantity) {
  for (int a = 0; a < 3; ++a) {
    ray->n[a] = d[a];
    ray->r[a] = (d[a] != 0.0) ? 1.0 / d[a] : 0.0;
    ray->o[a] = o[a];
  }
  ray->chis = chis;
  const double th = atan2(sqrt(d[0] * d[0] + d[1] * d[1]), d[2]);
  const double ph = atan2(d[1], d[0]);
  ray->st = sin(th);
  ray->ct = cos(th);
  ray->sp = sin(ph);
  ray->cp = cos(ph);
  ray->quantity = quantity;
}

/* Crossing parameter of the plane x_a = P: the ray p(chi) = o + chi n meets it
 * at chi = (P - o_a) / n_a (Eq. disttocross, with D = chi_A - chi). */
static inline double rro_tplane(const rro_ray* ray, int a, double P) {
  return (P - ray->o[a]) * ray->r[a];
}

/* Slab of axis a (plane spacing hl) that holds the ray at chi.  A ray sits in
 * slab m when t_exit(m) < chi <= t_entry(m): a point on a plane belongs to the
 * slab the ray is moving into (towards the observer). */
static inline int64_t rro_start_slab(const rro_ray* ray, int a, double chi, double hl) {
  const double n = ray->n[a];
  if (n == 0.0) return (int64_t)floor(ray->o[a] / hl);
  int64_t m = (int64_t)floor((ray->o[a] + chi * n) / hl);
  for (int it = 0; it < 64; ++it) {
    const double t0 = rro_tplane(ray, a, (double)m * hl);
    const double t1 = rro_tplane(ray, a, (double)(m + 1) * hl);
    const double texit = n > 0.0 ? t0 : t1;
    const double tentry = n > 0.0 ? t1 : t0;
    if (!(texit < chi)) {
      m += (n > 0.0) ? -1 : 1;
      continue;
    }
    if (!(chi <= tentry)) {
      m += (n > 0.0) ? 1 : -1;
      continue;
    }
    break;
  }
  return m;
}

/* Exit point of slab-cell m (level spacing hl): chi_B = max(chi_lo, t_exit,a)
 * (the face the ray travels least to reach, Eq. disttocross); ties keep the
 * earlier candidate, chi_lo first.  step[a] = 1 for every axis whose exit
 * plane is at chi_B. */
static inline double rro_exit(const rro_ray* ray, const int64_t* m, double hl, double chiA,
                              double lo, int* step) {
  (void)chiA;
  double te[3];
  double chiB = lo;
  for (int a = 0; a < 3; ++a) {
    te[a] = -INFINITY;
    if (ray->n[a] == 0.0) continue;
    const int64_t plane = ray->n[a] > 0.0 ? m[a] : m[a] + 1;
    te[a] = rro_tplane(ray, a, (double)plane * hl);
    if (te[a] > chiB) chiB = te[a];
  }
  for (int a = 0; a < 3; ++a) step[a] = (ray->n[a] != 0.0) && (te[a] == chiB);
  return chiB;
}

/* Projections of the tidal tensor T = (xx, yy, zz, xy, xz, yz).
 * Eq. (n1n1) and Eq. (n2n2); the mixed term of Eq. (n1n2) is taken without
 * its overall 1/sin(theta) (the flat-sky e_phi^T T e_theta). */
static inline double rro_n1n1(const rro_ray* ray, const double* T) {
  const double s2p = ray->sp * ray->sp, c2p = ray->cp * ray->cp;
  const double sin2p = 2.0 * ray->sp * ray->cp;
  return s2p * T[0] + c2p * T[1] - sin2p * T[3];
}
static inline double rro_n2n2(const rro_ray* ray, const double* T) {
  const double s2p = ray->sp * ray->sp, c2p = ray->cp * ray->cp;
  const double sin2p = 2.0 * ray->sp * ray->cp;
  const double c2t = ray->ct * ray->ct, s2t = ray->st * ray->st;
  const double sin2t = 2.0 * ray->st * ray->ct;
  return c2p * c2t * T[0] + s2p * c2t * T[1] + s2t * T[2] + sin2p * c2t * T[3] -
         ray->sp * sin2t * T[5] - ray->cp * sin2t * T[4];
}
static inline double rro_n1n2(const rro_ray* ray, const double* T) {
  const double c2p = ray->cp * ray->cp, s2p = ray->sp * ray->sp;
  return ray->ct * (ray->cp * ray->sp * (T[1] - T[0]) + (c2p - s2p) * T[3]) +
         ray->st * (ray->sp * T[4] - ray->cp * T[5]);
}
static inline double rro_quantity(const rro_ray* ray, const double* T) {
  switch (ray->quantity) {
    case 1: return rro_n1n1(ray, T) - rro_n2n2(ray, T);   /* Eq. (gamma1) */
    case 2: return 2.0 * rro_n1n2(ray, T);                /* Eq. (gamma2) */
    default: return rro_n1n1(ray, T) + rro_n2n2(ray, T);  /* Eq. (kappa) */
  }
}

/* The cubic Q(chi_A + s) = d_1 + d_2 s + d_3 s^2 + d_4 s^3 of the trilinear
 * field along the ray inside one cell (App. B, Eq. dns), from the vertex
 * values Q[1..8] of the paper's P_i (i = 1 + ix + 2 iy + 4 iz), lower corner
 * p1 and cell size h. */
static inline void rro_dn(const rro_ray* ray, const double* Q, const double* p1, double h,
                          double chiA, double* d) {
  /* Eq. (trilinear_coef) */
  double al[9];
  al[1] = Q[1];
  al[2] = Q[2] - Q[1];
  al[3] = Q[3] - Q[1];
  al[4] = Q[5] - Q[1];
  al[5] = Q[4] - Q[3] - Q[2] + Q[1];
  al[6] = Q[7] - Q[5] - Q[3] + Q[1];
  al[7] = Q[6] - Q[5] - Q[2] + Q[1];
  al[8] = Q[8] - Q[7] - Q[6] - Q[4] + Q[2] + Q[5] + Q[3] - Q[1];
  /* (a,b,c): point A relative to P_1 (Eq. Deltas) */
  const double a = ray->o[0] + chiA * ray->n[0] - p1[0];
  const double b = ray->o[1] + chiA * ray->n[1] - p1[1];
  const double c = ray->o[2] + chiA * ray->n[2] - p1[2];
  const double sx = ray->n[0], sy = ray->n[1], sz = ray->n[2];
  const double h2 = h * h, h3 = h * h * h;
  /* App. B, Eq. (dns) */
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

/* Eq. (Iclensing): I_c for one cell from the vertex values Q[1..8]. */
static inline double rro_integral_trilinear_q(const rro_ray* ray, const double* Q,
                                              const double* p1, double h, double chiA,
                                              double chiB) {
  double d[5];
  rro_dn(ray, Q, p1, h, chiA, d);
  /* Eq. (Iclensing) with R = chi_B - chi_A */
  const double chis = ray->chis;
  const double R = chiB - chiA;
  double sum = 0.0;
  double RN = 1.0;
  for (int N = 1; N <= 4; ++N) {
    RN *= R;
    sum += d[N] * (RN / N * (chiA - chis) * chiA + RN * R / (N + 1) * (2.0 * chiA - chis) +
                   RN * R * R / (N + 2));
  }
  return sum / chis;
}

/* The two integrals of Eq. (Isources) over one cell, int chi Q dchi and
 * int chi^2 Q dchi from chi_B to chi_A, from the same cubic: with
 * chi = chi_A + s and R = chi_B - chi_A,
 *   int chi Q   = -sum_N d_N (chi_A R^N / N + R^(N+1) / (N+1))
 *   int chi^2 Q = -sum_N d_N (chi_A^2 R^N / N + 2 chi_A R^(N+1) / (N+1) + R^(N+2) / (N+2)),
 * so that their combination A - B / chi_s is Eq. (Iclensing). */
static inline void rro_moments_trilinear_q(const rro_ray* ray, const double* Q, const double* p1,
                                           double h, double chiA, double chiB, double* ma,
                                           double* mb) {
  double d[5];
  rro_dn(ray, Q, p1, h, chiA, d);
  const double R = chiB - chiA;
  double sa = 0.0, sb = 0.0, RN = 1.0;
  for (int N = 1; N <= 4; ++N) {
    RN *= R;
    sa += d[N] * (chiA * RN / N + RN * R / (N + 1));
    sb += d[N] * (chiA * chiA * RN / N + 2.0 * chiA * RN * R / (N + 1) + RN * R * R / (N + 2));
  }
  *ma = -sa;
  *mb = -sb;
}

static inline double rro_integral_trilinear(const rro_ray* ray, const double tcorner[8][6],
                                            const double* p1, double h, double chiA,
                                            double chiB) {
  double Q[9];
  Q[0] = 0.0;
  for (int i = 1; i <= 8; ++i) Q[i] = rro_quantity(ray, tcorner[i - 1]);
  return rro_integral_trilinear_q(ray, Q, p1, h, chiA, chiB);
}

/* Eq. (Iclensing_ngp): cell-centre value times the integrated kernel. */
static inline double rro_integral_ngp(const rro_ray* ray, const double* tcentre, double chiA,
                                      double chiB) {
  const double Qc = rro_quantity(ray, tcentre);
  const double chis = ray->chis;
  return Qc / chis *
         (chis / 2.0 * (chiA * chiA - chiB * chiB) -
          (chiA * chiA * chiA - chiB * chiB * chiB) / 3.0);
}

#endif
