// rr_ray.hpp -- per-ray device helpers of the march kernels: crossing
// parameters (FP64), projections of the tidal tensor, the per-cell integral
// and the debug hash.
#pragma once

// Multiply-adds are fused only within one expression (explicit fma() calls
// and a * b + c written together), never across statements: the march is
// instantiated with and without the pass logic, and both instantiations must
// round every piece the same way.
#pragma clang fp contract(on)

#include "rr_internal.hpp"

namespace rr {

// Crossing parameter of plane x_a = P for a ray p(chi) = o + chi * n:
// chi = (P - o_a) * (1/n_a), FP64, never contracted.
__device__ __forceinline__ double tplane(double P, double o, double r) {
  return __dmul_rn(__dsub_rn(P, o), r);
}

// Slab of one axis holding the ray at chi (plane spacing hl):
// t_exit < chi <= t_entry, a point on a plane belongs to the slab the ray
// moves into.  Starts from floor((o + chi n) / hl) and corrects.
__device__ __forceinline__ int start_slab(double o, double n, double r, double chi, double hl) {
  if (n == 0.0) return (int)floor(o / hl);
  int m = (int)floor((o + chi * n) / hl);
  for (int it = 0; it < 8; ++it) {
    const double t0 = tplane((double)m * hl, o, r);
    const double t1 = tplane((double)(m + 1) * hl, o, r);
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

// Exit parameter of slab m on one axis (-inf when the ray never crosses it).
__device__ __forceinline__ double texit_of(int m, double o, double n, double r, double hl) {
  if (n == 0.0) return -__builtin_inf();
  const int plane = n > 0.0 ? m : m + 1;
  return tplane((double)plane * hl, o, r);
}

// Projection coefficients P_ab so that Q = sum_ab P_ab T_ab (components
// xx, yy, zz, xy, xz, yz; off-diagonals already doubled).
//   kappa : tr T - n^T T n                    (Eqs. n1n1 + n2n2)
//   gamma1: e_phi^T T e_phi - e_theta^T T e_theta  (Eq. gamma1)
//   gamma2: 2 e_phi^T T e_theta               (Eq. gamma2, flat-sky mixed term)
__device__ inline void projection(int quantity, double dx, double dy, double dz, double* P) {
  if (quantity == RR_Q_KAPPA) {
    P[0] = 1.0 - dx * dx;
    P[1] = 1.0 - dy * dy;
    P[2] = 1.0 - dz * dz;
    P[3] = -2.0 * dx * dy;
    P[4] = -2.0 * dx * dz;
    P[5] = -2.0 * dy * dz;
    return;
  }
  const double st = sqrt(dx * dx + dy * dy);
  const double cp = st > 0.0 ? dx / st : 1.0;
  const double sp = st > 0.0 ? dy / st : 0.0;
  const double ct = dz;
  const double et[3] = {ct * cp, ct * sp, -st};
  const double ep[3] = {-sp, cp, 0.0};
  if (quantity == RR_Q_GAMMA1) {
    P[0] = ep[0] * ep[0] - et[0] * et[0];
    P[1] = ep[1] * ep[1] - et[1] * et[1];
    P[2] = ep[2] * ep[2] - et[2] * et[2];
    P[3] = 2.0 * (ep[0] * ep[1] - et[0] * et[1]);
    P[4] = 2.0 * (ep[0] * ep[2] - et[0] * et[2]);
    P[5] = 2.0 * (ep[1] * ep[2] - et[1] * et[2]);
  } else {
    P[0] = 2.0 * ep[0] * et[0];
    P[1] = 2.0 * ep[1] * et[1];
    P[2] = 2.0 * ep[2] * et[2];
    P[3] = 2.0 * (ep[0] * et[1] + ep[1] * et[0]);
    P[4] = 2.0 * (ep[0] * et[2] + ep[2] * et[0]);
    P[5] = 2.0 * (ep[1] * et[2] + ep[2] * et[1]);
  }
}

// Three-point Gauss-Legendre on [chi_B, chi_A], nodes at chi_B + L * c_k.
// The integrand g(chi) * Q(p(chi)) is a polynomial of degree <= 5 in chi
// (cubic trilinear field along a line times the quadratic lensing kernel), so
// the rule reproduces Eq. (Iclensing) exactly up to rounding.
struct GL3 {
  static constexpr double c0 = 0.11270166537925831148;  // (1 - sqrt(3/5)) / 2
  static constexpr double c1 = 0.5;
  static constexpr double c2 = 0.88729833462074168852;  // (1 + sqrt(3/5)) / 2
  static constexpr double w0 = 5.0 / 18.0;              // weights on [0, 1]
  static constexpr double w1 = 8.0 / 18.0;
  static constexpr double w2 = 5.0 / 18.0;
};

// Trilinear value from the eight corner values at local coords (ux, uy, uz),
// with the x-differences precomputed (corner v = ix + 2 iy + 4 iz).
template <typename R>
__device__ __forceinline__ R trilerp(const R* q, const R* dq, R ux, R uy, R uz) {
  const R a00 = fma(ux, dq[0], q[0]);
  const R a10 = fma(ux, dq[1], q[2]);
  const R a01 = fma(ux, dq[2], q[4]);
  const R a11 = fma(ux, dq[3], q[6]);
  const R b0 = fma(uy, a10 - a00, a00);
  const R b1 = fma(uy, a11 - a01, a01);
  return fma(uz, b1 - b0, b0);
}

// int_{chi_B}^{chi_A} g(chi) Q dchi for one cell.  uA/uB: local coordinates
// (cell units) of the entry and exit points; L = chi_A - chi_B; chiB;
// DB = chi_s - chi_B; inv_chis = 1/chi_s.
template <typename R>
__device__ __forceinline__ R cell_integral(const R* q, const R* uA, const R* uB, R L, R chiB, R DB,
                                           R inv_chis) {
  R dq[4];
  dq[0] = q[1] - q[0];
  dq[1] = q[3] - q[2];
  dq[2] = q[5] - q[4];
  dq[3] = q[7] - q[6];
  const R du0 = uA[0] - uB[0], du1 = uA[1] - uB[1], du2 = uA[2] - uB[2];
  R acc;
  {
    const R c = (R)GL3::c0;
    const R qk = trilerp(q, dq, fma(du0, c, uB[0]), fma(du1, c, uB[1]), fma(du2, c, uB[2]));
    const R chik = fma(L, c, chiB);
    const R gk = chik * fma(-L, c, DB);
    acc = (R)GL3::w0 * gk * qk;
  }
  {
    const R c = (R)GL3::c1;
    const R qk = trilerp(q, dq, fma(du0, c, uB[0]), fma(du1, c, uB[1]), fma(du2, c, uB[2]));
    const R chik = fma(L, c, chiB);
    const R gk = chik * fma(-L, c, DB);
    acc = fma((R)GL3::w1 * gk, qk, acc);
  }
  {
    const R c = (R)GL3::c2;
    const R qk = trilerp(q, dq, fma(du0, c, uB[0]), fma(du1, c, uB[1]), fma(du2, c, uB[2]));
    const R chik = fma(L, c, chiB);
    const R gk = chik * fma(-L, c, DB);
    acc = fma((R)GL3::w2 * gk, qk, acc);
  }
  return acc * L * inv_chis;
}

// Method A (Eq. kappa2) for one cell: int g (c delta) + (dg/dchi) (n . grad Phi)
// over [chi_B, chi_A], both fields trilinear (qd, qg at the corners).  With
// g = chi (chi_s - chi) / chi_s and dg/dchi = (chi_s - 2 chi) / chi_s the
// integrand has degree <= 5: the same three-point rule is exact.
template <typename R>
__device__ __forceinline__ R cell_integral_a(const R* qd, const R* qg, const R* uA, const R* uB,
                                             R L, R chiB, R DB, R inv_chis) {
  R dd[4], dg[4];
  dd[0] = qd[1] - qd[0]; dd[1] = qd[3] - qd[2]; dd[2] = qd[5] - qd[4]; dd[3] = qd[7] - qd[6];
  dg[0] = qg[1] - qg[0]; dg[1] = qg[3] - qg[2]; dg[2] = qg[5] - qg[4]; dg[3] = qg[7] - qg[6];
  const R du0 = uA[0] - uB[0], du1 = uA[1] - uB[1], du2 = uA[2] - uB[2];
  const R cs[3] = {(R)GL3::c0, (R)GL3::c1, (R)GL3::c2};
  const R ws[3] = {(R)GL3::w0, (R)GL3::w1, (R)GL3::w2};
  R acc = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R c = cs[k];
    const R u0 = fma(du0, c, uB[0]), u1 = fma(du1, c, uB[1]), u2 = fma(du2, c, uB[2]);
    const R chik = fma(L, c, chiB);
    const R rest = fma(-L, c, DB);               // chi_s - chi
    const R vd = trilerp(qd, dd, u0, u1, u2);
    const R vg = trilerp(qg, dg, u0, u1, u2);
    acc = fma(ws[k], fma(chik * rest, vd, (rest - chik) * vg), acc);
  }
  return acc * L * inv_chis;
}

// The two integrals of the source-distance decomposition (Eq. Isources) over
// one cell: ma = int chi Q dchi and mb = int chi^2 Q dchi on [chi_B, chi_A]
// (degree <= 5 in chi: the three-point rule is exact).
template <typename R>
__device__ __forceinline__ void cell_moments(const R* q, const R* uA, const R* uB, R L, R chiB,
                                             R& ma, R& mb) {
  R dq[4];
  dq[0] = q[1] - q[0];
  dq[1] = q[3] - q[2];
  dq[2] = q[5] - q[4];
  dq[3] = q[7] - q[6];
  const R du0 = uA[0] - uB[0], du1 = uA[1] - uB[1], du2 = uA[2] - uB[2];
  const R cs[3] = {(R)GL3::c0, (R)GL3::c1, (R)GL3::c2};
  const R ws[3] = {(R)GL3::w0, (R)GL3::w1, (R)GL3::w2};
  R a = 0, b = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R c = cs[k];
    const R qk = trilerp(q, dq, fma(du0, c, uB[0]), fma(du1, c, uB[1]), fma(du2, c, uB[2]));
    const R chik = fma(L, c, chiB);
    const R wq = ws[k] * qk * chik;
    a += wq;
    b = fma(wq, chik, b);
  }
  ma = a * L;
  mb = b * L;
}

// int_{chi_B}^{chi_A} Q dchi of the trilinear field (a constant kernel, the
// ISW integrand): cubic in chi, so the three-point rule is exact.
template <typename R>
__device__ __forceinline__ R cell_integral_scalar(const R* q, const R* uA, const R* uB, R L) {
  R dq[4];
  dq[0] = q[1] - q[0];
  dq[1] = q[3] - q[2];
  dq[2] = q[5] - q[4];
  dq[3] = q[7] - q[6];
  const R du0 = uA[0] - uB[0], du1 = uA[1] - uB[1], du2 = uA[2] - uB[2];
  const R cs[3] = {(R)GL3::c0, (R)GL3::c1, (R)GL3::c2};
  const R ws[3] = {(R)GL3::w0, (R)GL3::w1, (R)GL3::w2};
  R acc = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R c = cs[k];
    acc = fma(ws[k], trilerp(q, dq, fma(du0, c, uB[0]), fma(du1, c, uB[1]), fma(du2, c, uB[2])),
              acc);
  }
  return acc * L;
}

// FNV-1a, 64 bit, over the 8 little-endian bytes of w.
__device__ __forceinline__ uint64_t fnv_word(uint64_t h, uint64_t w) {
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    h ^= (w >> (8 * b)) & 0xffull;
    h *= 0x100000001b3ull;
  }
  return h;
}
__device__ __forceinline__ uint64_t fnv_piece(uint64_t h, int64_t cell, double a, double b) {
  h = fnv_word(h, (uint64_t)cell);
  h = fnv_word(h, (uint64_t)__double_as_longlong(a));
  h = fnv_word(h, (uint64_t)__double_as_longlong(b));
  return h;
}
constexpr uint64_t kFnvOffset = 0xcbf29ce484222325ull;

struct LogRecord {
  int64_t cell;
  double chi_a, chi_b;
};

// Kahan step: (sum, comp) += x
__device__ __forceinline__ void kahan_add(float& sum, float& comp, float x) {
  const float y = __fsub_rn(x, comp);
  const float t = __fadd_rn(sum, y);
  comp = __fsub_rn(__fsub_rn(t, sum), y);
  sum = t;
}

// Position of the k-th 8 x 8 tile of a bundle's tiles_x x tiles_y tile grid
// in Z order (quadrants (0,0), (1,0), (0,1), (1,1) at every level of the
// enclosing power-of-two square, positions outside the grid skipped): tiles
// that are close in launch order are close on the sky, so the wavefronts
// working at the same time, and the ones that share a chiplet, gather from
// the same part of the field.  k is wavefront-uniform (scalar work).
__device__ __forceinline__ void zorder_tile(int64_t k, int W, int H, int& x, int& y) {
  int s = 1;
  while (s < W || s < H) s <<= 1;
  int x0 = 0, y0 = 0;
  while (s > 1) {
    const int h = s >> 1;
    const int64_t w0 = min(max(W - x0, 0), h), w1 = min(max(W - x0 - h, 0), h);
    const int64_t h0 = min(max(H - y0, 0), h), h1 = min(max(H - y0 - h, 0), h);
    s = h;
    if (k < w0 * h0) continue;
    k -= w0 * h0;
    if (k < w1 * h0) {
      x0 += h;
      continue;
    }
    k -= w1 * h0;
    if (k < w0 * h1) {
      y0 += h;
      continue;
    }
    k -= w0 * h1;
    x0 += h;
    y0 += h;
  }
  x = x0;
  y = y0;
}

// Persistent launches: one work counter per chiplet (XCD).  Workgroups are
// dealt to the eight XCDs round-robin, so workgroup b runs on XCD b % 8; the
// tiles are split into eight contiguous ranges of the launch order, each
// chiplet drains its own range first (its L2 sees one compact part of the
// sky) and then helps with the others.  Returns the next tile, or -1 once
// every range is empty (every wavefront reaches that exit).
constexpr int kQueues = 8;
__device__ __forceinline__ int64_t next_tile(unsigned long long* queue, int64_t n_tiles, int& q,
                                             int& tried, int lane) {
  while (tried < kQueues) {
    const int64_t lo = n_tiles * q / kQueues, hi = n_tiles * (q + 1) / kQueues;
    unsigned long long t = 0;
    if (lane == 0) t = atomicAdd(queue + q, 1ull);
    t = __shfl(t, 0, 64);
    const int64_t k = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(t >> 32))
                                 << 32) |
                                (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)t));
    if (k < hi - lo) return lo + k;
    q = q + 1 == kQueues ? 0 : q + 1;
    ++tried;
  }
  return -1;
}

// Work assignment: global tile index -> (bundle, tile within it).
__device__ __forceinline__ int find_bundle(const DevBundle* b, int nb, int64_t tile) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b[mid].tile_begin <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

}  // namespace rr
