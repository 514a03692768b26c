// rr_octree.hip -- tidal tensor and ray march on a 2:1-balanced AMR octree.
//
// Cells: base cells 0..n^3-1 ([z][y][x]), then oct k owns cells
// n^3 + 8k + (ix + 2 iy + 4 iz); octs are breadth first, so every level is a
// contiguous range of cells.  A level-l cell has size 2^-l base cells and
// integer coordinates I at that level; locating a level-l position walks the
// child_oct links down from its base cell (at most four loads).
//
// Build (Sec. IV C, Sec. III H):
//  1. centre tensor, level by level: each component uses the level's own
//     finite-difference stencil (Eq. tidalexample, h = 2^-l) when every
//     stencil cell exists at level l; otherwise it is the trilinear
//     interpolation (weights 3/4, 1/4 per axis) of the coarser level's
//     component from the eight coarse centres around the cell centre;
//  2. corner tensors of every leaf, level by level: a vertex whose incident
//     leaves share one level takes their mean; a vertex in the middle of a
//     coarse edge or face takes the mean of that coarse leaf's 2 or 4 corner
//     values (already built, coarser level); any other vertex on a refinement
//     boundary takes the mass-redistribution weights of Eqs. (alphac3d) and
//     (alphaf3d), N_fv,j being the number of corners of fine leaf j that
//     touch a coarse leaf.
// March (Sec. III F): the uniform crossing rule on the current leaf's level;
// past a face, a coarser neighbour is entered by halving the coordinates, a
// refined one by descending to the child next to the crossed face (slab rule
// on the other axes).
#include "rr_octree.hpp"
#include "rr_ray.hpp"

namespace rr {
namespace {

struct Tree {
  const int32_t* __restrict__ child;
  const int4* __restrict__ info;   // per oct: x, y, z of child 0 (its level), level
  int n;
  int64_t nb;
};

// Base cell holding level-l coordinates I; every caller passes a cell of the
// domain or one of its neighbours, so I >> l lies in [-1, n] and wraps with
// one comparison per side.
__device__ __forceinline__ int64_t base_of(const Tree& T, int l, const int* I) {
  int b[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int q = I[a] >> l;    // floor division by 2^l (arithmetic shift)
    b[a] = q < 0 ? q + T.n : (q >= T.n ? q - T.n : q);
  }
  return ((int64_t)b[2] * T.n + b[1]) * T.n + b[0];
}

// Cell at level l and coordinates I; if the tree stops above l, the covering
// leaf.  Returns the level of the cell found.
__device__ __forceinline__ int descend(const Tree& T, int l, const int* I, int64_t& cell) {
  int64_t c = base_of(T, l, I);
  for (int lev = 1; lev <= l; ++lev) {
    const int k = T.child[c];
    if (k < 0) {
      cell = c;
      return lev - 1;
    }
    const int s = l - lev;
    const int ch = ((I[0] >> s) & 1) | (((I[1] >> s) & 1) << 1) | (((I[2] >> s) & 1) << 2);
    c = T.nb + 8 * (int64_t)k + ch;
  }
  cell = c;
  return l;
}

__device__ __forceinline__ void cell_coords(const Tree& T, int64_t c, int& level, int* I) {
  if (c < T.nb) {
    level = 0;
    I[0] = (int)(c % T.n);
    I[1] = (int)((c / T.n) % T.n);
    I[2] = (int)(c / ((int64_t)T.n * T.n));
    return;
  }
  const int64_t k = (c - T.nb) >> 3;
  const int ch = (int)((c - T.nb) & 7);
  const int4 inf = T.info[k];
  level = inf.w;
  I[0] = inf.x + (ch & 1);
  I[1] = inf.y + ((ch >> 1) & 1);
  I[2] = inf.z + ((ch >> 2) & 1);
}

// ----------------------------------------------------------- centre tensor --
__constant__ int kMixed[3][4][3] = {
    {{1, 1, 0}, {1, -1, 0}, {-1, 1, 0}, {-1, -1, 0}},   // xy: (++) (+-) (-+) (--)
    {{1, 0, 1}, {1, 0, -1}, {-1, 0, 1}, {-1, 0, -1}},   // xz
    {{0, 1, 1}, {0, 1, -1}, {0, -1, 1}, {0, -1, -1}},   // yz
};

template <typename In, typename Acc>
__global__ __launch_bounds__(256) void centre_kernel(Tree T, const In* __restrict__ phi,
                                                     Acc* __restrict__ tc, int l, int64_t begin,
                                                     int64_t end) {
  const int64_t c = begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= end) return;
  int lev, I[3];
  cell_coords(T, c, lev, I);
  const Acc inv_h2 = (Acc)(double)(1u << (2 * l));   // 1/h^2 with h = 2^-l
  const Acc p0 = (Acc)phi[c];
  Acc out[6];
#pragma unroll
  for (int comp = 0; comp < 6; ++comp) {
    bool ok = true;
    Acc v = 0;
    if (comp < 3) {
      int Jm[3] = {I[0], I[1], I[2]}, Jp[3] = {I[0], I[1], I[2]};
      Jm[comp] -= 1;
      Jp[comp] += 1;
      int64_t cm, cp;
      ok = descend(T, l, Jm, cm) == l && descend(T, l, Jp, cp) == l;
      if (ok) v = (((Acc)phi[cp] - p0) - (p0 - (Acc)phi[cm])) * inv_h2;
    } else {
      Acc s[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int J[3] = {I[0] + kMixed[comp - 3][q][0], I[1] + kMixed[comp - 3][q][1],
                          I[2] + kMixed[comp - 3][q][2]};
        int64_t cc;
        if (descend(T, l, J, cc) != l) {
          ok = false;
          s[q] = 0;
        } else {
          s[q] = (Acc)phi[cc];
        }
      }
      if (ok) v = ((s[0] - s[1]) - (s[2] - s[3])) * ((Acc)0.25 * inv_h2);
    }
    if (!ok) {
      // trilinear interpolation of the level-(l-1) component
      int P[3], off[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        P[a] = I[a] >> 1;
        off[a] = (I[a] & 1) ? 1 : -1;
      }
      Acc acc = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        int J[3];
        Acc w = 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int nb_ = (q >> a) & 1;
          J[a] = P[a] + (nb_ ? off[a] : 0);
          w *= nb_ ? (Acc)0.25 : (Acc)0.75;
        }
        int64_t cc;
        descend(T, l - 1, J, cc);
        acc += w * tc[6 * cc + comp];
      }
      v = acc;
    }
    out[comp] = v;
  }
#pragma unroll
  for (int comp = 0; comp < 6; ++comp) tc[6 * c + comp] = out[comp];
}

// ---------------------------------------------------------- corner tensors --
// Leaf covering octant o (bit a set: above the vertex on axis a) around the
// level-lv lattice point V.
__device__ __forceinline__ int octant_leaf(const Tree& T, int lv, const int* V, int o,
                                           int64_t& cell) {
  const int J[3] = {V[0] - 1 + (o & 1), V[1] - 1 + ((o >> 1) & 1), V[2] - 1 + ((o >> 2) & 1)};
  int lev = descend(T, lv, J, cell);
  if (lev < lv) return lev;
  const int ch = (1 - (o & 1)) | ((1 - ((o >> 1) & 1)) << 1) | ((1 - ((o >> 2) & 1)) << 2);
  int k;
  while ((k = T.child[cell]) >= 0) {
    cell = T.nb + 8 * (int64_t)k + ch;
    ++lev;
  }
  return lev;
}

template <typename Acc>
__global__ __launch_bounds__(256) void corner_kernel(Tree T, const Acc* __restrict__ tc,
                                                     const uint8_t* __restrict__ nfv_leaf,
                                                     Acc* __restrict__ cv, int l, int64_t begin,
                                                     int64_t end) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = begin + (g >> 3);
  const int v = (int)(g & 7);
  if (c >= end) return;
  Acc* out = cv + 48 * c + 6 * v;
  // cells that are not leaves get NaN blocks: the march tells a leaf from a
  // refined cell by a finite corner value and reads the child link otherwise
  if (T.child[c] >= 0) {
    const Acc nan = (Acc)__builtin_nan("");
#pragma unroll
    for (int comp = 0; comp < 6; ++comp) out[comp] = nan;
    return;
  }
  int lev0, I[3];
  cell_coords(T, c, lev0, I);
  const int V[3] = {I[0] + (v & 1), I[1] + ((v >> 1) & 1), I[2] + ((v >> 2) & 1)};
  int64_t leaf[8];
  int lv[8];
  int lc = 99, lf = -1;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    lv[o] = octant_leaf(T, l, V, o, leaf[o]);
    lc = min(lc, lv[o]);
    lf = max(lf, lv[o]);
  }
  Acc res[6] = {0, 0, 0, 0, 0, 0};
  const int s = l - lc;
  const int mask = (1 << s) - 1;
  const bool fr[3] = {(V[0] & mask) != 0, (V[1] & mask) != 0, (V[2] & mask) != 0};
  if (fr[0] || fr[1] || fr[2]) {
    // hanging: mean of the coarse leaf's corners spanning the edge / face
    int oc = 0;
#pragma unroll
    for (int o = 7; o >= 0; --o)
      if (lv[o] == lc) oc = o;
    int lcc, IC[3];
    cell_coords(T, leaf[oc], lcc, IC);
    const int period = T.n << lc;    // the coarse leaf may sit across the periodic face
    int cnt = 0;
    for (int sel = 0; sel < 8; ++sel) {
      int corner = 0;
      bool skip = false;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int bit = (sel >> a) & 1;
        int cb;
        if (fr[a]) {
          cb = bit;
        } else {
          if (bit) skip = true;
          cb = (V[a] >> s) - IC[a];
          cb = cb < 0 ? cb + period : (cb >= period ? cb - period : cb);
          cb = cb > 1 ? 1 : cb;     // V lies on the leaf's boundary: 0 or 1
        }
        corner |= cb << a;
      }
      if (skip) continue;
      const Acc* src = cv + 48 * leaf[oc] + 6 * corner;
#pragma unroll
      for (int comp = 0; comp < 6; ++comp) res[comp] += src[comp];
      ++cnt;
    }
    const Acc inv = (Acc)1 / (Acc)cnt;
#pragma unroll
    for (int comp = 0; comp < 6; ++comp) res[comp] *= inv;
  } else if (lc == lf) {
    // regular: mean of the eight centre values
#pragma unroll
    for (int o = 0; o < 8; ++o)
#pragma unroll
      for (int comp = 0; comp < 6; ++comp) res[comp] += tc[6 * leaf[o] + comp];
#pragma unroll
    for (int comp = 0; comp < 6; ++comp) res[comp] *= (Acc)0.125;
  } else {
    // boundary vertex: Eqs. (alphac3d), (alphaf3d).  The tree is 2:1
    // balanced over faces, edges and corners, so the fine leaves here are one
    // level below lc and N_fv of each is its count of corners touching a
    // leaf one level coarser, stored per leaf (coarse_corner_kernel).
    int n_coarse = 0, nfv[8], sum_fv = 0;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      nfv[o] = 0;
      if (lv[o] == lc) {
        ++n_coarse;
        continue;
      }
      nfv[o] = nfv_leaf[leaf[o]];
      sum_fv += nfv[o];
    }
    const Acc ac = (Acc)1 / ((Acc)n_coarse + (Acc)0.125 * (Acc)sum_fv);
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const Acc w = lv[o] == lc ? ac : (Acc)0.125 * (Acc)nfv[o] * ac;
#pragma unroll
      for (int comp = 0; comp < 6; ++comp) res[comp] += w * tc[6 * leaf[o] + comp];
    }
  }
#pragma unroll
  for (int comp = 0; comp < 6; ++comp) out[comp] = res[comp];
}

// Per leaf of level l >= 1: how many of its eight corners touch a leaf of
// level l - 1 (N_fv of Eqs. alphac3d / alphaf3d).  A corner W touches one when
// one of the eight level-l cells around it does not exist (the region is
// covered by a coarser leaf); those cells all lie in the 3 x 3 x 3 block of
// level-l cells around the leaf, looked up once each.
__global__ __launch_bounds__(256) void coarse_corner_kernel(Tree T, uint8_t* __restrict__ out,
                                                            int l, int64_t begin, int64_t end) {
  const int64_t c = begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= end) return;
  if (T.child[c] >= 0) {
    out[c] = 0;
    return;
  }
  int lev, I[3];
  cell_coords(T, c, lev, I);
  uint32_t coarse = 0;   // bit (dx+1) + 3 (dy+1) + 9 (dz+1)
  for (int d = 0; d < 27; ++d) {
    const int J[3] = {I[0] + d % 3 - 1, I[1] + (d / 3) % 3 - 1, I[2] + d / 9 - 1};
    int64_t cc;
    if (descend(T, l, J, cc) == l - 1) coarse |= 1u << d;
  }
  int cnt = 0;
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    bool touch = false;
#pragma unroll
    for (int o2 = 0; o2 < 8; ++o2) {
      const int d = ((w & 1) + (o2 & 1)) + 3 * (((w >> 1) & 1) + ((o2 >> 1) & 1)) +
                    9 * (((w >> 2) & 1) + ((o2 >> 2) & 1));
      touch |= (coarse >> d) & 1u;
    }
    cnt += touch;
  }
  out[c] = (uint8_t)cnt;
}

// ------------------------------------------------------------------- march --
__device__ __forceinline__ int slab_child(double o, double r, int m, int l, double chi) {
  const double hl1 = ldexp(1.0, -(l + 1));
  const int mid = 2 * m + 1;
  if (r == 0.0) return ldexp(o, l + 1) >= (double)mid;
  const double tm = tplane((double)mid * hl1, o, r);
  return r > 0.0 ? (chi > tm) : (chi <= tm);
}

// One corner of a leaf's block (8 corners x 6 components) projected on P.
template <typename R, typename Off>
__device__ __forceinline__ R leaf_corner(const R* __restrict__ cv, Off cell, int corner,
                                         const R* P) {
  // byte offset in Off (32 bit when the whole block array is below 4 GiB)
  const Off off = cell * (Off)(48 * sizeof(R)) + (Off)(corner * 6 * (int)sizeof(R));
  const R* p = reinterpret_cast<const R*>(reinterpret_cast<const char*>(cv) + (uint64_t)off);
  R t[6];
  if constexpr (sizeof(R) == 4) {
    const float2* p2 = reinterpret_cast<const float2*>(p);
    const float2 x = p2[0], y = p2[1], z = p2[2];
    t[0] = x.x; t[1] = x.y; t[2] = y.x; t[3] = y.y; t[4] = z.x; t[5] = z.y;
  } else {
    const double2* p2 = reinterpret_cast<const double2*>(p);
    const double2 x = p2[0], y = p2[1], z = p2[2];
    t[0] = x.x; t[1] = x.y; t[2] = y.x; t[3] = y.y; t[4] = z.x; t[5] = z.y;
  }
  R acc = P[0] * t[0];
#pragma unroll
  for (int c = 1; c < 6; ++c) acc = fma(P[c], t[c], acc);
  return acc;
}

// All eight corners of a leaf in the ray's frame: slot c (bit a: 0 = the
// face the ray enters through along axis a, 1 = the face it leaves through)
// is block corner c ^ flip, flip bit a set where n_a > 0 (the ray enters
// through the upper face).  In two halves, at most four records in flight:
// this runs at the start of a ray, at level changes and edge crossings only.
template <typename R, typename Off>
__device__ __forceinline__ void load_leaf(const R* __restrict__ cv, Off cell, int flip,
                                          const R* P, R* q) {
#pragma unroll
  for (int c = 0; c < 4; ++c) q[c] = leaf_corner<R, Off>(cv, cell, c ^ flip, P);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int c = 4; c < 8; ++c) q[c] = leaf_corner<R, Off>(cv, cell, c ^ flip, P);
}

// Cell at level l and coordinates I below base cell `b`; if the tree stops
// above l, the covering leaf.  Returns the level of the cell found.
template <typename Off>
__device__ __forceinline__ int descend_from(const Tree& T, Off b, int l, const int* I, Off& cell) {
  Off c = b;
  for (int lev = 1; lev <= l; ++lev) {
    const int k = T.child[c];
    if (k < 0) {
      cell = c;
      return lev - 1;
    }
    const int s = l - lev;
    const int ch = ((I[0] >> s) & 1) | (((I[1] >> s) & 1) << 1) | (((I[2] >> s) & 1) << 2);
    c = (Off)T.nb + 8 * (Off)k + (Off)ch;
  }
  cell = c;
  return l;
}

// Integrands: the tidal tensor with the trilinear integral, the leaf's
// centre tensor (NGP), and the trilinear tensor against the two
// source-distance moments chi and chi^2 (the many-source walk).
constexpr int kOctTidal = 0, kOctNgp = 1, kOctSources = 3;

// One ray through the octree, in the ray's frame (as the uniform march):
// per axis the lane keeps, in FP64, the crossing parameter of the current
// leaf's exit plane and the level-l coordinates m, and the local coordinate
// f = 1 - |n_a| 2^l (chi - t_exit) runs from 0 on the entry face to exactly 1
// on the exit face.  The wrapped base cell is tracked incrementally (no
// division per crossing).  Crossing one face into a leaf of the same level
// keeps the four projected corner values of that face (same-level leaves
// share their face corners bit for bit: a vertex's value is computed from
// the vertex alone) and loads the new leaf's four exit-face corners together
// with its child link; level changes and edge crossings reload all eight.
// A crossing that stays on level 0 or inside the parent oct needs no walk
// from the base cell.  kOverlap: the next leaf's loads are issued before the
// integral of the leaf being left (see the target step below).
template <typename R, bool kDebug, int kMode, typename Off, bool kOverlap>
__device__ void trace_oct(const Tree& T, const R* __restrict__ cv, const TraceArgs& a,
                          const DevBundle& B, int64_t ray) {
  const int64_t out = B.ray_offset + ray;
  const int n = T.n;
  const double lo = B.chi_lo;
  double chiA = B.chi_hi;
  // a later pass resumes on the face where the last one stopped
  bool resumed = false;
  if (a.resume) {
    const double r0 = a.resume[out];
    if (!(r0 > lo)) return;   // done in an earlier pass
    resumed = r0 < chiA;
    chiA = resumed ? r0 : chiA;
    if (chiA <= a.pause_chi) return;   // starts in a later pass
  }
  R P[6];
  double r[3];
  int m[3], wb[3];
  R absd[3];
  int flip = 0;   // block corner of ray-frame slot c: c ^ flip
  {
    const double d[3] = {B.dir[3 * ray + 0], B.dir[3 * ray + 1], B.dir[3 * ray + 2]};
    const double nrm2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(fabs(nrm2 - 1.0) <= 1e-9)) {
      if (a.status) a.status[out] = RR_RAY_BAD_DIRECTION;
      return;
    }
    double Pd[6];
    projection(a.quantity, d[0], d[1], d[2], Pd);
#pragma unroll
    for (int c = 0; c < 6; ++c) P[c] = (R)Pd[c];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      r[k] = (d[k] != 0.0) ? 1.0 / d[k] : 0.0;
      m[k] = start_slab(a.o[k], d[k], r[k], chiA, 1.0);
      const int q = m[k] % n;
      wb[k] = q < 0 ? q + n : q;
      absd[k] = d[k] != 0.0 ? (R)fabs(d[k]) : (R)1e-30;
      flip |= (d[k] > 0.0) << k;
    }
  }
  Off blin = ((Off)wb[2] * (Off)n + (Off)wb[1]) * (Off)n + (Off)wb[0];
  int l = 0;
  Off cell = blin;
  {
    int k;
    while ((k = T.child[cell]) >= 0) {
      int ch = 0;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const int bit = slab_child(a.o[ax], r[ax], m[ax], l, chiA);
        m[ax] = 2 * m[ax] + bit;
        ch |= bit << ax;
      }
      cell = (Off)T.nb + 8 * (Off)k + (Off)ch;
      ++l;
    }
  }
  double te[3];
  // exit parameters and slopes of every axis at level l (the slope |n_a| 2^l
  // is carried from level to level by exact power-of-two scaling); an axis
  // the ray never crosses gets the slope 1e-30 and an exit parameter
  // (1 - f) 1e30 below any chi, which reproduces its fixed coordinate
  auto set_level = [&](int dl) {
    const double hl = ldexp(1.0, -l);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (r[k] != 0.0) {
        absd[k] = ldexp(absd[k], dl);
        te[k] = tplane((double)(r[k] > 0.0 ? m[k] : m[k] + 1) * hl, a.o[k], r[k]);
      } else {
        te[k] = -(1.0 - ldexp(a.o[k] - (double)m[k] * hl, l)) * 1e30;
      }
    }
  };
  set_level(l);
  R fA[3];
  {
    const double hl = ldexp(1.0, -l);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      fA[k] = (R)1 - absd[k] * (R)(chiA - te[k]);
      // on the entry face of a resumed leaf the coordinate is 0, as when the
      // march steps across that face without stopping
      if (resumed && r[k] != 0.0 &&
          chiA == tplane((double)(r[k] > 0.0 ? m[k] + 1 : m[k]) * hl, a.o[k], r[k]))
        fA[k] = (R)0;
    }
  }
  R q[8];
  if constexpr (kMode != kOctNgp) load_leaf<R, Off>(cv, cell, flip, P, q);

  const R inv_chis = (R)(1.0 / B.chi_s);
  const R scale = (R)a.kappa_scale;
  R sum;
  float comp = 0.0f;
  // many-source walk: (sum, comp) integrate chi Q, (sum2, comp2) chi^2 Q, and
  // the walk also stops at the next source distance src_j
  R sum2 = 0;
  float comp2 = 0.0f;
  int jn = 0;
  double src_j = -1.0;
  if constexpr (kMode == kOctSources) {
    if constexpr (sizeof(R) == 4) {
      const float4 mm = reinterpret_cast<const float4*>(a.kappa)[out];
      sum = mm.x; comp = mm.y; sum2 = mm.z; comp2 = mm.w;
    } else {
      const double2 mm = reinterpret_cast<const double2*>(a.kappa)[out];
      sum = mm.x; sum2 = mm.y;
    }
    while (jn < a.n_src && !(a.src[jn] < chiA)) ++jn;
    src_j = jn < a.n_src ? a.src[jn] : -1.0;
  } else if constexpr (sizeof(R) == 4) {
    sum = reinterpret_cast<float*>(a.kappa)[out];
    if (a.kappa_comp) comp = a.kappa_comp[out];
  } else {
    sum = reinterpret_cast<double*>(a.kappa)[out];
  }
  uint64_t hv = kFnvOffset;
  int64_t count = 0;
  int32_t st = RR_RAY_OK;
  const int64_t maxc = a.max_crossings > 0 ? a.max_crossings : INT64_MAX;
  bool paused = false;

  // the integral of the piece [chi_a, chiB] of the current leaf (corners q,
  // entry coordinates fA, exit coordinates fB), its accumulation and, in the
  // many-source walk, the hand-out at a source distance
  auto piece = [&](double chi_a, double chiB, const R* fB, R L) {
    R ic, ic2 = 0;
    if constexpr (kMode == kOctNgp) {
      // Eq. (Iclensing_ngp): the leaf's centre value times the integral of g,
      // L (g(mid) - L^2 / (12 chi_s)) with g(chi) = chi (chi_s - chi) / chi_s
      const R* tc = cv + 6 * (uint64_t)cell;
      R Qc = P[0] * tc[0];
#pragma unroll
      for (int c = 1; c < 6; ++c) Qc = fma(P[c], tc[c], Qc);
      const double mid = chiB + 0.5 * (chi_a - chiB);
      const R gm = (R)mid * (R)(B.chi_s - mid) - L * L * (R)(1.0 / 12.0);
      ic = Qc * (gm * L * inv_chis) * scale;
    } else if constexpr (kMode == kOctSources) {
      R ma, mb;
      cell_moments<R>(q, fA, fB, L, (R)chiB, ma, mb);
      ic = ma * scale;
      ic2 = mb * scale;
    } else {
      ic = cell_integral<R>(q, fA, fB, L, (R)chiB, (R)(B.chi_s - chiB), inv_chis) * scale;
    }
    if constexpr (sizeof(R) == 4) {
      kahan_add(sum, comp, ic);
      if constexpr (kMode == kOctSources) kahan_add(sum2, comp2, ic2);
    } else {
      sum += ic;
      if constexpr (kMode == kOctSources) sum2 += ic2;
    }
    if constexpr (kDebug) {
      if (a.hash) hv = fnv_piece(hv, (int64_t)cell, chi_a, chiB);
      if (a.log && count < a.log_stride) {
        LogRecord* L0 = reinterpret_cast<LogRecord*>(a.log) + out * a.log_stride + count;
        L0->cell = (int64_t)cell;
        L0->chi_a = chi_a;
        L0->chi_b = chiB;
      }
    }
    ++count;
    if constexpr (kMode == kOctSources) {
      if (src_j == chiB) {
        // hand out the two integrals accumulated since the previous stop
        double* pc = a.pieces + (out * a.n_src + jn) * 2;
        pc[0] = (double)sum - (double)comp;
        pc[1] = (double)sum2 - (double)comp2;
        sum = 0; comp = 0.0f; sum2 = 0; comp2 = 0.0f;
        ++jn;
        src_j = jn < a.n_src ? a.src[jn] : -1.0;
      }
    }
  };

  for (;;) {
    if (chiA <= a.pause_chi) {   // the rest of the window is a later pass's
      paused = true;
      break;
    }
    if (count >= maxc) {
      st = RR_RAY_MAX_STEPS;
      break;
    }
    double chiB = lo;
    if constexpr (kMode == kOctSources) chiB = src_j >= lo ? src_j : lo;
    chiB = te[0] > chiB ? te[0] : chiB;
    chiB = te[1] > chiB ? te[1] : chiB;
    chiB = te[2] > chiB ? te[2] : chiB;
    bool stepped[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) stepped[k] = te[k] == chiB;

    const R L = (R)(chiA - chiB);
    R fB[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) fB[k] = (R)1 - absd[k] * (R)(chiB - te[k]);
    const double chi_a = chiA;
    bool stop = chiB == lo;
    if constexpr (kMode == kOctSources) stop = stop || !(stepped[0] || stepped[1] || stepped[2]);
    if (stop) {
      piece(chi_a, chiB, fB, L);
      if (chiB == lo) break;
      // stopped at a source distance inside the leaf: same corners
      chiA = chiB;
#pragma unroll
      for (int k = 0; k < 3; ++k) fA[k] = fB[k];
      continue;
    }
    if constexpr (!kOverlap) piece(chi_a, chiB, fB, L);
    chiA = chiB;

    // step the crossed axes on level l; track the base cell
    const bool single = (int)stepped[0] + (int)stepped[1] + (int)stepped[2] == 1;
    Off nc;
    int lev = l;
    if (__ballot(l == 0 && single) == __ballot(1)) {
      // every lane is on level 0 and crosses one face: the new base cell
      // without branches (its index moves by the wrapped step times the
      // axis stride)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int st = stepped[k] ? (r[k] > 0.0 ? -1 : 1) : 0;
        m[k] += st;
        int w = wb[k] + st;
        w = w < 0 ? n - 1 : (w == n ? 0 : w);
        const int64_t stride = k == 0 ? 1 : (k == 1 ? (int64_t)n : (int64_t)n * n);
        blin += (Off)((int64_t)(w - wb[k]) * stride);
        wb[k] = w;
      }
      nc = blin;
    } else {
      const int ch_old = (m[0] & 1) | ((m[1] & 1) << 1) | ((m[2] & 1) << 2);
      bool sib = l > 0;
      bool moved = false;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (stepped[k]) {
          const int mo = m[k];
          const int s = r[k] > 0.0 ? -1 : 1;
          m[k] = mo + s;
          sib = sib && ((m[k] >> 1) == (mo >> 1));
          if ((m[k] >> l) != (mo >> l)) {
            const int w = wb[k] + s;
            wb[k] = w < 0 ? n - 1 : (w == n ? 0 : w);
            moved = true;
          }
        }
      }
      if (moved) blin = ((Off)wb[2] * (Off)n + (Off)wb[1]) * (Off)n + (Off)wb[0];
      // the level-l cell past the face: a base cell, a sibling, or a walk
      if (l == 0) {
        nc = blin;
      } else if (sib) {
        const int ch = (m[0] & 1) | ((m[1] & 1) << 1) | ((m[2] & 1) << 2);
        nc = cell + (Off)(ch - ch_old);
      } else {
        lev = descend_from<Off>(T, blin, l, m, nc);
      }
    }
    // the target: a same-level leaf across one face keeps four corner values
    // and loads the other four together with its child link; a refined target
    // (the loads are dropped), a coarser one or an edge crossing reloads all.
    // With kOverlap the four loads are issued for every target (each cell,
    // leaf or not, has its block, so they stay in bounds where they are not
    // used) and the integral of the leaf being left is computed while they
    // are in flight; otherwise the integral comes first and the loads only
    // for a same-level face crossing (the register budget of the persistent
    // march cannot hold the loads in flight across the integral).
    const int l_in = l;
    bool inner[3] = {false, false, false};   // a crossed plane inside the new (coarser) leaf
    int kc = kOverlap ? -1 : T.child[nc];
    bool kept = false;
    const bool k0 = stepped[0], k1 = stepped[1];
    const bool same = kMode != kOctNgp && lev == l && single;
    R F0 = 0, F1 = 0, F2 = 0, F3 = 0;
    if (kOverlap ? kMode != kOctNgp : same) {
      // slots of the new exit face: (1 << k) | i_a << a | i_b << b, a < b the other axes
      const int sk = k0 ? 1 : (k1 ? 2 : 4);
      const int sa = k0 ? 2 : 1;
      const int sb = k0 || k1 ? 4 : 2;
      F0 = leaf_corner<R, Off>(cv, nc, sk ^ flip, P);
      F1 = leaf_corner<R, Off>(cv, nc, (sk | sa) ^ flip, P);
      F2 = leaf_corner<R, Off>(cv, nc, (sk | sb) ^ flip, P);
      F3 = leaf_corner<R, Off>(cv, nc, (sk | sa | sb) ^ flip, P);
    }
    if constexpr (kOverlap) {
      piece(chi_a, chiB, fB, L);
      // the integral is computed here, between the issue of the loads and
      // the first use of their values: neither moves past these statements
      asm volatile("" ::"v"(sum), "v"(comp));
      asm volatile("" ::"v"(F0), "v"(F1), "v"(F2), "v"(F3));
      // the target's child link.  The blocks of cells that are not leaves
      // hold NaN (corner_kernel), so a finite corner value of a same-level
      // target shows a leaf and the link is read only where that does not
      // settle it (a NaN value, a level change or an edge crossing).  The
      // persistent march reads it for every target, ahead of its corner
      // loads: reading it only where needed made that march slower (batched
      // bundles 1.90 -> 2.36-2.38 s, with the other targets' links read
      // before or after the corner loads).
      if (!(same && F0 == F0)) kc = T.child[nc];
    }
    if constexpr (kMode != kOctNgp) {
      if (same) {
        if (__ballot(kc < 0 && !k0 && !k1) == __ballot(1)) {
          // every marching lane crossed a z face into a leaf of its level
          // (lines of sight near the z axis): no selects
          q[0] = q[4]; q[1] = q[5]; q[2] = q[6]; q[3] = q[7];
          q[4] = F0; q[5] = F1; q[6] = F2; q[7] = F3;
          kept = true;
        } else if (kc < 0) {
          const R n0 = k0 ? q[1] : (k1 ? q[2] : q[4]);
          const R n1 = k0 ? F0 : (k1 ? q[3] : q[5]);
          const R n2 = k0 ? q[3] : (k1 ? F0 : q[6]);
          const R n3 = k0 || k1 ? F1 : q[7];
          const R n4 = k0 ? q[5] : (k1 ? q[6] : F0);
          const R n5 = k0 ? F2 : (k1 ? q[7] : F1);
          const R n6 = k0 ? q[7] : F2;
          q[0] = n0; q[1] = n1; q[2] = n2; q[3] = n3;
          q[4] = n4; q[5] = n5; q[6] = n6; q[7] = F3;
          kept = true;
        }
      }
    }
    if (!kept) {
      // refined target: the child next to the crossed face(s), slab rule elsewhere
      while (kc >= 0) {
        int ch = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const int bit = stepped[ax] ? (r[ax] > 0.0 ? 1 : 0)
                                      : slab_child(a.o[ax], r[ax], m[ax], l, chiA);
          m[ax] = 2 * m[ax] + bit;
          ch |= bit << ax;
        }
        nc = (Off)T.nb + 8 * (Off)kc + (Off)ch;
        ++l;
        kc = T.child[nc];
      }
      if (lev < l_in) {
        // coarser neighbour.  Across an edge or a vertex, a crossed plane of
        // level l_in need not be a plane of level lev: along an axis on which
        // the ray stays within the refined cell's range it runs through the
        // coarser leaf's interior (there its entry coordinate is not 0)
        const int mask = (1 << (l_in - lev)) - 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int plane = r[k] > 0.0 ? m[k] + 1 : m[k];   // the crossed plane, if stepped
          inner[k] = stepped[k] && (plane & mask) != 0;
          m[k] >>= (l_in - lev);
        }
        l = lev;
      }
      if constexpr (kMode != kOctNgp) load_leaf<R, Off>(cv, nc, flip, P, q);
    }
    if (l != l_in) {
      set_level(l - l_in);
    } else {
      const double hl = ldexp(1.0, -l);
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (stepped[k])
          te[k] = tplane((double)(r[k] > 0.0 ? m[k] : m[k] + 1) * hl, a.o[k], r[k]);
    }
    // the entry point: on the crossed faces of the new leaf exactly 0,
    // elsewhere the exit coordinate of the last leaf (same level) or
    // recomputed at the new level.  In a finer leaf a point can lie exactly
    // on its entry face along an axis that was not stepped (a ray running in
    // a plane of the finer level): 0 there too, as a pass resuming at that
    // point sets it.  (A coarser leaf's entry face holds no such point: along
    // an axis it moves on, the ray left its entry plane with the last piece.)
    const double hl_new = ldexp(1.0, -l);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (stepped[k] && !inner[k]) {
        fA[k] = (R)0;
      } else if (l != l_in) {
        fA[k] = (R)1 - absd[k] * (R)(chiA - te[k]);
        if (l > l_in && r[k] != 0.0 &&
            chiA == tplane((double)(r[k] > 0.0 ? m[k] + 1 : m[k]) * hl_new, a.o[k], r[k]))
          fA[k] = (R)0;
      } else {
        fA[k] = fB[k];
      }
    }
    cell = nc;
  }
  if (!(sum == sum) || sum - sum != (R)0) st = RR_RAY_NONFINITE;
  if constexpr (kMode == kOctSources) {
    if (!(sum2 == sum2) || sum2 - sum2 != (R)0) st = RR_RAY_NONFINITE;
    if constexpr (sizeof(R) == 4)
      reinterpret_cast<float4*>(a.kappa)[out] = make_float4(sum, comp, sum2, comp2);
    else
      reinterpret_cast<double2*>(a.kappa)[out] = make_double2(sum, sum2);
  } else if constexpr (sizeof(R) == 4) {
    reinterpret_cast<float*>(a.kappa)[out] = sum;
    if (a.kappa_comp) a.kappa_comp[out] = comp;
  } else {
    reinterpret_cast<double*>(a.kappa)[out] = sum;
  }
  // stopped at the pass boundary: the next pass starts on the face ahead
  if (a.resume) a.resume[out] = paused ? chiA : -INFINITY;
  if (a.status) a.status[out] = st;
  if constexpr (kDebug) {
    if (a.hash) a.hash[out] = hv;
    if (a.count) a.count[out] = count;
  }
}

template <typename R, bool kDebug, int kMode, typename Off, bool kOverlap>
__device__ __forceinline__ void oct_tile(const Tree& T, const R* cv, const TraceArgs& a,
                                         int64_t tile, int lane) {
  const int b = find_bundle(a.bundles, a.n_bundles, tile);
  const DevBundle& B = a.bundles[b];
  int tx, ty;
  zorder_tile(tile - B.tile_begin, B.tiles_x, B.tiles_y, tx, ty);
  const int ix = tx * 8 + (lane & 7), iy = ty * 8 + (lane >> 3);
  if (ix < B.nx && iy < B.ny)
    trace_oct<R, kDebug, kMode, Off, kOverlap>(T, cv, a, B, (int64_t)iy * B.nx + ix);
}

template <typename R, bool kDebug, int kMode, typename Off>
__global__ __launch_bounds__(256) void march_octree_kernel(Tree T, const R* __restrict__ cv,
                                                           TraceArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nblk = gridDim.x, blk = blockIdx.x;
  const int64_t per = (nblk + 7) / 8;
  // the tile is the same for the 64 lanes: keep it (and the bundle) scalar
  const int64_t tile =
      ((blk % 8) * per + blk / 8) * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(wave);
  if (tile >= a.n_tiles) return;
  // the tidal march computes each integral while the next leaf's corner
  // loads are in flight (the register budget of a direct launch holds them)
  oct_tile<R, kDebug, kMode, Off, kMode == kOctTidal>(T, cv, a, tile, lane);
}

// The FP32 tidal march (no debug outputs, 32-bit offsets) fits 128 VGPRs
// without spilling: four waves per SIMD keep a 16-wave-per-CU persistent grid
// resident at once (at 132 VGPRs only three were; the 64 batched bundles
// 2.34 -> 2.02 s).  The other instantiations spill under that cap.  Under
// it the loads of the next leaf cannot stay in flight across an integral
// (the compiler then serialises them), so the integral comes first.
template <typename R, bool kDebug, int kMode, typename Off>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    sizeof(R) == 4 && kMode == 0 && !kDebug && sizeof(Off) == 4 ? 4 : 1)))
void march_octree_persistent(Tree T, const R* __restrict__ cv, TraceArgs a) {
  const int lane = threadIdx.x & 63;
  int q = blockIdx.x % kQueues, tried = 0;
  for (;;) {
    const int64_t tile = next_tile(a.queue, a.n_tiles, q, tried, lane);
    if (tile < 0) break;
    oct_tile<R, kDebug, kMode, Off, false>(T, cv, a, tile, lane);
  }
}

template <typename R, bool kDebug, int kMode, typename Off>
hipError_t launch_march(const Tree& T, const void* cv, const TraceArgs& a, int persistent,
                        int grid_waves, hipStream_t s) {
  if (persistent) {
    const int blocks = (grid_waves + 3) / 4;
    hipLaunchKernelGGL((march_octree_persistent<R, kDebug, kMode, Off>), dim3(blocks), dim3(256), 0, s, T,
                       (const R*)cv, a);
  } else {
    int64_t blocks = (a.n_tiles + 3) / 4;
    if (blocks == 0) return hipSuccess;
    blocks = (blocks + 7) / 8 * 8;
    hipLaunchKernelGGL((march_octree_kernel<R, kDebug, kMode, Off>), dim3((unsigned)blocks), dim3(256), 0, s,
                       T, (const R*)cv, a);
  }
  return hipGetLastError();
}

template <typename In, typename Acc>
hipError_t build_all(const OctreeTensor& t, const void* values, hipStream_t s) {
  Tree T{t.child_oct_dev, reinterpret_cast<const int4*>(t.oct_info), t.n,
         (int64_t)t.n * t.n * t.n};
  for (int l = 0; l <= t.max_level; ++l) {
    const int64_t b = t.level_begin[l], e = t.level_begin[l + 1];
    if (e <= b) continue;
    const int64_t blocks = (e - b + 255) / 256;
    hipLaunchKernelGGL((centre_kernel<In, Acc>), dim3((unsigned)blocks), dim3(256), 0, s, T,
                       (const In*)values, (Acc*)t.centre, l, b, e);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  for (int l = 0; l <= t.max_level; ++l) {
    const int64_t b = t.level_begin[l], e = t.level_begin[l + 1];
    if (e <= b) continue;
    const int64_t blocks = (8 * (e - b) + 255) / 256;
    hipLaunchKernelGGL((corner_kernel<Acc>), dim3((unsigned)blocks), dim3(256), 0, s, T,
                       (const Acc*)t.centre, (const uint8_t*)t.coarse_corners, (Acc*)t.corners,
                       l, b, e);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

}  // namespace

hipError_t OctreeTensor::count_coarse_corners(hipStream_t s) {
  Tree T{child_oct_dev, reinterpret_cast<const int4*>(oct_info), n, (int64_t)n * n * n};
  for (int l = 1; l <= max_level; ++l) {
    const int64_t b = level_begin[l], e = level_begin[l + 1];
    if (e <= b) continue;
    hipLaunchKernelGGL(coarse_corner_kernel, dim3((unsigned)((e - b + 255) / 256)), dim3(256), 0,
                       s, T, coarse_corners, l, b, e);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t OctreeTensor::build(const void* values, int dtype, hipStream_t s) {
  if (precision == RR_PREC_FP32_KAHAN)
    return dtype == RR_F32 ? build_all<float, float>(*this, values, s)
                           : build_all<double, float>(*this, values, s);
  return dtype == RR_F32 ? build_all<float, double>(*this, values, s)
                         : build_all<double, double>(*this, values, s);
}

namespace {

template <typename R, int kMode>
hipError_t launch_march_w(const Tree& T, const void* cv, int64_t n_cells, const TraceArgs& a,
                          int persistent, int grid_waves, hipStream_t s) {
  const bool dbg = a.hash || a.log || a.count;
  // 32-bit cell indices and byte offsets when the corner blocks are below 4 GiB
  const bool small = n_cells * 48 * (int64_t)sizeof(R) < (1ll << 32);
  if (small)
    return dbg ? launch_march<R, true, kMode, uint32_t>(T, cv, a, persistent, grid_waves, s)
               : launch_march<R, false, kMode, uint32_t>(T, cv, a, persistent, grid_waves, s);
  return dbg ? launch_march<R, true, kMode, uint64_t>(T, cv, a, persistent, grid_waves, s)
             : launch_march<R, false, kMode, uint64_t>(T, cv, a, persistent, grid_waves, s);
}

}  // namespace

hipError_t OctreeTensor::march(const TraceArgs& a, int persistent, int grid_waves,
                               hipStream_t s) {
  if (a.n_tiles == 0) return hipSuccess;
  Tree T{child_oct_dev, reinterpret_cast<const int4*>(oct_info), n, (int64_t)n * n * n};
  if (a.mode == kOctNgp) {   // cell-centre records, 6 per cell
    if (precision == RR_PREC_FP32_KAHAN)
      return launch_march_w<float, kOctNgp>(T, centre, n_cells, a, persistent, grid_waves, s);
    return launch_march_w<double, kOctNgp>(T, centre, n_cells, a, persistent, grid_waves, s);
  }
  if (a.mode == kOctSources) {
    if (precision == RR_PREC_FP32_KAHAN)
      return launch_march_w<float, kOctSources>(T, corners, n_cells, a, persistent, grid_waves, s);
    return launch_march_w<double, kOctSources>(T, corners, n_cells, a, persistent, grid_waves, s);
  }
  if (precision == RR_PREC_FP32_KAHAN)
    return launch_march_w<float, kOctTidal>(T, corners, n_cells, a, persistent, grid_waves, s);
  return launch_march_w<double, kOctTidal>(T, corners, n_cells, a, persistent, grid_waves, s);
}

}  // namespace rr
