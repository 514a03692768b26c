// rr_march_uniform.hip -- cell-by-cell ray march through a uniform grid
// (Sec. III F, Eqs. rayposition - disttocross) with the per-cell lensing
// integral of the trilinear vertex reconstruction (Eqs. trilinear_int,
// Iclensing) and its accumulation along the ray (Eq. sumIc).
//
// Work decomposition: a wavefront owns an 8 x 8 tile of a bundle's ray map,
// so its 64 lanes start from neighbouring directions, visit neighbouring
// cells (coalesced, cache-friendly gathers) and take similar numbers of steps.
// Tiles are either mapped one per wavefront from the grid (XCD-striped so a
// chiplet's L2 sees a contiguous part of the sky) or pulled from a device
// queue by persistent workgroups.
#include <climits>

#include "rr_ray.hpp"

namespace rr {
namespace {

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Vertex record at byte offset `off` of the tensor (6 components: three
// 8-byte accesses in FP32, three 16-byte accesses in FP64).  A 32-bit offset
// lets the load take the array base from scalar registers.
template <typename R, typename Off>
__device__ __forceinline__ void load_vertex(const R* __restrict__ tv, Off off, R* t) {
  const char* b = reinterpret_cast<const char*>(tv) + (uint64_t)off;
  if constexpr (sizeof(R) == 4) {
    const float2* p = reinterpret_cast<const float2*>(b);
    const float2 x = p[0], y = p[1], z = p[2];
    t[0] = x.x; t[1] = x.y; t[2] = y.x; t[3] = y.y; t[4] = z.x; t[5] = z.y;
  } else {
    const double2* p = reinterpret_cast<const double2*>(b);
    const double2 x = p[0], y = p[1], z = p[2];
    t[0] = x.x; t[1] = x.y; t[2] = y.x; t[3] = y.y; t[4] = z.x; t[5] = z.y;
  }
}

// Q_v = P : T_v for the vertex record at byte offset off.
template <typename R, typename Off>
__device__ __forceinline__ R project(const R* __restrict__ tv, Off off, const R* P) {
  R t[6];
  load_vertex<R, Off>(tv, off, t);
  R acc = P[0] * t[0];
#pragma unroll
  for (int c = 1; c < 6; ++c) acc = fma(P[c], t[c], acc);
  return acc;
}

// Integrand modes: the tidal tensor with the trilinear integral, the tidal
// tensor at cell centres (NGP), Method A's (c delta, grad Phi) fields, the
// tidal tensor against the two source-distance moments chi and chi^2, and a
// vertex scalar with a constant kernel (ISW).
constexpr int kTidal = 0, kNgp = 1, kMethodA = 2, kSources = 3, kScalar = 4;

// Corner value(s) of the record at `off`: Q = P : T (tidal modes),
// (c delta, n . grad Phi) with P[0..2] = n (Method A), or the scalar (ISW).
template <typename R, typename Off, int kMode>
__device__ __forceinline__ void corner_value(const R* __restrict__ tv, Off off, const R* P, R& q,
                                             R& q2) {
  if constexpr (kMode == kScalar) {
    q = *reinterpret_cast<const R*>(reinterpret_cast<const char*>(tv) + (uint64_t)off);
    q2 = (R)0;
  } else if constexpr (kMode == kMethodA) {
    const char* b = reinterpret_cast<const char*>(tv) + (uint64_t)off;
    R t[4];
    if constexpr (sizeof(R) == 4) {
      const float4 x = *reinterpret_cast<const float4*>(b);
      t[0] = x.x; t[1] = x.y; t[2] = x.z; t[3] = x.w;
    } else {
      const double2* p = reinterpret_cast<const double2*>(b);
      const double2 x = p[0], y = p[1];
      t[0] = x.x; t[1] = x.y; t[2] = y.x; t[3] = y.y;
    }
    q = t[0];
    q2 = fma(P[2], t[3], fma(P[1], t[2], P[0] * t[1]));
  } else {
    q = project<R, Off>(tv, off, P);
    q2 = (R)0;
  }
}

// All eight corners (c = b0 + 2 b1 + 4 b2), loaded in two halves so that at
// most four vertex records are in flight: this path runs only at the start of
// a ray and after edge or vertex crossings, and must not set the register
// budget of the whole loop.
template <typename R, typename Off, int kMode>
__device__ __forceinline__ void load_corners(const R* __restrict__ tv, Off base, const Off* dX,
                                             const R* P, R* q, R* q2) {
  const Off v2 = base + dX[1];
  corner_value<R, Off, kMode>(tv, base, P, q[0], q2[0]);
  corner_value<R, Off, kMode>(tv, base + dX[0], P, q[1], q2[1]);
  corner_value<R, Off, kMode>(tv, v2, P, q[2], q2[2]);
  corner_value<R, Off, kMode>(tv, v2 + dX[0], P, q[3], q2[3]);
  __builtin_amdgcn_sched_barrier(0);
  const Off v4 = base + dX[2];
  const Off v6 = v4 + dX[1];
  corner_value<R, Off, kMode>(tv, v4, P, q[4], q2[4]);
  corner_value<R, Off, kMode>(tv, v4 + dX[0], P, q[5], q2[5]);
  corner_value<R, Off, kMode>(tv, v6, P, q[6], q2[6]);
  corner_value<R, Off, kMode>(tv, v6 + dX[0], P, q[7], q2[7]);
}

// One face crossed along axis k (one-hot k0, k1, k2 = neither): the four
// values of that face move to the entry face, the four of the new exit face
// F_j (j = i_a + 2 i_b over the two other axes a < b) come in (Method A's two
// corner sets; the tidal path writes the same selects inline).  The selects
// operate on register values: the empty asm statements keep the compiler
// from turning a select of two array elements into an indexed load, which
// would move the array to LDS.
template <typename R>
__device__ __forceinline__ void shift_face(R* q, bool k0, bool k1, R F0, R F1, R F2, R F3) {
  R a[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    a[c] = q[c];
    asm volatile("" : "+v"(a[c]));
  }
  const R n0 = k0 ? a[1] : (k1 ? a[2] : a[4]);
  const R n1 = k0 ? F0 : (k1 ? a[3] : a[5]);
  const R n2 = k0 ? a[3] : (k1 ? F0 : a[6]);
  const R n3 = k0 || k1 ? F1 : a[7];
  const R n4 = k0 ? a[5] : (k1 ? a[6] : F0);
  const R n5 = k0 ? F2 : (k1 ? a[7] : F1);
  const R n6 = k0 ? a[7] : F2;
  q[0] = n0; q[1] = n1; q[2] = n2; q[3] = n3;
  q[4] = n4; q[5] = n5; q[6] = n6; q[7] = F3;
}

// One ray, in the ray's own frame: along each axis, corner bit 0 is the
// vertex layer of the face the ray enters through and bit 1 the layer of the
// face it leaves through, and the local coordinate f runs from 0 (entry face)
// to 1 (exit face).  A crossing of one face then keeps the four projected
// corner values of that face (they become the entry face of the next cell)
// and loads only the four of the new exit face; a crossing through an edge or
// a vertex reloads all eight.
//
// Per axis the lane keeps, in FP64, the crossing parameter of the exit plane
// (f = 1 - |n_a| (chi - t_exit) inside the slab) and its reciprocal
// direction, and as integers the exit plane's lattice coordinate and the
// wrapped index of the exit vertex layer; the cell's entry corner is one byte
// offset into the vertex array (32 bit when the tensor is below 4 GiB), with
// per-axis steps to the exit layer (modular arithmetic).
template <typename R, bool kDebug, typename Off, int kMode, bool kPass>
__device__ void trace_one(const R* __restrict__ tv, const TraceArgs& a, const DevBundle& B,
                          int64_t ray) {
  const int64_t out = B.ray_offset + ray;
  const double d[3] = {B.dir[3 * ray + 0], B.dir[3 * ray + 1], B.dir[3 * ray + 2]};
  // Only unit directions are traced: that bounds the number of crossings by
  // the chi window validated on the host, so every lane terminates.
  const double nrm2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  if (!(fabs(nrm2 - 1.0) <= 1e-9)) {
    if (a.status) a.status[out] = RR_RAY_BAD_DIRECTION;
    return;
  }
  R P[6];
  if constexpr (kMode == kMethodA || kMode == kScalar) {
#pragma unroll
    for (int c = 0; c < 3; ++c) P[c] = (R)d[c];
  } else {
    double Pd[6];
    projection(a.quantity, d[0], d[1], d[2], Pd);
#pragma unroll
    for (int c = 0; c < 6; ++c) P[c] = (R)Pd[c];
  }

  const int n = a.n;
  constexpr Off kRec =
      (Off)((kMode == kMethodA ? 4 : (kMode == kScalar ? 1 : 6)) * sizeof(R));  // bytes per record
  const Off stride[3] = {kRec, kRec * (Off)n, kRec * (Off)n * (Off)n};
  const double lo = B.chi_lo;
  double chiA = B.chi_hi;
  // a later pass resumes on the face where the last one stopped
  if constexpr (kPass) {
    const double r0 = a.resume[out];
    if (!(r0 > lo)) return;             // done in an earlier pass
    chiA = fmin(r0, chiA);              // +inf before the first pass
    if (chiA <= a.pause_chi) return;    // starts in a later pass
  }
  double r[3], te[3];
  R absd[3];         // f(chi) = 1 - absd (chi - t_exit)
  int px[3];         // lattice coordinate of the exit plane (unwrapped, replicated box)
  int xl[3];         // exit vertex layer, wrapped into [0, n)
  Off base = 0;      // byte offset of the corner on all three entry layers
  Off dX[3];         // byte step from the entry to the exit layer
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r[k] = (d[k] != 0.0) ? 1.0 / d[k] : 0.0;
    const int m = start_slab(a.o[k], d[k], r[k], chiA, 1.0);
    // n_a > 0: the march runs down the lattice, leaving through plane m;
    // otherwise up, leaving through plane m + 1 (never reached if n_a = 0)
    px[k] = d[k] > 0.0 ? m : m + 1;
    if (d[k] != 0.0) {
      te[k] = tplane((double)px[k], a.o[k], r[k]);
      absd[k] = (R)fabs(d[k]);
    } else {
      // never crossed: a slope of 1e-30 with an exit parameter (1 - f) 1e30
      // below reproduces the fixed coordinate f = o~ - m to rounding, and the
      // parameter is never the largest (chi_lo >= 0)
      te[k] = -(1.0 - (a.o[k] - (double)m)) * 1e30;
      absd[k] = (R)1e-30;
    }
    int lm = m % n;
    lm = lm < 0 ? lm + n : lm;                       // layer of plane m
    const int lp = lm + 1 == n ? 0 : lm + 1;         // layer of plane m + 1
    const int el = d[k] > 0.0 ? lp : lm;
    xl[k] = d[k] > 0.0 ? lm : lp;
    base += (Off)el * stride[k];
    dX[k] = (Off)xl[k] * stride[k] - (Off)el * stride[k];
  }
  R fA[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    fA[k] = (R)1 - absd[k] * (R)(chiA - te[k]);
    // on the entry face (a resumed ray, or a window that starts on a face)
    // the coordinate is 0, as when the march steps across that face
    if (kPass && d[k] != 0.0 &&
        chiA == tplane((double)(d[k] > 0.0 ? px[k] + 1 : px[k] - 1), a.o[k], r[k]))
      fA[k] = (R)0;
  }

  R q[8], q2[8];  // corner values (q2: Method A's gradient term), c = b0 + 2 b1 + 4 b2
  if constexpr (kMode != kNgp) load_corners<R, Off, kMode>(tv, base, dX, P, q, q2);

  const R inv_chis = (R)(1.0 / B.chi_s);
  const R scale = (R)a.kappa_scale;
  R sum;
  float comp = 0.0f;
  // source-distance moments: (sum, comp) integrate chi Q, (sum2, comp2)
  // chi^2 Q; the walk also stops at the next source distance src_j
  R sum2 = 0;
  float comp2 = 0.0f;
  int jn = 0;
  double src_j = -1.0;
  if constexpr (kMode == kSources) {
    if constexpr (sizeof(R) == 4) {
      const float4 m = reinterpret_cast<const float4*>(a.kappa)[out];
      sum = m.x; comp = m.y; sum2 = m.z; comp2 = m.w;
    } else {
      const double2 m = reinterpret_cast<const double2*>(a.kappa)[out];
      sum = m.x; sum2 = m.y;
    }
    // this window stops at the sources with chi_lo <= chi_s,j < chi_hi
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

  for (;;) {
    if (a.open) {
      bool outside = false;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int m = r[k] > 0.0 ? px[k] : px[k] - 1;
        outside |= m < 2 || m > n - 3;
      }
      if (outside) {
        st = RR_RAY_OUT_OF_DOMAIN;
        break;
      }
    }
    if constexpr (kPass) {
      if (chiA <= a.pause_chi) break;   // the rest of the window is a later pass's
    }
    if (count >= maxc) {
      st = RR_RAY_MAX_STEPS;
      break;
    }
    // exit point: chi_B = max(chi_lo, t_exit,x, t_exit,y, t_exit,z), ties keep the earlier
    // (the next source distance takes the place of chi_lo when it lies above it)
    double chiB = lo;
    if constexpr (kMode == kSources) chiB = src_j >= lo ? src_j : lo;
    chiB = te[0] > chiB ? te[0] : chiB;
    chiB = te[1] > chiB ? te[1] : chiB;
    chiB = te[2] > chiB ? te[2] : chiB;
    bool stepped[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) stepped[k] = te[k] == chiB;

    // local coordinates of the exit point; exactly 1 on the crossed faces
    R fB[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) fB[k] = (R)1 - absd[k] * (R)(chiB - te[k]);
    const R L = (R)(chiA - chiB);
    R ic, ic2 = 0;
    if constexpr (kMode == kSources) {
      R ma, mb;
      cell_moments<R>(q, fA, fB, L, (R)chiB, ma, mb);
      ic = ma * scale;
      ic2 = mb * scale;
    } else if constexpr (kMode == kScalar) {
      ic = cell_integral_scalar<R>(q, fA, fB, L) * scale;
    } else if constexpr (kMode == kMethodA) {
      // Eq. (kappa2): c delta against g, n . grad Phi against dg/dchi, and the
      // step's surface term -[g n . grad Phi] at its first and last point
      R s = cell_integral_a<R>(q, q2, fA, fB, L, (R)chiB, (R)(B.chi_s - chiB), inv_chis);
      const bool first = count == 0 && chiA == B.chi_hi, last = chiB == lo;
      if (first || last) {
        R dq[4];
        dq[0] = q2[1] - q2[0]; dq[1] = q2[3] - q2[2]; dq[2] = q2[5] - q2[4]; dq[3] = q2[7] - q2[6];
        if (first) {
          const R g = (R)chiA * (R)(B.chi_s - chiA) * inv_chis;
          s -= g * trilerp<R>(q2, dq, fA[0], fA[1], fA[2]);
        }
        if (last) {
          const R g = (R)chiB * (R)(B.chi_s - chiB) * inv_chis;
          s += g * trilerp<R>(q2, dq, fB[0], fB[1], fB[2]);
        }
      }
      ic = s * scale;
    } else if constexpr (kMode == kNgp) {
      // Eq. (Iclensing_ngp): the cell-centre value times the integral of g over
      // the piece, L (g(mid) - L^2 / (12 chi_s)) with g(chi) = chi (chi_s - chi) / chi_s
      Off cellv = base;
#pragma unroll
      for (int k = 0; k < 3; ++k) cellv += r[k] > 0.0 ? dX[k] : (Off)0;
      const R Qc = project<R, Off>(tv, cellv, P);
      const double mid = chiB + 0.5 * (chiA - chiB);
      const R gm = (R)mid * (R)(B.chi_s - mid) - L * L * (R)(1.0 / 12.0);
      ic = Qc * (gm * L * inv_chis) * scale;
    } else {
      ic = cell_integral<R>(q, fA, fB, L, (R)chiB, (R)(B.chi_s - chiB), inv_chis) * scale;
    }
    if constexpr (sizeof(R) == 4) {
      kahan_add(sum, comp, ic);
      if constexpr (kMode == kSources) kahan_add(sum2, comp2, ic2);
    } else {
      sum += ic;
      if constexpr (kMode == kSources) sum2 += ic2;
    }
    if constexpr (kDebug) {
      // cell id = vertex id of its lower corner: the exit layer where n_a > 0
      Off low = base;
#pragma unroll
      for (int k = 0; k < 3; ++k) low += r[k] > 0.0 ? dX[k] : (Off)0;
      const int64_t cell = (int64_t)(low / kRec);
      if (a.hash) hv = fnv_piece(hv, cell, chiA, chiB);
      if (a.log && count < a.log_stride) {
        LogRecord* L0 = reinterpret_cast<LogRecord*>(a.log) + out * a.log_stride + count;
        L0->cell = cell;
        L0->chi_a = chiA;
        L0->chi_b = chiB;
      }
    }
    ++count;
    if constexpr (kMode == kSources) {
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
    if (chiB == lo) {
      chiA = lo;
      break;
    }
    // step every axis whose exit plane is at chi_B: the exit layer becomes
    // the entry layer, the next layer along the march the exit layer
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      fA[k] = fB[k];
      if (stepped[k]) {
        fA[k] = (R)0;
        const bool down = r[k] > 0.0;
        px[k] += down ? -1 : 1;
        te[k] = tplane((double)px[k], a.o[k], r[k]);
        base += dX[k];
        const Off wrapstep = (Off)(n - 1) * stride[k];
        if (down) {
          const bool wrap = xl[k] == 0;
          xl[k] = wrap ? n - 1 : xl[k] - 1;
          dX[k] = wrap ? wrapstep : (Off)0 - stride[k];
        } else {
          const bool wrap = xl[k] == n - 1;
          xl[k] = wrap ? 0 : xl[k] + 1;
          dX[k] = wrap ? (Off)0 - wrapstep : stride[k];
        }
      }
    }
    const int n_stepped = (int)stepped[0] + (int)stepped[1] + (int)stepped[2];
    if constexpr (kMode == kNgp) {
      // one record per cell: nothing carried from cell to cell
    } else if (kMode == kSources && n_stepped == 0) {
      // stopped at a source distance inside the cell: same corners
    } else if (n_stepped == 1) {
      // one face crossed (axis k): keep its four values, load the new exit face,
      // whose corners F_j (j = i_a + 2 i_b over the two other axes a < b)
      const bool k0 = stepped[0], k1 = stepped[1];
      const Off dk = k0 ? dX[0] : (k1 ? dX[1] : dX[2]);
      const Off da = k0 ? dX[1] : dX[0];
      const Off db = k0 || k1 ? dX[2] : dX[1];
      const Off w0 = base + dk, w1 = w0 + da;
      if constexpr (kMode == kMethodA || kMode == kScalar) {
        R F[4], G[4];
        corner_value<R, Off, kMode>(tv, w0, P, F[0], G[0]);
        corner_value<R, Off, kMode>(tv, w1, P, F[1], G[1]);
        corner_value<R, Off, kMode>(tv, w0 + db, P, F[2], G[2]);
        corner_value<R, Off, kMode>(tv, w1 + db, P, F[3], G[3]);
        shift_face<R>(q, k0, k1, F[0], F[1], F[2], F[3]);
        if constexpr (kMode == kMethodA) shift_face<R>(q2, k0, k1, G[0], G[1], G[2], G[3]);
      } else {
        const R F0 = project<R, Off>(tv, w0, P);
        const R F1 = project<R, Off>(tv, w1, P);
        const R F2 = project<R, Off>(tv, w0 + db, P);
        const R F3 = project<R, Off>(tv, w1 + db, P);
        if (__ballot(!k0 && !k1) == __ballot(1)) {
          // every marching lane crossed a z face (lines of sight near the z
          // axis): the old exit face becomes the entry face, no selects
          q[0] = q[4]; q[1] = q[5]; q[2] = q[6]; q[3] = q[7];
          q[4] = F0; q[5] = F1; q[6] = F2; q[7] = F3;
          chiA = chiB;
          continue;
        }
        const R n0 = k0 ? q[1] : (k1 ? q[2] : q[4]);
        const R n1 = k0 ? F0 : (k1 ? q[3] : q[5]);
        const R n2 = k0 ? q[3] : (k1 ? F0 : q[6]);
        const R n3 = k0 || k1 ? F1 : q[7];
        const R n4 = k0 ? q[5] : (k1 ? q[6] : F0);
        const R n5 = k0 ? F2 : (k1 ? q[7] : F1);
        const R n6 = k0 ? q[7] : F2;
        q[0] = n0; q[1] = n1; q[2] = n2; q[3] = n3;
        q[4] = n4; q[5] = n5; q[6] = n6; q[7] = F3;
      }
    } else {
      load_corners<R, Off, kMode>(tv, base, dX, P, q, q2);
    }
    chiA = chiB;
  }
  // a ray that ended without reaching chi_lo or an error stopped at a pass boundary
  const bool paused = st == RR_RAY_OK && chiA > lo;
  if (!(sum == sum) || sum - sum != (R)0) st = RR_RAY_NONFINITE;
  if constexpr (kMode == kSources) {
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
  if constexpr (kPass) a.resume[out] = paused ? chiA : -INFINITY;
  if (a.status) a.status[out] = st;
  if constexpr (kDebug) {
    if (a.hash) a.hash[out] = hv;
    if (a.count) a.count[out] = count;
  }
}

template <typename R, bool kDebug, typename Off, int kMode, bool kPass>
__device__ __forceinline__ void run_tile(const R* __restrict__ tv, const TraceArgs& a,
                                         int64_t tile, int lane) {
  const int b = find_bundle(a.bundles, a.n_bundles, tile);
  const DevBundle& B = a.bundles[b];
  int tx, ty;
  zorder_tile(tile - B.tile_begin, B.tiles_x, B.tiles_y, tx, ty);
  const int ix = tx * 8 + (lane & 7), iy = ty * 8 + (lane >> 3);
  if (ix < B.nx && iy < B.ny) trace_one<R, kDebug, Off, kMode, kPass>(tv, a, B, (int64_t)iy * B.nx + ix);
}

// One wavefront per tile.  Workgroups are dealt round-robin to the 8 XCDs;
// remap so that XCD x gets the x-th contiguous slice of tiles.  The FP32 loop
// is held to 96 VGPRs (5 wavefronts per SIMD): the march waits on dependent
// gathers, and the fifth wavefront hides more of that latency than the
// compiler's unconstrained schedule (100 VGPRs, 4 wavefronts) gains.
template <typename R, bool kDebug, typename Off, int kMode, bool kPass>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 5 : 1)))
void march_uniform_kernel(const R* __restrict__ tv,
                                                            TraceArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t nblk = gridDim.x;
  const int64_t blk = blockIdx.x;
  const int64_t per = (nblk + 7) / 8;
  const int64_t xcd = blk % 8, slot = blk / 8;
  const int64_t vblk = xcd * per + slot;
  // the tile is the same for the 64 lanes: keep it (and the bundle) scalar
  const int64_t tile = vblk * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(wave);
  if (tile >= a.n_tiles) return;
  run_tile<R, kDebug, Off, kMode, kPass>(tv, a, tile, lane);
}

// Persistent workgroups: every wavefront pulls tiles from its chiplet's
// counter, then from the others', until all are drained (every wave reaches
// the exit test).  The tile is the same for the 64 lanes: it (and the
// bundle) stays scalar.
template <typename R, bool kDebug, typename Off, int kMode, bool kPass>
__global__ __launch_bounds__(256) void march_uniform_persistent(const R* __restrict__ tv,
                                                                TraceArgs a) {
  const int lane = threadIdx.x & 63;
  int q = blockIdx.x % kQueues, tried = 0;
  for (;;) {
    const int64_t tile = next_tile(a.queue, a.n_tiles, q, tried, lane);
    if (tile < 0) break;
    run_tile<R, kDebug, Off, kMode, kPass>(tv, a, tile, lane);
  }
}

__global__ void queue_reset_kernel(unsigned long long* q) {
  if (threadIdx.x < kQueues) q[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(256) void fill_kernel(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// kappa of every source (Eqs. Isources, Isources1) once the walk has reached
// the observer: the moment state holds what lies below the nearest source,
// and summing the pieces from the observer outwards gives int chi Q and
// int chi^2 Q below each source in turn, kappa_j = A_j - B_j / chi_s,j.
// FP64 throughout; one thread per ray.
template <typename R>
__global__ __launch_bounds__(256) void kappa_from_pieces_kernel(const R* __restrict__ mom,
                                                                const double* __restrict__ pieces,
                                                                const double* __restrict__ src,
                                                                int ns, int64_t nr,
                                                                double* __restrict__ kappa) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  double A, B;
  if constexpr (sizeof(R) == 4) {
    const float4 m = reinterpret_cast<const float4*>(mom)[r];
    A = (double)m.x - (double)m.y;
    B = (double)m.z - (double)m.w;
  } else {
    const double2 m = reinterpret_cast<const double2*>(mom)[r];
    A = m.x;
    B = m.y;
  }
  for (int j = ns - 1; j >= 0; --j) {
    kappa[r * ns + j] = A - B / src[j];
    A += pieces[(r * ns + j) * 2 + 0];
    B += pieces[(r * ns + j) * 2 + 1];
  }
}

template <typename R, bool kDebug, typename Off, int kMode, bool kPass>
hipError_t launch3(const void* tv, const TraceArgs& a, int persistent, int block, int grid_waves,
                   hipStream_t s) {
  const int wpb = block / 64;
  if (persistent) {
    const int blocks = (grid_waves + wpb - 1) / wpb;
    hipLaunchKernelGGL((march_uniform_persistent<R, kDebug, Off, kMode, kPass>), dim3(blocks), dim3(block), 0, s,
                       (const R*)tv, a);
  } else {
    int64_t blocks = (a.n_tiles + wpb - 1) / wpb;
    if (blocks == 0) return hipSuccess;
    blocks = (blocks + 7) / 8 * 8;   // the XCD remap is a bijection on multiples of 8
    hipLaunchKernelGGL((march_uniform_kernel<R, kDebug, Off, kMode, kPass>), dim3((unsigned)blocks), dim3(block),
                       0, s, (const R*)tv, a);
  }
  return hipGetLastError();
}

template <typename R, int kMode>
hipError_t launch_mode(const void* tv, const TraceArgs& a, bool small, int persistent, int block,
                       int grid_waves, hipStream_t s) {
  const bool dbg = a.hash || a.log || a.count;
  // split marches never carry debug outputs (the host keeps those in one pass)
  if (a.resume)
    return small ? launch3<R, false, uint32_t, kMode, true>(tv, a, persistent, block, grid_waves, s)
                 : launch3<R, false, uint64_t, kMode, true>(tv, a, persistent, block, grid_waves, s);
  if (dbg)
    return small ? launch3<R, true, uint32_t, kMode, false>(tv, a, persistent, block, grid_waves, s)
                 : launch3<R, true, uint64_t, kMode, false>(tv, a, persistent, block, grid_waves, s);
  return small ? launch3<R, false, uint32_t, kMode, false>(tv, a, persistent, block, grid_waves, s)
               : launch3<R, false, uint64_t, kMode, false>(tv, a, persistent, block, grid_waves, s);
}

template <typename R>
hipError_t launch(const void* tv, const TraceArgs& a, int persistent, int block, int grid_waves,
                  hipStream_t s) {
  // 32-bit byte offsets when the whole tensor is below 4 GiB
  const int words = a.mode == kMethodA ? 4 : (a.mode == kScalar ? 1 : 6);
  const bool small = (int64_t)a.n * a.n * a.n * (int64_t)(words * sizeof(R)) < (1ll << 32);
  switch (a.mode) {
    case kNgp: return launch_mode<R, kNgp>(tv, a, small, persistent, block, grid_waves, s);
    case kMethodA: return launch_mode<R, kMethodA>(tv, a, small, persistent, block, grid_waves, s);
    case kSources: return launch_mode<R, kSources>(tv, a, small, persistent, block, grid_waves, s);
    case kScalar: return launch_mode<R, kScalar>(tv, a, small, persistent, block, grid_waves, s);
    default: return launch_mode<R, kTidal>(tv, a, small, persistent, block, grid_waves, s);
  }
}

}  // namespace

hipError_t launch_march_uniform(int precision, const void* tv, const TraceArgs& a, int persistent,
                                int block, int grid_waves, hipStream_t s) {
  if (precision == RR_PREC_FP32_KAHAN) return launch<float>(tv, a, persistent, block, grid_waves, s);
  return launch<double>(tv, a, persistent, block, grid_waves, s);
}

hipError_t launch_kappa_from_pieces(int precision, const void* moments, const double* pieces,
                                    const double* src, int n_src, int64_t n_rays, double* kappa,
                                    hipStream_t s) {
  const int64_t blocks = (n_rays + 255) / 256;
  if (blocks == 0) return hipSuccess;
  if (precision == RR_PREC_FP32_KAHAN)
    hipLaunchKernelGGL(kappa_from_pieces_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const float*)moments, pieces, src, n_src, n_rays, kappa);
  else
    hipLaunchKernelGGL(kappa_from_pieces_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const double*)moments, pieces, src, n_src, n_rays, kappa);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  const int64_t blocks = (n + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_queue_reset(unsigned long long* q, hipStream_t s) {
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, s, q);
  return hipGetLastError();
}

}  // namespace rr
