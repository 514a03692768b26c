// rr_adjoint_uniform.hip -- gradient of L = sum_r w_r kappa_r with respect to
// the potential of a uniform periodic grid.
//
// kappa is linear in Phi (straight rays, Born approximation, Sec. IV A), so
// dL/dPhi = A^T w for the forward chain A = (per-cell integrals) o (vertex
// mean, Sec. III F) o (finite differences, Eq. tidalexample):
//   1. scatter: re-walk every ray; the integral over one cell is
//      sum_v omega_v Q_v with Q_v = P . T_v, so the cell adds
//      w * scale * omega_v * P_ab to Lambda_v,ab = dL/dT_v,ab.  A corner's
//      weights are summed in registers while the ray stays next to it and
//      flushed with FP32 atomics when the ray moves away from it.
//   2. transpose: dL/dPhi = sum_ab D_ab^T Avg^T Lambda_ab.  Both operators are
//      convolutions on the periodic grid; composed per axis they become
//      S'f(c) = (f(c+2) - f(c+1)) - (f(c) - f(c-1))   (second difference)
//      D'f(c) = (f(c+2) - f(c)) + (f(c+1) - f(c-1))   (first difference)
//      B'f(c) = f(c) + f(c+1)                           (vertex sum)
//      dL/dPhi = (1/8)(S'x B'y B'z Lxx + B'x S'y B'z Lyy + B'x B'y S'z Lzz)
//              + (1/32)(D'x D'y B'z Lxy + D'x B'y D'z Lxz + B'x D'y D'z Lyz).
#include "rr_octree.hpp"
#include "rr_ray.hpp"

namespace rr {
namespace {

__global__ void fill_zero_kernel(float* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < n; k += stride) p[k] = 0.0f;
}

// Per-corner weights of the three-point Gauss-Legendre integral of one cell:
// omega_v = L/chi_s * sum_k w_k g(chi_k) N_v(u_k), N_v the trilinear basis.
__device__ __forceinline__ void corner_weights(const float* uA, const float* uB, float L,
                                               float chiB, float DB, float inv_chis, float* om) {
  const float cs[3] = {(float)GL3::c0, (float)GL3::c1, (float)GL3::c2};
  const float ws[3] = {(float)GL3::w0, (float)GL3::w1, (float)GL3::w2};
#pragma unroll
  for (int v = 0; v < 8; ++v) om[v] = 0.0f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float c = cs[k];
    const float ux = fmaf(uA[0] - uB[0], c, uB[0]);
    const float uy = fmaf(uA[1] - uB[1], c, uB[1]);
    const float uz = fmaf(uA[2] - uB[2], c, uB[2]);
    const float chik = fmaf(L, c, chiB);
    const float W = ws[k] * chik * fmaf(-L, c, DB);
    const float z1 = W * uz, z0 = W - z1;
    const float y1z0 = uy * z0, y0z0 = z0 - y1z0, y1z1 = uy * z1, y0z1 = z1 - y1z1;
    om[0] = fmaf(1.0f - ux, y0z0, om[0]);
    om[1] = fmaf(ux, y0z0, om[1]);
    om[2] = fmaf(1.0f - ux, y1z0, om[2]);
    om[3] = fmaf(ux, y1z0, om[3]);
    om[4] = fmaf(1.0f - ux, y0z1, om[4]);
    om[5] = fmaf(ux, y0z1, om[5]);
    om[6] = fmaf(1.0f - ux, y1z1, om[6]);
    om[7] = fmaf(ux, y1z1, om[7]);
  }
  const float s = L * inv_chis;
#pragma unroll
  for (int v = 0; v < 8; ++v) om[v] *= s;
}

// x of another lane of the same row of 16, picked by a DPP lane pattern.
template <int kCtrl>
__device__ __forceinline__ float dpp_lane(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xf, 0xf, false));
}

// Sum over the 64 lanes (every lane active), returned as a wavefront-uniform
// value.  Within each row of 16 lanes: add lane i ^ 1, lane i ^ 2 (quad
// permutes), then the mirrored lane of the half row (the other quad of eight)
// and of the row (the other eight); the four row sums are then read out of
// lanes 0, 16, 32 and 48.  Lane moves, no LDS traffic.
__device__ __forceinline__ float wave_sum(float x) {
  x += dpp_lane<0xb1>(x);    // quad_perm [1,0,3,2]
  x += dpp_lane<0x4e>(x);    // quad_perm [2,3,0,1]
  x += dpp_lane<0x141>(x);   // row_half_mirror
  x += dpp_lane<0x140>(x);   // row_mirror
  const int b = __float_as_int(x);
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(b, 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(b, 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(b, 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(b, 48));
  return (r0 + r1) + (r2 + r3);
}

// Retire one corner of every lane that has weight on it (acc != 0): its six
// tensor components get acc * P_ab.  The rays of a tile run side by side and
// every cell is crossed by many rays, so per-lane atomics on one address
// would serialise: the retiring lanes are grouped by vertex (one group per
// distinct vertex, usually one or two per wavefront), each group's six sums
// are reduced across the wavefront and its first lane issues the global
// atomics.  Called with all 64 lanes active (acc = 0 for lanes that retire
// nothing, including lanes whose ray has ended).
__device__ __forceinline__ void flush_corner(float* __restrict__ lam, uint64_t vid, float acc,
                                             const float* P, int lane) {
  bool want = acc != 0.0f;
  unsigned long long m = __ballot(want);
  while (m != 0ull) {
    const int leader = __builtin_ctzll(m);
    const uint64_t lv =
        ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(vid >> 32), leader) << 32) |
        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)vid, leader);
    const bool mine = want && vid == lv;
    float sums[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) sums[c] = wave_sum(mine ? acc * P[c] : 0.0f);
    if (lane == leader) {
      float* dst = lam + lv * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) atomicAdd(dst + c, sums[c]);
    }
    want = want && !mine;
    m = __ballot(want);
  }
}

// One 8 x 8 tile of rays, all 64 lanes kept active to the end (lanes without
// a ray, or whose ray has ended, take part in the wavefront reductions with
// nothing to add).
__device__ void scatter_tile(const TraceArgs& a, const DevBundle& B, int ix, int iy, int lane,
                             const float* __restrict__ wts, float* __restrict__ lam) {
  bool alive = ix < B.nx && iy < B.ny;
  const int64_t ray = alive ? (int64_t)iy * B.nx + ix : 0;
  const int64_t out = B.ray_offset + ray;
  float wr = 0.0f;
  double d[3] = {0.0, 0.0, 1.0};
  if (alive) {
    wr = wts[out] * (float)a.kappa_scale;
    const double e0 = B.dir[3 * ray + 0], e1 = B.dir[3 * ray + 1], e2 = B.dir[3 * ray + 2];
    const double nrm2 = e0 * e0 + e1 * e1 + e2 * e2;
    alive = wr != 0.0f && fabs(nrm2 - 1.0) <= 1e-9;
    if (alive) {
      d[0] = e0;
      d[1] = e1;
      d[2] = e2;
    }
  }
  double Pd[6];
  projection(RR_Q_KAPPA, d[0], d[1], d[2], Pd);
  float P[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) P[c] = (float)Pd[c] * wr;

  const int n = a.n;
  const uint64_t nI = (uint64_t)n, nnI = nI * nI;
  const uint64_t stride[3] = {1, nI, nnI};
  const double lo = B.chi_lo;
  double chiA = B.chi_hi;
  double r[3], pe[3], te[3], cpos[3], sgn[3];
  int w[3];
  uint64_t off0[3], off1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r[k] = (d[k] != 0.0) ? 1.0 / d[k] : 0.0;
    const int m = start_slab(a.o[k], d[k], r[k], chiA, 1.0);
    sgn[k] = d[k] > 0.0 ? -1.0 : 1.0;
    pe[k] = (double)(d[k] > 0.0 ? m : m + 1);
    te[k] = d[k] != 0.0 ? tplane(pe[k], a.o[k], r[k]) : -__builtin_inf();
    cpos[k] = a.o[k] - (double)m;
    const int ww = m % n;
    w[k] = ww < 0 ? ww + n : ww;
    off0[k] = (uint64_t)w[k] * stride[k];
    off1[k] = (uint64_t)(w[k] + 1 == n ? 0 : w[k] + 1) * stride[k];
  }
  float uA[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) uA[k] = (float)fma(chiA, d[k], cpos[k]);
  const float inv_chis = (float)(1.0 / B.chi_s);
  const int64_t maxc = a.max_crossings > 0 ? a.max_crossings : INT64_MAX;
  float acc[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) acc[v] = 0.0f;
  int64_t count = 0;
  bool stopped = false;   // ended by max_crossings: its open corners still retire

  while (__ballot(alive) != 0ull) {
    bool stepped[3] = {false, false, false};
    float uB[3] = {0.0f, 0.0f, 0.0f};
    double chiB = lo;
    int retire = 0;
    int kk = -1;
    bool last = false;
    if (alive) {
      if (count >= maxc) {
        alive = false;
        stopped = true;
      } else {
        chiB = te[0] > chiB ? te[0] : chiB;
        chiB = te[1] > chiB ? te[1] : chiB;
        chiB = te[2] > chiB ? te[2] : chiB;
#pragma unroll
        for (int k = 0; k < 3; ++k) stepped[k] = te[k] == chiB;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const float face = d[k] > 0.0 ? 0.0f : 1.0f;
          uB[k] = stepped[k] ? face : (float)fma(chiB, d[k], cpos[k]);
        }
        float om[8];
        corner_weights(uA, uB, (float)(chiA - chiB), (float)chiB, (float)(B.chi_s - chiB),
                       inv_chis, om);
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[v] += om[v];
        ++count;
        last = chiB == lo;
        const int nstep = (int)stepped[0] + (int)stepped[1] + (int)stepped[2];
        // corners that retire: all eight at the end of the ray or after an
        // edge/vertex crossing; after a single-axis step along k the face the
        // ray leaves behind (the crossed face is shared with the next cell)
        retire = 0xff;
        if (!last && nstep == 1) {
          kk = stepped[0] ? 0 : (stepped[1] ? 1 : 2);
          const int bit = 1 << kk;
          const int keep = d[kk] > 0.0 ? 0 : bit;   // corners on the crossed face
          retire = 0;
#pragma unroll
          for (int v = 0; v < 8; ++v)
            if ((v & bit) != keep) retire |= 1 << v;
        }
      }
    }
    if (stopped) retire = 0xff;
    // corner ids of the current cell (v = ix + 2 iy + 4 iz)
    uint64_t vid[8];
    {
      const uint64_t zy00 = off0[2] + off0[1], zy01 = off0[2] + off1[1];
      const uint64_t zy10 = off1[2] + off0[1], zy11 = off1[2] + off1[1];
      vid[0] = zy00 + off0[0]; vid[1] = zy00 + off1[0]; vid[2] = zy01 + off0[0];
      vid[3] = zy01 + off1[0]; vid[4] = zy10 + off0[0]; vid[5] = zy10 + off1[0];
      vid[6] = zy11 + off0[0]; vid[7] = zy11 + off1[0];
    }
#pragma unroll
    for (int v = 0; v < 8; ++v)
      flush_corner(lam, vid[v], ((retire >> v) & 1) ? acc[v] : 0.0f, P, lane);
    if (stopped) {
#pragma unroll
      for (int v = 0; v < 8; ++v) acc[v] = 0.0f;
      stopped = false;
    }
    if (!alive) continue;
    if (last) {
      alive = false;
      continue;
    }
    if (kk < 0) {
#pragma unroll
      for (int v = 0; v < 8; ++v) acc[v] = 0.0f;
    } else {
      // the crossed face becomes the opposite face of the next cell
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k != kk) continue;
        const int bit = 1 << k;
        const int keep = d[k] > 0.0 ? 0 : bit;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          if ((v & bit) != keep) {
            acc[v] = acc[v ^ bit];
            acc[v ^ bit] = 0.0f;
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uA[k] = uB[k];
      if (stepped[k]) {
        pe[k] += sgn[k];
        te[k] = tplane(pe[k], a.o[k], r[k]);
        cpos[k] -= sgn[k];
        uA[k] = 1.0f - uB[k];
        const int s = d[k] > 0.0 ? -1 : 1;
        int ww = w[k] + s;
        ww = ww < 0 ? ww + n : (ww >= n ? ww - n : ww);
        w[k] = ww;
        off0[k] = (uint64_t)ww * stride[k];
        off1[k] = (uint64_t)(ww + 1 == n ? 0 : ww + 1) * stride[k];
      }
    }
    chiA = chiB;
  }
}

__global__ __launch_bounds__(256) void scatter_kernel(TraceArgs a, const float* __restrict__ wts,
                                                      float* __restrict__ lam) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t nblk = gridDim.x, blk = blockIdx.x;
  const int64_t per = (nblk + 7) / 8;
  const int64_t tile = ((blk % 8) * per + blk / 8) * (blockDim.x >> 6) +
                       __builtin_amdgcn_readfirstlane(wave);
  if (tile >= a.n_tiles) return;
  const int b = find_bundle(a.bundles, a.n_bundles, tile);
  const DevBundle& B = a.bundles[b];
  const int64_t local = tile - B.tile_begin;
  const int tx = (int)(local % B.tiles_x), ty = (int)(local / B.tiles_x);
  scatter_tile(a, B, tx * 8 + (lane & 7), ty * 8 + (lane >> 3), lane, wts, lam);
}

// Transpose stencil: one thread per cell, all inputs from L2 (Lambda is
// written by the scatter just before and fits the last-level caches for the
// grids this path targets).
__device__ __forceinline__ int wrapn(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__global__ __launch_bounds__(256) void transpose_kernel(const float* __restrict__ lam,
                                                        float* __restrict__ dphi, int n) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (c >= nn * n) return;
  const int i = (int)(c % n), j = (int)((c / n) % n), k = (int)(c / nn);
  int xs[4], ys[4], zs[4];   // c-1, c, c+1, c+2 (wrapped)
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    xs[t] = wrapn(i - 1 + t, n);
    ys[t] = wrapn(j - 1 + t, n);
    zs[t] = wrapn(k - 1 + t, n);
  }
  auto L = [&](int tz, int ty, int tx, int comp) -> float {
    return lam[(((int64_t)zs[tz] * n + ys[ty]) * n + xs[tx]) * 6 + comp];
  };
  // S' along one axis with B' on the other two: the cell's vertices are
  // offsets 1, 2 (t index), the stencil spans t = 0..3
  float sxx = 0.f, syy = 0.f, szz = 0.f, dxy = 0.f, dxz = 0.f, dyz = 0.f;
#pragma unroll
  for (int p = 1; p <= 2; ++p)
#pragma unroll
    for (int q = 1; q <= 2; ++q) {
      sxx += (L(p, q, 3, 0) - L(p, q, 2, 0)) - (L(p, q, 1, 0) - L(p, q, 0, 0));
      syy += (L(p, 3, q, 1) - L(p, 2, q, 1)) - (L(p, 1, q, 1) - L(p, 0, q, 1));
      szz += (L(3, p, q, 2) - L(2, p, q, 2)) - (L(1, p, q, 2) - L(0, p, q, 2));
    }
  auto Dx = [&](int tz, int ty, int comp) {
    return (L(tz, ty, 3, comp) - L(tz, ty, 1, comp)) + (L(tz, ty, 2, comp) - L(tz, ty, 0, comp));
  };
  auto Dy = [&](int tz, int tx, int comp) {
    return (L(tz, 3, tx, comp) - L(tz, 1, tx, comp)) + (L(tz, 2, tx, comp) - L(tz, 0, tx, comp));
  };
#pragma unroll
  for (int p = 1; p <= 2; ++p) {
    dxy += (Dx(p, 3, 3) - Dx(p, 1, 3)) + (Dx(p, 2, 3) - Dx(p, 0, 3));
    dxz += (Dx(3, p, 4) - Dx(1, p, 4)) + (Dx(2, p, 4) - Dx(0, p, 4));
    dyz += (Dy(3, p, 5) - Dy(1, p, 5)) + (Dy(2, p, 5) - Dy(0, p, 5));
  }
  dphi[c] += (sxx + syy + szz) * 0.125f + (dxy + dxz + dyz) * 0.03125f;
}

}  // namespace

hipError_t launch_adjoint_uniform(const TraceArgs& a, const float* dl_dkappa, float* lam,
                                  float* dl_dphi, hipStream_t s) {
  const int64_t nv = (int64_t)a.n * a.n * a.n;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(2048), dim3(256), 0, s, lam, nv * 6);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.n_tiles > 0) {
    int64_t blocks = (a.n_tiles + 3) / 4;
    blocks = (blocks + 7) / 8 * 8;
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, dl_dkappa, lam);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t tb = (nv + 255) / 256;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)tb), dim3(256), 0, s, (const float*)lam,
                     dl_dphi, a.n);
  return hipGetLastError();
}

}  // namespace rr
