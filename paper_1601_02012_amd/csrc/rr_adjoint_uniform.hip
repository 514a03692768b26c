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

// A wavefront's cache of retired vertex sums in LDS, direct-mapped on the low
// bits of the vertex coordinates: the lanes of a tile drift apart by a step
// or two, so a vertex is often retired by several groups of lanes a few steps
// apart; their sums meet in the cache, and a vertex goes to global memory
// (six FP32 atomics) when its slot is taken by another vertex or the tile
// ends.  Only group leaders touch it, one at a time.
struct CacheSlot {
  uint64_t tag;   // vertex id, or kEmpty
  float v[6];
};
constexpr int kSlots = 256;   // x & 7, y & 7, z & 3
constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ void flush_slot(float* __restrict__ lam, const CacheSlot& e) {
  if (e.tag != kEmpty) {
    float* dst = lam + e.tag * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) atomicAdd(dst + c, e.v[c]);
  }
}

// Retire one corner of every lane that has weight on it (acc != 0): its six
// tensor components get acc * P_ab.  The rays of a tile run side by side and
// every cell is crossed by many rays, so per-lane atomics on one address
// would serialise: the retiring lanes are grouped by vertex (one group per
// distinct vertex, usually one or two per wavefront), each group's six sums
// are reduced across the wavefront and its first lane adds them to the
// wavefront's cache.  Called with all 64 lanes active (acc = 0 for lanes
// that retire nothing, including lanes whose ray has ended).
__device__ __forceinline__ void flush_corner(float* __restrict__ lam, CacheSlot* cache,
                                             uint64_t vid, int slot, float acc, const float* P,
                                             int lane) {
  bool want = acc != 0.0f;
  unsigned long long m = __ballot(want);
  while (m != 0ull) {
    const int leader = __builtin_ctzll(m);
    const uint64_t lv =
        ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(vid >> 32), leader) << 32) |
        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)vid, leader);
    const int ls = __builtin_amdgcn_readlane(slot, leader);
    const bool mine = want && vid == lv;
    float sums[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) sums[c] = wave_sum(mine ? acc * P[c] : 0.0f);
    if (lane == leader) {
      CacheSlot& e = cache[ls];
      if (e.tag == lv) {
#pragma unroll
        for (int c = 0; c < 6; ++c) e.v[c] += sums[c];
      } else {
        flush_slot(lam, e);
        e.tag = lv;
#pragma unroll
        for (int c = 0; c < 6; ++c) e.v[c] = sums[c];
      }
    }
    want = want && !mine;
    m = __ballot(want);
  }
}

// One 8 x 8 tile of rays, all 64 lanes kept active to the end (lanes without
// a ray, or whose ray has ended, take part in the wavefront reductions with
// nothing to add).
__device__ void scatter_tile(const TraceArgs& a, const DevBundle& B, int ix, int iy, int lane,
                             const float* __restrict__ wts, float* __restrict__ lam,
                             CacheSlot* cache) {
  for (int e = lane; e < kSlots; e += 64) cache[e].tag = kEmpty;
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
    int slot[8];
    {
      int cx[2], cy[2], cz[2];
      cx[0] = w[0]; cx[1] = w[0] + 1 == n ? 0 : w[0] + 1;
      cy[0] = w[1]; cy[1] = w[1] + 1 == n ? 0 : w[1] + 1;
      cz[0] = w[2]; cz[1] = w[2] + 1 == n ? 0 : w[2] + 1;
#pragma unroll
      for (int v = 0; v < 8; ++v)
        slot[v] = (cx[v & 1] & 7) | ((cy[(v >> 1) & 1] & 7) << 3) | ((cz[v >> 2] & 3) << 6);
    }
    {
      const uint64_t zy00 = off0[2] + off0[1], zy01 = off0[2] + off1[1];
      const uint64_t zy10 = off1[2] + off0[1], zy11 = off1[2] + off1[1];
      vid[0] = zy00 + off0[0]; vid[1] = zy00 + off1[0]; vid[2] = zy01 + off0[0];
      vid[3] = zy01 + off1[0]; vid[4] = zy10 + off0[0]; vid[5] = zy10 + off1[0];
      vid[6] = zy11 + off0[0]; vid[7] = zy11 + off1[0];
    }
#pragma unroll
    for (int v = 0; v < 8; ++v)
      flush_corner(lam, cache, vid[v], slot[v], ((retire >> v) & 1) ? acc[v] : 0.0f, P, lane);
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
  for (int e = lane; e < kSlots; e += 64) flush_slot(lam, cache[e]);
}

__global__ __launch_bounds__(256) void scatter_kernel(TraceArgs a, const float* __restrict__ wts,
                                                      float* __restrict__ lam) {
  __shared__ CacheSlot cache[4][kSlots];
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
  scatter_tile(a, B, tx * 8 + (lane & 7), ty * 8 + (lane >> 3), lane, wts, lam,
               cache[__builtin_amdgcn_readfirstlane(wave)]);
}

// Transpose stencil, built like the forward tensor: a workgroup owns a
// 64 x 16 column of cells and marches 16 cells along z; each step stages one
// vertex plane of Lambda (six components, with a halo of one vertex below and
// two above in x and y) in LDS, each thread loading its share of the next
// plane while the current one is used.  Cell c uses vertices c-1 .. c+2 on
// each axis (t = 0..3); per plane the thread forms the in-plane parts of the
// six terms, keeps the raw per-column values of the two z-differenced ones,
// and combines four planes.
constexpr int kTX = 64, kTY = 16, kTZ = 16;

__global__ __launch_bounds__(kTX * kTY) void transpose_kernel(const float* __restrict__ lam,
                                                              float* __restrict__ dphi, int n,
                                                              int ntx, int nty) {
  constexpr int NT = kTX * kTY;
  constexpr int PX = kTX + 3, PY = kTY + 3;
  constexpr int PL = PX * PY;
  constexpr int kN = (PL + NT - 1) / NT;
  __shared__ float sl[2][6][PL];
  const int b = blockIdx.x;
  const int bx = b % ntx, by = (b / ntx) % nty, bz = b / (ntx * nty);
  const int i0 = bx * kTX, j0 = by * kTY, k0 = bz * kTZ;
  const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
  const int i = i0 + tx, j = j0 + ty;
  const bool mine = i < n && j < n;
  const int64_t nn = (int64_t)n * n;
  const int k_end = min(k0 + kTZ, n);       // cells k0 .. k_end - 1

  int off[kN];
  bool act[kN];
#pragma unroll
  for (int u = 0; u < kN; ++u) {
    const int e = threadIdx.x + NT * u;
    act[u] = e < PL;
    int wx = (i0 - 1 + e % PX) % n, wy = (j0 - 1 + e / PX) % n;
    wx = wx < 0 ? wx + n : wx;
    wy = wy < 0 ? wy + n : wy;
    off[u] = wy * n + wx;
  }
  float2 pre[kN][3];
  auto fetch = [&](int gz) {
    const float* src = lam + (int64_t)gz * nn * 6;
#pragma unroll
    for (int u = 0; u < kN; ++u)
      if (act[u]) {
        const float2* r = reinterpret_cast<const float2*>(src + (int64_t)off[u] * 6);
        pre[u][0] = r[0];
        pre[u][1] = r[1];
        pre[u][2] = r[2];
      }
  };

  // histories over the planes t = 0..3 (vertex planes p-3 .. p)
  float AXX[4] = {}, AYY[4] = {}, AXY[4] = {};   // in-plane S'x B'y, B'x S'y, D'x D'y
  float ZZ[4][4] = {};                           // Lzz at the 2x2 columns
  float XZ[4][2] = {}, YZ[4][2] = {};            // D'x Lxz on rows j, j+1; D'y Lyz on columns i, i+1
  int slot = 0;
  int gz = (k0 - 1) % n;
  if (gz < 0) gz += n;
  fetch(gz);
  for (int p = k0 - 1; p <= k_end + 1; ++p, slot ^= 1) {
#pragma unroll
    for (int u = 0; u < kN; ++u)
      if (act[u]) {
        const int e = threadIdx.x + NT * u;
        sl[slot][0][e] = pre[u][0].x; sl[slot][1][e] = pre[u][0].y;
        sl[slot][2][e] = pre[u][1].x; sl[slot][3][e] = pre[u][1].y;
        sl[slot][4][e] = pre[u][2].x; sl[slot][5][e] = pre[u][2].y;
      }
    if (++gz == n) gz = 0;
    __syncthreads();
    if (p < k_end + 1) fetch(gz);
    auto L = [&](int comp, int ty_, int tx_) { return sl[slot][comp][(ty + ty_) * PX + tx + tx_]; };
    float axx = 0.f, ayy = 0.f, azz[2][2], xz[2], yz[2];
#pragma unroll
    for (int q = 1; q <= 2; ++q)
      axx += (L(0, q, 3) - L(0, q, 2)) - (L(0, q, 1) - L(0, q, 0));
#pragma unroll
    for (int c = 1; c <= 2; ++c)
      ayy += (L(1, 3, c) - L(1, 2, c)) - (L(1, 1, c) - L(1, 0, c));
#pragma unroll
    for (int q = 1; q <= 2; ++q)
#pragma unroll
      for (int c = 1; c <= 2; ++c) azz[q - 1][c - 1] = L(2, q, c);
    float dx3[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) dx3[r] = (L(3, r, 3) - L(3, r, 1)) + (L(3, r, 2) - L(3, r, 0));
    const float axy = (dx3[3] - dx3[1]) + (dx3[2] - dx3[0]);
#pragma unroll
    for (int q = 1; q <= 2; ++q) xz[q - 1] = (L(4, q, 3) - L(4, q, 1)) + (L(4, q, 2) - L(4, q, 0));
#pragma unroll
    for (int c = 1; c <= 2; ++c) yz[c - 1] = (L(5, 3, c) - L(5, 1, c)) + (L(5, 2, c) - L(5, 0, c));
#pragma unroll
    for (int h = 0; h < 3; ++h) {
      AXX[h] = AXX[h + 1]; AYY[h] = AYY[h + 1]; AXY[h] = AXY[h + 1];
#pragma unroll
      for (int c = 0; c < 4; ++c) ZZ[h][c] = ZZ[h + 1][c];
      XZ[h][0] = XZ[h + 1][0]; XZ[h][1] = XZ[h + 1][1];
      YZ[h][0] = YZ[h + 1][0]; YZ[h][1] = YZ[h + 1][1];
    }
    AXX[3] = axx; AYY[3] = ayy; AXY[3] = axy;
    ZZ[3][0] = azz[0][0]; ZZ[3][1] = azz[0][1]; ZZ[3][2] = azz[1][0]; ZZ[3][3] = azz[1][1];
    XZ[3][0] = xz[0]; XZ[3][1] = xz[1];
    YZ[3][0] = yz[0]; YZ[3][1] = yz[1];
    if (p >= k0 + 2 && mine) {
      // cell k = p - 2: the histories hold vertex planes k-1 .. k+2
      const int k = p - 2;
      const float sxx = AXX[1] + AXX[2], syy = AYY[1] + AYY[2], dxy = AXY[1] + AXY[2];
      float szz = 0.f, dxz = 0.f, dyz = 0.f;
#pragma unroll
      for (int c = 0; c < 4; ++c) szz += (ZZ[3][c] - ZZ[2][c]) - (ZZ[1][c] - ZZ[0][c]);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        dxz += (XZ[3][c] - XZ[1][c]) + (XZ[2][c] - XZ[0][c]);
        dyz += (YZ[3][c] - YZ[1][c]) + (YZ[2][c] - YZ[0][c]);
      }
      float* dst = dphi + (int64_t)k * nn + (int64_t)j * n + i;
      *dst += (sxx + syy + szz) * 0.125f + (dxy + dxz + dyz) * 0.03125f;
    }
  }
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
  const int ntx = (a.n + kTX - 1) / kTX, nty = (a.n + kTY - 1) / kTY;
  const int64_t tb = (int64_t)ntx * nty * ((a.n + kTZ - 1) / kTZ);
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)tb), dim3(kTX * kTY), 0, s,
                     (const float*)lam, dl_dphi, a.n, ntx, nty);
  return hipGetLastError();
}

}  // namespace rr
