// rr_adjoint_uniform.hip -- gradient of L = sum_r w_r kappa_r with respect to
// the potential of a uniform periodic grid.
//
// kappa is linear in Phi (straight rays, Born approximation, Sec. IV A), so
// dL/dPhi = A^T w for the forward chain A = (per-cell integrals) o (vertex
// mean, Sec. III H) o (finite differences, Eq. tidalexample):
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
  const float s = L * inv_chis;
#pragma unroll
  for (int v = 0; v < 8; ++v) om[v] = 0.0f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float c = cs[k];
    const float ux = fmaf(uA[0] - uB[0], c, uB[0]);
    const float uy = fmaf(uA[1] - uB[1], c, uB[1]);
    const float uz = fmaf(uA[2] - uB[2], c, uB[2]);
    const float chik = fmaf(L, c, chiB);
    const float W = (ws[k] * s) * chik * fmaf(-L, c, DB);
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
}

// x of another lane of the same row of 16, picked by a DPP lane pattern.
template <int kCtrl>
__device__ __forceinline__ float dpp_lane(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xf, 0xf, false));
}

// One step of a wavefront reduce-scatter over 2 kHalf values per lane: the
// lane sends the half of its values it does not keep to the lane that the DPP
// pattern kCtrl reads it from, and adds the same half of its own source's
// values to the half it keeps (the high half if `hi`).  Source and receiver
// differ in exactly the bit that picks the half.
template <int kCtrl, int kHalf>
__device__ __forceinline__ void fold(float* x, bool hi) {
#pragma unroll
  for (int i = 0; i < kHalf; ++i) {
    const float keep = hi ? x[i + kHalf] : x[i];
    const float send = hi ? x[i] : x[i + kHalf];
    x[i] = keep + dpp_lane<kCtrl>(send);
  }
}

// A wavefront's cache of retired vertex sums in LDS, direct-mapped on the low
// bits of the vertex coordinates (taken before the periodic wrap, so the
// corners of one cell always fall in distinct slots): the lanes of a tile
// drift apart by a step or two, so a vertex is often retired by several
// groups of lanes a few steps apart; their sums meet in the cache, and a
// vertex goes to global memory (six FP32 atomics) when its slot is taken by
// another vertex or the tile ends.
// Vertex ids are 32 bit when the grid has fewer than 2^32 - 1 vertices.
template <typename Id>
struct CacheSlot {
  Id tag;         // vertex id, or empty (all bits set)
  float v[6];
};
constexpr int kSlots = 256;   // x & 7, y & 7, z & 3

template <typename Id>
__device__ __forceinline__ void flush_slot(float* __restrict__ lam, const CacheSlot<Id>& e) {
  if (e.tag != (Id)~(Id)0) {
    float* dst = lam + (uint64_t)e.tag * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) atomicAdd(dst + c, e.v[c]);
  }
}

// Retire face F of cell (W0, W1, W2) for the lanes with `mine` set: corner j
// of the face gets sum over those lanes of acc_v * P_ab.  The 4 x 6 sums are
// reduced jointly over the wavefront: three halving steps (lane bits 0, 1
// and 2, lane moves within quads and rows) leave every lane with 3 of the 24
// values summed over 8 lanes, which the row (bit 3) and the other rows
// (register swaps of 16- and 32-lane groups) then complete; lanes 0..7 hold
// all 24 sums, corner 2 b0 + b1 and components 3 b2 .. 3 b2 + 2, and update
// the cache side by side.  Called with all 64 lanes active; F and W are
// wavefront-uniform, so the four corners' vertex ids and cache slots are
// formed once per wavefront (scalar registers) and each lane picks its own.
template <typename Id>
__device__ __forceinline__ void retire_face(float* __restrict__ lam, CacheSlot<Id>* cache,
                                            const float* acc, const float* P, bool mine, int F,
                                            int W0, int W1, int W2, int n, int lane) {
  float a[4];
  switch (F) {
    case 0: a[0] = acc[0]; a[1] = acc[2]; a[2] = acc[4]; a[3] = acc[6]; break;
    case 1: a[0] = acc[1]; a[1] = acc[3]; a[2] = acc[5]; a[3] = acc[7]; break;
    case 2: a[0] = acc[0]; a[1] = acc[1]; a[2] = acc[4]; a[3] = acc[5]; break;
    case 3: a[0] = acc[2]; a[1] = acc[3]; a[2] = acc[6]; a[3] = acc[7]; break;
    case 4: a[0] = acc[0]; a[1] = acc[1]; a[2] = acc[2]; a[3] = acc[3]; break;
    default: a[0] = acc[4]; a[1] = acc[5]; a[2] = acc[6]; a[3] = acc[7]; break;
  }
  // the face's corners j = i_a + 2 i_b (a < b the two axes other than the
  // face's axis k = F / 2, which sits at layer F % 2): their lattice
  // coordinates take one of two values per axis, formed once per wavefront.
  // Lanes 0..7 will hold the sums of corner 2 b0 + b1 (lane bits 1, 0),
  // components 3 b2 .. 3 b2 + 2; every lane reads its slot of the cache now
  // (lanes 8..63 a slot of the same face, unused), so that the LDS reads are
  // in flight during the reduction.
  const int k = F >> 1, sd = F & 1;
  const int X1 = W0 + 1 == n ? 0 : W0 + 1, Y1 = W1 + 1 == n ? 0 : W1 + 1;
  const int Z1 = W2 + 1 == n ? 0 : W2 + 1;
  const int ia = (lane >> 1) & 1, ib = lane & 1;
  const int bx = k == 0 ? sd : ia;
  const int by = k == 1 ? sd : (k == 0 ? ia : ib);
  const int bz = k == 2 ? sd : ib;
  const int cx = bx ? X1 : W0, cy = by ? Y1 : W1, cz = bz ? Z1 : W2;
  const Id my_vid = ((Id)cz * (Id)n + (Id)cy) * (Id)n + (Id)cx;
  const int my_slot = ((W0 + bx) & 7) | (((W1 + by) & 7) << 3) | (((W2 + bz) & 3) << 6);
  const int cb = (lane & 4) ? 3 : 0;
  CacheSlot<Id>& e = cache[my_slot];
  const Id tag = e.tag;
  float held[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) held[i] = e.v[cb + i];
  __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the reduction
  // the first halving step is taken on the products as they are formed: a
  // lane with bit 0 set keeps corners 2 and 3 and sends 0 and 1, a lane
  // with it clear the reverse (the sent products are added by the DPP move
  // itself: keep * P is rounded on its own first)
  const bool h0 = (lane & 1) != 0;
  float x[12];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float al = mine ? a[j] : 0.0f, ah = mine ? a[j + 2] : 0.0f;
    const float keep = h0 ? ah : al, send = h0 ? al : ah;
#pragma unroll
    for (int c = 0; c < 6; ++c)
      x[6 * j + c] = __fmul_rn(keep, P[c]) + dpp_lane<0xb1>(__fmul_rn(send, P[c]));
  }                                      // quad_perm [1,0,3,2]: lane ^ 1
  fold<0x4e, 6>(x, (lane & 2) != 0);     // quad_perm [2,3,0,1]: lane ^ 2
  fold<0x124, 3>(x, (lane & 4) != 0);    // row_ror:4: lane - 4 within the row
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    x[i] += dpp_lane<0x128>(x[i]);       // row_ror:8: lane ^ 8
    // the 16-lane rows and then the 32-lane halves swapped in registers: the
    // two results hold x of the lane and of lane ^ 16 (^ 32), in either order
    const auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(x[i]), __float_as_uint(x[i]),
                                                      false, false);
    x[i] = __uint_as_float(r16[0]) + __uint_as_float(r16[1]);
    const auto r32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[i]), __float_as_uint(x[i]),
                                                      false, false);
    x[i] = __uint_as_float(r32[0]) + __uint_as_float(r32[1]);
  }
  if (lane < 8) {
    if (tag == my_vid) {
#pragma unroll
      for (int i = 0; i < 3; ++i) e.v[cb + i] = held[i] + x[i];
    } else {
      if (tag != (Id)~(Id)0) {
#pragma unroll
        for (int i = 0; i < 3; ++i) atomicAdd(lam + (uint64_t)tag * 6 + cb + i, held[i]);
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) e.v[cb + i] = x[i];
      if (cb == 0) e.tag = my_vid;
    }
  }
}

// One 8 x 8 tile of rays, all 64 lanes kept active to the end (lanes without
// a ray, or whose ray has ended, take part in the wavefront reductions with
// nothing to add).
template <typename Id>
__device__ void scatter_tile(const TraceArgs& a, const DevBundle& B, int ix, int iy, int lane,
                             const float* __restrict__ wts, float* __restrict__ lam,
                             CacheSlot<Id>* cache) {
  for (int e = lane; e < kSlots; e += 64) cache[e].tag = (Id)~(Id)0;
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
  const double lo = B.chi_lo;
  double chiA = B.chi_hi;
  // per axis: bit k of dpos set when d_k > 0 (the march runs down the lattice)
  const int dpos = (d[0] > 0.0 ? 1 : 0) | (d[1] > 0.0 ? 2 : 0) | (d[2] > 0.0 ? 4 : 0);
  double r[3], te[3], cpos[3];
  int px[3];   // lattice coordinate of the exit plane
  int w[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r[k] = (d[k] != 0.0) ? 1.0 / d[k] : 0.0;
    const int m = start_slab(a.o[k], d[k], r[k], chiA, 1.0);
    px[k] = d[k] > 0.0 ? m : m + 1;
    te[k] = d[k] != 0.0 ? tplane((double)px[k], a.o[k], r[k]) : -__builtin_inf();
    cpos[k] = a.o[k] - (double)m;
    const int ww = m % n;
    w[k] = ww < 0 ? ww + n : ww;
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
    // the corners that retire are one face of the cell, F = 2 axis + side,
    // or all eight (both z faces, f0 = 4 and f1 = 5)
    int f0 = -1, f1 = -1;
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
          const float face = ((dpos >> k) & 1) ? 0.0f : 1.0f;
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
        // ray leaves behind (the crossed face is shared with the next cell;
        // the ray moves along -d, so it leaves the high face when d_k > 0)
        if (!last && nstep == 1) {
          kk = stepped[0] ? 0 : (stepped[1] ? 1 : 2);
          f0 = 2 * kk + ((dpos >> kk) & 1);
        } else {
          f0 = 4;
          f1 = 5;
        }
      }
    }
    if (stopped) {
      f0 = 4;
      f1 = 5;
    }
    // one round per distinct (cell, face) among the lanes, usually one
    for (;;) {
      const unsigned long long m = __ballot(f0 >= 0);
      if (m == 0ull) break;
      const int leader = __builtin_ctzll(m);
      const int F = __builtin_amdgcn_readlane(f0, leader);
      const int W0 = __builtin_amdgcn_readlane(w[0], leader);
      const int W1 = __builtin_amdgcn_readlane(w[1], leader);
      const int W2 = __builtin_amdgcn_readlane(w[2], leader);
      const bool mine = f0 == F && w[0] == W0 && w[1] == W1 && w[2] == W2;
      retire_face<Id>(lam, cache, acc, P, mine, F, W0, W1, W2, n, lane);
      if (mine) {
        f0 = f1;
        f1 = -1;
      }
    }
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
        const int keep = ((dpos >> k) & 1) ? 0 : bit;
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
        const bool down = (dpos >> k) & 1;
        px[k] += down ? -1 : 1;
        te[k] = tplane((double)px[k], a.o[k], r[k]);
        cpos[k] += down ? 1.0 : -1.0;
        uA[k] = 1.0f - uB[k];
        const int s = down ? -1 : 1;
        int ww = w[k] + s;
        ww = ww < 0 ? ww + n : (ww >= n ? ww - n : ww);
        w[k] = ww;
      }
    }
    chiA = chiB;
  }
  for (int e = lane; e < kSlots; e += 64) flush_slot(lam, cache[e]);
}

template <typename Id>
__global__ __launch_bounds__(256) void scatter_kernel(TraceArgs a, const float* __restrict__ wts,
                                                      float* __restrict__ lam) {
  __shared__ CacheSlot<Id> cache[4][kSlots];
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
  scatter_tile<Id>(a, B, tx * 8 + (lane & 7), ty * 8 + (lane >> 3), lane, wts, lam,
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
    if (nv < (int64_t)0xffffffffll)
      hipLaunchKernelGGL(scatter_kernel<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s, a,
                         dl_dkappa, lam);
    else
      hipLaunchKernelGGL(scatter_kernel<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, s, a,
                         dl_dkappa, lam);
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
