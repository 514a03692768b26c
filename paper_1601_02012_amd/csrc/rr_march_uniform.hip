// rr_march_uniform.hip -- cell-by-cell ray march through a uniform grid
// (Sec. III E, Eqs. rayposition - disttocross) with the per-cell lensing
// integral of the trilinear vertex reconstruction (Eqs. trilinear_int,
// Iclensing) and its accumulation along the ray (Eq. sumIc).
//
// Work decomposition: a wavefront owns an 8 x 8 tile of a bundle's ray map,
// so its 64 lanes start from neighbouring directions, visit neighbouring
// cells (coalesced, cache-friendly gathers) and take similar numbers of steps.
// Tiles are either mapped one per wavefront from the grid (XCD-striped so a
// chiplet's L2 sees a contiguous part of the sky) or pulled from a device
// queue by persistent workgroups.
#include "rr_ray.hpp"

namespace rr {
namespace {

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

template <typename R>
__device__ __forceinline__ void load_vertex(const R* __restrict__ tv, uint64_t v, R* t);

template <>
__device__ __forceinline__ void load_vertex<float>(const float* __restrict__ tv, uint64_t v,
                                                   float* t) {
  const float2* p = reinterpret_cast<const float2*>(tv + v * 6);
  const float2 a = p[0], b = p[1], c = p[2];
  t[0] = a.x; t[1] = a.y; t[2] = b.x; t[3] = b.y; t[4] = c.x; t[5] = c.y;
}
template <>
__device__ __forceinline__ void load_vertex<double>(const double* __restrict__ tv, uint64_t v,
                                                    double* t) {
  const double2* p = reinterpret_cast<const double2*>(tv + v * 6);
  const double2 a = p[0], b = p[1], c = p[2];
  t[0] = a.x; t[1] = a.y; t[2] = b.x; t[3] = b.y; t[4] = c.x; t[5] = c.y;
}

// One ray.  Per axis the lane keeps, in FP64, the coordinate of the exit
// plane, its crossing parameter and the local-coordinate offset o~ - m; the
// cell's wrapped indices are kept as integer offsets into the vertex array, so
// a crossing costs no integer division and no int->float conversion.
template <typename R, bool kDebug, typename Idx>
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
  double Pd[6];
  projection(a.quantity, d[0], d[1], d[2], Pd);
  R P[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) P[c] = (R)Pd[c];

  const int n = a.n;
  const Idx nI = (Idx)n, nnI = (Idx)n * (Idx)n;
  const double lo = B.chi_lo;
  double chiA = B.chi_hi;
  double r[3], pe[3], te[3], cpos[3], sgn[3];
  int m[3], w[3];
  Idx off0[3], off1[3];           // wrapped offsets of the cell's lower / upper vertex layer
  const Idx stride[3] = {(Idx)1, nI, nnI};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r[k] = (d[k] != 0.0) ? 1.0 / d[k] : 0.0;
    m[k] = start_slab(a.o[k], d[k], r[k], chiA, 1.0);
    sgn[k] = d[k] > 0.0 ? -1.0 : 1.0;            // step of m along the march
    pe[k] = (double)(d[k] > 0.0 ? m[k] : m[k] + 1);
    te[k] = d[k] != 0.0 ? tplane(pe[k], a.o[k], r[k]) : -__builtin_inf();
    cpos[k] = a.o[k] - (double)m[k];
    int ww = m[k] % n;
    w[k] = ww < 0 ? ww + n : ww;
    off0[k] = (Idx)w[k] * stride[k];
    off1[k] = (Idx)(w[k] + 1 == n ? 0 : w[k] + 1) * stride[k];
  }
  R uA[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) uA[k] = (R)fma(chiA, d[k], cpos[k]);

  const R inv_chis = (R)(1.0 / B.chi_s);
  const R scale = (R)a.kappa_scale;
  R sum;
  float comp = 0.0f;
  if constexpr (sizeof(R) == 4) {
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
    if (a.open && (m[0] < 2 || m[1] < 2 || m[2] < 2 || m[0] > n - 3 || m[1] > n - 3 ||
                   m[2] > n - 3)) {
      st = RR_RAY_OUT_OF_DOMAIN;
      break;
    }
    if (count >= maxc) {
      st = RR_RAY_MAX_STEPS;
      break;
    }
    // exit point: chi_B = max(chi_lo, t_exit,x, t_exit,y, t_exit,z), ties keep the earlier
    double chiB = lo;
    chiB = te[0] > chiB ? te[0] : chiB;
    chiB = te[1] > chiB ? te[1] : chiB;
    chiB = te[2] > chiB ? te[2] : chiB;
    bool stepped[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) stepped[k] = te[k] == chiB;

    // the eight corners (v = ix + 2 iy + 4 iz), projected on the ray's P
    R q[8];
    {
      const Idx zy00 = off0[2] + off0[1], zy01 = off0[2] + off1[1];
      const Idx zy10 = off1[2] + off0[1], zy11 = off1[2] + off1[1];
      const Idx vid[8] = {zy00 + off0[0], zy00 + off1[0], zy01 + off0[0], zy01 + off1[0],
                          zy10 + off0[0], zy10 + off1[0], zy11 + off0[0], zy11 + off1[0]};
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        R t[6];
        load_vertex<R>(tv, (uint64_t)vid[v], t);
        R acc = P[0] * t[0];
#pragma unroll
        for (int c = 1; c < 6; ++c) acc = fma(P[c], t[c], acc);
        q[v] = acc;
      }
    }
    // local coordinates of the exit point; exact on the crossed faces
    R uB[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const R face = d[k] > 0.0 ? (R)0 : (R)1;
      uB[k] = stepped[k] ? face : (R)fma(chiB, d[k], cpos[k]);
    }
    const R L = (R)(chiA - chiB);
    const R ic = cell_integral<R>(q, uA, uB, L, (R)chiB, (R)(B.chi_s - chiB), inv_chis) * scale;
    if constexpr (sizeof(R) == 4) {
      kahan_add(sum, comp, ic);
    } else {
      sum += ic;
    }
    if constexpr (kDebug) {
      const int64_t cell = (int64_t)(off0[2] + off0[1] + off0[0]);
      if (a.hash) hv = fnv_piece(hv, cell, chiA, chiB);
      if (a.log && count < a.log_stride) {
        LogRecord* L0 = reinterpret_cast<LogRecord*>(a.log) + out * a.log_stride + count;
        L0->cell = cell;
        L0->chi_a = chiA;
        L0->chi_b = chiB;
      }
    }
    ++count;
    if (chiB == lo) break;
    // step every axis whose exit plane is at chi_B; the entry point of the
    // next cell is the exit point of this one
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uA[k] = uB[k];
      if (stepped[k]) {
        pe[k] += sgn[k];
        te[k] = tplane(pe[k], a.o[k], r[k]);
        cpos[k] -= sgn[k];
        uA[k] = (R)1 - uB[k];
        const int s = d[k] > 0.0 ? -1 : 1;
        m[k] += s;
        int ww = w[k] + s;
        ww = ww < 0 ? ww + n : (ww >= n ? ww - n : ww);
        w[k] = ww;
        off0[k] = (Idx)ww * stride[k];
        off1[k] = (Idx)(ww + 1 == n ? 0 : ww + 1) * stride[k];
      }
    }
    chiA = chiB;
  }
  if (!(sum == sum) || sum - sum != (R)0) st = RR_RAY_NONFINITE;
  if constexpr (sizeof(R) == 4) {
    reinterpret_cast<float*>(a.kappa)[out] = sum;
    if (a.kappa_comp) a.kappa_comp[out] = comp;
  } else {
    reinterpret_cast<double*>(a.kappa)[out] = sum;
  }
  if (a.status) a.status[out] = st;
  if constexpr (kDebug) {
    if (a.hash) a.hash[out] = hv;
    if (a.count) a.count[out] = count;
  }
}

template <typename R, bool kDebug, typename Idx>
__device__ __forceinline__ void run_tile(const R* __restrict__ tv, const TraceArgs& a,
                                         int64_t tile, int lane) {
  const int b = find_bundle(a.bundles, a.n_bundles, tile);
  const DevBundle& B = a.bundles[b];
  const int64_t local = tile - B.tile_begin;
  const int tx = (int)(local % B.tiles_x), ty = (int)(local / B.tiles_x);
  const int ix = tx * 8 + (lane & 7), iy = ty * 8 + (lane >> 3);
  if (ix < B.nx && iy < B.ny) trace_one<R, kDebug, Idx>(tv, a, B, (int64_t)iy * B.nx + ix);
}

// One wavefront per tile.  Workgroups are dealt round-robin to the 8 XCDs;
// remap so that XCD x gets the x-th contiguous slice of tiles.
template <typename R, bool kDebug, typename Idx>
__global__ __launch_bounds__(256) void march_uniform_kernel(const R* __restrict__ tv,
                                                            TraceArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t nblk = gridDim.x;
  const int64_t blk = blockIdx.x;
  const int64_t per = (nblk + 7) / 8;
  const int64_t xcd = blk % 8, slot = blk / 8;
  const int64_t vblk = xcd * per + slot;
  const int64_t tile = vblk * (blockDim.x >> 6) + wave;
  if (tile >= a.n_tiles) return;
  run_tile<R, kDebug, Idx>(tv, a, tile, lane);
}

// Persistent workgroups: every wavefront pulls tiles from a device counter
// until the queue is drained (every wave reaches the exit test).
template <typename R, bool kDebug, typename Idx>
__global__ __launch_bounds__(256) void march_uniform_persistent(const R* __restrict__ tv,
                                                                TraceArgs a) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    unsigned long long t = 0;
    if (lane == 0) t = atomicAdd(a.queue, 1ull);
    t = __shfl(t, 0, 64);
    if ((int64_t)t >= a.n_tiles) break;
    run_tile<R, kDebug, Idx>(tv, a, (int64_t)t, lane);
  }
}

__global__ void queue_reset_kernel(unsigned long long* q) { *q = 0ull; }

template <typename R, bool kDebug, typename Idx>
hipError_t launch3(const void* tv, const TraceArgs& a, int persistent, int block, int grid_waves,
                   hipStream_t s) {
  const int wpb = block / 64;
  if (persistent) {
    const int blocks = (grid_waves + wpb - 1) / wpb;
    hipLaunchKernelGGL((march_uniform_persistent<R, kDebug, Idx>), dim3(blocks), dim3(block), 0, s,
                       (const R*)tv, a);
  } else {
    int64_t blocks = (a.n_tiles + wpb - 1) / wpb;
    if (blocks == 0) return hipSuccess;
    blocks = (blocks + 7) / 8 * 8;   // the XCD remap is a bijection on multiples of 8
    hipLaunchKernelGGL((march_uniform_kernel<R, kDebug, Idx>), dim3((unsigned)blocks), dim3(block),
                       0, s, (const R*)tv, a);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch(const void* tv, const TraceArgs& a, int persistent, int block, int grid_waves,
                  hipStream_t s) {
  const bool dbg = a.hash || a.log || a.count;
  const bool small = (int64_t)a.n * a.n * a.n < (1ll << 32);
  if (dbg)
    return small ? launch3<R, true, uint32_t>(tv, a, persistent, block, grid_waves, s)
                 : launch3<R, true, uint64_t>(tv, a, persistent, block, grid_waves, s);
  return small ? launch3<R, false, uint32_t>(tv, a, persistent, block, grid_waves, s)
               : launch3<R, false, uint64_t>(tv, a, persistent, block, grid_waves, s);
}

}  // namespace

hipError_t launch_march_uniform(int precision, const void* tv, const TraceArgs& a, int persistent,
                                int block, int grid_waves, hipStream_t s) {
  if (precision == RR_PREC_FP32_KAHAN) return launch<float>(tv, a, persistent, block, grid_waves, s);
  return launch<double>(tv, a, persistent, block, grid_waves, s);
}

hipError_t launch_queue_reset(unsigned long long* q, hipStream_t s) {
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(1), 0, s, q);
  return hipGetLastError();
}

}  // namespace rr
