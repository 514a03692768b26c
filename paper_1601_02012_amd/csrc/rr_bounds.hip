// rr_bounds.hip -- the vertex box a set of rays reads: lattice bounds of the
// rays' end points over their chi windows (the march between them stays in
// the box they span).
#include <climits>

#include "rr_ray.hpp"

namespace rr {
namespace {

// Lattice bounds of the rays' end points (the walk between them stays in the
// box they span).  A bounded grid strides over the tiles (one wavefront per
// tile at a time); the bounds are reduced across the wavefront, then across
// the workgroup, before one atomic per bound and workgroup.
__global__ __launch_bounds__(256) void ray_bounds_kernel(TraceArgs a, int* out) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < a.n_tiles;
       tile += (int64_t)gridDim.x * 4) {
    const int b = find_bundle(a.bundles, a.n_bundles, tile);
    const DevBundle& B = a.bundles[b];
    const int64_t local = tile - B.tile_begin;
    const int tx = (int)(local % B.tiles_x), ty = (int)(local / B.tiles_x);
    const int ix = tx * 8 + (lane & 7), iy = ty * 8 + (lane >> 3);
    if (ix < B.nx && iy < B.ny) {
      const int64_t ray = (int64_t)iy * B.nx + ix;
      const double d[3] = {B.dir[3 * ray + 0], B.dir[3 * ray + 1], B.dir[3 * ray + 2]};
      const double nrm2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (fabs(nrm2 - 1.0) <= 1e-9) {   // other rays are not traced
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int p0 = (int)floor(fma(B.chi_hi, d[k], a.o[k]));
          const int p1 = (int)floor(fma(B.chi_lo, d[k], a.o[k]));
          lo[k] = min(lo[k], min(p0, p1));
          hi[k] = max(hi[k], max(p0, p1));
        }
      }
    }
  }
#pragma unroll
  for (int sh = 32; sh > 0; sh >>= 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lo[k] = min(lo[k], __shfl_xor(lo[k], sh, 64));
      hi[k] = max(hi[k], __shfl_xor(hi[k], sh, 64));
    }
  }
  __shared__ int red[4][6];
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      red[wave][k] = lo[k];
      red[wave][3 + k] = hi[k];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      int l = red[0][k], h = red[0][3 + k];
      for (int w = 1; w < 4; ++w) {
        l = min(l, red[w][k]);
        h = max(h, red[w][3 + k]);
      }
      if (l != INT_MAX) atomicMin(out + k, l);
      if (h != INT_MIN) atomicMax(out + 3 + k, h);
    }
  }
}

}  // namespace

hipError_t launch_ray_bounds(const TraceArgs& a, int* out, hipStream_t s) {
  int64_t blocks = (a.n_tiles + 3) / 4;
  if (blocks == 0) return hipSuccess;
  blocks = blocks < 2048 ? blocks : 2048;
  hipLaunchKernelGGL(ray_bounds_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, out);
  return hipGetLastError();
}

}  // namespace rr
