// rr_tensor_uniform.hip -- tidal tensor at cell centres (Eq. tidalexample) fused
// with its interpolation to cell vertices (Sec. III F, regular vertices).
//
// One workgroup builds a TX x TY x TZ block of vertices.  It stages the
// potential of the block plus a two-cell halo in LDS, evaluates the centre
// tensor of the (TX+1)(TY+1)(TZ+1) cells that touch those vertices into LDS,
// and writes every vertex as the mean of its eight cells.  Vertex (i,j,k) is
// the lower corner of cell (i,j,k).  Second differences are formed as
// differences of neighbour differences, which are exact in floating point
// for neighbours within a factor two of each other (Sterbenz).
#include "rr_internal.hpp"

namespace rr {
namespace {

template <typename Acc>
struct TileShape;
template <>
struct TileShape<float> {  // 64x4x4 vertices: LDS 3283*4 + 1625*24 = 52 KB
  static constexpr int TX = 64, TY = 4, TZ = 4;
};
template <>
struct TileShape<double> {  // 32x4x4 vertices: LDS 2695... see below, < 64 KB
  static constexpr int TX = 32, TY = 4, TZ = 4;
};

__device__ inline int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

template <typename In, typename Acc, typename Out>
__global__ __launch_bounds__(256) void vertex_tensor_uniform_kernel(const In* __restrict__ phi,
                                                                    Out* __restrict__ tv, int n,
                                                                    int open, int ntx, int nty) {
  constexpr int TX = TileShape<Acc>::TX, TY = TileShape<Acc>::TY, TZ = TileShape<Acc>::TZ;
  constexpr int PX = TX + 3, PY = TY + 3, PZ = TZ + 3;   // potential tile (halo 2 below, 1 above)
  constexpr int CX = TX + 1, CY = TY + 1, CZ = TZ + 1;   // centre-tensor tile
  constexpr int RW = VertexRecord<Out>::kWords;
  __shared__ Acc sphi[PZ * PY * PX];
  __shared__ Acc sten[6][CZ * CY * CX];

  // workgroup -> tile (x fastest)
  const int b = blockIdx.x;
  const int bx = b % ntx;
  const int by = (b / ntx) % nty;
  const int bz = b / (ntx * nty);
  const int i0 = bx * TX, j0 = by * TY, k0 = bz * TZ;

  // stage 0: potential with halo, x fastest for coalescing
  for (int e = threadIdx.x; e < PZ * PY * PX; e += blockDim.x) {
    const int x = e % PX, y = (e / PX) % PY, z = e / (PX * PY);
    int gi = i0 - 2 + x, gj = j0 - 2 + y, gk = k0 - 2 + z;
    Acc v;
    if (open) {
      const bool in = gi >= 0 && gj >= 0 && gk >= 0 && gi < n && gj < n && gk < n;
      v = in ? (Acc)phi[((int64_t)gk * n + gj) * n + gi] : (Acc)0;
    } else {
      gi = wrapi(gi, n);
      gj = wrapi(gj, n);
      gk = wrapi(gk, n);
      v = (Acc)phi[((int64_t)gk * n + gj) * n + gi];
    }
    sphi[e] = v;
  }
  __syncthreads();

  // stage 1: centre tensor of cells i0-1 .. i0+TX-1 (etc.)
  for (int e = threadIdx.x; e < CZ * CY * CX; e += blockDim.x) {
    const int x = e % CX, y = (e / CX) % CY, z = e / (CX * CY);
    // cell (i0-1+x) sits at potential-tile index x+1
    const int px = x + 1, py = y + 1, pz = z + 1;
#define P(dx, dy, dz) sphi[((pz + (dz)) * PY + (py + (dy))) * PX + (px + (dx))]
    const Acc c = P(0, 0, 0);
    Acc txx = (P(1, 0, 0) - c) - (c - P(-1, 0, 0));
    Acc tyy = (P(0, 1, 0) - c) - (c - P(0, -1, 0));
    Acc tzz = (P(0, 0, 1) - c) - (c - P(0, 0, -1));
    Acc txy = ((P(1, 1, 0) - P(1, -1, 0)) - (P(-1, 1, 0) - P(-1, -1, 0))) * (Acc)0.25;
    Acc txz = ((P(1, 0, 1) - P(1, 0, -1)) - (P(-1, 0, 1) - P(-1, 0, -1))) * (Acc)0.25;
    Acc tyz = ((P(0, 1, 1) - P(0, 1, -1)) - (P(0, -1, 1) - P(0, -1, -1))) * (Acc)0.25;
#undef P
    if (open) {
      const int gi = i0 - 1 + x, gj = j0 - 1 + y, gk = k0 - 1 + z;
      const bool in = gi >= 1 && gj >= 1 && gk >= 1 && gi <= n - 2 && gj <= n - 2 && gk <= n - 2;
      if (!in) {
        const Acc nan = (Acc)__builtin_nan("");
        txx = tyy = tzz = txy = txz = tyz = nan;
      }
    }
    sten[0][e] = txx;
    sten[1][e] = tyy;
    sten[2][e] = tzz;
    sten[3][e] = txy;
    sten[4][e] = txz;
    sten[5][e] = tyz;
  }
  __syncthreads();

  // stage 2: vertices, mean of the eight cells around each
  for (int e = threadIdx.x; e < TZ * TY * TX; e += blockDim.x) {
    const int x = e % TX, y = (e / TX) % TY, z = e / (TX * TY);
    const int gi = i0 + x, gj = j0 + y, gk = k0 + z;
    if (gi >= n || gj >= n || gk >= n) continue;
    // vertex (gi,gj,gk) touches cells gi-1, gi -> centre-tile x, x+1
    Out rec[RW];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const Acc* s = sten[c];
#define C(dx, dy, dz) s[((z + (dz)) * CY + (y + (dy))) * CX + (x + (dx))]
      const Acc s0 = (C(0, 0, 0) + C(1, 0, 0)) + (C(0, 1, 0) + C(1, 1, 0));
      const Acc s1 = (C(0, 0, 1) + C(1, 0, 1)) + (C(0, 1, 1) + C(1, 1, 1));
#undef C
      rec[c] = (Out)((s0 + s1) * (Acc)0.125);
    }
#pragma unroll
    for (int c = 6; c < RW; ++c) rec[c] = (Out)0;
    Out* dst = tv + (((int64_t)gk * n + gj) * n + gi) * RW;
    if constexpr (RW == 8) {
      float4* d4 = reinterpret_cast<float4*>(dst);
      d4[0] = make_float4(rec[0], rec[1], rec[2], rec[3]);
      d4[1] = make_float4(rec[4], rec[5], rec[6], rec[7]);
    } else {
      double2* d2 = reinterpret_cast<double2*>(dst);
      d2[0] = make_double2(rec[0], rec[1]);
      d2[1] = make_double2(rec[2], rec[3]);
      d2[2] = make_double2(rec[4], rec[5]);
    }
  }
}

template <typename In, typename Acc, typename Out>
hipError_t launch_vt(int n, int open, const void* phi, void* tv, hipStream_t s) {
  constexpr int TX = TileShape<Acc>::TX, TY = TileShape<Acc>::TY, TZ = TileShape<Acc>::TZ;
  const int ntx = (n + TX - 1) / TX, nty = (n + TY - 1) / TY, ntz = (n + TZ - 1) / TZ;
  const int64_t blocks = (int64_t)ntx * nty * ntz;
  hipLaunchKernelGGL((vertex_tensor_uniform_kernel<In, Acc, Out>), dim3((unsigned)blocks),
                     dim3(256), 0, s, (const In*)phi, (Out*)tv, n, open, ntx, nty);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_vertex_tensor_uniform(int precision, int dtype, int n, int open,
                                        const void* phi, void* tv, hipStream_t s) {
  if (precision == RR_PREC_FP32_KAHAN) {
    if (dtype == RR_F32) return launch_vt<float, float, float>(n, open, phi, tv, s);
    return launch_vt<double, float, float>(n, open, phi, tv, s);
  }
  if (dtype == RR_F32) return launch_vt<float, double, double>(n, open, phi, tv, s);
  return launch_vt<double, double, double>(n, open, phi, tv, s);
}

}  // namespace rr
