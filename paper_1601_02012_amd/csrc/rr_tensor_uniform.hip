// rr_tensor_uniform.hip -- tidal tensor at cell centres (Eq. tidalexample) fused
// with its interpolation to cell vertices (Sec. III F, regular vertices).
//
// Vertex (i,j,k) is the lower corner of cell (i,j,k) and takes the mean of the
// centre tensors of cells {i-1,i} x {j-1,j} x {k-1,k}.  Summing the centre
// stencils over those eight cells factorises per axis into
//   second difference summed over two cells: S f(i) = (f(i+1) - f(i)) - (f(i-1) - f(i-2))
//   first difference summed over two cells:  D f(i) = (f(i+1) - f(i-1)) + (f(i) - f(i-2))
//   plain sum over the two cells:            B f(i) = f(i-1) + f(i)
// so that   T_xx = (1/8) S_x B_y B_z Phi,   T_xy = (1/32) D_x D_y B_z Phi, ...
// Differences are always taken first on the raw potential (exact for
// neighbours within a factor two, Sterbenz), sums afterwards.
//
// The vertices built are a periodic box [o, o + size) of the lattice (the
// whole grid, or the part a set of rays can reach).
//
// Layout of the work: a workgroup owns a 64 x 4 column of vertices in x-y and
// marches along z.  Each step stages one potential plane (plus a two-cell
// halo) in LDS; every thread reads its 4 x 4 patch of that plane once and
// keeps the per-plane partial stencils of the last four planes in registers,
// so each potential value is read from HBM about once and each vertex costs
// 16 LDS reads and ~80 arithmetic operations.
#include "rr_internal.hpp"

namespace rr {
namespace {

constexpr int TX = 64, TY = 4;          // vertices per workgroup in x, y
constexpr int PX = TX + 3, PY = TY + 3; // staged plane: halo 2 below, 1 above
constexpr int KZ = 32;                  // vertices per workgroup along z

__device__ inline int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

template <typename Out>
__device__ inline void store_vertex(Out* dst, const Out* rec);
template <>
__device__ inline void store_vertex<float>(float* dst, const float* r) {
  float2* d2 = reinterpret_cast<float2*>(dst);
  d2[0] = make_float2(r[0], r[1]);
  d2[1] = make_float2(r[2], r[3]);
  d2[2] = make_float2(r[4], r[5]);
}
template <>
__device__ inline void store_vertex<double>(double* dst, const double* r) {
  double2* d2 = reinterpret_cast<double2*>(dst);
  d2[0] = make_double2(r[0], r[1]);
  d2[1] = make_double2(r[2], r[3]);
  d2[2] = make_double2(r[4], r[5]);
}

struct VertexBox {
  int ox, oy, oz;   // origin, wrapped into [0, n)
  int sx, sy, sz;   // extent, at most n
  int ntx, nty;     // workgroup tiles in x and y
};

template <typename In, typename Acc>
__global__ __launch_bounds__(256) void vertex_tensor_uniform_kernel(const In* __restrict__ phi,
                                                                    Acc* __restrict__ tv, int n,
                                                                    int open, VertexBox V) {
  constexpr int RW = VertexRecord<Acc>::kWords;
  __shared__ Acc plane[2][PY * PX];

  const int b = blockIdx.x;
  const int bx = b % V.ntx;
  const int by = (b / V.ntx) % V.nty;
  const int bz = b / (V.ntx * V.nty);
  // box-local origin of this workgroup's column; lattice indices wrap
  const int li0 = bx * TX, lj0 = by * TY, lk0 = bz * KZ;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const bool mine = li0 + tx < V.sx && lj0 + ty < V.sy;
  int i = V.ox + li0 + tx, j = V.oy + lj0 + ty;
  i = i >= n ? i - n : i;
  j = j >= n ? j - n : j;
  const int64_t nn = (int64_t)n * n;

  // per-plane partial stencils, history over planes (index 0 = oldest)
  Acc XX[2], YY[2], XY[2];     // planes k-1, k
  Acc Z[4][4];                 // raw Phi of the 2x2 column box, planes k-2..k+1
  Acc DX[4][2], DY[4][2];      // D_x on rows j-1, j and D_y on columns i-1, i, planes k-2..k+1

  // staging: each thread copies at most two elements of every plane; their
  // (wrapped) x-y offsets are fixed for the whole march
  constexpr int kStage = (PX * PY + 255) / 256;
  int soff[kStage];
  bool sin_[kStage], sact[kStage];
#pragma unroll
  for (int u = 0; u < kStage; ++u) {
    const int e = threadIdx.x + 256 * u;
    sact[u] = e < PX * PY;
    const int lx = e % PX, ly = e / PX;
    // unwrapped lattice coordinates (the open boundary pads outside [0, n))
    const int gx = V.ox + li0 - 2 + lx, gy = V.oy + lj0 - 2 + ly;
    sin_[u] = gx >= 0 && gy >= 0 && gx < n && gy < n;
    int wx = gx % n, wy = gy % n;
    wx = wx < 0 ? wx + n : wx;
    wy = wy < 0 ? wy + n : wy;
    soff[u] = wy * n + wx;
  }

  const int k0 = V.oz + lk0;                       // unwrapped
  const int k_end = k0 + min(KZ, V.sz - lk0);
  int slot = 0;
  int gz = (k0 - 2) % n;
  if (gz < 0) gz += n;
  for (int p = k0 - 2; p <= k_end; ++p, slot ^= 1) {
    // stage plane p (x fastest, wrapped or zero-padded)
    Acc* pl = plane[slot];
    const bool zin = p >= 0 && p < n;
    const In* src = phi + (int64_t)gz * nn;
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      if (!sact[u]) continue;
      Acc v;
      if (open)
        v = (sin_[u] && zin) ? (Acc)src[soff[u]] : (Acc)0;
      else
        v = (Acc)src[soff[u]];
      pl[threadIdx.x + 256 * u] = v;
    }
    if (++gz == n) gz = 0;
    __syncthreads();
    // 4x4 patch: rows y = j-2..j+1, columns x = i-2..i+1
    Acc q[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) q[r][c] = pl[(ty + r) * PX + (tx + c)];

    Acc dx[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) dx[r] = (q[r][3] - q[r][1]) + (q[r][2] - q[r][0]);
    const Acc sxx = ((q[1][3] - q[1][2]) - (q[1][1] - q[1][0])) +
                    ((q[2][3] - q[2][2]) - (q[2][1] - q[2][0]));
    const Acc syy = ((q[3][1] - q[2][1]) - (q[1][1] - q[0][1])) +
                    ((q[3][2] - q[2][2]) - (q[1][2] - q[0][2]));
    const Acc dxy = (dx[3] - dx[1]) + (dx[2] - dx[0]);
    const Acc dy1 = (q[3][1] - q[1][1]) + (q[2][1] - q[0][1]);
    const Acc dy2 = (q[3][2] - q[1][2]) + (q[2][2] - q[0][2]);

    // shift the z histories so that Z/DX/DY[0..3] hold planes p-3..p
#pragma unroll
    for (int h = 0; h < 3; ++h) {
#pragma unroll
      for (int c = 0; c < 4; ++c) Z[h][c] = Z[h + 1][c];
      DX[h][0] = DX[h + 1][0]; DX[h][1] = DX[h + 1][1];
      DY[h][0] = DY[h + 1][0]; DY[h][1] = DY[h + 1][1];
    }
    Z[3][0] = q[1][1]; Z[3][1] = q[1][2]; Z[3][2] = q[2][1]; Z[3][3] = q[2][2];
    DX[3][0] = dx[1]; DX[3][1] = dx[2];
    DY[3][0] = dy1; DY[3][1] = dy2;

    if (p >= k0 + 1 && mine) {
      // vertex k = p - 1: Z/DX/DY[0..3] are planes k-2..k+1; XX/YY/XY[0..1] are k-1, k
      const int k = p - 1 >= n ? p - 1 - n : p - 1;
      Acc rec[6];
      rec[0] = (XX[0] + XX[1]) * (Acc)0.125;
      rec[1] = (YY[0] + YY[1]) * (Acc)0.125;
      Acc zz = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) zz += (Z[3][c] - Z[2][c]) - (Z[1][c] - Z[0][c]);
      rec[2] = zz * (Acc)0.125;
      rec[3] = (XY[0] + XY[1]) * (Acc)0.03125;
      Acc xz = 0, yz = 0;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        xz += (DX[3][c] - DX[1][c]) + (DX[2][c] - DX[0][c]);
        yz += (DY[3][c] - DY[1][c]) + (DY[2][c] - DY[0][c]);
      }
      rec[4] = xz * (Acc)0.03125;
      rec[5] = yz * (Acc)0.03125;
      if (open && (i < 2 || j < 2 || k < 2 || i > n - 2 || j > n - 2 || k > n - 2)) {
        const Acc nan = (Acc)__builtin_nan("");
#pragma unroll
        for (int c = 0; c < 6; ++c) rec[c] = nan;
      }
      store_vertex<Acc>(tv + ((int64_t)k * nn + (int64_t)j * n + i) * RW, rec);
    }
    // XX/YY/XY hold planes (p-2, p-1) during step p; push plane p
    XX[0] = XX[1]; YY[0] = YY[1]; XY[0] = XY[1];
    XX[1] = sxx; YY[1] = syy; XY[1] = dxy;
  }
}

template <typename In, typename Acc>
hipError_t launch_vt(int n, int open, const int* lo, const int* size, const void* phi, void* tv,
                     hipStream_t s) {
  VertexBox V;
  int o[3];
  for (int a = 0; a < 3; ++a) {
    o[a] = lo[a] % n;
    if (o[a] < 0) o[a] += n;
  }
  V.ox = o[0]; V.oy = o[1]; V.oz = o[2];
  V.sx = size[0]; V.sy = size[1]; V.sz = size[2];
  V.ntx = (V.sx + TX - 1) / TX;
  V.nty = (V.sy + TY - 1) / TY;
  const int ntz = (V.sz + KZ - 1) / KZ;
  const int64_t blocks = (int64_t)V.ntx * V.nty * ntz;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((vertex_tensor_uniform_kernel<In, Acc>), dim3((unsigned)blocks), dim3(256),
                     0, s, (const In*)phi, (Acc*)tv, n, open, V);
  return hipGetLastError();
}

}  // namespace

// Vertices of the periodic box [lo, lo + size) (size[a] <= n; the host
// layer validates).
hipError_t launch_vertex_tensor_uniform(int precision, int dtype, int n, int open, const int* lo,
                                        const int* size, const void* phi, void* tv,
                                        hipStream_t s) {
  if (precision == RR_PREC_FP32_KAHAN) {
    if (dtype == RR_F32) return launch_vt<float, float>(n, open, lo, size, phi, tv, s);
    return launch_vt<double, float>(n, open, lo, size, phi, tv, s);
  }
  if (dtype == RR_F32) return launch_vt<float, double>(n, open, lo, size, phi, tv, s);
  return launch_vt<double, double>(n, open, lo, size, phi, tv, s);
}

}  // namespace rr
