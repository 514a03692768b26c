// rr_tensor_uniform.hip -- tidal tensor at cell centres (Eq. tidalexample) fused
// with its interpolation to cell vertices (Sec. III H, regular vertices).
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
// Layout of the work: a workgroup owns a 64 x TY column of vertices in x-y
// and marches KZ vertices along z.  Each step stages one potential plane
// (plus a two-cell halo) in LDS; every thread reads its 4 x 4 patch of that
// plane once and keeps the per-plane partial stencils of the last four planes
// in registers, so each vertex costs 16 LDS reads and ~80 arithmetic
// operations.  Whole-grid builds take 64 x 16 x 16 columns (1024 threads;
// staging with the halo reads 1.5 potential values per vertex) and write the
// records with non-temporal stores (the 3 GiB tensor of a 512^3 grid does not
// fit any cache); small boxes take 64 x 4 x 32 columns and ordinary stores,
// since the march reads them right away.
#include "rr_internal.hpp"

namespace rr {
namespace {

constexpr int TX = 64;                  // vertices per workgroup in x

__device__ inline int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <bool kNT>
__device__ inline void store_vertex(float* dst, const float* r) {
  f32x2* d = reinterpret_cast<f32x2*>(dst);
  const f32x2 a = {r[0], r[1]}, b = {r[2], r[3]}, c = {r[4], r[5]};
  if constexpr (kNT) {
    __builtin_nontemporal_store(a, d);
    __builtin_nontemporal_store(b, d + 1);
    __builtin_nontemporal_store(c, d + 2);
  } else {
    d[0] = a; d[1] = b; d[2] = c;
  }
}
template <bool kNT>
__device__ inline void store_vertex(double* dst, const double* r) {
  f64x2* d = reinterpret_cast<f64x2*>(dst);
  const f64x2 a = {r[0], r[1]}, b = {r[2], r[3]}, c = {r[4], r[5]};
  if constexpr (kNT) {
    __builtin_nontemporal_store(a, d);
    __builtin_nontemporal_store(b, d + 1);
    __builtin_nontemporal_store(c, d + 2);
  } else {
    d[0] = a; d[1] = b; d[2] = c;
  }
}

struct VertexBox {
  int ox, oy, oz;   // origin, wrapped into [0, n)
  int sx, sy, sz;   // extent, at most n
  int ntx, nty;     // workgroup tiles in x and y
};

template <typename In, typename Acc, int TY, int KZ, bool kNT>
__global__ __launch_bounds__(64 * TY) void vertex_tensor_uniform_kernel(const In* __restrict__ phi,
                                                                        Acc* __restrict__ tv,
                                                                        int n, int open,
                                                                        VertexBox V) {
  constexpr int RW = VertexRecord<Acc>::kWords;
  constexpr int NT = TX * TY;                 // threads
  constexpr int PX = TX + 3, PY = TY + 3;     // staged plane: halo 2 below, 1 above
  __shared__ Acc plane[2][PY * PX];
  // FP64 records of whole-grid builds leave through LDS: each wavefront (one
  // row of 64 vertices) writes its 3 KiB row with contiguous 16-byte stores
  // instead of three 16-byte stores per lane at a 48-byte stride (2.2 ->
  // 1.8 ms for 512^3).  FP32 rows keep per-lane stores: the staging buffer
  // would cost the second workgroup per CU (0.78 -> 0.99 ms).
  constexpr bool kRowStore = kNT && sizeof(Acc) == 8;
  __shared__ __align__(16) Acc rowbuf[kRowStore ? TY : 1][kRowStore ? TX * RW : 1];

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
  // the wavefront's row is whole, does not wrap and starts 16-byte aligned
  int i_row = V.ox + li0;
  i_row = i_row >= n ? i_row - n : i_row;
  const bool row_ok = kRowStore && li0 + TX <= V.sx && lj0 + ty < V.sy && i_row + TX <= n;

  // per-plane partial stencils, history over planes (index 0 = oldest)
  Acc XX[2], YY[2], XY[2];     // planes k-1, k
  Acc Z[4][4];                 // raw Phi of the 2x2 column box, planes k-2..k+1
  Acc DX[4][2], DY[4][2];      // D_x on rows j-1, j and D_y on columns i-1, i, planes k-2..k+1

  // staging: each thread copies at most two elements of every plane; their
  // (wrapped) x-y offsets are fixed for the whole march
  constexpr int kStage = (PX * PY + NT - 1) / NT;
  int soff[kStage];
  bool sin_[kStage], sact[kStage];
#pragma unroll
  for (int u = 0; u < kStage; ++u) {
    const int e = threadIdx.x + NT * u;
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
  // this thread's part of plane p (x fastest, wrapped or zero-padded), read
  // one plane ahead, so that the loads of plane p + 1 are in flight while
  // plane p is differenced and its vertices stored.  FP64 records written
  // with three per-lane stores each (vertex boxes) read each plane when it
  // is staged: there reading ahead was slower (3.3 against 2.2 ms for
  // 512^3); with their rows leaving through LDS it is faster (1.76 -> 1.38).
  constexpr bool kAhead = sizeof(Acc) == 4 || kRowStore;
  In pre[kStage];
  auto fetch = [&](int p, int gzp) {
    const bool zin = p >= 0 && p < n;
    const In* src = phi + (int64_t)gzp * nn;
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      if (!sact[u] || (open && !(sin_[u] && zin)))
        pre[u] = (In)0;
      else
        pre[u] = src[soff[u]];
    }
  };
  if constexpr (kAhead) fetch(k0 - 2, gz);
  for (int p = k0 - 2; p <= k_end; ++p, slot ^= 1) {
    Acc* pl = plane[slot];
    if constexpr (!kAhead) fetch(p, gz);
#pragma unroll
    for (int u = 0; u < kStage; ++u)
      if (sact[u]) pl[threadIdx.x + NT * u] = (Acc)pre[u];
    if (++gz == n) gz = 0;
    __syncthreads();
    if constexpr (kAhead) {
      if (p < k_end) fetch(p + 1, gz);
    }
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
      if (row_ok) {
        // lanes write their records side by side in LDS, then read back
        // 16-byte chunks of the row in order (LDS operations of one
        // wavefront complete in order; the empty asm statements keep the
        // compiler from moving the accesses across each other)
        Acc* rb = rowbuf[kRowStore ? ty : 0];
#pragma unroll
        for (int c = 0; c < RW; ++c) rb[tx * RW + c] = rec[c];
        __asm__ volatile("" ::: "memory");
        typedef Acc chunk_t __attribute__((ext_vector_type(16 / sizeof(Acc))));
        constexpr int kE = 16 / sizeof(Acc), kChunks = TX * RW / kE;
        Acc* dst = tv + ((int64_t)k * nn + (int64_t)j * n + i_row) * RW;
#pragma unroll
        for (int m = tx; m < kChunks; m += TX)
          __builtin_nontemporal_store(*reinterpret_cast<const chunk_t*>(rb + m * kE),
                                      reinterpret_cast<chunk_t*>(dst + m * kE));
        __asm__ volatile("" ::: "memory");
      } else {
        store_vertex<kNT>(tv + ((int64_t)k * nn + (int64_t)j * n + i) * RW, rec);
      }
    }
    // XX/YY/XY hold planes (p-2, p-1) during step p; push plane p
    XX[0] = XX[1]; YY[0] = YY[1]; XY[0] = XY[1];
    XX[1] = sxx; YY[1] = syy; XY[1] = dxy;
  }
}

// Cell-centre tensor (Eq. tidalexample, cell size 1), one cell per thread,
// for the nearest-grid-point integral (Eq. Iclensing_ngp).  Second
// differences as differences of differences, mixed ones over the four
// diagonal neighbours; open grids leave the outer cell layer NaN (no stencil).
template <typename In, typename Acc>
__global__ __launch_bounds__(256) void centre_tensor_uniform_kernel(const In* __restrict__ phi,
                                                                    Acc* __restrict__ tc, int n,
                                                                    int open) {
  const int64_t nn = (int64_t)n * n;
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= nn * n) return;
  const int i = (int)(c % n), j = (int)((c / n) % n), k = (int)(c / nn);
  Acc rec[6];
  if (open && (i < 1 || j < 1 || k < 1 || i > n - 2 || j > n - 2 || k > n - 2)) {
#pragma unroll
    for (int u = 0; u < 6; ++u) rec[u] = (Acc)__builtin_nan("");
  } else {
    const int im = i == 0 ? n - 1 : i - 1, ip = i + 1 == n ? 0 : i + 1;
    const int jm = j == 0 ? n - 1 : j - 1, jp = j + 1 == n ? 0 : j + 1;
    const int km = k == 0 ? n - 1 : k - 1, kp = k + 1 == n ? 0 : k + 1;
    auto P = [&](int x, int y, int z) -> Acc { return (Acc)phi[(int64_t)z * nn + (int64_t)y * n + x]; };
    const Acc c0 = P(i, j, k);
    rec[0] = (P(ip, j, k) - c0) - (c0 - P(im, j, k));
    rec[1] = (P(i, jp, k) - c0) - (c0 - P(i, jm, k));
    rec[2] = (P(i, j, kp) - c0) - (c0 - P(i, j, km));
    rec[3] = ((P(ip, jp, k) - P(ip, jm, k)) - (P(im, jp, k) - P(im, jm, k))) * (Acc)0.25;
    rec[4] = ((P(ip, j, kp) - P(ip, j, km)) - (P(im, j, kp) - P(im, j, km))) * (Acc)0.25;
    rec[5] = ((P(i, jp, kp) - P(i, jp, km)) - (P(i, jm, kp) - P(i, jm, km))) * (Acc)0.25;
  }
  store_vertex<false>(tc + c * 6, rec);
}

template <typename In, typename Acc>
hipError_t launch_ct(int n, int open, const void* phi, void* tc, hipStream_t s) {
  const int64_t blocks = ((int64_t)n * n * n + 255) / 256;
  hipLaunchKernelGGL((centre_tensor_uniform_kernel<In, Acc>), dim3((unsigned)blocks), dim3(256),
                     0, s, (const In*)phi, (Acc*)tc, n, open);
  return hipGetLastError();
}

template <typename In, typename Acc, int TY, int KZ, bool kNT>
hipError_t launch_shape(const VertexBox& box, int n, int open, const void* phi, void* tv,
                        hipStream_t s) {
  VertexBox V = box;
  V.ntx = (V.sx + TX - 1) / TX;
  V.nty = (V.sy + TY - 1) / TY;
  const int ntz = (V.sz + KZ - 1) / KZ;
  const int64_t blocks = (int64_t)V.ntx * V.nty * ntz;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((vertex_tensor_uniform_kernel<In, Acc, TY, KZ, kNT>),
                     dim3((unsigned)blocks), dim3(TX * TY), 0, s, (const In*)phi, (Acc*)tv, n,
                     open, V);
  return hipGetLastError();
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
  const int64_t nv = (int64_t)V.sx * V.sy * V.sz;
  // boxes beyond 1/8 of the grid stream through HBM like the whole grid
  if (8 * nv > (int64_t)n * n * n)
    return launch_shape<In, Acc, 16, 16, true>(V, n, open, phi, tv, s);
  return launch_shape<In, Acc, 4, 32, false>(V, n, open, phi, tv, s);
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

hipError_t launch_centre_tensor_uniform(int precision, int dtype, int n, int open,
                                        const void* phi, void* tc, hipStream_t s) {
  if (precision == RR_PREC_FP32_KAHAN) {
    if (dtype == RR_F32) return launch_ct<float, float>(n, open, phi, tc, s);
    return launch_ct<double, float>(n, open, phi, tc, s);
  }
  if (dtype == RR_F32) return launch_ct<float, double>(n, open, phi, tc, s);
  return launch_ct<double, double>(n, open, phi, tc, s);
}

}  // namespace rr
