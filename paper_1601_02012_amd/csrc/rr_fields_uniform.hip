// rr_fields_uniform.hip -- the other vertex fields of a uniform grid, each the
// mean over the eight cells incident on a vertex (Sec. III H, regular
// vertices):
//   Method A (Eq. kappa2): c delta and the central-difference gradient of Phi;
//   ISW (Sec. VII): the rate (Phi_curr - Phi_prev) / dt of consecutive steps.
//
// Vertex (i,j,k) averages cells {i-1,i} x {j-1,j} x {k-1,k}.  With
//   B f(i) = f(i-1) + f(i)                                  (sum over the two cells)
//   D f(i) = (f(i+1) - f(i-1)) + (f(i) - f(i-2))            (central difference, summed)
// the records are c delta = (c/8) B_x B_y B_z delta, dPhi/dx = D_x B_y B_z Phi / 16
// (and the same for y, z), and the ISW value = (inv_dt/8) B_x B_y B_z (Phi_curr -
// Phi_prev).  Differences are taken on raw values first, sums afterwards.
//
// Layout of the work, as for the tidal tensor: a workgroup owns a 64 x 16
// column of vertices in x-y and marches 16 vertices along z; each step
// stages one plane of its inputs (with halo) in LDS, and every thread loads
// its share of the next plane while the current one is differenced and its
// records are stored.  The records go out with non-temporal stores (a 512^3
// field does not fit any cache).  Open grids: the vertices whose stencil
// would leave the grid are NaN, so the staged halo is always read wrapped.
#include "rr_internal.hpp"

namespace rr {
namespace {

constexpr int TX = 64;   // vertices per workgroup in x
constexpr int TY = 16;   // ... in y
constexpr int KZ = 16;   // ... marched along z

// This thread's share of a staged PX x PY window of every plane whose lower
// corner is lattice point (x0, y0) (unwrapped): offsets within a plane,
// wrapped into [0, n)^2, fixed for the whole march.
template <int NT, int PX, int PY>
struct Stage {
  static constexpr int kN = (PX * PY + NT - 1) / NT;
  int off[kN];
  bool act[kN];
  __device__ __forceinline__ void init(int x0, int y0, int n) {
#pragma unroll
    for (int u = 0; u < kN; ++u) {
      const int e = threadIdx.x + NT * u;
      act[u] = e < PX * PY;
      int wx = (x0 + e % PX) % n, wy = (y0 + e / PX) % n;
      wx = wx < 0 ? wx + n : wx;
      wy = wy < 0 ? wy + n : wy;
      off[u] = wy * n + wx;
    }
  }
};

template <typename T>
__device__ __forceinline__ void store_nt(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

// Method A: per vertex (c delta, dPhi/dx, dPhi/dy, dPhi/dz).
template <typename In, typename Acc>
__global__ __launch_bounds__(TX * TY) void method_a_fields_kernel(const In* __restrict__ delta,
                                                                  const In* __restrict__ phi,
                                                                  Acc* __restrict__ fv, int n,
                                                                  int open, double cdelta,
                                                                  int ntx, int nty) {
  constexpr int NT = TX * TY;
  constexpr int PX = TX + 3, PY = TY + 3;   // halo: two cells below, one above
  __shared__ Acc sp[2][PY * PX];
  __shared__ Acc sd[2][PY * PX];
  const int b = blockIdx.x;
  const int bx = b % ntx, by = (b / ntx) % nty, bz = b / (ntx * nty);
  const int i0 = bx * TX, j0 = by * TY, k0 = bz * KZ;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = i0 + tx, j = j0 + ty;
  const bool mine = i < n && j < n;
  const int64_t nn = (int64_t)n * n;
  const int k_end = min(k0 + KZ, n);        // vertices k0 .. k_end - 1

  Stage<NT, PX, PY> S;
  S.init(i0 - 2, j0 - 2, n);
  In pp[S.kN], pd[S.kN];
  auto fetch = [&](int gz) {
    const In* a = phi + (int64_t)gz * nn;
    const In* d = delta + (int64_t)gz * nn;
#pragma unroll
    for (int u = 0; u < S.kN; ++u) {
      if (S.act[u]) {
        pp[u] = a[S.off[u]];
        pd[u] = d[S.off[u]];
      }
    }
  };

  Acc Z[4][4] = {};       // raw Phi of the 2x2 column box, planes k-2 .. k+1
  Acc GX[2] = {}, GY[2] = {}, DS[2] = {};  // D_x B_y Phi, B_x D_y Phi, B_x B_y delta, planes k-1, k
  const Acc cd = (Acc)(cdelta * 0.125);
  int slot = 0;
  int gz = (k0 - 2) % n;
  if (gz < 0) gz += n;
  fetch(gz);
  for (int p = k0 - 2; p <= k_end; ++p, slot ^= 1) {
#pragma unroll
    for (int u = 0; u < S.kN; ++u)
      if (S.act[u]) {
        sp[slot][threadIdx.x + NT * u] = (Acc)pp[u];
        sd[slot][threadIdx.x + NT * u] = (Acc)pd[u];
      }
    if (++gz == n) gz = 0;
    __syncthreads();
    if (p < k_end) fetch(gz);
    // 4x4 patch of Phi: rows y = j-2 .. j+1, columns x = i-2 .. i+1
    const Acc* pl = sp[slot];
    Acc q[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) q[r][c] = pl[(ty + r) * PX + (tx + c)];
    const Acc* dl = sd[slot];
    const Acc e11 = dl[(ty + 1) * PX + tx + 1], e12 = dl[(ty + 1) * PX + tx + 2];
    const Acc e21 = dl[(ty + 2) * PX + tx + 1], e22 = dl[(ty + 2) * PX + tx + 2];
    const Acc gx = ((q[1][3] - q[1][1]) + (q[1][2] - q[1][0])) +
                   ((q[2][3] - q[2][1]) + (q[2][2] - q[2][0]));
    const Acc gy = ((q[3][1] - q[1][1]) + (q[2][1] - q[0][1])) +
                   ((q[3][2] - q[1][2]) + (q[2][2] - q[0][2]));
    const Acc ds = (e11 + e12) + (e21 + e22);
#pragma unroll
    for (int h = 0; h < 3; ++h)
#pragma unroll
      for (int c = 0; c < 4; ++c) Z[h][c] = Z[h + 1][c];
    Z[3][0] = q[1][1]; Z[3][1] = q[1][2]; Z[3][2] = q[2][1]; Z[3][3] = q[2][2];

    if (p >= k0 + 1 && mine) {
      // vertex k = p - 1: Z[0..3] are planes k-2 .. k+1; GX/GY/DS[0..1] are k-1, k
      const int k = p - 1;
      Acc gz_ = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) gz_ += (Z[3][c] - Z[1][c]) + (Z[2][c] - Z[0][c]);
      Acc rec[4];
      rec[0] = (DS[0] + DS[1]) * cd;
      rec[1] = (GX[0] + GX[1]) * (Acc)0.0625;
      rec[2] = (GY[0] + GY[1]) * (Acc)0.0625;
      rec[3] = gz_ * (Acc)0.0625;
      if (open && (i < 2 || j < 2 || k < 2 || i > n - 2 || j > n - 2 || k > n - 2)) {
#pragma unroll
        for (int c = 0; c < 4; ++c) rec[c] = (Acc)__builtin_nan("");
      }
      const int64_t v = (int64_t)k * nn + (int64_t)j * n + i;
      if constexpr (sizeof(Acc) == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 r = {rec[0], rec[1], rec[2], rec[3]};
        store_nt(reinterpret_cast<f4*>(fv) + v, r);
      } else {
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2 r0 = {rec[0], rec[1]}, r1 = {rec[2], rec[3]};
        store_nt(reinterpret_cast<d2*>(fv) + 2 * v, r0);
        store_nt(reinterpret_cast<d2*>(fv) + 2 * v + 1, r1);
      }
    }
    GX[0] = GX[1]; GY[0] = GY[1]; DS[0] = DS[1];
    GX[1] = gx; GY[1] = gy; DS[1] = ds;
  }
}

// ISW: per vertex the mean rate (Phi_curr - Phi_prev) * inv_dt.  The
// potentials of consecutive steps are close, so the staged differences and
// the sum are FP64, rounded once.
template <typename In, typename Acc>
__global__ __launch_bounds__(TX * TY) void isw_field_kernel(const In* __restrict__ curr,
                                                            const In* __restrict__ prev,
                                                            Acc* __restrict__ qv, int n, int open,
                                                            double inv_dt, int ntx, int nty) {
  constexpr int NT = TX * TY;
  constexpr int PX = TX + 1, PY = TY + 1;   // halo: one cell below
  __shared__ double sd[2][PY * PX];
  const int b = blockIdx.x;
  const int bx = b % ntx, by = (b / ntx) % nty, bz = b / (ntx * nty);
  const int i0 = bx * TX, j0 = by * TY, k0 = bz * KZ;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = i0 + tx, j = j0 + ty;
  const bool mine = i < n && j < n;
  const int64_t nn = (int64_t)n * n;
  const int k_end = min(k0 + KZ, n);        // vertices k0 .. k_end - 1

  Stage<NT, PX, PY> S;
  S.init(i0 - 1, j0 - 1, n);
  In pc[S.kN], pv[S.kN];
  auto fetch = [&](int gz) {
    const In* a = curr + (int64_t)gz * nn;
    const In* c = prev + (int64_t)gz * nn;
#pragma unroll
    for (int u = 0; u < S.kN; ++u) {
      if (S.act[u]) {
        pc[u] = a[S.off[u]];
        pv[u] = c[S.off[u]];
      }
    }
  };

  double H = 0;           // in-plane sum of plane k-1
  const double scale = inv_dt * 0.125;
  int slot = 0;
  int gz = (k0 - 1) % n;
  if (gz < 0) gz += n;
  fetch(gz);
  for (int p = k0 - 1; p < k_end; ++p, slot ^= 1) {
#pragma unroll
    for (int u = 0; u < S.kN; ++u)
      if (S.act[u]) sd[slot][threadIdx.x + NT * u] = (double)pc[u] - (double)pv[u];
    if (++gz == n) gz = 0;
    __syncthreads();
    if (p + 1 < k_end) fetch(gz);
    // cells (i-1, i) x (j-1, j) of plane p
    const double* pl = sd[slot];
    const double h = (pl[ty * PX + tx] + pl[ty * PX + tx + 1]) +
                     (pl[(ty + 1) * PX + tx] + pl[(ty + 1) * PX + tx + 1]);
    if (p >= k0 && mine) {
      const int k = p;
      Acc out = (Acc)((H + h) * scale);
      if (open && (i < 1 || j < 1 || k < 1)) out = (Acc)__builtin_nan("");
      store_nt(qv + (int64_t)k * nn + (int64_t)j * n + i, out);
    }
    H = h;
  }
}

template <typename In, typename Acc>
hipError_t launch_ma(int n, int open, const void* delta, const void* phi, double cdelta, void* fv,
                     hipStream_t s) {
  const int ntx = (n + TX - 1) / TX, nty = (n + TY - 1) / TY, ntz = (n + KZ - 1) / KZ;
  const int64_t blocks = (int64_t)ntx * nty * ntz;
  hipLaunchKernelGGL((method_a_fields_kernel<In, Acc>), dim3((unsigned)blocks), dim3(TX * TY), 0,
                     s, (const In*)delta, (const In*)phi, (Acc*)fv, n, open, cdelta, ntx, nty);
  return hipGetLastError();
}

template <typename In, typename Acc>
hipError_t launch_isw(int n, int open, const void* curr, const void* prev, double inv_dt,
                      void* qv, hipStream_t s) {
  const int ntx = (n + TX - 1) / TX, nty = (n + TY - 1) / TY, ntz = (n + KZ - 1) / KZ;
  const int64_t blocks = (int64_t)ntx * nty * ntz;
  hipLaunchKernelGGL((isw_field_kernel<In, Acc>), dim3((unsigned)blocks), dim3(TX * TY), 0, s,
                     (const In*)curr, (const In*)prev, (Acc*)qv, n, open, inv_dt, ntx, nty);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_method_a_vertex_fields(int precision, int dtype, int n, int open,
                                         const void* delta, const void* phi, double cdelta,
                                         void* fv, hipStream_t s) {
  if (precision == RR_PREC_FP32_KAHAN) {
    if (dtype == RR_F32) return launch_ma<float, float>(n, open, delta, phi, cdelta, fv, s);
    return launch_ma<double, float>(n, open, delta, phi, cdelta, fv, s);
  }
  if (dtype == RR_F32) return launch_ma<float, double>(n, open, delta, phi, cdelta, fv, s);
  return launch_ma<double, double>(n, open, delta, phi, cdelta, fv, s);
}

hipError_t launch_isw_vertex_field(int precision, int dtype, int n, int open, const void* curr,
                                   const void* prev, double inv_dt, void* qv, hipStream_t s) {
  if (precision == RR_PREC_FP32_KAHAN) {
    if (dtype == RR_F32) return launch_isw<float, float>(n, open, curr, prev, inv_dt, qv, s);
    return launch_isw<double, float>(n, open, curr, prev, inv_dt, qv, s);
  }
  if (dtype == RR_F32) return launch_isw<float, double>(n, open, curr, prev, inv_dt, qv, s);
  return launch_isw<double, double>(n, open, curr, prev, inv_dt, qv, s);
}

}  // namespace rr
