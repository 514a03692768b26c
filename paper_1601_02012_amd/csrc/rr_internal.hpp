// rr_internal.hpp -- data shared by the host layer and the HIP kernels of
// librayramses.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rayramses.h"

namespace rr {

// Base-cell units: h0 = L / n, o~ = o / h0, chi~ = chi / h0 (host FP64 divides).
struct DevBundle {
  const double* dir;   // n_rays x 3
  int64_t ray_offset;
  int64_t n_rays;
  int32_t nx, ny;
  int32_t tiles_x, tiles_y;
  int64_t tile_begin;  // prefix over bundles in launch order
  double chi_s, chi_hi, chi_lo;  // base-cell units
};

struct TraceArgs {
  const DevBundle* bundles;
  int32_t n_bundles;
  int64_t n_tiles;           // total 8x8 tiles over all bundles
  double o[3];               // observer, base-cell units
  double kappa_scale;
  int32_t n;                 // base cells per side
  int32_t open;              // RR_BOUNDARY_OPEN
  int32_t quantity;
  int32_t integral;
  int32_t mode;              // integrand: 0 tidal tensor, 1 tidal tensor at centres (NGP),
                             // 2 Method A, 3 the two source-distance moments,
                             // 4 a vertex scalar with a constant kernel (ISW)
  int64_t max_crossings;
  // outputs
  void* kappa;
  float* kappa_comp;
  int32_t* status;
  uint64_t* hash;
  int64_t* count;
  void* log;
  int64_t log_stride;
  // work queue (persistent mode)
  unsigned long long* queue;
  // source-distance moments (mode 3): kappa holds the per-ray moment state,
  // src the source distances (base-cell units, decreasing), pieces the pairs
  // handed out at each of them
  const double* src;
  int32_t n_src;
  double* pieces;
  // passes (resume != nullptr): per ray the chi where the next pass starts
  // (+inf: the window's chi_hi; -inf: done); a pass stops a ray on the first
  // face at or below pause_chi (base-cell units; -inf: run to chi_lo)
  double* resume;
  double pause_chi;
};

// Uniform vertex tensor record: 6 components, FP32 (24 B, three 8-byte
// accesses) or FP64 (48 B, three 16-byte accesses).
template <typename Real>
struct VertexRecord;
template <>
struct VertexRecord<float> {
  static constexpr int kWords = 6;
};
template <>
struct VertexRecord<double> {
  static constexpr int kWords = 6;
};

// host launchers (defined in the .hip files)
hipError_t launch_vertex_tensor_uniform(int precision, int dtype, int n, int open, const int* lo,
                                        const int* size, const void* phi, void* tv,
                                        hipStream_t s);
// Method A vertex records (c delta, grad Phi): 4 components per vertex
hipError_t launch_method_a_vertex_fields(int precision, int dtype, int n, int open,
                                         const void* delta, const void* phi, double cdelta,
                                         void* fv, hipStream_t s);
// ISW vertex scalars: mean over the eight incident cells of (curr - prev) * inv_dt
hipError_t launch_isw_vertex_field(int precision, int dtype, int n, int open, const void* curr,
                                   const void* prev, double inv_dt, void* qv, hipStream_t s);
// cell-centre tensor records (one per cell, same layout as the vertex records)
hipError_t launch_centre_tensor_uniform(int precision, int dtype, int n, int open,
                                        const void* phi, void* tc, hipStream_t s);
// min / max over the rays of the floor of their lattice coordinates at both
// ends of their chi windows: out[0..2] min, out[3..5] max (atomics; the
// caller initialises out)
hipError_t launch_ray_bounds(const TraceArgs& a, int* out, hipStream_t s);
hipError_t launch_march_uniform(int precision, const void* tv, const TraceArgs& a, int persistent,
                                int block, int grid_waves, hipStream_t s);
hipError_t launch_queue_reset(unsigned long long* q, hipStream_t s);
// The allocation-free trace: bundles it takes at most, and the addresses (on
// the current device) of the queue counter and the bundle table inside the
// library's fixed device scratch array (resolved once per device).
constexpr int kNoallocMaxBundles = 1024;
hipError_t noalloc_scratch(void** queue, DevBundle** table);
// dst[0..count) = host[0..count), by kernels whose arguments carry the entries
hipError_t launch_put_bundles(DevBundle* dst, const DevBundle* host, int count, hipStream_t s);
// p[0..n) = v (a kernel: safe inside a graph capture)
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);
// kappa of every source from the moment state and the pieces (mode 3)
hipError_t launch_kappa_from_pieces(int precision, const void* moments, const double* pieces,
                                    const double* src, int n_src, int64_t n_rays, double* kappa,
                                    hipStream_t s);

}  // namespace rr
