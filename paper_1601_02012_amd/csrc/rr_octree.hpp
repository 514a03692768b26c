// rr_octree.hpp -- octree tidal tensor and march (host object + launchers).
#pragma once

#include <string>

#include "rr_internal.hpp"

namespace rr {

constexpr int kMaxLevel = 4;

// Device-resident description of a 2:1-balanced octree plus its per-leaf
// corner tensors (8 corners x 6 components per cell record).
struct OctreeTensor {
  int32_t n = 0;
  int32_t max_level = 0;
  int32_t precision = 0;
  int64_t n_cells = 0;
  int64_t n_octs = 0;
  const int32_t* child_oct_dev = nullptr;   // caller-owned
  int32_t* oct_info = nullptr;              // per oct: level coords of child 0 (x,y,z), level
  void* centre = nullptr;                   // per cell: 6 components (precision-typed)
  void* corners = nullptr;                  // per cell: 8 x 6 components
  uint8_t* coarse_corners = nullptr;        // per leaf of level >= 1: corners touching a coarser leaf
  int32_t corner_record_bytes = 0;
  int64_t level_begin[kMaxLevel + 2] = {0};  // first cell index of each level (levels contiguous)

  static OctreeTensor* create(const rr_field_desc* f, int precision, rr_status* st,
                              std::string* msg);
  hipError_t count_coarse_corners(hipStream_t s);   // once, at creation (tree only)
  hipError_t build(const void* values, int dtype, hipStream_t s);
  hipError_t march(const TraceArgs& a, int persistent, int grid_waves, hipStream_t s);
  ~OctreeTensor();
};

hipError_t launch_adjoint_uniform(const TraceArgs& a, const float* dl_dkappa, float* lam,
                                  float* dl_dphi, hipStream_t s);

}  // namespace rr
