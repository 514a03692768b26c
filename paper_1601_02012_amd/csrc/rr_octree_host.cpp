// rr_octree_host.cpp -- placeholder until the octree kernels land.
#include "rr_octree.hpp"

namespace rr {

OctreeTensor* OctreeTensor::create(const rr_field_desc*, int, rr_status* st, std::string* msg) {
  *st = RR_ERR_UNSUPPORTED;
  *msg = "octree grids are not built into this library yet";
  return nullptr;
}
hipError_t OctreeTensor::build(const void*, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t OctreeTensor::march(const TraceArgs&, int, int, hipStream_t) {
  return hipErrorNotSupported;
}
OctreeTensor::~OctreeTensor() {}

}  // namespace rr
