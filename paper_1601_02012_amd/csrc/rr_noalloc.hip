// rr_noalloc.hip -- the fixed device scratch array behind rr_trace_rays_noalloc.
//
// The array holds what a plan otherwise allocates for a trace: the work-queue
// counter of persistent launches and the device copy of the bundle table.
// Each GPU the library runs on holds its own copy of the array (until the
// process ends); host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device, never through the
// array's name, which is a host-side stand-in.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rr_internal.hpp"

namespace rr {

namespace {

static_assert(sizeof(DevBundle) == 72, "bundle table entries are 72 bytes");

constexpr size_t kTableOffset = 256;    // bytes [0, 256): queue counter (+ spare)
constexpr size_t kScratchBytes = kTableOffset + sizeof(DevBundle) * kNoallocMaxBundles;

static __device__ __align__(256) unsigned char scratch[(kScratchBytes + 255) / 256 * 256];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Bundle-table entries passed by value: a launch's arguments are copied when
// it is enqueued, so the table needs neither a host staging buffer nor a
// copy from pageable memory (and a capture records a kernel node).
constexpr int kPutChunk = 48;   // 48 x 72 B = 3456 B of kernel arguments
struct BundleChunk {
  DevBundle b[kPutChunk];
};

__global__ __launch_bounds__(64) void put_bundles_kernel(DevBundle* __restrict__ dst,
                                                         BundleChunk c, int count) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = c.b[i];
}

}  // namespace

hipError_t noalloc_scratch(void** queue, DevBundle** table) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    // once per device, with that device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *queue = g_ptr[dev];
  *table = reinterpret_cast<DevBundle*>(static_cast<char*>(g_ptr[dev]) + kTableOffset);
  return hipSuccess;
}

hipError_t launch_put_bundles(DevBundle* dst, const DevBundle* host, int count, hipStream_t s) {
  for (int k = 0; k < count; k += kPutChunk) {
    BundleChunk c;
    const int m = count - k < kPutChunk ? count - k : kPutChunk;
    for (int i = 0; i < m; ++i) c.b[i] = host[k + i];
    hipLaunchKernelGGL(put_bundles_kernel, dim3(1), dim3(64), 0, s, dst + k, c, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rr
