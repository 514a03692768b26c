// rr_octree_host.cpp -- host set-up of an octree field: validates the
// breadth-first layout and the 2:1 balance (faces, edges and corners), derives
// every oct's level and integer coordinates, and owns the device buffers of
// the centre tensor and of the per-leaf corner tensors.
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "rr_octree.hpp"

namespace rr {

namespace {

struct HostTree {
  int n = 0;
  int64_t nb = 0;
  const std::vector<int32_t>* child = nullptr;
  const std::vector<int32_t>* info = nullptr;   // 4 per oct: x, y, z, level

  // cell at level l with level coords I, or the leaf above; returns the level reached
  int descend(int l, const int64_t* I, int64_t* cell) const {
    int64_t b[3];
    for (int a = 0; a < 3; ++a) {
      int64_t q = I[a] >> l;   // arithmetic shift: floor division by 2^l
      q %= n;
      if (q < 0) q += n;
      b[a] = q;
    }
    int64_t c = (b[2] * n + b[1]) * n + b[0];
    for (int lev = 1; lev <= l; ++lev) {
      const int32_t k = (*child)[c];
      if (k < 0) {
        *cell = c;
        return lev - 1;
      }
      int ch = 0;
      for (int a = 0; a < 3; ++a) ch |= (int)((I[a] >> (l - lev)) & 1) << a;
      c = nb + 8 * (int64_t)k + ch;
    }
    *cell = c;
    return l;
  }
};

}  // namespace

OctreeTensor* OctreeTensor::create(const rr_field_desc* f, int precision, rr_status* st,
                                   std::string* msg) {
  const int n = f->n_base;
  const int64_t nb = (int64_t)n * n * n;
  const int64_t n_cells = f->n_cells;
  const int64_t n_octs = (n_cells - nb) / 8;
  if (n_octs > (int64_t)INT32_MAX) {
    *st = RR_ERR_OCTREE;
    *msg = "too many octs for int32 child indices";
    return nullptr;
  }
  std::vector<int32_t> child(n_cells);
  hipError_t e = hipMemcpy(child.data(), f->child_oct, sizeof(int32_t) * n_cells,
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    *st = RR_ERR_HIP;
    *msg = std::string("child_oct copy: ") + hipGetErrorString(e);
    return nullptr;
  }
  // breadth-first layout: scanning cells in index order, refined cells must
  // name octs 0, 1, 2, ... in sequence, and an oct's cells come after its parent
  std::vector<int32_t> info((size_t)n_octs * 4, 0);
  int64_t next = 0;
  int max_level = 0;
  auto fail = [&](const char* what) -> OctreeTensor* {
    *st = RR_ERR_OCTREE;
    *msg = what;
    return nullptr;
  };
  for (int64_t c = 0; c < n_cells; ++c) {
    const int32_t k = child[c];
    if (k < 0) {
      if (k != -1) return fail("child_oct entries must be an oct index or -1");
      continue;
    }
    if (k != next) return fail("octs are not in breadth-first order (child_oct must number them "
                               "in the order of their parent cells)");
    int level;
    int64_t I[3];
    if (c < nb) {
      level = 0;
      I[0] = c % n;
      I[1] = (c / n) % n;
      I[2] = c / ((int64_t)n * n);
    } else {
      const int64_t p = (c - nb) / 8;
      if (p >= k) return fail("an oct's parent cell must precede it");
      const int ch = (int)((c - nb) % 8);
      level = info[4 * p + 3];
      for (int a = 0; a < 3; ++a) I[a] = info[4 * p + a] + ((ch >> a) & 1);
    }
    if (level + 1 > kMaxLevel) return fail("refinement deeper than 4 levels");
    for (int a = 0; a < 3; ++a) info[4 * k + a] = (int32_t)(2 * I[a]);
    info[4 * k + 3] = level + 1;
    if (level + 1 > max_level) max_level = level + 1;
    ++next;
  }
  if (next != n_octs) return fail("some octs have no parent cell");
  if (max_level > f->max_level) return fail("tree is deeper than max_level");
  // levels must be contiguous in oct order (breadth first)
  for (int64_t k = 1; k < n_octs; ++k)
    if (info[4 * k + 3] < info[4 * (k - 1) + 3]) return fail("octs are not ordered by level");
  // 2:1 balance over faces, edges and corners
  HostTree T;
  T.n = n;
  T.nb = nb;
  T.child = &child;
  T.info = &info;
  for (int64_t c = 0; c < n_cells; ++c) {
    if (child[c] < 0) continue;
    int level;
    int64_t I[3];
    if (c < nb) {
      level = 0;
      I[0] = c % n;
      I[1] = (c / n) % n;
      I[2] = c / ((int64_t)n * n);
    } else {
      const int64_t p = (c - nb) / 8;
      const int ch = (int)((c - nb) % 8);
      level = info[4 * p + 3];
      for (int a = 0; a < 3; ++a) I[a] = info[4 * p + a] + ((ch >> a) & 1);
    }
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int64_t J[3] = {I[0] + dx, I[1] + dy, I[2] + dz};
          int64_t cc;
          if (T.descend(level, J, &cc) != level)
            return fail("octree is not 2:1 balanced: a refined cell has a missing neighbour");
        }
  }

  std::unique_ptr<OctreeTensor> t(new OctreeTensor);
  t->n = n;
  t->max_level = max_level;
  t->precision = precision;
  t->n_cells = n_cells;
  t->n_octs = n_octs;
  t->child_oct_dev = f->child_oct;
  t->level_begin[0] = 0;
  t->level_begin[1] = nb;
  for (int l = 1; l <= kMaxLevel; ++l) {
    int64_t first = n_octs;
    for (int64_t k = 0; k < n_octs; ++k)
      if (info[4 * k + 3] > l) {
        first = k;
        break;
      }
    t->level_begin[l + 1] = nb + 8 * first;
  }
  const size_t rs = precision == RR_PREC_FP32_KAHAN ? 4 : 8;
  t->corner_record_bytes = (int32_t)(48 * rs);
  void* p = nullptr;
  if (n_octs > 0) {
    e = hipMalloc(&p, sizeof(int32_t) * 4 * n_octs);
    if (e != hipSuccess) goto oom;
    t->oct_info = (int32_t*)p;
    e = hipMemcpy(t->oct_info, info.data(), sizeof(int32_t) * 4 * n_octs, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      *st = RR_ERR_HIP;
      *msg = std::string("oct info upload: ") + hipGetErrorString(e);
      return nullptr;
    }
  }
  e = hipMalloc(&p, rs * 6 * (size_t)n_cells);
  if (e != hipSuccess) goto oom;
  t->centre = p;
  e = hipMalloc(&p, rs * 48 * (size_t)n_cells);
  if (e != hipSuccess) goto oom;
  t->corners = p;
  e = hipMalloc(&p, (size_t)n_cells);
  if (e != hipSuccess) goto oom;
  t->coarse_corners = (uint8_t*)p;
  // the counts depend on the tree only: computed once here, on the null
  // stream, and waited for (later builds may run on any stream)
  e = t->count_coarse_corners(nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    *st = RR_ERR_HIP;
    *msg = std::string("octree corner counts: ") + hipGetErrorString(e);
    return nullptr;
  }
  *st = RR_OK;
  return t.release();
oom:
  *st = RR_ERR_OOM;
  *msg = std::string("octree tensor allocation: ") + hipGetErrorString(e);
  return nullptr;
}

OctreeTensor::~OctreeTensor() {
  if (oct_info) (void)hipFree(oct_info);
  if (centre) (void)hipFree(centre);
  if (corners) (void)hipFree(corners);
  if (coarse_corners) (void)hipFree(coarse_corners);
}

}  // namespace rr
