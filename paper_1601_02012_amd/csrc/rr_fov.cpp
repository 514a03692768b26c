// rr_fov.cpp -- host-side ray directions of a flat-sky map (Sec. III E,
// Eqs. txty and rayid) with the gnomonic mapping about the map centre.
//
// Every operation is rounded on its own (no fused multiply-add), in the
// order the header states, so that any caller evaluating the same formula
// in the same order obtains the same bits.
#include <cmath>
#include <cstdint>

#include "../../include/rayramses.h"

namespace rr {
rr_status fov_fail(rr_status s, const char* what);
}

#pragma clang fp contract(off)

namespace {

// Orthonormal frame (e1, e2, e3) of a map centred on c (c finite, non-zero).
void map_frame(const double c[3], double e1[3], double e2[3], double e3[3]) {
  const double r = std::sqrt((c[0] * c[0] + c[1] * c[1]) + c[2] * c[2]);
  for (int a = 0; a < 3; ++a) e3[a] = c[a] / r;
  if (e3[0] == 0.0 && e3[1] == 0.0) {
    // on the z axis: the map's x axis is x^, its y axis +-y^ (right-handed)
    e1[0] = 1.0, e1[1] = 0.0, e1[2] = 0.0;
    e2[0] = 0.0, e2[1] = e3[2] < 0.0 ? -1.0 : 1.0, e2[2] = 0.0;
    return;
  }
  const double h[3] = {std::fabs(e3[2]) < 0.9 ? 0.0 : 1.0, 0.0,
                       std::fabs(e3[2]) < 0.9 ? 1.0 : 0.0};
  // e1 = normalise(h x e3)
  double u[3] = {h[1] * e3[2] - h[2] * e3[1], h[2] * e3[0] - h[0] * e3[2],
                 h[0] * e3[1] - h[1] * e3[0]};
  const double ru = std::sqrt((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
  for (int a = 0; a < 3; ++a) e1[a] = u[a] / ru;
  // e2 = e3 x e1
  e2[0] = e3[1] * e1[2] - e3[2] * e1[1];
  e2[1] = e3[2] * e1[0] - e3[0] * e1[2];
  e2[2] = e3[0] * e1[1] - e3[1] * e1[0];
}

// Eq. txty: theta_i = fov / (N - 1) * (i - 1) - fov / 2, i = 1..N; N = 1 -> 0.
double map_angle(double fov, int32_t n, int32_t i0) {
  if (n == 1) return 0.0;
  const double step = fov / (double)(n - 1);
  return step * (double)i0 - fov / 2.0;
}

}  // namespace

extern "C" rr_status rr_fov_directions(const double center_dir[3], double fov_x, double fov_y,
                                       int32_t nx, int32_t ny, double* dir_host) {
  if (!center_dir || !dir_host)
    return rr::fov_fail(RR_ERR_INVALID_ARG, "center_dir and dir_host must be non-NULL");
  if (!std::isfinite(center_dir[0]) || !std::isfinite(center_dir[1]) ||
      !std::isfinite(center_dir[2]) || !std::isfinite(fov_x) || !std::isfinite(fov_y))
    return rr::fov_fail(RR_ERR_NONFINITE, "center_dir and the fields of view must be finite");
  if (center_dir[0] == 0.0 && center_dir[1] == 0.0 && center_dir[2] == 0.0)
    return rr::fov_fail(RR_ERR_INVALID_ARG, "center_dir is the zero vector");
  if (nx < 1 || ny < 1 || nx > 65536 || ny > 65536)
    return rr::fov_fail(RR_ERR_INVALID_ARG, "map shape outside [1, 65536] per axis");
  if (!(fov_x >= 0.0 && fov_x < M_PI) || !(fov_y >= 0.0 && fov_y < M_PI))
    return rr::fov_fail(RR_ERR_INVALID_ARG, "fields of view must lie in [0, pi)");
  if ((nx > 1 && !(fov_x > 0.0)) || (ny > 1 && !(fov_y > 0.0)))
    return rr::fov_fail(RR_ERR_INVALID_ARG, "an axis with several rays needs a positive fov");
  // the centre is normalised first so that its scale does not change any bit
  const double r = std::sqrt((center_dir[0] * center_dir[0] + center_dir[1] * center_dir[1]) +
                             center_dir[2] * center_dir[2]);
  if (!(r > 0.0) || !std::isfinite(r))
    return rr::fov_fail(RR_ERR_INVALID_ARG, "center_dir has no usable length");
  double e1[3], e2[3], e3[3];
  map_frame(center_dir, e1, e2, e3);
  for (int32_t iy = 0; iy < ny; ++iy) {
    const double ty = std::tan(map_angle(fov_y, ny, iy));
    for (int32_t ix = 0; ix < nx; ++ix) {
      const double tx = std::tan(map_angle(fov_x, nx, ix));
      double d[3];
      for (int a = 0; a < 3; ++a) d[a] = (tx * e1[a] + ty * e2[a]) + e3[a];
      const double nd = std::sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
      double* o = dir_host + 3 * ((int64_t)iy * nx + ix);
      for (int a = 0; a < 3; ++a) o[a] = d[a] / nd;
    }
  }
  return RR_OK;
}
