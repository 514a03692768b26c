/* trace_client.c -- a plain C caller of librayramses (no Python, no C++):
 * the field of view and its ray directions (Sec. III E, Eqs. txty, rayid),
 * the vertex tensor of a uniform periodic potential (Eq. tidalexample,
 * Sec. III H) and one trace of every ray (Eqs. sumIc, Iclensing), with the
 * per-ray crossing hashes, counts and status, through the C ABI declared in
 * include/rayramses.h.  Device memory comes from the HIP runtime.
 *
 * usage: trace_client PHI N BOX PREC FOV_DEG NX CHI_S OUT
 *   PHI   raw little-endian FP64 potential, N^3 values [z][y][x]
 *   PREC  0: FP64 path (potential FP64); 1: FP32-Kahan path (potential
 *         rounded to FP32 on the host)
 *   OUT   written: int64 n_rays, int32 prec, kappa (n_rays x 8 or 4 bytes),
 *         kappa_comp (FP32 path only, n_rays x 4), hash (n_rays x 8),
 *         count (n_rays x 8), status (n_rays x 4)
 * The observer sits at the origin and looks along +z; the window is
 * [0, CHI_S].  Exit status 0 on success; a failing call prints
 * rr_last_error() and exits 1. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "rayramses.h"

static int check_rr(rr_status s, const char* what) {
  if (s != RR_OK) {
    fprintf(stderr, "%s -> %d: %s\n", what, (int)s, rr_last_error());
    return 1;
  }
  return 0;
}

static int check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return 1;
  }
  return 0;
}

#define RR(call) do { if (check_rr((call), #call)) return 1; } while (0)
#define HIP(call) do { if (check_hip((call), #call)) return 1; } while (0)

int main(int argc, char** argv) {
  if (argc != 9) {
    fprintf(stderr, "usage: %s PHI N BOX PREC FOV_DEG NX CHI_S OUT\n", argv[0]);
    return 2;
  }
  const char* phi_path = argv[1];
  const int n = atoi(argv[2]);
  const double box = atof(argv[3]);
  const int fp32 = atoi(argv[4]) != 0;
  const double fov = atof(argv[5]) * (3.14159265358979323846 / 180.0);
  const int nx = atoi(argv[6]);
  const double chi_s = atof(argv[7]);
  const char* out_path = argv[8];
  if (n < 4 || nx < 1 || !(box > 0.0) || !(chi_s > 0.0)) {
    fprintf(stderr, "bad arguments\n");
    return 2;
  }
  const int64_t nc = (int64_t)n * n * n, nr = (int64_t)nx * nx;
  printf("librayramses version %d\n", (int)rr_version());

  /* potential: host file -> device, FP64 or rounded to FP32 */
  double* phi = (double*)malloc((size_t)nc * sizeof(double));
  FILE* fp = fopen(phi_path, "rb");
  if (!phi || !fp || fread(phi, sizeof(double), (size_t)nc, fp) != (size_t)nc) {
    fprintf(stderr, "cannot read %s\n", phi_path);
    return 2;
  }
  fclose(fp);
  void* phi_d = NULL;
  const size_t vbytes = (size_t)nc * (fp32 ? sizeof(float) : sizeof(double));
  HIP(hipMalloc(&phi_d, vbytes));
  if (fp32) {
    float* p32 = (float*)malloc((size_t)nc * sizeof(float));
    for (int64_t i = 0; i < nc; ++i) p32[i] = (float)phi[i];
    HIP(hipMemcpy(phi_d, p32, vbytes, hipMemcpyHostToDevice));
    free(p32);
  } else {
    HIP(hipMemcpy(phi_d, phi, vbytes, hipMemcpyHostToDevice));
  }
  free(phi);

  rr_field_desc f = {0};
  f.kind = RR_GRID_UNIFORM;
  f.field = RR_FIELD_PHI;
  f.boundary = RR_BOUNDARY_PERIODIC;
  f.dtype = fp32 ? RR_F32 : RR_F64;
  f.n_base = n;
  f.max_level = 0;
  f.box_size = box;
  f.values = phi_d;
  rr_tensor t = NULL;
  RR(rr_tensor_create(&f, fp32 ? RR_PREC_FP32_KAHAN : RR_PREC_FP64, &t));
  RR(rr_build_tidal_tensor(t, &f, NULL));

  /* ray directions on the host (gnomonic map about +z), then to the device */
  const double centre[3] = {0.0, 0.0, 1.0};
  double* dir = (double*)malloc((size_t)nr * 3 * sizeof(double));
  RR(rr_fov_directions(centre, fov, fov, nx, nx, dir));
  void* dir_d = NULL;
  HIP(hipMalloc(&dir_d, (size_t)nr * 3 * sizeof(double)));
  HIP(hipMemcpy(dir_d, dir, (size_t)nr * 3 * sizeof(double), hipMemcpyHostToDevice));
  free(dir);

  rr_bundle b = {0};
  b.ray_offset = 0;
  b.n_rays = nr;
  b.dir = (const double*)dir_d;
  b.nx = nx;
  b.ny = nx;
  b.chi_s = chi_s;
  b.chi_hi = chi_s;
  b.chi_lo = 0.0;
  b.center_dir[2] = 1.0;
  b.fov_x = fov;
  b.fov_y = fov;

  void *kap_d = NULL, *comp_d = NULL, *hash_d = NULL, *count_d = NULL, *stat_d = NULL;
  const size_t kbytes = (size_t)nr * (fp32 ? sizeof(float) : sizeof(double));
  HIP(hipMalloc(&kap_d, kbytes));
  HIP(hipMemset(kap_d, 0, kbytes));
  if (fp32) {
    HIP(hipMalloc(&comp_d, (size_t)nr * sizeof(float)));
    HIP(hipMemset(comp_d, 0, (size_t)nr * sizeof(float)));
  }
  HIP(hipMalloc(&hash_d, (size_t)nr * 8));
  HIP(hipMalloc(&count_d, (size_t)nr * 8));
  HIP(hipMalloc(&stat_d, (size_t)nr * 4));

  rr_trace_params tp;
  memset(&tp, 0, sizeof tp);
  tp.observer[0] = tp.observer[1] = tp.observer[2] = 0.0;
  tp.kappa_scale = 1.0;
  tp.precision = fp32 ? RR_PREC_FP32_KAHAN : RR_PREC_FP64;
  tp.quantity = RR_Q_KAPPA;
  tp.integral = RR_INTEGRAL_TRILINEAR;
  tp.persistent = 0;
  tp.max_crossings = 0;
  tp.crossing_hash = (uint64_t*)hash_d;
  tp.crossing_count = (int64_t*)count_d;

  rr_plan plan = NULL;
  RR(rr_plan_create(&plan));
  /* a window outside [0, chi_s] is refused on the host, before any launch */
  rr_bundle bad = b;
  bad.chi_hi = 2.0 * chi_s;
  if (rr_trace_rays(plan, t, &tp, &bad, 1, kap_d, (float*)comp_d, (int32_t*)stat_d, NULL) !=
      RR_ERR_INVALID_ARG) {
    fprintf(stderr, "a chi window beyond chi_s was accepted\n");
    return 1;
  }
  printf("refused as expected: %s\n", rr_last_error());
  RR(rr_trace_rays(plan, t, &tp, &b, 1, kap_d, (float*)comp_d, (int32_t*)stat_d, NULL));
  HIP(hipDeviceSynchronize());

  void* host = malloc((size_t)nr * 8);
  FILE* fo = fopen(out_path, "wb");
  if (!host || !fo) {
    fprintf(stderr, "cannot write %s\n", out_path);
    return 2;
  }
  const int32_t prec = fp32;
  fwrite(&nr, 8, 1, fo);
  fwrite(&prec, 4, 1, fo);
  HIP(hipMemcpy(host, kap_d, kbytes, hipMemcpyDeviceToHost));
  fwrite(host, 1, kbytes, fo);
  if (fp32) {
    HIP(hipMemcpy(host, comp_d, (size_t)nr * 4, hipMemcpyDeviceToHost));
    fwrite(host, 4, (size_t)nr, fo);
  }
  HIP(hipMemcpy(host, hash_d, (size_t)nr * 8, hipMemcpyDeviceToHost));
  fwrite(host, 8, (size_t)nr, fo);
  HIP(hipMemcpy(host, count_d, (size_t)nr * 8, hipMemcpyDeviceToHost));
  fwrite(host, 8, (size_t)nr, fo);
  HIP(hipMemcpy(host, stat_d, (size_t)nr * 4, hipMemcpyDeviceToHost));
  fwrite(host, 4, (size_t)nr, fo);
  fclose(fo);
  free(host);

  RR(rr_plan_destroy(plan));
  RR(rr_tensor_destroy(t));
  HIP(hipFree(kap_d));
  if (comp_d) HIP(hipFree(comp_d));
  HIP(hipFree(hash_d));
  HIP(hipFree(count_d));
  HIP(hipFree(stat_d));
  HIP(hipFree(dir_d));
  HIP(hipFree(phi_d));
  printf("traced %lld rays\n", (long long)nr);
  return 0;
}
