/* A plain C consumer of the library: no Python, no PyTorch. Builds a 64x64
 * periodic droplet (R = 16, W = 4, rho 1 / 0.1, sigma 0.01, M 0.1,
 * tau 0.8), runs 200 steps in FP64 and in FP32 and checks that the total
 * of phi is conserved (FP64: to 1e-12 relative; FP32: exactly, the stored
 * order parameter being fixed point); then the same for a 32^3 droplet
 * (R = 8) through the three-dimensional header, 100 steps, walls normal to
 * z with gravity in FP32. Exit status 0 on success. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "qilbm.h"
#include "qilbm3d.h"

#define CHECK_HIP(x)                                                   \
  do {                                                                 \
    hipError_t e_ = (x);                                               \
    if (e_ != hipSuccess) {                                            \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));          \
      return 2;                                                        \
    }                                                                  \
  } while (0)
#define CHECK_LBM(x)                                                   \
  do {                                                                 \
    lbm_status s_ = (x);                                               \
    if (s_ != LBM_OK) {                                                \
      fprintf(stderr, "%s: %s\n", #x, lbm_strerror(s_));               \
      return 3;                                                        \
    }                                                                  \
  } while (0)

static int run(int precision, double tol) {
  const int nx = 64, ny = 64;
  lbm_params p = {nx, ny, 1.0, 0.1, 0.01, 4.0, 0.1, 0.8, 0.8, 0.0, 0.0, 1.0,
                  LBM_BC_PERIODIC, precision, 0u};
  double* phi0 = (double*)malloc(sizeof(double) * nx * ny);
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const double r = sqrt((x - 32.0) * (x - 32.0) + (y - 32.0) * (y - 32.0));
      phi0[y * nx + x] = 0.5 + 0.5 * tanh(2.0 * (16.0 - r) / 4.0);
    }
  const size_t ws_bytes = lbm_workspace_bytes(&p);
  if (ws_bytes == 0) return 4;
  void* ws = NULL;
  double* phi0_dev = NULL;
  CHECK_HIP(hipMalloc(&ws, ws_bytes));
  CHECK_HIP(hipMalloc((void**)&phi0_dev, sizeof(double) * nx * ny));
  CHECK_HIP(hipMemcpy(phi0_dev, phi0, sizeof(double) * nx * ny, hipMemcpyHostToDevice));
  lbm_ctx* ctx = NULL;
  CHECK_LBM(lbm_init(&ctx, &p, ws, ws_bytes, phi0_dev, NULL));
  double m0[4], m1[4];
  CHECK_LBM(lbm_mass(ctx, m0));
  CHECK_LBM(lbm_step(ctx, 200));
  CHECK_LBM(lbm_mass(ctx, m1));
  const double drift = fabs(m1[0] - m0[0]) / fabs(m0[0]);
  printf("precision %d: sum phi %.15g -> %.15g (relative drift %.3g), t = %lld\n", precision,
         m0[0], m1[0], drift, (long long)lbm_time(ctx));
  lbm_destroy(ctx);
  CHECK_HIP(hipFree(phi0_dev));
  CHECK_HIP(hipFree(ws));
  free(phi0);
  return drift <= tol ? 0 : 1;
}

static int run3(int precision, int bc, double tol) {
  const int n = 32;
  const size_t N = (size_t)n * n * n;
  lbm3_params p = {n,   n,   n,   1.0, 0.1,          0.01, 4.0,      0.1, 0.8,
                   0.8, 0.0, 0.0, bc ? -1e-5 : 0.0, 0.55, bc,      precision, 0u};
  double* phi0 = (double*)malloc(sizeof(double) * N);
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const double r = sqrt((x - 16.0) * (x - 16.0) + (y - 16.0) * (y - 16.0) +
                              (z - 16.0) * (z - 16.0));
        phi0[((size_t)z * n + y) * n + x] = 0.5 + 0.5 * tanh(2.0 * (8.0 - r) / 4.0);
      }
  const size_t ws_bytes = lbm3_workspace_bytes(&p);
  if (ws_bytes == 0) return 4;
  void* ws = NULL;
  double* phi0_dev = NULL;
  CHECK_HIP(hipMalloc(&ws, ws_bytes));
  CHECK_HIP(hipMalloc((void**)&phi0_dev, sizeof(double) * N));
  CHECK_HIP(hipMemcpy(phi0_dev, phi0, sizeof(double) * N, hipMemcpyHostToDevice));
  lbm3_ctx* ctx = NULL;
  CHECK_LBM(lbm3_init(&ctx, &p, ws, ws_bytes, phi0_dev, NULL));
  double m0[5], m1[5];
  CHECK_LBM(lbm3_mass(ctx, m0));
  CHECK_LBM(lbm3_step(ctx, 100));
  CHECK_LBM(lbm3_mass(ctx, m1));
  const double drift = fabs(m1[0] - m0[0]) / fabs(m0[0]);
  printf("3-D precision %d bc %d: sum phi %.15g -> %.15g (relative drift %.3g), t = %lld\n",
         precision, bc, m0[0], m1[0], drift, (long long)lbm3_time(ctx));
  lbm3_destroy(ctx);
  CHECK_HIP(hipFree(phi0_dev));
  CHECK_HIP(hipFree(ws));
  free(phi0);
  return drift <= tol ? 0 : 1;
}

int main(void) {
  if (lbm_abi_version() != QILBM_ABI_VERSION) {
    fprintf(stderr, "library interface version %d, header %d\n", (int)lbm_abi_version(),
            QILBM_ABI_VERSION);
    return 1;
  }
  int rc = run(LBM_FP64, 1e-12);
  if (rc == 0) rc = run(LBM_FP32, 0.0);
  if (rc == 0) rc = run3(LBM_FP64, LBM_BC_PERIODIC, 1e-12);
  if (rc == 0) rc = run3(LBM_FP32, 1, 0.0);
  printf(rc == 0 ? "abi example ok\n" : "abi example FAILED (%d)\n", rc);
  return rc;
}
