/* A C caller of the library, with no Python and no torch: device memory from the HIP runtime,
 * the flow of a linear intensity ramp moved by a quarter pixel (the method recovers the shift
 * exactly away from the borders), and an invalid plan rejected with an error text. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "ofmi.h"

#define H 40
#define W 64

static int check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return 1;
  }
  return 0;
}

int main(void) {
  static unsigned char h1[H * W], h2[H * W];
  static float u[H * W], v[H * W];
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      h1[y * W + x] = (unsigned char)(4 * x);
      h2[y * W + x] = (unsigned char)(4 * x - 1 < 0 ? 0 : 4 * x - 1);
    }
  if (of_plan_create(0, 5, 1, 1, 1) != NULL || of_last_error()[0] == '\0') {
    fprintf(stderr, "an invalid plan was not rejected\n");
    return 1;
  }
  void *d1 = NULL, *d2 = NULL;
  float *du = NULL, *dv = NULL;
  if (check(hipMalloc(&d1, H * W), "hipMalloc") || check(hipMalloc(&d2, H * W), "hipMalloc") ||
      check(hipMalloc((void**)&du, sizeof(u)), "hipMalloc") ||
      check(hipMalloc((void**)&dv, sizeof(v)), "hipMalloc") ||
      check(hipMemcpy(d1, h1, H * W, hipMemcpyHostToDevice), "hipMemcpy") ||
      check(hipMemcpy(d2, h2, H * W, hipMemcpyHostToDevice), "hipMemcpy"))
    return 1;
  of_plan* p = of_plan_create(H, W, 1, 3, 1);
  if (!p) {
    fprintf(stderr, "of_plan_create: %s\n", of_last_error());
    return 1;
  }
  if (of_compute(p, d1, d2, du, dv, NULL) != OF_OK) {
    fprintf(stderr, "of_compute: %s\n", of_last_error());
    return 1;
  }
  if (check(hipDeviceSynchronize(), "sync") ||
      check(hipMemcpy(u, du, sizeof(u), hipMemcpyDeviceToHost), "hipMemcpy") ||
      check(hipMemcpy(v, dv, sizeof(v), hipMemcpyDeviceToHost), "hipMemcpy"))
    return 1;
  double worst = 0.0;
  for (int y = 0; y < H; ++y)
    for (int x = 6; x < W - 6; ++x) {
      const double du_ = fabs(u[y * W + x] - 0.25), dv_ = fabs(v[y * W + x]);
      if (du_ > worst) worst = du_;
      if (dv_ > worst) worst = dv_;
    }
  of_plan_destroy(p);
  hipFree(d1);
  hipFree(d2);
  hipFree(du);
  hipFree(dv);
  printf("C caller: quarter-pixel ramp shift recovered to %.2e px\n", worst);
  return worst <= 1e-6 ? 0 : 1;
}
