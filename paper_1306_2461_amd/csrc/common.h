// Device helpers shared by the HIP kernels: element loads/stores per storage type, the
// clamped bilinear sample with split coordinates, the prolongation read and the 2x2 solve.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ofmi {

constexpr float kTau = 1e-5f;   // relative singularity threshold of the 2x2 solve

// Field source of an iteration: the previous iteration at the same level, the coarser
// level's result (prolongation u <- 2 bilinear(u_c, x/2, y/2)), or zero (coarsest level).
enum FlowMode : int { kFlowSame = 0, kFlowCoarse = 1, kFlowZero = 2 };

struct IterArgs {
  const void* I1;      // frame 1 at this level
  const void* I2;      // frame 2 at this level
  const float* uin;    // source field (same level or coarse level), unused for kFlowZero
  const float* vin;
  float* uout;         // destination field, this level
  float* vout;
  int H, W;            // level size
  int Hc, Wc;          // coarse level size (kFlowCoarse)
  int mode;            // FlowMode
};

__device__ __forceinline__ float ld(const uint8_t* p, int i) { return (float)p[i]; }
__device__ __forceinline__ float ld(const float* p, int i) { return p[i]; }
__device__ __forceinline__ float ld(const __half* p, int i) { return __half2float(p[i]); }

__device__ __forceinline__ void st(float* p, int i, float x) { p[i] = x; }
__device__ __forceinline__ void st(__half* p, int i, float x) { p[i] = __float2half_rn(x); }

// Integer base and fraction of the sample coordinate x + d along one axis of length n,
// clamped into [0, n-1].  Splitting d = floor(d) + frac keeps the coordinate exact in FP32
// (x + d itself would round to the spacing of |x|).  Returns base; frac is 0 when clamped.
__device__ __forceinline__ int split_coord(int x, float d, int n, float& frac) {
  float fd = floorf(d);
  frac = d - fd;
  fd = fminf(fmaxf(fd, -1048576.f), 1048576.f);
  int b = x + (int)fd;
  if (b < 0) { b = 0; frac = 0.f; }
  else if (b >= n - 1) { b = n - 1; frac = 0.f; }
  return b;
}

// I(x + u, y + v) by bilinear interpolation with clamped coordinates.
template <typename T>
__device__ __forceinline__ float warp_sample(const T* __restrict__ I, int H, int W, int x, int y,
                                             float u, float v) {
  float a, b;
  const int xi = split_coord(x, u, W, a);
  const int yi = split_coord(y, v, H, b);
  const int x1 = min(xi + 1, W - 1);
  const int y1 = min(yi + 1, H - 1);
  const float z00 = ld(I, yi * W + xi), z01 = ld(I, yi * W + x1);
  const float z10 = ld(I, y1 * W + xi), z11 = ld(I, y1 * W + x1);
  const float t = fmaf(a, z01 - z00, z00);
  const float s = fmaf(a, z11 - z10, z10);
  return fmaf(b, s - t, t);
}

// Field value at in-image pixel (x, y) of the current level for the iteration's source.
__device__ __forceinline__ void read_flow(const IterArgs& a, int x, int y, float& u, float& v) {
  if (a.mode == kFlowSame) {
    const int i = y * a.W + x;
    u = a.uin[i];
    v = a.vin[i];
  } else if (a.mode == kFlowCoarse) {
    // 2 * bilinear(coarse, x/2, y/2): base floor(x/2), fraction 0 or 1/2.
    const int x0 = x >> 1, y0 = y >> 1;
    const int x1 = min(x0 + 1, a.Wc - 1), y1 = min(y0 + 1, a.Hc - 1);
    const float fa = (x & 1) ? 0.5f : 0.f, fb = (y & 1) ? 0.5f : 0.f;
    const int i00 = y0 * a.Wc + x0, i01 = y0 * a.Wc + x1, i10 = y1 * a.Wc + x0, i11 = y1 * a.Wc + x1;
    float t = fmaf(fa, a.uin[i01] - a.uin[i00], a.uin[i00]);
    float s = fmaf(fa, a.uin[i11] - a.uin[i10], a.uin[i10]);
    u = 2.f * fmaf(fb, s - t, t);
    t = fmaf(fa, a.vin[i01] - a.vin[i00], a.vin[i00]);
    s = fmaf(fa, a.vin[i11] - a.vin[i10], a.vin[i10]);
    v = 2.f * fmaf(fb, s - t, t);
  } else {
    u = 0.f;
    v = 0.f;
  }
}

// New estimate at a pixel from its window sums and its current estimate (u, v).
// D = AC - B^2 uses Kahan's FMA-compensated difference of products.
__device__ __forceinline__ void solve_update(float A, float B, float C, float sx, float sy,
                                             float u, float v, float& un, float& vn) {
  const float bx = fmaf(B, v, fmaf(A, u, sx));
  const float by = fmaf(C, v, fmaf(B, u, sy));
  const float T = A + C;
  const float w = B * B;
  const float e = fmaf(-B, B, w);
  const float D = fmaf(A, C, -w) + e;
  float du = 0.f, dv = 0.f;
  if (D > kTau * (T * T)) {
    const float inv = 1.0f / D;
    du = -(fmaf(C, bx, -B * by)) * inv;
    dv = -(fmaf(A, by, -B * bx)) * inv;
  } else if (T > 0.f) {
    const float inv = 1.0f / (T * T);
    du = -(fmaf(A, bx, B * by)) * inv;
    dv = -(fmaf(B, bx, C * by)) * inv;
  }
  un = u + du;
  vn = v + dv;
}

}  // namespace ofmi
