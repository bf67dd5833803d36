// Device helpers shared by the HIP kernels: element loads/stores per storage type, the
// clamped bilinear sample with split coordinates, the prolongation read and the 2x2 solve.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ofmi {

constexpr float kTau = 1e-5f;   // relative singularity threshold of the 2x2 solve
constexpr int kMaxTaps = 25;    // window taps for the largest supported radius (2*12 + 1)

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
  const uint8_t* mask; // this level's mask (nonzero = computed) or nullptr (no mask)
  const uint8_t* tiles; // plain launches with a mask: one flag per iteration tile: 0 = no
                        // unmasked output pixel, 1 = some masked pixels, 2 = no masked pixel
                        // (batched launches carry the flag in the work item)
  float taps[kMaxTaps]; // Gaussian-weighted window: separable taps g[0..2r] (unused for the box)
  // Recirculation-bubble count (eq. 3), final iteration of a plan only: when bcount is set,
  // the launch adds to *bcount the number of written u values <= *bthr.
  const float* bthr;
  unsigned long long* bcount;
};

// Element access by an unsigned 32-bit element index whose byte offset is formed in 32 bits
// (planes are below 4 GiB), through the global address space: with the base pointer in
// scalar registers this selects the scalar-base + 32-bit vector-offset global addressing
// form, also where the pointer itself was read from memory (work lists) and the compiler
// could not infer the address space (it would otherwise emit flat accesses).
template <typename T>
using global_t = __attribute__((address_space(1))) T;

template <typename T>
__device__ __forceinline__ const global_t<T>& at(const T* p, unsigned i) {
  return *((const global_t<T>*)((const global_t<char>*)p + i * (unsigned)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ global_t<T>& at(T* p, unsigned i) {
  return *((global_t<T>*)((global_t<char>*)p + i * (unsigned)sizeof(T)));
}

__device__ __forceinline__ float ld(const uint8_t* p, unsigned i) { return (float)at(p, i); }
__device__ __forceinline__ float ld(const float* p, unsigned i) { return at(p, i); }
__device__ __forceinline__ float ld(const __half* p, unsigned i) {
  return __half2float(__ushort_as_half(at(reinterpret_cast<const unsigned short*>(p), i)));
}

__device__ __forceinline__ void st(float* p, unsigned i, float x) { at(p, i) = x; }
__device__ __forceinline__ void st(__half* p, unsigned i, float x) {
  at(reinterpret_cast<unsigned short*>(p), i) = __half_as_ushort(__float2half_rn(x));
}

// Row-major offset y * W + x with a 24-bit multiply: the full-rate v_mul_u32_u24 (the 32-bit
// integer multiply issues at a quarter of the rate).  Plans keep H and W below 2^24 and H * W
// below 2^30, so every product of an in-image row and a width fits.
__device__ __forceinline__ unsigned rowofs(int y, int W, int x) {
  return __umul24((unsigned)y, (unsigned)W) + (unsigned)x;
}

// i / D and i % D for a compile-time divisor D and 0 <= i < LIMIT: a 24-bit multiply by
// floor(2^20 / D) + 1 and a shift (instead of the quarter-rate 32-bit high multiply), checked
// exact for every i in range at compile time.
template <int D, int LIMIT>
struct ConstDiv {
  static constexpr unsigned S = 20, M = (1u << S) / D + 1;
  static constexpr bool exact() {
    for (unsigned i = 0; i < (unsigned)LIMIT; ++i)
      if (((i * M) >> S) != i / (unsigned)D) return false;
    return true;
  }
  static_assert(D > 0 && (unsigned long long)LIMIT * M < (1ull << 32) && exact(),
                "24-bit reciprocal multiply not exact over the index range");
  __device__ static __forceinline__ unsigned q(unsigned i) {
    if constexpr ((D & (D - 1)) == 0) return i / (unsigned)D;
    else return __umul24(i, M) >> S;
  }
  // (a signed 24-bit multiply by -D, so that the subtraction folds into one full-rate
  // multiply-add rather than a 32-bit one)
  __device__ static __forceinline__ unsigned r(unsigned i, unsigned q) {
    return i + (unsigned)__mul24((int)q, -D);
  }
};

// Integer base and fraction of the sample coordinate x + d along one axis of length n,
// clamped into [0, n-1].  Splitting d = floor(d) + frac keeps the coordinate exact in FP32
// (x + d itself would round to the spacing of |x|).  The sample is interior when its base
// lies in [0, n-2]; otherwise the base is clamped and the fraction is 0.  Returns the base;
// `step` is 1 for an interior sample (the second tap is the next element) and 0 otherwise.
__device__ __forceinline__ int split_coord(int x, float d, int n, float& frac, unsigned& step) {
  const float fd = floorf(d);
  const int bu = x + (int)fminf(fmaxf(fd, -1048576.f), 1048576.f);
  const bool inside = (unsigned)bu < (unsigned)(n - 1);
  frac = inside ? d - fd : 0.f;
  step = inside ? 1u : 0u;
  return min(max(bu, 0), n - 1);
}

// I(x + u, y + v) by bilinear interpolation with clamped coordinates.
template <typename T>
__device__ __forceinline__ float warp_sample(const T* __restrict__ I, int H, int W, int x, int y,
                                             float u, float v) {
  float a, b;
  unsigned sx, sy;
  const int xi = split_coord(x, u, W, a, sx);
  const int yi = split_coord(y, v, H, b, sy);
  const unsigned o00 = rowofs(yi, W, xi);
  const unsigned dy = sy * (unsigned)W;
  const float z00 = ld(I, o00), z01 = ld(I, o00 + sx);
  const float z10 = ld(I, o00 + dy), z11 = ld(I, o00 + dy + sx);
  const float t = fmaf(a, z01 - z00, z00);
  const float s = fmaf(a, z11 - z10, z10);
  return fmaf(b, s - t, t);
}

// Field value at in-image pixel (x, y) of the current level for the iteration's source.
// The source mode is a compile-time parameter so every kernel reads its field straight-line.
template <int MODE>
__device__ __forceinline__ void read_flow(const IterArgs& a, int x, int y, float& u, float& v) {
  if constexpr (MODE == kFlowSame) {
    const unsigned i = rowofs(y, a.W, x);
    u = at(a.uin, i);
    v = at(a.vin, i);
  } else if constexpr (MODE == kFlowCoarse) {
    // 2 * bilinear(coarse, x/2, y/2): base floor(x/2), fraction 0 or 1/2.
    const int x0 = x >> 1, y0 = y >> 1;
    const unsigned dx = x0 < a.Wc - 1 ? 1u : 0u;
    const unsigned dy = y0 < a.Hc - 1 ? (unsigned)a.Wc : 0u;
    const float fa = (x & 1) ? 0.5f : 0.f, fb = (y & 1) ? 0.5f : 0.f;
    const unsigned i00 = rowofs(y0, a.Wc, x0);
    const unsigned i01 = i00 + dx, i10 = i00 + dy, i11 = i00 + dy + dx;
    const float u00 = at(a.uin, i00), u01 = at(a.uin, i01), u10 = at(a.uin, i10), u11 = at(a.uin, i11);
    const float v00 = at(a.vin, i00), v01 = at(a.vin, i01), v10 = at(a.vin, i10), v11 = at(a.vin, i11);
    float t = fmaf(fa, u01 - u00, u00);
    float s = fmaf(fa, u11 - u10, u10);
    u = 2.f * fmaf(fb, s - t, t);
    t = fmaf(fa, v01 - v00, v00);
    s = fmaf(fa, v11 - v10, v10);
    v = 2.f * fmaf(fb, s - t, t);
  } else {
    u = 0.f;
    v = 0.f;
  }
}

// 1/x from the hardware reciprocal (1 ulp) refined by one Newton-Raphson step.
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
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
  // D > tau T^2 > 0 keeps the reciprocals finite.
  if (D > kTau * (T * T)) {
    const float inv = recip(D);
    du = -(fmaf(C, bx, -B * by)) * inv;
    dv = -(fmaf(A, by, -B * bx)) * inv;
  } else if (T > 0.f) {
    const float inv = recip(T * T);
    du = -(fmaf(A, bx, B * by)) * inv;
    dv = -(fmaf(B, bx, C * by)) * inv;
  }
  un = u + du;
  vn = v + dv;
}

}  // namespace ofmi
