// One fused Gauss-Newton iteration of the dense window-based Lucas-Kanade method at one
// pyramid level (Sec. 2.4): warp of frame 2 by the current field, central-difference
// gradients of the warped frame, the five window sums, the 2x2 solve and the update.
//
// A workgroup owns a TW x TH tile of output pixels.  It stages in LDS the warped frame over
// the tile grown by r + 1 px, then the five products over the tile grown by r px, then
// row sums of the products, and finishes with column sums and the per-pixel solve.
#include "kernels.h"

namespace ofmi {

namespace {

constexpr int TW = 16, TH = 16, NT = TW * TH;

template <typename T>
__global__ __launch_bounds__(NT) void lk_iter_tile(IterArgs a, int R) {
  extern __shared__ float sm[];
  const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH;
  const int PW = TW + 2 * R, PH = TH + 2 * R;   // product region
  const int WW = PW + 2, WH = PH + 2;           // warped-frame region
  float* w2 = sm;
  float* pr = w2 + WW * WH;                      // 5 planes PH x PW
  float* rs = pr + 5 * PW * PH;                  // 5 planes PH x TW
  const int tid = threadIdx.x;
  const int H = a.H, W = a.W;
  const T* I1 = (const T*)a.I1;
  const T* I2 = (const T*)a.I2;

  // Warped frame; positions outside the image hold the clamped neighbour's value, which is
  // exactly what the clamped central difference needs.
  for (int i = tid; i < WW * WH; i += NT) {
    const int ly = i / WW, lx = i - ly * WW;
    const int gx = min(max(x0 - R - 1 + lx, 0), W - 1);
    const int gy = min(max(y0 - R - 1 + ly, 0), H - 1);
    float u, v;
    read_flow(a, gx, gy, u, v);
    w2[i] = warp_sample(I2, H, W, gx, gy, u, v);
  }
  __syncthreads();

  // Products; zero outside the image (truncated window).
  const int PP = PW * PH;
  for (int i = tid; i < PP; i += NT) {
    const int ly = i / PW, lx = i - ly * PW;
    const int gx = x0 - R + lx, gy = y0 - R + ly;
    float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f, p4 = 0.f;
    if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
      const int c = (ly + 1) * WW + lx + 1;
      const float ix = 0.5f * (w2[c + 1] - w2[c - 1]);
      const float iy = 0.5f * (w2[c + WW] - w2[c - WW]);
      float u, v;
      read_flow(a, gx, gy, u, v);
      float it = w2[c] - ld(I1, gy * W + gx);
      it = fmaf(-ix, u, it);
      it = fmaf(-iy, v, it);
      p0 = ix * ix;
      p1 = ix * iy;
      p2 = iy * iy;
      p3 = ix * it;
      p4 = iy * it;
    }
    pr[i] = p0;
    pr[PP + i] = p1;
    pr[2 * PP + i] = p2;
    pr[3 * PP + i] = p3;
    pr[4 * PP + i] = p4;
  }
  __syncthreads();

  // Row sums over dx for the TW output columns.
  const int RP = PH * TW;
  for (int i = tid; i < RP; i += NT) {
    const int ly = i / TW, lx = i - ly * TW;
    const int base = ly * PW + lx;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      float s = 0.f;
      for (int dx = 0; dx <= 2 * R; ++dx) s += pr[k * PP + base + dx];
      rs[k * RP + i] = s;
    }
  }
  __syncthreads();

  // Column sums over dy, solve, update.
  const int lx = tid % TW, ly = tid / TW;
  const int gx = x0 + lx, gy = y0 + ly;
  if (gx < W && gy < H) {
    float S[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      float s = 0.f;
      for (int dy = 0; dy <= 2 * R; ++dy) s += rs[k * RP + (ly + dy) * TW + lx];
      S[k] = s;
    }
    float u, v, un, vn;
    read_flow(a, gx, gy, u, v);
    solve_update(S[0], S[1], S[2], S[3], S[4], u, v, un, vn);
    a.uout[gy * W + gx] = un;
    a.vout[gy * W + gx] = vn;
  }
}

template <typename T>
hipError_t go(const IterArgs& a, int R, hipStream_t s) {
  const int PW = TW + 2 * R, PH = TH + 2 * R;
  const size_t lds = sizeof(float) * ((size_t)(PW + 2) * (PH + 2) + 5 * PW * PH + 5 * PH * TW);
  dim3 grid((a.W + TW - 1) / TW, (a.H + TH - 1) / TH);
  hipLaunchKernelGGL(lk_iter_tile<T>, grid, dim3(NT), lds, s, a, R);
  return hipGetLastError();
}

__global__ void zero_kernel(float* u, float* v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    u[i] = 0.f;
    v[i] = 0.f;
  }
}

}  // namespace

hipError_t launch_iter(Elem t, const IterArgs& a, int R, hipStream_t s) {
  switch (t) {
    case Elem::U8: return go<uint8_t>(a, R, s);
    case Elem::F32: return go<float>(a, R, s);
    case Elem::F16: return go<__half>(a, R, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_zero(float* u, float* v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0,
                     s, u, v, n);
  return hipGetLastError();
}

}  // namespace ofmi
