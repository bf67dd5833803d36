// Pyramid reduction: separable binomial [1 4 6 4 1]/16 blur (rows first, then columns),
// clamp-to-edge, keep even rows and columns (factor 4 in area per level, Sec. 2.4).
#include "kernels.h"

namespace ofmi {

namespace {

constexpr float kB0 = 1.f / 16.f, kB1 = 4.f / 16.f, kB2 = 6.f / 16.f;

template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void reduce_kernel(const Tin* __restrict__ in1,
                                                      const Tin* __restrict__ in2, int H, int W,
                                                      Tout* __restrict__ out1,
                                                      Tout* __restrict__ out2, int Ho, int Wo) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= Ho || j >= Wo) return;
  const Tin* in = blockIdx.z ? in2 : in1;
  Tout* out = blockIdx.z ? out2 : out1;
  const float k[5] = {kB0, kB1, kB2, kB1, kB0};
  unsigned rows[5];
#pragma unroll
  for (int a = 0; a < 5; ++a) rows[a] = (unsigned)min(max(2 * i + a - 2, 0), H - 1) * (unsigned)W;
  float acc = 0.f;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    const unsigned xx = (unsigned)min(max(2 * j + b - 2, 0), W - 1);
    float col = 0.f;
#pragma unroll
    for (int a = 0; a < 5; ++a) col = fmaf(k[a], ld(in, rows[a] + xx), col);
    acc = fmaf(k[b], col, acc);
  }
  st(out, (unsigned)i * (unsigned)Wo + (unsigned)j, acc);
}

// Batched reduction: workgroups stride over a list of (job, block) items; a block is 64x4
// output pixels of one job's output plane.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void reduce_batch_kernel(const ReduceJob* __restrict__ jobs,
                                                            const int2* __restrict__ items,
                                                            int nitems) {
  const float k[5] = {kB0, kB1, kB2, kB1, kB0};
  for (int t = blockIdx.x; t < nitems; t += gridDim.x) {
    const int2 it = items[t];
    const ReduceJob jb = jobs[it.x];
    const int bxn = (jb.Wo + 63) / 64;
    const int j = (it.y % bxn) * 64 + (threadIdx.x & 63);
    const int i = (it.y / bxn) * 4 + (threadIdx.x >> 6);
    if (i >= jb.Ho || j >= jb.Wo) continue;
    const Tin* in = (const Tin*)jb.in;
    unsigned rows[5];
#pragma unroll
    for (int a = 0; a < 5; ++a)
      rows[a] = (unsigned)min(max(2 * i + a - 2, 0), jb.H - 1) * (unsigned)jb.W;
    float acc = 0.f;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const unsigned xx = (unsigned)min(max(2 * j + b - 2, 0), jb.W - 1);
      float col = 0.f;
#pragma unroll
      for (int a = 0; a < 5; ++a) col = fmaf(k[a], ld(in, rows[a] + xx), col);
      acc = fmaf(k[b], col, acc);
    }
    st((Tout*)jb.out, (unsigned)i * (unsigned)jb.Wo + (unsigned)j, acc);
  }
}

template <typename Tin, typename Tout>
hipError_t go_batch(const ReduceJob* jobs, const int2* items, int nitems, int grid, hipStream_t s) {
  hipLaunchKernelGGL((reduce_batch_kernel<Tin, Tout>), dim3(grid), dim3(256), 0, s, jobs, items,
                     nitems);
  return hipGetLastError();
}

template <typename Tin, typename Tout>
hipError_t go(const void* in1, const void* in2, int H, int W, void* out1, void* out2, int Ho,
              int Wo, hipStream_t s) {
  dim3 grid((Wo + 63) / 64, (Ho + 3) / 4, in2 ? 2 : 1);
  hipLaunchKernelGGL((reduce_kernel<Tin, Tout>), grid, dim3(256), 0, s, (const Tin*)in1,
                     (const Tin*)in2, H, W, (Tout*)out1, (Tout*)out2, Ho, Wo);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_reduce_batch(Elem tin, Elem tout, const ReduceJob* jobs, const int2* items,
                               int nitems, int grid, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (tout == Elem::F32) {
    if (tin == Elem::U8) return go_batch<uint8_t, float>(jobs, items, nitems, grid, s);
    if (tin == Elem::F32) return go_batch<float, float>(jobs, items, nitems, grid, s);
  } else if (tout == Elem::F16) {
    if (tin == Elem::U8) return go_batch<uint8_t, __half>(jobs, items, nitems, grid, s);
    if (tin == Elem::F32) return go_batch<float, __half>(jobs, items, nitems, grid, s);
    if (tin == Elem::F16) return go_batch<__half, __half>(jobs, items, nitems, grid, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(Elem tin, Elem tout, const void* in1, const void* in2, int H, int W,
                         void* out1, void* out2, int Ho, int Wo, hipStream_t s) {
  if (tout == Elem::F32) {
    if (tin == Elem::U8) return go<uint8_t, float>(in1, in2, H, W, out1, out2, Ho, Wo, s);
    if (tin == Elem::F32) return go<float, float>(in1, in2, H, W, out1, out2, Ho, Wo, s);
  } else if (tout == Elem::F16) {
    if (tin == Elem::U8) return go<uint8_t, __half>(in1, in2, H, W, out1, out2, Ho, Wo, s);
    if (tin == Elem::F32) return go<float, __half>(in1, in2, H, W, out1, out2, Ho, Wo, s);
    if (tin == Elem::F16) return go<__half, __half>(in1, in2, H, W, out1, out2, Ho, Wo, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace ofmi
