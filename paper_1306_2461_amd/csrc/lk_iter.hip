// Dispatch of the fused iteration kernel by frame element type, and the zero fill.
#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace ofmi {

hipError_t launch_iter_u8(const IterArgs* a, const BatchLaunch* b, int R, int mode, int nb,
                          int variant, hipStream_t s);
hipError_t launch_iter_f32(const IterArgs* a, const BatchLaunch* b, int R, int mode, int nb,
                          int variant, hipStream_t s);
hipError_t launch_iter_f16(const IterArgs* a, const BatchLaunch* b, int R, int mode, int nb,
                          int variant, hipStream_t s);

int strip_width_for(int R) {
  // Mirrors strip_width<R>(): the LDS footprint of 64-column strips stays within 64 KB for
  // every supported radius (0..12).
  (void)R;
  return 64;
}

namespace {

__global__ void zero_kernel(float* u, float* v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    u[i] = 0.f;
    v[i] = 0.f;
  }
}

// Zero flow over listed tiles of many pairs (batch work items: pair in the low 16 bits of x,
// tile x, first row, rows; tiles TW columns wide), written into each pair's output planes of
// its arguments.  One workgroup per tile at a time, TW-column rows (TW divides the workgroup
// size).
__global__ __launch_bounds__(256) void zero_tiles_kernel(const IterArgs* __restrict__ args,
                                                         const int4* __restrict__ tiles,
                                                         int ntiles, int tw) {
  const int c = (int)threadIdx.x % tw, rstep = (int)blockDim.x / tw;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int4 w = tiles[t];
    const int p = w.x & 0xffff;
    float* __restrict__ u = args[p].uout;
    float* __restrict__ v = args[p].vout;
    const int W = args[p].W, H = args[p].H;
    const int x = w.y * tw + c, y0 = w.z, y1 = min(H, y0 + w.w);
    if (x >= W) continue;
    for (int y = y0 + (int)threadIdx.x / tw; y < y1; y += rstep) {
      const size_t o = (size_t)y * W + x;
      u[o] = 0.f;
      v[o] = 0.f;
    }
  }
}

// dst[0..bytes) = src[0..bytes): 16-byte words when both are 16-byte aligned, then the tail.
__global__ void copy_kernel(char* __restrict__ dst, const char* __restrict__ src, size_t bytes) {
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t done = 0;
  if ((((uintptr_t)dst | (uintptr_t)src) & 15) == 0) {
    const size_t n16 = bytes / 16;
    for (size_t i = tid; i < n16; i += stride)
      reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
    done = n16 * 16;
  }
  for (size_t i = done + tid; i < bytes; i += stride) dst[i] = src[i];
}

}  // namespace

hipError_t launch_zero_tiles(const IterArgs* args, const int4* tiles, int ntiles, int tw,
                             hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (tw < 1 || tw > 256 || 256 % tw != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(zero_tiles_kernel, dim3(std::min(ntiles, 4096)), dim3(256), 0, s, args, tiles,
                     ntiles, tw);
  return hipGetLastError();
}

hipError_t prime_zero_tiles() {
  hipFuncAttributes attr;
  return hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&zero_tiles_kernel));
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const size_t words = (bytes + 15) / 16;
  const unsigned grid = (unsigned)std::min<size_t>((words + 255) / 256, 1024);
  hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, s, (char*)dst, (const char*)src, bytes);
  return hipGetLastError();
}

hipError_t launch_iter(Elem t, const IterArgs& a, int R, int nb, int variant, hipStream_t s) {
  switch (t) {
    case Elem::U8: return launch_iter_u8(&a, nullptr, R, a.mode, nb, variant, s);
    case Elem::F32: return launch_iter_f32(&a, nullptr, R, a.mode, nb, variant, s);
    case Elem::F16: return launch_iter_f16(&a, nullptr, R, a.mode, nb, variant, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_iter_batch(Elem t, const BatchLaunch& b, int R, int mode, hipStream_t s) {
  if (b.ntiles <= 0) return hipSuccess;
  switch (t) {
    case Elem::U8: return launch_iter_u8(nullptr, &b, R, mode, 0, b.variant, s);
    case Elem::F32: return launch_iter_f32(nullptr, &b, R, mode, 0, b.variant, s);
    case Elem::F16: return launch_iter_f16(nullptr, &b, R, mode, 0, b.variant, s);
  }
  return hipErrorInvalidValue;
}

namespace {
__global__ void zero_count_kernel(unsigned long long* c) {
  if (threadIdx.x == 0) *c = 0ull;
}
}  // namespace

hipError_t launch_zero_count(unsigned long long* c, hipStream_t s) {
  hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(64), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_zero(float* u, float* v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0,
                     s, u, v, n);
  return hipGetLastError();
}

}  // namespace ofmi
