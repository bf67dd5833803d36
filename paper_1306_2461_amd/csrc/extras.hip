// Steps around the flow: local equalisation of raw frames (Sec. 2.4, eq. 2 read as
// (I - local mean) / (local standard deviation + eps) over a (2r+1)^2 window truncated at the
// border) and the field statistics behind the recirculation-bubble surface (Sec. 3.2, eq. 3:
// running mean field, its extremes, and the count of vectors at or below a threshold).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ofmi.h"
#include "kernels.h"
#include "runtime.h"

namespace ofmi {

namespace {

constexpr int NTW = 64, NTH = 16;    // output tile of the normalisation kernel

// Window sums in FP64 (float frames; 8-bit frames take the integer kernel below), separable: the tile's input window is staged
// in LDS first (every load of a thread in flight together; pixels outside the image held as
// 0), then row sums of the tile's rows into LDS, then column sums per output pixel.  The sums
// run over the in-image pixels in ascending order, as a direct sum over the frame would.
constexpr int kNormRowsMax = NTH + 2 * OF_MAX_NORMALIZE_RADIUS;
constexpr int kNormColsMax = NTW + 2 * OF_MAX_NORMALIZE_RADIUS;

inline size_t normalize_lds_bytes(int r) {
  const size_t rows = NTH + 2 * (size_t)r, cols = NTW + 2 * (size_t)r;
  return 2 * sizeof(double) * rows * NTW + sizeof(float) * rows * cols;
}

template <typename T>
__global__ __launch_bounds__(256) void normalize_kernel(const T* __restrict__ in, float* __restrict__ out,
                                                        int H, int W, int r, float eps) {
  extern __shared__ double rs[];     // [rows * NTW] sums, the same of squares, then the window
  const int x0 = blockIdx.x * NTW, y0 = blockIdx.y * NTH;
  const int rows = NTH + 2 * r, cols = NTW + 2 * r;
  double* s1 = rs;
  double* s2 = rs + rows * NTW;
  float* win = reinterpret_cast<float*>(s2 + rows * NTW);   // [rows][cols] from (y0-r, x0-r)
  {
    constexpr int NL = (kNormRowsMax * kNormColsMax + 255) / 256;
    const int n = rows * cols;
    float v[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      if (256 * k >= n) break;   // uniform across the workgroup
      const int e = min((int)threadIdx.x + 256 * k, n - 1);
      const int ly = e / cols, lx = e - ly * cols;
      const int gy = y0 - r + ly, gx = x0 - r + lx;
      const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
      const unsigned o = (unsigned)min(max(gy, 0), H - 1) * (unsigned)W + (unsigned)min(max(gx, 0), W - 1);
      const float val = ld(in, o);
      v[k] = inside ? val : 0.f;
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      if (256 * k >= n) break;
      win[min((int)threadIdx.x + 256 * k, n - 1)] = v[k];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < rows * NTW; i += 256) {
    const int ly = i / NTW, lx = i - ly * NTW;
    const int gy = y0 - r + ly, gx = x0 + lx;
    double a = 0.0, b = 0.0;
    if (gy >= 0 && gy < H && gx < W) {
      const float* row = win + ly * cols;   // row[x - (x0 - r)] = frame value at column x
      const int xa = max(gx - r, 0), xb = min(gx + r, W - 1);
      for (int x = xa; x <= xb; ++x) {
        const double v = (double)row[x - (x0 - r)];
        a += v;
        b += v * v;
      }
    }
    s1[i] = a;
    s2[i] = b;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NTH * NTW; i += 256) {
    const int ly = i / NTW, lx = i - ly * NTW;
    const int gy = y0 + ly, gx = x0 + lx;
    if (gy >= H || gx >= W) continue;
    double a = 0.0, b = 0.0;
    for (int dy = 0; dy <= 2 * r; ++dy) {
      a += s1[(ly + dy) * NTW + lx];
      b += s2[(ly + dy) * NTW + lx];
    }
    const int nx = min(gx + r, W - 1) - max(gx - r, 0) + 1;
    const int ny = min(gy + r, H - 1) - max(gy - r, 0) + 1;
    const double n = (double)nx * ny;
    const double m = a / n, m2 = b / n;
    const double sd = sqrt(fmax(m2 - m * m, 0.0));
    const unsigned o = (unsigned)gy * (unsigned)W + (unsigned)gx;
    const double c = (double)win[(ly + r) * cols + lx + r];
    at(out, o) = (float)((c - m) / (sd + (double)eps));
  }
}

// 8-bit frames: the window sums of I and I^2 are integers below 2^31 (at most 33 x 33 x 255^2),
// so they are formed exactly in int32 as sliding sums (one addition and one subtraction per
// step instead of 2r+1 FP64 additions): the same values as the FP64 sums above, hence the
// same bits after the FP64 division and square root below.
constexpr int kSeg = 8;              // outputs per thread of a sliding row or column sum

inline size_t normalize_u8_lds_bytes(int r) {
  const size_t rows = NTH + 2 * (size_t)r, cols = NTW + 2 * (size_t)r;
  return sizeof(int) * (2 * rows * NTW + rows * cols);
}

__global__ __launch_bounds__(256) void normalize_u8_kernel(const uint8_t* __restrict__ in,
                                                           float* __restrict__ out, int H, int W,
                                                           int r, float eps) {
  extern __shared__ int ri[];        // [rows * NTW] sums of I, the same of I^2, then the window
  const int x0 = blockIdx.x * NTW, y0 = blockIdx.y * NTH;
  const int rows = NTH + 2 * r, cols = NTW + 2 * r;
  int* s1 = ri;
  int* s2 = ri + rows * NTW;
  int* win = s2 + rows * NTW;        // [rows][cols] from (y0-r, x0-r), 0 outside the image
  {
    constexpr int NL = (kNormRowsMax * kNormColsMax + 255) / 256;
    const int n = rows * cols;
    int v[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      if (256 * k >= n) break;   // uniform across the workgroup
      const int e = min((int)threadIdx.x + 256 * k, n - 1);
      const int ly = e / cols, lx = e - ly * cols;
      const int gy = y0 - r + ly, gx = x0 - r + lx;
      const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
      const unsigned o = (unsigned)min(max(gy, 0), H - 1) * (unsigned)W + (unsigned)min(max(gx, 0), W - 1);
      const int val = (int)at(in, o);
      v[k] = inside ? val : 0;
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      if (256 * k >= n) break;
      win[min((int)threadIdx.x + 256 * k, n - 1)] = v[k];
    }
  }
  __syncthreads();
  // row sums: output column lx covers window columns lx .. lx + 2r (pixels outside the image
  // are 0, which truncates the window at the border)
  for (int i = threadIdx.x; i < rows * (NTW / kSeg); i += 256) {
    const int ly = i / (NTW / kSeg), lx0 = (i - ly * (NTW / kSeg)) * kSeg;
    const int* row = win + ly * cols;
    int a = 0, b = 0;
    for (int x = lx0; x <= lx0 + 2 * r; ++x) {
      a += row[x];
      b += row[x] * row[x];
    }
    s1[ly * NTW + lx0] = a;
    s2[ly * NTW + lx0] = b;
#pragma unroll
    for (int j = 1; j < kSeg; ++j) {
      const int add = row[lx0 + j + 2 * r], sub = row[lx0 + j - 1];
      a += add - sub;
      b += add * add - sub * sub;
      s1[ly * NTW + lx0 + j] = a;
      s2[ly * NTW + lx0 + j] = b;
    }
  }
  __syncthreads();
  // column sums and the equalised value: thread (column, group of NTH/4 rows), sliding down
  constexpr int RG = NTH / 4;
  const int lx = threadIdx.x % NTW, ly0 = (threadIdx.x / NTW) * RG;
  const int gx = x0 + lx;
  int a = 0, b = 0;
  for (int dy = 0; dy <= 2 * r; ++dy) {
    a += s1[(ly0 + dy) * NTW + lx];
    b += s2[(ly0 + dy) * NTW + lx];
  }
  for (int j = 0; j < RG; ++j) {
    if (j > 0) {
      a += s1[(ly0 + j + 2 * r) * NTW + lx] - s1[(ly0 + j - 1) * NTW + lx];
      b += s2[(ly0 + j + 2 * r) * NTW + lx] - s2[(ly0 + j - 1) * NTW + lx];
    }
    const int gy = y0 + ly0 + j;
    if (gy >= H || gx >= W) continue;
    const int nx = min(gx + r, W - 1) - max(gx - r, 0) + 1;
    const int ny = min(gy + r, H - 1) - max(gy - r, 0) + 1;
    const double n = (double)nx * ny;
    const double m = (double)a / n, m2 = (double)b / n;
    const double sd = sqrt(fmax(m2 - m * m, 0.0));
    const double c = (double)win[(ly0 + j + r) * cols + lx + r];
    at(out, (unsigned)gy * (unsigned)W + (unsigned)gx) = (float)((c - m) / (sd + (double)eps));
  }
}

__global__ void mean_update_kernel(float* __restrict__ mean, const float* __restrict__ x,
                                   long long n, float inv) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    mean[i] = fmaf(x[i] - mean[i], inv, mean[i]);
}

__device__ __forceinline__ float wave_min(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Monotone map of a float onto unsigned ints (for atomic min/max on floats).
__device__ __forceinline__ unsigned ordered(float f) {
  const unsigned b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float unordered(unsigned u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__global__ void stats_init_kernel(unsigned* mm, unsigned long long* cnt) {
  if (threadIdx.x == 0) {
    if (mm) {
      mm[0] = 0xffffffffu;    // min
      mm[1] = 0u;             // max
    }
    if (cnt) *cnt = 0ull;
  }
}

__global__ __launch_bounds__(256) void minmax_kernel(const float* __restrict__ x, long long n,
                                                     unsigned* mm) {
  float lo = INFINITY, hi = -INFINITY;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    lo = fminf(lo, x[i]);
    hi = fmaxf(hi, x[i]);
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&mm[0], ordered(lo));
    atomicMax(&mm[1], ordered(hi));
  }
}

__global__ void minmax_finish_kernel(unsigned* mm, float* out) {
  if (threadIdx.x == 0) {
    out[0] = unordered(mm[0]);
    out[1] = unordered(mm[1]);
  }
}

__global__ __launch_bounds__(256) void count_kernel(const float* __restrict__ x, long long n,
                                                    float thr, unsigned long long* cnt) {
  unsigned long long c = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    c += x[i] <= thr ? 1ull : 0ull;
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(cnt, c);
}

__global__ __launch_bounds__(256) void count_dev_kernel(const float* __restrict__ x, long long n,
                                                        const float* __restrict__ thr,
                                                        unsigned long long* cnt) {
  const float t = *thr;
  unsigned long long c = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    c += x[i] <= t ? 1ull : 0ull;
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(cnt, c);
}

// eq. 3 step, device side only.  mean <- mean + (u - mean) / (t + 1) (t = 0: mean <- u) with
// the extremes of the new mean reduced into mm (ordered uints).
__global__ __launch_bounds__(256) void mean_minmax_kernel(float* __restrict__ mean,
                                                          const float* __restrict__ u, long long n,
                                                          float inv, int first, unsigned* mm) {
  float lo = INFINITY, hi = -INFINITY;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float m = first ? u[i] : fmaf(u[i] - mean[i], inv, mean[i]);
    mean[i] = m;
    lo = fminf(lo, m);
    hi = fmaxf(hi, m);
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&mm[0], ordered(lo));
    atomicMax(&mm[1], ordered(hi));
  }
}

// surface <- count / n (when `surface_first` is 0: before the threshold moves), threshold <-
// (min + max) / 2 of the new mean; the min/max work cells are reset for the next call.
__global__ void bubble_finish_kernel(unsigned* mm, float* thr, const unsigned long long* cnt,
                                     long long n, float* surface) {
  if (threadIdx.x == 0) {
    if (surface && cnt) *surface = (float)((double)*cnt / (double)n);
    *thr = 0.5f * (unordered(mm[0]) + unordered(mm[1]));
    mm[0] = 0xffffffffu;
    mm[1] = 0u;
  }
}

__global__ void bubble_surface_kernel(const unsigned long long* cnt, long long n, float* surface) {
  if (threadIdx.x == 0) *surface = (float)((double)*cnt / (double)n);
}

unsigned grid_for(long long n) {
  const long long b = (n + 255) / 256;
  return (unsigned)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

}  // namespace

hipError_t launch_count_at_most(const float* x, long long n, const float* thr,
                                unsigned long long* c, hipStream_t s) {
  hipLaunchKernelGGL(stats_init_kernel, dim3(1), dim3(64), 0, s, (unsigned*)nullptr, c);
  hipLaunchKernelGGL(count_dev_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, thr, c);
  return hipGetLastError();
}

hipError_t launch_normalize(Elem t, const void* in, float* out, int H, int W, int r, float eps,
                            hipStream_t s) {
  if (r < 0 || r > OF_MAX_NORMALIZE_RADIUS) return hipErrorInvalidValue;
  dim3 grid((W + NTW - 1) / NTW, (H + NTH - 1) / NTH);
  const size_t lds = normalize_lds_bytes(r);
  // Up to 67.5 KB at the largest radius: opt in to more than 64 KB of dynamic LDS, once.
  static const hipError_t opt32 = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&normalize_kernel<float>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)normalize_lds_bytes(OF_MAX_NORMALIZE_RADIUS));
  if (t == Elem::U8) {
    hipLaunchKernelGGL(normalize_u8_kernel, grid, dim3(256), normalize_u8_lds_bytes(r), s,
                       (const uint8_t*)in, out, H, W, r, eps);
  } else if (t == Elem::F32) {
    if (opt32 != hipSuccess) return opt32;
    hipLaunchKernelGGL(normalize_kernel<float>, grid, dim3(256), lds, s, (const float*)in, out, H,
                       W, r, eps);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ofmi

using namespace ofmi;

extern "C" {

of_status of_normalize(const void* in, float* out, int H, int W, int radius, float eps,
                       unsigned flags, void* stream) {
  if (!in || !out) return set_error("NULL plane"), OF_EINVAL;
  if (H < 1 || W < 1 || (long long)H * W >= (1ll << 30)) return set_error("bad size"), OF_EINVAL;
  if (radius < 0 || radius > OF_MAX_NORMALIZE_RADIUS) return set_error("radius out of range"), OF_EINVAL;
  if (!(eps >= 0.f)) return set_error("eps must be >= 0"), OF_EINVAL;
  if (flags & ~OF_FLAG_INPUT_F32) return set_error("unknown flags"), OF_EINVAL;
  if ((void*)out == in) return set_error("in and out must differ"), OF_EINVAL;
  hipError_t e = launch_normalize((flags & OF_FLAG_INPUT_F32) ? Elem::F32 : Elem::U8, in, out, H,
                                  W, radius, eps, (hipStream_t)stream);
  if (e != hipSuccess) return set_error(std::string("normalize: ") + hipGetErrorString(e)), OF_EHIP;
  return OF_OK;
}

of_status of_field_mean_update(float* mean, const float* x, long long n, int t, void* stream) {
  if (!mean || !x || n < 1 || t < 0) return set_error("bad argument"), OF_EINVAL;
  hipLaunchKernelGGL(mean_update_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     mean, x, n, 1.0f / (float)(t + 1));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(hipGetErrorString(e)), OF_EHIP;
  return OF_OK;
}

of_status of_field_minmax(const float* x, long long n, float* out2, void* work, void* stream) {
  if (!x || !out2 || !work || n < 1) return set_error("bad argument"), OF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned* mm = (unsigned*)work;
  hipLaunchKernelGGL(stats_init_kernel, dim3(1), dim3(64), 0, s, mm, (unsigned long long*)nullptr);
  hipLaunchKernelGGL(minmax_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, mm);
  hipLaunchKernelGGL(minmax_finish_kernel, dim3(1), dim3(64), 0, s, mm, out2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(hipGetErrorString(e)), OF_EHIP;
  return OF_OK;
}

of_status of_bubble_step(float* mean, const float* u, long long n, int t,
                         unsigned long long* count, float* threshold, float* surface, void* work,
                         void* stream) {
  if (!mean || !u || !count || !threshold || !surface || !work || n < 1 || t < 0)
    return set_error("bad argument"), OF_EINVAL;
  if (((uintptr_t)work & 3) || ((uintptr_t)count & 7)) return set_error("misaligned work or count"), OF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned* mm = (unsigned*)work;
  hipLaunchKernelGGL(stats_init_kernel, dim3(1), dim3(64), 0, s, mm, (unsigned long long*)nullptr);
  if (t > 0)   // count holds u <= the threshold in force while u was computed
    hipLaunchKernelGGL(bubble_surface_kernel, dim3(1), dim3(64), 0, s, count, n, surface);
  hipLaunchKernelGGL(mean_minmax_kernel, dim3(grid_for(n)), dim3(256), 0, s, mean, u, n,
                     1.0f / (float)(t + 1), t == 0 ? 1 : 0, mm);
  hipLaunchKernelGGL(bubble_finish_kernel, dim3(1), dim3(64), 0, s, mm, threshold,
                     (const unsigned long long*)nullptr, n, (float*)nullptr);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && t == 0) {   // the first field against its own threshold
    e = launch_count_at_most(u, n, threshold, count, s);
    if (e == hipSuccess) hipLaunchKernelGGL(bubble_surface_kernel, dim3(1), dim3(64), 0, s, count, n, surface);
    if (e == hipSuccess) e = hipGetLastError();
  }
  if (e != hipSuccess) return set_error(hipGetErrorString(e)), OF_EHIP;
  return OF_OK;
}

of_status of_count_at_most(const float* x, long long n, float threshold,
                           unsigned long long* count, void* stream) {
  if (!x || !count || n < 1) return set_error("bad argument"), OF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(stats_init_kernel, dim3(1), dim3(64), 0, s, (unsigned*)nullptr, count);
  hipLaunchKernelGGL(count_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, threshold, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(hipGetErrorString(e)), OF_EHIP;
  return OF_OK;
}

}  // extern "C"
