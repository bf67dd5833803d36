// Pyramid reduction: separable binomial [1 4 6 4 1]/16 blur (rows first, then columns),
// clamp-to-edge, keep even rows and columns (factor 4 in area per level, Sec. 2.4).
// Each row and column filter is the fused-multiply-add chain over the taps in order.
#include "kernels.h"

namespace ofmi {

namespace {

constexpr float kB0 = 1.f / 16.f, kB1 = 4.f / 16.f, kB2 = 6.f / 16.f;

// One output tile (kReduceTileW x kReduceTileH pixels of the coarser level) of one frame.
// The clamped input window of the tile (2*TW+3 columns, 2*TH+3 rows) is staged in LDS with
// row-contiguous loads; the row pass then filters the staged rows at the even columns, the
// column pass filters those results at the even rows.  Input elements are loaded once per
// tile instead of 25 times per output pixel.
constexpr int TW = kReduceTileW, TH = kReduceTileH;
constexpr int IW = 2 * TW + 3, IH = 2 * TH + 3;   // staged input window
constexpr int IWP = IW + 1;                        // its LDS row pitch

template <typename Tin, typename Tout>
__device__ __forceinline__ void reduce_tile(const Tin* __restrict__ in, int H, int W,
                                            Tout* __restrict__ out, int Ho, int Wo, int bx, int by,
                                            float* win, float* hrow) {
  const int i0 = by * TH, j0 = bx * TW;             // first output row / column
  const int r0 = 2 * i0 - 2, c0 = 2 * j0 - 2;       // first input row / column of the window
  // All of a thread's window loads in flight together (a load-then-store loop would wait for
  // each in turn); items past the end repeat the last element, same value to the same slot.
  constexpr int NL = (IH * IW + 255) / 256;
  float v[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int e = min((int)threadIdx.x + 256 * k, IH * IW - 1);
    const int ry = e / IW, rx = e - ry * IW;
    const int y = min(max(r0 + ry, 0), H - 1), x = min(max(c0 + rx, 0), W - 1);
    v[k] = ld(in, (unsigned)y * (unsigned)W + (unsigned)x);
  }
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int e = min((int)threadIdx.x + 256 * k, IH * IW - 1);
    const int ry = e / IW;
    win[ry * IWP + (e - ry * IW)] = v[k];
  }
  __syncthreads();
  // Row pass at the even columns 2j of every staged row.
  for (int e = threadIdx.x; e < IH * TW; e += 256) {
    const int ry = e / TW, q = e - ry * TW;
    const float* w = win + ry * IWP + 2 * q;
    float acc = kB0 * w[0];
    acc = fmaf(kB1, w[1], acc);
    acc = fmaf(kB2, w[2], acc);
    acc = fmaf(kB1, w[3], acc);
    acc = fmaf(kB0, w[4], acc);
    hrow[ry * TW + q] = acc;
  }
  __syncthreads();
  // Column pass at the even rows 2i.
  for (int e = threadIdx.x; e < TH * TW; e += 256) {
    const int p = e / TW, q = e - p * TW;
    const int i = i0 + p, j = j0 + q;
    if (i < Ho && j < Wo) {
      const float* h = hrow + 2 * p * TW + q;
      float acc = kB0 * h[0];
      acc = fmaf(kB1, h[TW], acc);
      acc = fmaf(kB2, h[2 * TW], acc);
      acc = fmaf(kB1, h[3 * TW], acc);
      acc = fmaf(kB0, h[4 * TW], acc);
      st(out, (unsigned)i * (unsigned)Wo + (unsigned)j, acc);
    }
  }
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void reduce_kernel(const Tin* __restrict__ in1,
                                                      const Tin* __restrict__ in2, int H, int W,
                                                      Tout* __restrict__ out1,
                                                      Tout* __restrict__ out2, int Ho, int Wo) {
  __shared__ float win[IH * IWP];
  __shared__ float hrow[IH * TW];
  reduce_tile<Tin, Tout>(blockIdx.z ? in2 : in1, H, W, blockIdx.z ? out2 : out1, Ho, Wo,
                         blockIdx.x, blockIdx.y, win, hrow);
}

// Direct form for small planes (latency bound: no staging barriers): one thread per output
// pixel reads its 5x5 input window itself.  Same arithmetic, in the same order, as
// reduce_tile, so both give identical bits.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void reduce_direct_kernel(const Tin* __restrict__ in1,
                                                             const Tin* __restrict__ in2, int H,
                                                             int W, Tout* __restrict__ out1,
                                                             Tout* __restrict__ out2, int Ho,
                                                             int Wo) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= Ho || j >= Wo) return;
  const Tin* in = blockIdx.z ? in2 : in1;
  Tout* out = blockIdx.z ? out2 : out1;
  unsigned cols[5];
#pragma unroll
  for (int b = 0; b < 5; ++b) cols[b] = (unsigned)min(max(2 * j + b - 2, 0), W - 1);
  float h[5];
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    const unsigned row = (unsigned)min(max(2 * i + a - 2, 0), H - 1) * (unsigned)W;
    float acc = kB0 * ld(in, row + cols[0]);
    acc = fmaf(kB1, ld(in, row + cols[1]), acc);
    acc = fmaf(kB2, ld(in, row + cols[2]), acc);
    acc = fmaf(kB1, ld(in, row + cols[3]), acc);
    acc = fmaf(kB0, ld(in, row + cols[4]), acc);
    h[a] = acc;
  }
  float acc = kB0 * h[0];
  acc = fmaf(kB1, h[1], acc);
  acc = fmaf(kB2, h[2], acc);
  acc = fmaf(kB1, h[3], acc);
  acc = fmaf(kB0, h[4], acc);
  st(out, (unsigned)i * (unsigned)Wo + (unsigned)j, acc);
}

// Batched reduction: workgroups stride over a list of (job, output tile) items.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void reduce_batch_kernel(const ReduceJob* __restrict__ jobs,
                                                            const int2* __restrict__ items,
                                                            int nitems) {
  __shared__ float win[IH * IWP];
  __shared__ float hrow[IH * TW];
  for (int t = blockIdx.x; t < nitems; t += gridDim.x) {
    const int2 it = items[t];
    const ReduceJob jb = jobs[it.x];
    const int bxn = (jb.Wo + TW - 1) / TW;
    reduce_tile<Tin, Tout>((const Tin*)jb.in, jb.H, jb.W, (Tout*)jb.out, jb.Ho, jb.Wo,
                           it.y % bxn, it.y / bxn, win, hrow);
    __syncthreads();
  }
}

template <typename Tin, typename Tout>
hipError_t go_batch(const ReduceJob* jobs, const int2* items, int nitems, int grid, hipStream_t s) {
  hipLaunchKernelGGL((reduce_batch_kernel<Tin, Tout>), dim3(grid), dim3(256), 0, s, jobs, items,
                     nitems);
  return hipGetLastError();
}

// Planes of up to 2^20 output pixels take the direct form (a single pair's pyramid step is
// latency bound), larger ones the staged form.
template <typename Tin, typename Tout>
hipError_t go(const void* in1, const void* in2, int H, int W, void* out1, void* out2, int Ho,
              int Wo, hipStream_t s) {
  if ((long long)Ho * Wo <= (1ll << 20)) {
    dim3 grid((Wo + 63) / 64, (Ho + 3) / 4, in2 ? 2 : 1);
    hipLaunchKernelGGL((reduce_direct_kernel<Tin, Tout>), grid, dim3(256), 0, s, (const Tin*)in1,
                       (const Tin*)in2, H, W, (Tout*)out1, (Tout*)out2, Ho, Wo);
  } else {
    dim3 grid((Wo + TW - 1) / TW, (Ho + TH - 1) / TH, in2 ? 2 : 1);
    hipLaunchKernelGGL((reduce_kernel<Tin, Tout>), grid, dim3(256), 0, s, (const Tin*)in1,
                       (const Tin*)in2, H, W, (Tout*)out1, (Tout*)out2, Ho, Wo);
  }
  return hipGetLastError();
}

// Fused reduction chain (one launch for D levels of one pair's pyramid, which is latency
// bound level by level).  A workgroup owns a T x T tile of the deepest level and rebuilds
// the tile's clamped footprint at every level of the chain in LDS: S_D = T rows and columns
// from o_D = (by T, bx T), and S_{d-1} = 2 S_d + 3 from o_{d-1} = 2 o_d - 2 at the level
// above.  Footprint entry k of a level holds that level's value at the clamped position
// clamp(o + k), so every value is computed exactly as reduce_tile computes it (row filter at
// the clamped columns, then column filter at the clamped rows, the same FMA chains), rounded
// to the storage type before the next level reads it: the chain gives the bits of D single
// reductions.  Each level's own part of the tile (T 2^(D-d) square, at footprint offset
// 2^(D-d+1) - 2) is written out.
constexpr int chain_span(int D, int T, int d) { return d >= D ? T : 2 * chain_span(D, T, d + 1) + 3; }

template <typename T>
__device__ __forceinline__ float stored(float x);
template <>
__device__ __forceinline__ float stored<float>(float x) { return x; }
template <>
__device__ __forceinline__ float stored<__half>(float x) { return __half2float(__float2half_rn(x)); }

// Level d of the chain from level d-1's footprint `src` (row pass into `fr`, column pass into
// `dst`); Hd x Wd is level d's size, (tyD, txD) the tile's origin at the deepest level.
template <typename Tout, int D, int T, int d, int NTH>
__device__ __forceinline__ void chain_level(const float* src, float* dst, float* fr, int Hd, int Wd,
                                            Tout* out, int tyD, int txD) {
  constexpr int Sp = chain_span(D, T, d - 1), Sd = chain_span(D, T, d);
  constexpr int k = D - d;
  // footprint origin at level d: o_d = 2^(D-d) o_D - 2^(D-d+1) + 2
  const int oyd = (tyD << k) - (2 << k) + 2, oxd = (txD << k) - (2 << k) + 2;
  // Row pass: every footprint row of level d-1 at the columns of level d's footprint.
  for (int e = threadIdx.x; e < Sp * Sd; e += NTH) {
    const int r = e / Sd, q = e - r * Sd;
    const int cx = min(max(oxd + q, 0), Wd - 1) - oxd;
    const float* w = src + r * Sp + 2 * cx;
    float acc = kB0 * w[0];
    acc = fmaf(kB1, w[1], acc);
    acc = fmaf(kB2, w[2], acc);
    acc = fmaf(kB1, w[3], acc);
    acc = fmaf(kB0, w[4], acc);
    fr[r * Sd + q] = acc;
  }
  __syncthreads();
  // Column pass at the rows of level d's footprint; the tile's own part goes out.
  constexpr int own0 = (2 << k) - 2, own = T << k;
  for (int e = threadIdx.x; e < Sd * Sd; e += NTH) {
    const int p = e / Sd, q = e - p * Sd;
    const int cy = min(max(oyd + p, 0), Hd - 1) - oyd;
    const float* h = fr + 2 * cy * Sd + q;
    float acc = kB0 * h[0];
    acc = fmaf(kB1, h[Sd], acc);
    acc = fmaf(kB2, h[2 * Sd], acc);
    acc = fmaf(kB1, h[3 * Sd], acc);
    acc = fmaf(kB0, h[4 * Sd], acc);
    dst[p * Sd + q] = stored<Tout>(acc);
    const int i = oyd + p, j = oxd + q;
    if (p >= own0 && p < own0 + own && q >= own0 && q < own0 + own && i < Hd && j < Wd)
      st(out, (unsigned)i * (unsigned)Wd + (unsigned)j, acc);
  }
  __syncthreads();
}

// NTH threads per workgroup: the chain is latency bound, so more threads per tile shorten
// every phase (fewer footprint entries per thread).
template <typename Tin, typename Tout, int D, int T, int NTH>
__global__ __launch_bounds__(NTH) void reduce_chain_kernel(ReduceChain a, int tiles_x) {
  constexpr int S0 = chain_span(D, T, 0), S1 = chain_span(D, T, 1);
  __shared__ float fa[S0 * S0];   // footprints of levels 0, 2
  __shared__ float fr[S0 * S1];   // row-pass results
  __shared__ float fb[S1 * S1];   // footprints of levels 1, 3
  const bool f2 = blockIdx.z != 0;
  const int by = blockIdx.x / tiles_x, bx = blockIdx.x - by * tiles_x;
  const int tyD = by * T, txD = bx * T;
  {
    const Tin* in = (const Tin*)(f2 ? a.in[1] : a.in[0]);
    const int H = a.H[0], W = a.W[0];
    const int oy0 = (tyD << D) - (2 << D) + 2, ox0 = (txD << D) - (2 << D) + 2;
    // All loads in flight together: items past the end repeat the last entry (same value to
    // the same slot), so neither loads nor stores need a guard.
    constexpr int NL = (S0 * S0 + NTH - 1) / NTH;
    float v[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int e = min((int)threadIdx.x + NTH * k, S0 * S0 - 1);
      const int ry = e / S0, rx = e - ry * S0;
      const int y = min(max(oy0 + ry, 0), H - 1), x = min(max(ox0 + rx, 0), W - 1);
      v[k] = ld(in, (unsigned)y * (unsigned)W + (unsigned)x);
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) fa[min((int)threadIdx.x + NTH * k, S0 * S0 - 1)] = v[k];
  }
  __syncthreads();
  chain_level<Tout, D, T, 1, NTH>(fa, fb, fr, a.H[1], a.W[1], (Tout*)(f2 ? a.out[1][0] : a.out[0][0]),
                             tyD, txD);
  chain_level<Tout, D, T, 2, NTH>(fb, fa, fr, a.H[2], a.W[2], (Tout*)(f2 ? a.out[1][1] : a.out[0][1]),
                             tyD, txD);
  if constexpr (D == 3)
    chain_level<Tout, D, T, 3, NTH>(fa, fb, fr, a.H[3], a.W[3], (Tout*)(f2 ? a.out[1][2] : a.out[0][2]),
                               tyD, txD);
}

constexpr int kChainThreads = 1024;

template <typename Tin, typename Tout>
hipError_t go_chain(const ReduceChain& c, hipStream_t s) {
  const int nf = c.in[1] ? 2 : 1;
  constexpr int NTH = kChainThreads;
  if (c.D == 2) {
    constexpr int T = 16;
    const int tx = (c.W[2] + T - 1) / T, ty = (c.H[2] + T - 1) / T;
    hipLaunchKernelGGL((reduce_chain_kernel<Tin, Tout, 2, T, NTH>), dim3(tx * ty, 1, nf),
                       dim3(NTH), 0, s, c, tx);
  } else if (c.D == 3) {
    constexpr int T = 8;
    const int tx = (c.W[3] + T - 1) / T, ty = (c.H[3] + T - 1) / T;
    hipLaunchKernelGGL((reduce_chain_kernel<Tin, Tout, 3, T, NTH>), dim3(tx * ty, 1, nf),
                       dim3(NTH), 0, s, c, tx);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Mask pyramid: a coarse pixel is unmasked when any of its (up to) four finer pixels is.
__global__ __launch_bounds__(256) void mask_reduce_kernel(const uint8_t* __restrict__ in, int H,
                                                           int W, uint8_t* __restrict__ out,
                                                           int Ho, int Wo) {
  const long long n = (long long)Ho * Wo;
  for (long long e = blockIdx.x * 256ll + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    const int i = (int)(e / Wo), j = (int)(e - (long long)i * Wo);
    const unsigned r0 = (unsigned)(2 * i) * (unsigned)W, r1 = (unsigned)min(2 * i + 1, H - 1) * (unsigned)W;
    const unsigned c0 = (unsigned)(2 * j), c1 = (unsigned)min(2 * j + 1, W - 1);
    const bool on = at(in, r0 + c0) | at(in, r0 + c1) | at(in, r1 + c0) | at(in, r1 + c1);
    at(out, (unsigned)e) = on ? 1 : 0;
  }
}

}  // namespace

hipError_t launch_mask_reduce(const uint8_t* in, int H, int W, uint8_t* out, int Ho, int Wo,
                              hipStream_t s) {
  const long long n = (long long)Ho * Wo;
  const long long blocks = (n + 255) / 256;
  hipLaunchKernelGGL(mask_reduce_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)),
                     dim3(256), 0, s, in, H, W, out, Ho, Wo);
  return hipGetLastError();
}

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

hipError_t launch_reduce_chain(Elem tin, Elem tout, const ReduceChain& c, hipStream_t s) {
  if (tout == Elem::F32) {
    if (tin == Elem::U8) return go_chain<uint8_t, float>(c, s);
    if (tin == Elem::F32) return go_chain<float, float>(c, s);
  } else if (tout == Elem::F16) {
    if (tin == Elem::U8) return go_chain<uint8_t, __half>(c, s);
    if (tin == Elem::F32) return go_chain<float, __half>(c, s);
    if (tin == Elem::F16) return go_chain<__half, __half>(c, s);
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
