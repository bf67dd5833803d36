// Host-side launchers of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "common.h"

namespace ofmi {

enum class Elem : int { U8 = 0, F32 = 1, F16 = 2 };

inline size_t elem_bytes(Elem e) { return e == Elem::U8 ? 1 : (e == Elem::F16 ? 2 : 4); }

// One plane reduction job of a batched pyramid step.
struct ReduceJob {
  const void* in;
  void* out;
  int H, W, Ho, Wo;
};

// Output tile of the pyramid reduction kernels (columns x rows of the coarser level).
constexpr int kReduceTileW = 64, kReduceTileH = 16;
inline int reduce_blocks(int Ho, int Wo) {
  return ((Wo + kReduceTileW - 1) / kReduceTileW) * ((Ho + kReduceTileH - 1) / kReduceTileH);
}

// Batched pyramid step over (job, output tile) work items.
hipError_t launch_reduce_batch(Elem tin, Elem tout, const ReduceJob* jobs, const int2* items,
                               int nitems, int grid, hipStream_t s);

// Mask pyramid step: out(i, j) = 1 if any of in(2i..2i+1, 2j..2j+1) (clamped) is nonzero.
hipError_t launch_mask_reduce(const uint8_t* in, int H, int W, uint8_t* out, int Ho, int Wo,
                              hipStream_t s);

// D = 2 or 3 successive pyramid reductions of up to two frames in one launch (levels f+1 ..
// f+D from level f; in[1] null for one frame): sizes H[0..D], W[0..D] of levels f .. f+D,
// out[frame][d-1] = level f+d.  Same bits as D launch_reduce calls.
struct ReduceChain {
  const void* in[2];
  void* out[2][3];
  int H[4], W[4];
  int D;
};
hipError_t launch_reduce_chain(Elem tin, Elem tout, const ReduceChain& c, hipStream_t s);

// One pyramid reduction of up to two frames of the same geometry (out = reduce(in)).
hipError_t launch_reduce(Elem tin, Elem tout, const void* in1, const void* in2, int H, int W,
                         void* out1, void* out2, int Ho, int Wo, hipStream_t s);

// Tile variants of the iteration kernel:
//   narrow     5 threads per output column, item indices recomputed every band;
//   wide       10 threads per output column, item indices kept in registers (shortest
//              dependent path per band: launches with about one tile per CU);
//   wide lean  10 threads per output column, indices recomputed every band (fewer live
//              registers, so more resident workgroups: launches with many tiles).
//   wide 32 /  the wide variant on strips of 32 or 16 output columns (plain launches of the
//   wide 16    box window): small levels spread over more CUs, fewer waves per SIMD per tile,
//              hence a shorter path per band where a level has fewer tiles than CUs.
//   wide 32x2 / the same strips with two bands per pass and 20 threads per output column
//   wide 16x2   (plain launches of the box window, r <= kMaxPairRadius): a tile of one output
//              band runs its priming band and its output band together, one dependent path.
//   lean 32x2   wide 32x2 with the item indices recomputed every pass (as wide lean): fewer
//              live registers, so several workgroups share a CU (levels with more tiles).
enum TileVariant : int { kTileNarrow = 0, kTileWide = 1, kTileWideLean = 2, kTileWide32 = 3,
                         kTileWide16 = 4, kTileWide32x2 = 5, kTileWide16x2 = 6, kTileLean32x2 = 7 };
constexpr int kTileVariants = 8;
// Largest window radius of the two-bands-per-pass variants (their LDS stays within 64 KB).
constexpr int kMaxPairRadius = 8;
// Added to a plain launch's variant: Gaussian-weighted window sums (taps in IterArgs::taps).
constexpr int kTileGauss = 16;

// Batched iteration launch: `grid` workgroups stride over `ntiles` work items (pair | tile
// flag << 16, tile x, first output row, output rows) with per-pair arguments args[pair]
// (device arrays); the flag (0 no unmasked pixel, 1 some masked pixels, 2 none) is read for
// pairs with a mask.
struct BatchLaunch {
  const IterArgs* args;
  const int4* tiles;
  int ntiles;
  int grid;
  int variant;   // TileVariant (narrow, wide, wide lean), plus kTileGauss for the Gaussian window
  bool masked;   // some pair of the launch has a mask (IterArgs::mask)
  // Load the kernel this launch would run on the current device, without launching it (a
  // kernel's first launch loads its code: milliseconds that a latency-bound caller primes
  // ahead instead of paying on a request).
  bool prime = false;
};

// Strip width (output columns per tile) of the iteration kernel for radius R (variants 0-2).
int strip_width_for(int R);
// Strip width of a plain launch's tile variant.
inline int tile_width(int variant, int R) {
  if (variant == kTileWide32 || variant == kTileWide32x2 || variant == kTileLean32x2) return 32;
  if (variant == kTileWide16 || variant == kTileWide16x2) return 16;
  return strip_width_for(R);
}
// Whether a plain launch of radius R (Gaussian-weighted window or not) has tile variant
// `variant`: narrow strips only with the box window, two bands per pass only up to
// kMaxPairRadius.
inline bool tile_variant_valid(int variant, int R, bool gaussian) {
  if (variant < kTileNarrow || variant >= kTileVariants) return false;
  if (gaussian && variant > kTileWideLean) return false;
  if ((variant == kTileWide32x2 || variant == kTileWide16x2 || variant == kTileLean32x2) &&
      R > kMaxPairRadius)
    return false;
  return true;
}

// One fused Gauss-Newton iteration at one level (frames of element type `t`), tiles of height
// (2R+1)*nb, tile variant `variant` (TileVariant).
hipError_t launch_iter(Elem t, const IterArgs& a, int R, int nb, int variant, hipStream_t s);

// The same over a work list of many pairs' tiles at one (level, iteration) phase.
hipError_t launch_iter_batch(Elem t, const BatchLaunch& b, int R, int mode, hipStream_t s);

// Local equalisation of one frame (uint8 or float32 in, float32 out).
hipError_t launch_normalize(Elem t, const void* in, float* out, int H, int W, int r, float eps,
                            hipStream_t s);

// u = v = 0 over n elements (a fill kernel, safe under stream capture).
hipError_t launch_zero(float* u, float* v, size_t n, hipStream_t s);
// Zero flow over a work list of tiles (batch work items: pair in the low 16 bits of x, tile x,
// first row, rows; tw columns wide) into the output planes of args[pair] (tw divides 256).
hipError_t launch_zero_tiles(const IterArgs* args, const int4* tiles, int ntiles, int tw,
                             hipStream_t s);
// Loads the zero-tiles kernel's code on the current device (no launch).
hipError_t prime_zero_tiles();
// Copy of `bytes` bytes by a kernel on stream s (device memory, or pinned host memory through
// its device mapping).
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// *c = 0 (a one-thread kernel, safe under stream capture).
hipError_t launch_zero_count(unsigned long long* c, hipStream_t s);

// *c = number of x[i] <= *thr over n elements (the threshold read on the device).
hipError_t launch_count_at_most(const float* x, long long n, const float* thr,
                                unsigned long long* c, hipStream_t s);

}  // namespace ofmi
