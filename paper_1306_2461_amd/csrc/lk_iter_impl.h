// One fused Gauss-Newton iteration of the dense window-based Lucas-Kanade method at one
// pyramid level (Sec. 2.4): warp of frame 2 by the current field, central-difference
// gradients of the warped frame, the five window sums, the 2x2 solve and the update.
//
// Work decomposition (gfx950, wave64):
//   * a workgroup of 5*TW threads (narrow) or at least 10*TW threads (wide, rounded up so the
//     warped-frame positions of a band take few rounds per thread) owns a strip of TW output
//     columns and TH output rows;
//   * it walks down the strip in bands of N = 2r+1 product rows; per band:
//       P1  warped frame for the band's new rows into an LDS ring; all global loads of the
//           band (field, frame 1, centre field of the band's outputs) are issued here;
//       P2  the five products Ix^2, IxIy, Iy^2, Ix It, Iy It of the band's rows into LDS;
//       P3  horizontal window sums: one thread per (channel, row, 8-column segment); every
//           window of a segment holds one common column, so each window is a suffix sum plus
//           a prefix sum of its own values (no subtraction of values leaving the window);
//           r <= 3 takes direct sums (segments sit on multiples of 8 of the level's columns);
//           the Gaussian-weighted window takes a direct weighted sum per output instead;
//       P4  vertical window sums: one thread per (channel, column) holds the previous
//           band's horizontal sums in registers; the window of the band's row i is the
//           suffix sum of the previous band from row i+1 plus the prefix sum of the current
//           band up to row i (fixed order; bands sit on a global grid of period N), or the
//           direct weighted sum over the same rows for the Gaussian-weighted window;
//       P5  per-pixel 2x2 solve and update for the band's output rows.
//   The window sums therefore do not depend on how the image is cut into tiles.
//   * two-bands-per-pass variants run the five phases once over two bands' rows with twice
//     the threads (20*TW), so a one-band tile (output band plus priming band) is one trip;
//   * coarse-field launches of the wide one-band variants keep the interpolated field of the
//     warped-frame positions in an LDS ring for P2 and P5.
#pragma once

#include "kernels.h"

namespace ofmi {

namespace {

// Adds every lane's count to *dst: a wave sum, then one atomic per wave.
__device__ __forceinline__ void add_count(unsigned long long* dst, unsigned c) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(dst, (unsigned long long)c);
}

// Threads per workgroup.  Narrow variants: 5 per output column.  Wide variants: at least 10
// per column, and enough that the warped-frame positions of a steady pass (every pass but a
// tile's first, which also samples the two rows above) take the fewest rounds of items per
// thread that a workgroup of at most 1024 allows, rounded up to whole groups of four waves (one
// per SIMD of the CU): e.g. r = 8 on 64-column strips samples 17 x 82 positions per band, 3
// rounds at 640 threads (73 % of the lanes busy) and 2 at 768; on 32-column strips 17 x 50
// positions, one round at 1024.
template <int R, int TW, bool WIDE, int BB>
constexpr int group_threads() {
  if (!WIDE) return 5 * TW * BB;
  const int N = 2 * R + 1, WC = TW + 2 * R + 2;
  const int items = (BB == 1 ? N : BB * N + 2) * WC;
  const int base = 10 * TW * BB;
  const int k = (items + 1023) / 1024;
  int nt = ((items + k - 1) / k + 255) / 256 * 256;
  if (nt < base) nt = base;
  if (nt > 1024) nt = base;
  return nt;
}

template <int R, int TW_, bool WIDE = false, int BB = 1>
struct Cfg {
  static constexpr int N = 2 * R + 1;                 // band height = window height
  static constexpr int NR = BB * N;                   // product rows per pass (BB bands)
  static constexpr int TW = TW_;                      // output columns per strip
  static constexpr int NT = group_threads<R, TW_, WIDE, BB>();   // threads per workgroup
  static constexpr int PC = TW + 2 * R;               // product columns
  static constexpr int WC = PC + 2;                   // warped-frame columns
  static constexpr int HL = 8 + 2 * R;                // products read per horizontal segment
  static constexpr int HL4 = (HL + 3) / 4;            // ... in float4 units
  static constexpr int PP = ((TW + 4 * HL4 - 8) + 3) / 4 * 4 + 4;  // product row pitch
  static constexpr int WP = WC + 1;                   // warped-frame row pitch
  // Warped-frame rows held in LDS: one band per pass keeps a power-of-two ring (the two rows
  // shared with the next band stay); two bands per pass sample all NR + 2 rows every pass.
  static constexpr int RING = N + 2 <= 16 ? 16 : 32;
  static constexpr int WROWS = BB == 1 ? RING : NR + 2;
  static constexpr int NSEG = TW / 8;
  static constexpr int P1_ROWS_MAX = NR + 2;
  static constexpr int K1 = (P1_ROWS_MAX * WC + NT - 1) / NT;   // P1 items per thread
  // ... in a pass after a tile's first (one band per pass: N new rows)
  static constexpr int K1S = ((BB == 1 ? N : P1_ROWS_MAX) * WC + NT - 1) / NT;
  static constexpr int K2 = (NR * PC + NT - 1) / NT;            // P2 items per thread
  static constexpr int K3 = (5 * NR * NSEG + NT - 1) / NT;      // P3 items per thread
  static constexpr int K5 = (NR * TW + NT - 1) / NT;            // P5 items per thread
  // The window sums [5][NR][TW] reuse the product buffer [5][NR][PP] once P3 has read it, or
  // (SPLIT) have a region of their own after the warped rows, which saves P3's second barrier.
  static constexpr size_t LDS_FLOATS = 5 * (size_t)NR * PP + (size_t)WROWS * WP;
  static constexpr size_t HS_FLOATS = 5 * (size_t)NR * TW;
  // Field ring (launches that read a field, one band per pass): u and v of the warped-frame
  // positions, kept for FRING rows so that P2 and P5 read them from LDS instead of loading
  // (and, from a coarser field, re-interpolating) them again.
  static constexpr int FRING = 64;
  static constexpr size_t FR_FLOATS = 2 * (size_t)FRING * WP;
  static constexpr bool SPLIT_FITS = (LDS_FLOATS + HS_FLOATS) * sizeof(float) <= 65536;
};

// Separate window-sum region for the wide (latency) variant where it fits in 64 KB: that
// variant runs about one workgroup per CU, so the larger LDS footprint costs no occupancy.
template <int R, int TW, bool WIDE, bool LEAN, int BB = 1>
constexpr bool split_hs() {
  return WIDE && !LEAN && Cfg<R, TW, WIDE, BB>::SPLIT_FITS;
}
template <int R, int TW, bool WIDE, bool LEAN, int BB = 1, bool FR = false>
constexpr size_t lds_bytes() {
  using C = Cfg<R, TW, WIDE, BB>;
  return (C::LDS_FLOATS + (split_hs<R, TW, WIDE, LEAN, BB>() ? C::HS_FLOATS : 0) +
          (FR ? C::FR_FLOATS : 0)) * sizeof(float);
}
// Plain launches of the wide variants with one band per pass keep the field ring when they
// read a field (its 2*64 rows cost LDS that only these latency-bound launches can spare); the
// batched kernel keeps it in every variant (measured faster there as well).
template <int MODE, bool WIDE, bool LEAN, int BB>
constexpr bool field_ring() {
  return MODE != kFlowZero && WIDE && !LEAN && BB == 1;
}

// One tile: TW output columns from x0 = bx*TW and TH output rows from row y0, walked in
// nbands bands (TH is a multiple of N; nbands = TH/N + 1).  `sm4` is the workgroup's LDS.
// INTERIOR: the tile's whole warped-frame region (the tile grown by r + 1 px, all bands)
// lies inside the image, so no position needs clamping or an in-image test.
// LEAN: the item indices are recomputed every band instead of being kept in registers
// across the band loop: a few more VALU instructions per band for far fewer live registers,
// i.e. more resident workgroups per CU (launches with many tiles); without it each band's
// dependent path is shorter (launches with about one tile per CU).
// pixel_mask: the tile holds masked pixels, whose flow is written as zero.
// GAUSS: window sums weighted by the separable taps a.taps[0..2r] (Gaussian-weighted window)
// instead of the unweighted box: every horizontal and vertical sum is a direct 2r+1-term
// weighted sum in a fixed order, so results remain independent of the tiling.
// BUB: the launch may carry the eq. 3 count (plain launches; checked at run time there).
// BB: bands per pass.  With BB = 2 the phases run over two bands' rows at once with twice the
// threads, so a tile of two bands (one output band and the band that primes the vertical
// sums) is one pass of the dependent path instead of two; P4 walks the two bands in order,
// with the same additions as two single-band passes.  nbands is then even.
// FR (a field is read, one band per pass): P1 stores the field of every warped-frame position
// (interpolated from the coarser level in the coarse-field mode) in a ring of FRING rows; P2
// and P5 read theirs from it (the same value at the same clamped position) instead of loading
// it again (eight loads per value from a coarser field, one from the current one).  The next band's P1 may overwrite
// ring rows while slower threads are still in P5: it writes rows tb+N+1 .. tb+2N while P5
// reads rows tb-R .. tb+R, at most 5R+2 < FRING apart, so no slot is shared.
template <typename T, int R, int TW, int MODE, bool WIDE, bool DEFER, bool INTERIOR, bool LEAN,
          bool GAUSS = false, int BB = 1, bool FR = false, bool BUB = false>
__device__ __forceinline__ void strip_tile(const IterArgs& a, int TH, int nbands, int bx, int y0,
                                           bool pixel_mask, float4* sm4) {
  using C = Cfg<R, TW, WIDE, BB>;
  constexpr int N = C::N, NR = C::NR, NT = C::NT, PC = C::PC, WC = C::WC, PP = C::PP, WP = C::WP;
  constexpr int RMASK = C::RING - 1;
  static_assert(BB == 1 || BB == 2, "one or two bands per pass");
  static_assert(!FR || (MODE != kFlowZero && BB == 1 && 5 * R + 2 < C::FRING),
                "field ring: launches that read a field, one band per pass");
  float* sm = reinterpret_cast<float*>(sm4);
  constexpr bool kSplit = split_hs<R, TW, WIDE, LEAN, BB>();
  float* pr = sm;                               // [5][NR][PP] products (16-byte aligned rows)
  float* w2 = pr + 5 * NR * PP;                 // [WROWS][WP] warped frame
  // [5][NR][TW] horizontal, then window sums (16-byte aligned: WROWS*WP is a multiple of 4
  // here or the region aliases the products)
  float* hs = kSplit ? w2 + C::WROWS * WP : pr;
  float* fru = kSplit ? hs + C::HS_FLOATS : w2 + C::WROWS * WP;   // [FRING][WP] (FR only)
  float* frv = fru + C::FRING * WP;
  constexpr int FMASK = C::FRING - 1;

  const int tid0 = threadIdx.x;
  const int H = a.H, W = a.W;
  const int x0 = bx * TW;
  const T* __restrict__ I1 = (const T*)a.I1;
  const T* __restrict__ I2 = (const T*)a.I2;

  // P4 ownership: channel and column of this thread (the first 5*TW threads).
  const int vk = tid0 / TW, vc = tid0 - vk * TW;
  const bool p4 = vk < 5;
  float prev[N];
#pragma unroll
  for (int i = 0; i < N; ++i) prev[i] = 0.f;

  // eq. 3 count of the final iteration: u values at or below the threshold written by this
  // thread (one atomic per wave at the end)
  const bool bub = BUB && a.bcount != nullptr;
  const float bthr = bub ? at(a.bthr, 0u) : 0.f;
  unsigned bcnt = 0;
  for (int b = 0; b < nbands; b += BB) {
    const int tb = N * b;                        // first product row of the pass
    // LEAN: the thread index is re-materialised per band, opaque to the optimiser, so the
    // item indices derived from it are not hoisted out of the loop.
    int tid = tid0;
    if constexpr (LEAN) asm volatile("" : "+v"(tid));
    // ---------------------------------------------------------------- P1
    // Every global load of the band is issued here, branch-free (clamped addresses; results
    // for items outside the image or the band are discarded): the field at the warped-frame
    // positions, the four frame-2 samples of every warped-frame position, then frame 1 and the
    // field at this thread's P2 items and the centre field of its P5 items.  In the lean
    // variants a scheduling barrier keeps the last group after the samples are stored: issued
    // together the groups are all live at once (the kernel's register peak); the split costs
    // one more dependent load round per band and buys resident workgroups.
    const int wfirst = (BB == 2 || b == 0) ? tb - 1 : tb + 1;
    const int nw = ((BB == 2 || b == 0) ? NR + 2 : N) * WC;
    int wofs[C::K1], wgx[C::K1], wgy[C::K1];
    float wu[C::K1], wv[C::K1];
#pragma unroll
    for (int k = 0; k < C::K1; ++k) {
      if (k >= C::K1S && b != 0) break;   // uniform: only a tile's first pass has these
      using DW = ConstDiv<WC, C::P1_ROWS_MAX * WC>;
      const unsigned i = (unsigned)min(tid + k * NT, nw - 1), qi = DW::q(i);
      const int w = wfirst + (int)qi, lx = (int)DW::r(i, qi);
      if constexpr (INTERIOR) {
        wgx[k] = x0 - R - 1 + lx;
        wgy[k] = y0 - R + w;
      } else {
        wgx[k] = min(max(x0 - R - 1 + lx, 0), W - 1);
        wgy[k] = min(max(y0 - R + w, 0), H - 1);
      }
      wofs[k] = (BB == 1 ? (w & RMASK) : w - (tb - 1)) * WP + lx;
      read_flow<MODE>(a, wgx[k], wgy[k], wu[k], wv[k]);
      if constexpr (FR) {
        fru[(w & FMASK) * WP + lx] = wu[k];
        frv[(w & FMASK) * WP + lx] = wv[k];
      }
    }
    // In the coarse-field mode each field value costs eight loads: where registers are tight
    // (DEFER) the field at this thread's P2 and P5 items is read in those phases rather than
    // held in flight here.
    constexpr bool kDefer = DEFER && MODE == kFlowCoarse && !FR;
    constexpr bool kLoadField = !kDefer && !FR;   // P2/P5 field loads issued in P1
    float i1v[C::K2], pu[C::K2], pv[C::K2];
    float cu[C::K5], cv[C::K5];
    // (The same loads are written twice, before the samples for the default variants and
    // after them for the lean ones, so that each keeps its own straight-line schedule.)
    if constexpr (!LEAN) {
#pragma unroll
      for (int k = 0; k < C::K2; ++k) {
        using DP = ConstDiv<PC, NR * PC>;
        const unsigned i = (unsigned)min(tid + k * NT, NR * PC - 1), qi = DP::q(i);
        int gx = x0 - R + (int)DP::r(i, qi), gy = y0 - R + tb + (int)qi;
        if constexpr (!INTERIOR) {
          gx = min(max(gx, 0), W - 1);
          gy = min(max(gy, 0), H - 1);
        }
        i1v[k] = ld(I1, rowofs(gy, W, gx));
        if constexpr (kLoadField) read_flow<MODE>(a, gx, gy, pu[k], pv[k]);
      }
      if constexpr (kLoadField) {
#pragma unroll
        for (int k = 0; k < C::K5; ++k) {
          const int i = min(tid + k * NT, NR * TW - 1);
          const int gx = INTERIOR ? x0 + (int)((unsigned)i % TW) : min(x0 + (int)((unsigned)i % TW), W - 1);
          const int gy = min(max(y0 + tb + (int)((unsigned)i / TW) - 2 * R, 0), H - 1);
          read_flow<MODE>(a, gx, gy, cu[k], cv[k]);
        }
      }
    }
    // Items past the end repeat the last position (clamped index) and store the identical
    // value to the identical slot, so the stores need no guard: a guard lets the compiler
    // sink each item's gathers into its own branch and wait for them one item at a time.
#pragma unroll
    for (int k = 0; k < C::K1; ++k) {
      if (k >= C::K1S && b != 0) break;
      w2[wofs[k]] = warp_sample(I2, H, W, wgx[k], wgy[k], wu[k], wv[k]);
    }
    if constexpr (LEAN) {
      __builtin_amdgcn_sched_barrier(0);   // compiler-only fence
#pragma unroll
      for (int k = 0; k < C::K2; ++k) {
        using DP = ConstDiv<PC, NR * PC>;
        const unsigned i = (unsigned)min(tid + k * NT, NR * PC - 1), qi = DP::q(i);
        int gx = x0 - R + (int)DP::r(i, qi), gy = y0 - R + tb + (int)qi;
        if constexpr (!INTERIOR) {
          gx = min(max(gx, 0), W - 1);
          gy = min(max(gy, 0), H - 1);
        }
        i1v[k] = ld(I1, rowofs(gy, W, gx));
        if constexpr (kLoadField) read_flow<MODE>(a, gx, gy, pu[k], pv[k]);
      }
      if constexpr (kLoadField) {
#pragma unroll
        for (int k = 0; k < C::K5; ++k) {
          const int i = min(tid + k * NT, NR * TW - 1);
          const int gx = INTERIOR ? x0 + (int)((unsigned)i % TW) : min(x0 + (int)((unsigned)i % TW), W - 1);
          const int gy = min(max(y0 + tb + (int)((unsigned)i / TW) - 2 * R, 0), H - 1);
          read_flow<MODE>(a, gx, gy, cu[k], cv[k]);
        }
      }
    }
    __syncthreads();
    // ---------------------------------------------------------------- P2
    if constexpr (kDefer) {
#pragma unroll
      for (int k = 0; k < C::K2; ++k) {
        using DP = ConstDiv<PC, NR * PC>;
        const unsigned i = (unsigned)min(tid + k * NT, NR * PC - 1), qi = DP::q(i);
        int gx = x0 - R + (int)DP::r(i, qi), gy = y0 - R + tb + (int)qi;
        if constexpr (!INTERIOR) {
          gx = min(max(gx, 0), W - 1);
          gy = min(max(gy, 0), H - 1);
        }
        read_flow<MODE>(a, gx, gy, pu[k], pv[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < C::K2; ++k) {
      const int i = tid + k * NT;
      if (i < NR * PC) {
        using DP = ConstDiv<PC, NR * PC>;
        const int r = (int)DP::q((unsigned)i), c = (int)DP::r((unsigned)i, (unsigned)r);
        const int t = tb + r;
        const int gx = x0 - R + c, gy = y0 - R + t;
        float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f, p4 = 0.f;
        if (INTERIOR || (gx >= 0 && gx < W && gy >= 0 && gy < H)) {
          // warped row t sits in ring slot t & RMASK, or (two bands per pass) in row r + 1
          const int s0 = BB == 1 ? t & RMASK : r + 1;
          const int sm1 = BB == 1 ? (t - 1) & RMASK : r;
          const int sp1 = BB == 1 ? (t + 1) & RMASK : r + 2;
          const float* row = w2 + s0 * WP + c + 1;
          const float ix = 0.5f * (row[1] - row[-1]);
          const float iy = 0.5f * (w2[sp1 * WP + c + 1] - w2[sm1 * WP + c + 1]);
          float fu, fv;   // field at the product position
          if constexpr (FR) {
            fu = fru[(t & FMASK) * WP + c + 1];
            fv = frv[(t & FMASK) * WP + c + 1];
          } else {
            fu = pu[k];
            fv = pv[k];
          }
          float it = row[0] - i1v[k];
          it = fmaf(-ix, fu, it);
          it = fmaf(-iy, fv, it);
          p0 = ix * ix;
          p1 = ix * iy;
          p2 = iy * iy;
          p3 = ix * it;
          p4 = iy * it;
        }
        float* q = pr + r * PP + c;
        q[0] = p0;
        q[NR * PP] = p1;
        q[2 * NR * PP] = p2;
        q[3 * NR * PP] = p3;
        q[4 * NR * PP] = p4;
      }
    }
    __syncthreads();
    // ---------------------------------------------------------------- P3
    // Where the window sums overwrite the products they are made from, every thread first
    // reads and sums its segments, then all write after a barrier.
    float hv[C::K3][8];
#pragma unroll
    for (int k = 0; k < C::K3; ++k) {
      const int i = tid + k * NT;
      if (i < 5 * NR * C::NSEG) {
        const int seg = (int)((unsigned)i % C::NSEG), rr = (int)((unsigned)i / C::NSEG);   // ch * NR + row
        typedef float f4v __attribute__((ext_vector_type(4)));
        const f4v* src = reinterpret_cast<const f4v*>(pr + rr * PP + 8 * seg);
        float vbuf[4 * C::HL4];
#pragma unroll
        for (int q = 0; q < C::HL4; ++q) {
          // The empty asm takes the four values as one 128-bit register operand, so each read
          // stays one 128-bit LDS load (the sums below use the values out of order, and the
          // loads were otherwise split into 32-bit pairs).
          f4v f = src[q];
          asm volatile("" : "+v"(f));
          vbuf[4 * q] = f.x;
          vbuf[4 * q + 1] = f.y;
          vbuf[4 * q + 2] = f.z;
          vbuf[4 * q + 3] = f.w;
        }
        if constexpr (GAUSS) {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            float s = a.taps[0] * vbuf[j];
#pragma unroll
            for (int q = 1; q <= 2 * R; ++q) s = fmaf(a.taps[q], vbuf[j + q], s);
            hv[k][j] = s;
          }
        } else if constexpr (2 * R >= 7) {
          // Every window of the segment holds column 2R (the last column of window 0), so
          // window j is the suffix vbuf[j..2R] plus the prefix vbuf[2R+1..2R+j]: sums of
          // values inside the window only.  (A running sum that subtracts the value leaving
          // the window carries a rounding error relative to the largest product of the
          // segment rather than of the window, which ill-conditioned windows amplify.)
          float suf = vbuf[7];   // vbuf[7..2R], in load order
#pragma unroll
          for (int q = 8; q <= 2 * R; ++q) suf += vbuf[q];
          float sj[8];
          sj[7] = suf;
#pragma unroll
          for (int j = 6; j >= 0; --j) sj[j] = vbuf[j] + sj[j + 1];
          hv[k][0] = sj[0];
          float pre = 0.f;
#pragma unroll
          for (int j = 1; j < 8; ++j) {
            pre = j == 1 ? vbuf[2 * R + 1] : pre + vbuf[2 * R + j];
            hv[k][j] = sj[j] + pre;
          }
        } else {
          // r <= 3: direct sums, at most 6 additions per output
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            float s = vbuf[j];
#pragma unroll
            for (int q = 1; q <= 2 * R; ++q) s += vbuf[j + q];
            hv[k][j] = s;
          }
        }
      }
    }
    if constexpr (!kSplit) __syncthreads();
#pragma unroll
    for (int k = 0; k < C::K3; ++k) {
      const int i = tid + k * NT;
      if (i < 5 * NR * C::NSEG) {
        const int seg = (int)((unsigned)i % C::NSEG), rr = (int)((unsigned)i / C::NSEG);
        float4* dst = reinterpret_cast<float4*>(hs + rr * C::TW + 8 * seg);
        dst[0] = make_float4(hv[k][0], hv[k][1], hv[k][2], hv[k][3]);
        dst[1] = make_float4(hv[k][4], hv[k][5], hv[k][6], hv[k][7]);
      }
    }
    __syncthreads();
    // ---------------------------------------------------------------- P4
    static_assert(!GAUSS || BB == 1, "Gaussian-weighted window: one band per pass");
    if (GAUSS && p4) {
      // Output row r of the band: previous-band rows r+1..N-1 then current rows 0..r, i.e.
      // window offsets 0..N-1 from its top row, weighted by the taps in that order.
      float* col = hs + vk * N * TW + vc;
      float cur[N];
#pragma unroll
      for (int r = 0; r < N; ++r) cur[r] = col[r * TW];
#pragma unroll
      for (int r = 0; r < N; ++r) {
        float s = 0.f;
#pragma unroll
        for (int m = r + 1; m < N; ++m) s = fmaf(a.taps[m - r - 1], prev[m], s);
#pragma unroll
        for (int m = 0; m <= r; ++m) s = fmaf(a.taps[N - 1 - r + m], cur[m], s);
        col[r * TW] = s;
      }
#pragma unroll
      for (int r = 0; r < N; ++r) prev[r] = cur[r];
    } else if (p4) {
#pragma unroll
      for (int bb = 0; bb < BB; ++bb) {
        float* col = hs + vk * NR * TW + bb * N * TW + vc;
        // prev[r] <- prev[r] + ... + prev[N-1] (suffix sums of the previous band, in place)
#pragma unroll
        for (int r = N - 2; r >= 0; --r) prev[r] += prev[r + 1];
        float pre = 0.f;
#pragma unroll
        for (int r = 0; r < N; ++r) {
          const float c = col[r * TW];
          pre = r == 0 ? c : pre + c;
          col[r * TW] = r + 1 < N ? prev[r + 1] + pre : pre;
          prev[r] = c;
        }
      }
    }
    __syncthreads();
    // ---------------------------------------------------------------- P5
    if constexpr (kDefer) {
#pragma unroll
      for (int k = 0; k < C::K5; ++k) {
        const int i = min(tid + k * NT, NR * TW - 1);
        const int gx = INTERIOR ? x0 + (int)((unsigned)i % TW) : min(x0 + (int)((unsigned)i % TW), W - 1);
        const int gy = min(max(y0 + tb + (int)((unsigned)i / TW) - 2 * R, 0), H - 1);
        read_flow<MODE>(a, gx, gy, cu[k], cv[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < C::K5; ++k) {
      const int i = tid + k * NT;
      if (i < NR * TW) {
        const int r = (int)((unsigned)i / TW), c = (int)((unsigned)i % TW);
        const int j = tb + r - 2 * R;
        const int gx = x0 + c, gy = y0 + j;
        if (j >= 0 && j < TH && (INTERIOR || (gx < W && gy < H))) {
          const float* s = hs + r * TW + c;
          float fu, fv;   // field at the output pixel: warped row j + R, column c + R + 1
          if constexpr (FR) {
            fu = fru[((j + R) & FMASK) * WP + c + R + 1];
            fv = frv[((j + R) & FMASK) * WP + c + R + 1];
          } else {
            fu = cu[k];
            fv = cv[k];
          }
          float un, vn;
          solve_update(s[0], s[NR * TW], s[2 * NR * TW], s[3 * NR * TW], s[4 * NR * TW], fu, fv,
                       un, vn);
          const unsigned o = rowofs(gy, W, gx);
          if (pixel_mask && at(a.mask, o) == 0) {   // masked-out pixel: zero flow
            un = 0.f;
            vn = 0.f;
          }
          at(a.uout, o) = un;
          at(a.vout, o) = vn;
          if constexpr (BUB) {
            if (bub) bcnt += un <= bthr ? 1u : 0u;
          }
        }
      }
    }
    // The next pass's P1 writes only warped rows that this pass's P2 finished reading before
    // the barriers above; its P2 rewrites the product/window-sum buffer after the P1 barrier,
    // when every thread has finished this pass's P5.
  }
  if constexpr (BUB) {
    if (bub) add_count(a.bcount, bcnt);
  }
}

// True when every warped-frame position of the tile (columns x0-R-1 .. x0+TW+R, rows
// y0-R-1 .. y0-R+N*nbands) lies inside the image.
template <int R, int TW>
__device__ __forceinline__ bool tile_interior(const IterArgs& a, int nbands, int bx, int y0) {
  constexpr int N = 2 * R + 1;
  const int x0 = bx * TW;
  return x0 - R - 1 >= 0 && x0 + TW + R <= a.W - 1 && y0 - R - 1 >= 0 &&
         y0 - R + N * nbands <= a.H - 1;
}

// Masked plans: a tile without an unmasked output pixel (TW columns from x0, TH rows from
// y0) is not computed; its workgroup writes zero flow over it (and counts those zeros for the
// eq. 3 count when the threshold is not negative).
template <int TW>
__device__ __forceinline__ void zero_tile(const IterArgs& a, int TH, int bx, int y0) {
  const int x0 = bx * TW;
  const int w = min(TW, a.W - x0), h = min(TH, a.H - y0);
  for (int i = threadIdx.x; i < w * h; i += blockDim.x) {
    const int r = i / w, c = i - r * w;
    const unsigned o = (unsigned)(y0 + r) * (unsigned)a.W + (unsigned)(x0 + c);
    at(a.uout, o) = 0.f;
    at(a.vout, o) = 0.f;
  }
  if (a.bcount != nullptr && threadIdx.x == 0 && 0.f <= at(a.bthr, 0u))
    atomicAdd(a.bcount, (unsigned long long)w * (unsigned long long)h);
}

// Workgroup index -> work index so that the workgroups one XCD runs (hardware dispatch is
// round-robin over the 8 XCDs) take a contiguous range of tiles, which share halos in L2.
__device__ __forceinline__ int xcd_order(int b, int nblocks) {
  constexpr int kXcd = 8;
  const int per = (nblocks + kXcd - 1) / kXcd;
  return (b % kXcd) * per + b / kXcd;
}

template <typename T, int R, int TW, int MODE, bool WIDE, bool LEAN, bool GAUSS, int BB>
__global__ __launch_bounds__((group_threads<R, TW, WIDE, BB>())) void lk_iter_strip(IterArgs a, int TH,
                                                                           int nbands, int tiles_x,
                                                                           int ntiles) {
  extern __shared__ float4 sm4[];
  const int t = xcd_order(blockIdx.x, gridDim.x);
  if (t >= ntiles) return;
  const int bx = t % tiles_x, y0 = t / tiles_x * TH;
  bool pixel_mask = false;
  if (a.mask) {
    const int f = a.tiles[t];
    if (f == 0) {
      zero_tile<TW>(a, TH, bx, y0);
      return;
    }
    pixel_mask = f == 1;
  }
  constexpr bool kDefer = WIDE || R > 8;
  constexpr bool kFR = field_ring<MODE, WIDE, LEAN, BB>();
  if (R <= 8 && tile_interior<R, TW>(a, nbands, bx, y0))
    strip_tile<T, R, TW, MODE, WIDE, kDefer, true, LEAN, GAUSS, BB, kFR, true>(a, TH, nbands, bx,
                                                                               y0, pixel_mask, sm4);
  else
    strip_tile<T, R, TW, MODE, WIDE, kDefer, false, LEAN, GAUSS, BB, kFR, true>(a, TH, nbands, bx,
                                                                                y0, pixel_mask, sm4);
}

// Batched form: workgroups stride over a work list of tiles of many pairs at the same
// (level, iteration) phase.  Work item = (pair | tile flag << 16, tile x, first output row,
// output rows, a multiple of 2r+1).  For a pair with a mask (in its arguments) the flag tells
// a tile without an unmasked pixel (0, zero-filled), one with masked pixels (1) and one
// without (2).
// MASK: launches of batches with masks (the mask code costs the unmasked launches about 5 %
// more instructions and is compiled out of them).
template <typename T, int R, int TW, int MODE, bool WIDE, bool LEAN, bool GAUSS, bool MASK>
__global__ __launch_bounds__((group_threads<R, TW, WIDE, 1>())) void lk_iter_batch(const IterArgs* __restrict__ args,
                                                                      const int4* __restrict__ tiles,
                                                                      int ntiles) {
  extern __shared__ float4 sm4[];
  using C = Cfg<R, TW, WIDE>;
  const int stride = (int)gridDim.x;
  for (int t = xcd_order(blockIdx.x, gridDim.x); t < ntiles; t += stride) {
    const int4 w = tiles[t];
    const IterArgs a = args[w.x & 0xffff];
    const int nb = w.w / C::N + 1;
    bool pixel_mask = false;
    if constexpr (MASK) {
      if (a.mask) {
        const int f = (int)((unsigned)w.x >> 16);
        if (f == 0) {
          zero_tile<TW>(a, w.w, w.y, w.z);
          continue;
        }
        pixel_mask = f == 1;
      }
    }
    constexpr bool kFR = MODE != kFlowZero;
    if (R <= 8 && tile_interior<R, TW>(a, nb, w.y, w.z))
      strip_tile<T, R, TW, MODE, WIDE, true, true, LEAN, GAUSS, 1, kFR>(a, w.w, nb, w.y, w.z,
                                                                        pixel_mask, sm4);
    else
      strip_tile<T, R, TW, MODE, WIDE, true, false, LEAN, GAUSS, 1, kFR>(a, w.w, nb, w.y, w.z,
                                                                         pixel_mask, sm4);
    __syncthreads();
  }
}

// 64-column strips while the LDS footprint stays within 64 KB, else 32-column strips.
template <int R>
constexpr int strip_width() {
  return Cfg<R, 64>::LDS_FLOATS * sizeof(float) <= 65536 ? 64 : 32;
}

// nb output bands per tile take nb + 1 bands (the first primes the vertical sums), rounded up
// to whole passes of BB bands (a band past the tile's rows writes nothing).
template <typename T, int R, int MODE, bool WIDE, bool LEAN, bool GAUSS, int TWV = 0, int BB = 1>
hipError_t go_plain_v(const IterArgs& a, int nb, hipStream_t s) {
  constexpr int TW = TWV ? TWV : strip_width<R>();
  using C = Cfg<R, TW, WIDE, BB>;
  constexpr bool kFR = field_ring<MODE, WIDE, LEAN, BB>();
  constexpr size_t kLds = lds_bytes<R, TW, WIDE, LEAN, BB, kFR>();
  static_assert(kLds <= 160 * 1024, "LDS footprint above 160 KB");
  const int TH = C::N * nb;
  const int tx = (a.W + TW - 1) / TW, ty = (a.H + TH - 1) / TH;
  const int ntiles = tx * ty;
  const int grid = (ntiles + 7) / 8 * 8;
  const int nbands = (nb + 1 + BB - 1) / BB * BB;
  if constexpr (kLds > 65536) {
    // Opt in to more than 64 KB of dynamic LDS (gfx950 has 160 KB per workgroup), once.
    static const hipError_t opt = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&lk_iter_strip<T, R, TW, MODE, WIDE, LEAN, GAUSS, BB>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLds);
    if (opt != hipSuccess) return opt;
  }
  hipLaunchKernelGGL((lk_iter_strip<T, R, TW, MODE, WIDE, LEAN, GAUSS, BB>), dim3(grid),
                     dim3(C::NT), kLds, s, a, TH, nbands, tx, ntiles);
  return hipGetLastError();
}

template <typename T, int R, int MODE, bool GAUSS>
hipError_t go_plain_g(const IterArgs& a, int nb, int variant, hipStream_t s) {
  switch (variant) {
    case kTileNarrow: return go_plain_v<T, R, MODE, false, true, GAUSS>(a, nb, s);
    case kTileWide: return go_plain_v<T, R, MODE, true, false, GAUSS>(a, nb, s);
    case kTileWideLean: return go_plain_v<T, R, MODE, true, true, GAUSS>(a, nb, s);
  }
  if constexpr (!GAUSS) {   // narrow strips: box window only
    switch (variant) {
      case kTileWide32: return go_plain_v<T, R, MODE, true, false, false, 32>(a, nb, s);
      case kTileWide16: return go_plain_v<T, R, MODE, true, false, false, 16>(a, nb, s);
    }
    if constexpr (R <= kMaxPairRadius) {   // two bands per pass
      switch (variant) {
        case kTileWide32x2: return go_plain_v<T, R, MODE, true, false, false, 32, 2>(a, nb, s);
        case kTileWide16x2: return go_plain_v<T, R, MODE, true, false, false, 16, 2>(a, nb, s);
        case kTileLean32x2: return go_plain_v<T, R, MODE, true, true, false, 32, 2>(a, nb, s);
      }
    }
  }
  return hipErrorInvalidValue;
}

// variant bit kTileGauss selects the Gaussian-weighted window.
template <typename T, int R, int MODE>
hipError_t go_plain(const IterArgs& a, int nb, int variant, hipStream_t s) {
  if (variant & kTileGauss) return go_plain_g<T, R, MODE, true>(a, nb, variant & ~kTileGauss, s);
  return go_plain_g<T, R, MODE, false>(a, nb, variant, s);
}

template <typename T, int R, int MODE, bool WIDE, bool LEAN, bool GAUSS, bool MASK>
hipError_t go_batch_m(const BatchLaunch& b, hipStream_t s) {
  constexpr int TW = strip_width<R>();
  using C = Cfg<R, TW, WIDE>;
  constexpr size_t kLds = lds_bytes<R, TW, WIDE, LEAN, 1, MODE != kFlowZero>();
  if constexpr (kLds > 65536) {
    static const hipError_t opt = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&lk_iter_batch<T, R, TW, MODE, WIDE, LEAN, GAUSS, MASK>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLds);
    if (opt != hipSuccess) return opt;
  }
  if (b.prime) {
    hipFuncAttributes attr;
    return hipFuncGetAttributes(
        &attr, reinterpret_cast<const void*>(&lk_iter_batch<T, R, TW, MODE, WIDE, LEAN, GAUSS, MASK>));
  }
  hipLaunchKernelGGL((lk_iter_batch<T, R, TW, MODE, WIDE, LEAN, GAUSS, MASK>), dim3(b.grid),
                     dim3(C::NT), kLds, s, b.args, b.tiles, b.ntiles);
  return hipGetLastError();
}

template <typename T, int R, int MODE, bool WIDE, bool LEAN, bool GAUSS>
hipError_t go_batch_v(const BatchLaunch& b, hipStream_t s) {
  return b.masked ? go_batch_m<T, R, MODE, WIDE, LEAN, GAUSS, true>(b, s)
                  : go_batch_m<T, R, MODE, WIDE, LEAN, GAUSS, false>(b, s);
}

// b.variant: OF_TILE_NARROW, _WIDE or _WIDE_LEAN, plus kTileGauss for the Gaussian window.
template <typename T, int R, int MODE>
hipError_t go_batch(const BatchLaunch& b, hipStream_t s) {
  switch (b.variant) {
    case kTileNarrow: return go_batch_v<T, R, MODE, false, true, false>(b, s);
    case kTileWide: return go_batch_v<T, R, MODE, true, false, false>(b, s);
    case kTileWideLean: return go_batch_v<T, R, MODE, true, true, false>(b, s);
    case kTileNarrow | kTileGauss: return go_batch_v<T, R, MODE, false, true, true>(b, s);
    case kTileWide | kTileGauss: return go_batch_v<T, R, MODE, true, false, true>(b, s);
    case kTileWideLean | kTileGauss: return go_batch_v<T, R, MODE, true, true, true>(b, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, int R>
hipError_t go_r(const IterArgs* a, const BatchLaunch* b, int mode, int nb, int variant,
                hipStream_t s) {
  switch (mode) {
    case kFlowSame:
      return a ? go_plain<T, R, kFlowSame>(*a, nb, variant, s) : go_batch<T, R, kFlowSame>(*b, s);
    case kFlowCoarse:
      return a ? go_plain<T, R, kFlowCoarse>(*a, nb, variant, s) : go_batch<T, R, kFlowCoarse>(*b, s);
    case kFlowZero:
      return a ? go_plain<T, R, kFlowZero>(*a, nb, variant, s) : go_batch<T, R, kFlowZero>(*b, s);
  }
  return hipErrorInvalidValue;
}

// Plain launch (a != nullptr; tile height N*nb, tile variant `variant`) or batched launch
// (b != nullptr; its own variant).
template <typename T>
hipError_t launch_iter_t(const IterArgs* a, const BatchLaunch* b, int R, int mode, int nb,
                         int variant, hipStream_t s) {
  switch (R) {
    case 0: return go_r<T, 0>(a, b, mode, nb, variant, s);
    case 1: return go_r<T, 1>(a, b, mode, nb, variant, s);
    case 2: return go_r<T, 2>(a, b, mode, nb, variant, s);
    case 3: return go_r<T, 3>(a, b, mode, nb, variant, s);
    case 4: return go_r<T, 4>(a, b, mode, nb, variant, s);
    case 5: return go_r<T, 5>(a, b, mode, nb, variant, s);
    case 6: return go_r<T, 6>(a, b, mode, nb, variant, s);
    case 7: return go_r<T, 7>(a, b, mode, nb, variant, s);
    case 8: return go_r<T, 8>(a, b, mode, nb, variant, s);
    case 9: return go_r<T, 9>(a, b, mode, nb, variant, s);
    case 10: return go_r<T, 10>(a, b, mode, nb, variant, s);
    case 11: return go_r<T, 11>(a, b, mode, nb, variant, s);
    case 12: return go_r<T, 12>(a, b, mode, nb, variant, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

}  // namespace ofmi
