// Plan geometry and the per-pair schedule shared by the plain, batched and session paths.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ofmi.h"
#include "kernels.h"

namespace ofmi {

struct Geometry {
  int L, R, K;
  unsigned flags;
  int H[OF_MAX_LEVELS], W[OF_MAX_LEVELS];
  Elem ein;                         // element type of the caller's frames
  Elem e0;                          // level-0 plane element type (float32 when normalised)
  size_t off_norm[2];               // normalised level-0 planes (OF_FLAG_NORMALIZE)
  Elem ep;                          // element type of pyramid levels >= 1
  size_t off_p1[OF_MAX_LEVELS];     // workspace offsets of the pyramid levels (>= 1)
  size_t off_p2[OF_MAX_LEVELS];
  size_t off_flow[4];               // ping-pong u0, u1, v0, v1 (level-0 size each)
  int nb[OF_MAX_LEVELS];            // iteration tile height per level, in bands of 2R+1 rows
  int variant[OF_MAX_LEVELS];       // tile variant of the iteration kernel (TileVariant)
  const uint8_t* mask[OF_MAX_LEVELS];   // per-level masks (of_plan_set_mask) or nullptr
  const uint8_t* tflags[OF_MAX_LEVELS]; // per-level iteration-tile flags (with a mask)
  const float* bthr;                // eq. 3 count of the final field (of_plan_set_bubble)
  unsigned long long* bcount;
  size_t bytes;
  Elem elem(int l) const;
};

// Optional event timing (of_plan_set_timing / of_plan_read_timing): one event pair around
// every launch (mode OF_TIMING_LAUNCH), or around the pyramid launches and around each level's
// iteration launches (OF_TIMING_LEVEL: no events between the launches of a span).
struct KernelTimer {
  struct Rec {
    int kernel;
    hipEvent_t a, b;
    double units, bytes;
    long long launches;
  };
  bool on = false;
  int mode = OF_TIMING_LAUNCH;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  bool per_launch() const { return on && mode == OF_TIMING_LAUNCH; }
  bool per_level() const { return on && mode == OF_TIMING_LEVEL; }
  hipError_t begin(hipStream_t s, hipEvent_t* a);
  hipError_t end(hipStream_t s, hipEvent_t a, int kernel, double units, double bytes,
                 long long launches = 1);
  hipError_t read(int kernel, double* ms, long long* n, double* units, double* bytes);
  ~KernelTimer();
};

// Captured schedules replayed with hipGraphLaunch, keyed by the caller's buffer pointers.
// Capture runs on a private stream; a replay is enqueued on the caller's stream.
struct GraphCache {
  struct Entry {
    std::vector<uintptr_t> key;
    hipGraphExec_t exec;
    unsigned long long used;
  };
  std::vector<Entry> entries;
  hipStream_t cap = nullptr;
  unsigned long long tick = 0;
  size_t max_entries = 64;
  template <class F>
  hipError_t run(const std::vector<uintptr_t>& key, hipStream_t s, F&& enqueue);
  bool contains(const std::vector<uintptr_t>& key) const {
    for (const Entry& e : entries)
      if (e.key == key) return true;
    return false;
  }
  // Index of the least recently used entry (entries must not be empty).
  size_t lru() const {
    size_t i = 0;
    for (size_t j = 1; j < entries.size(); ++j)
      if (entries[j].used < entries[i].used) i = j;
    return i;
  }
  // Drops entry i (the caller has made sure no replay of it is still in flight).
  void erase(size_t i) {
    hipGraphExecDestroy(entries[i].exec);
    entries.erase(entries.begin() + i);
  }
  void clear();
  ~GraphCache();
};

template <class F>
hipError_t GraphCache::run(const std::vector<uintptr_t>& key, hipStream_t s, F&& enqueue) {
  for (Entry& e : entries) {
    if (e.key == key) {
      e.used = ++tick;
      return hipGraphLaunch(e.exec, s);
    }
  }
  hipError_t err;
  if (!cap) {
    err = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (err != hipSuccess) return err;
  }
  err = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
  if (err != hipSuccess) return err;
  hipError_t eq = enqueue(cap);
  hipGraph_t graph = nullptr;
  err = hipStreamEndCapture(cap, &graph);
  if (eq != hipSuccess || err != hipSuccess) {
    if (graph) hipGraphDestroy(graph);
    return eq != hipSuccess ? eq : err;
  }
  hipGraphExec_t exec = nullptr;
  err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (err != hipSuccess) return err;
  if (entries.size() >= max_entries) {
    hipDeviceSynchronize();   // the evicted graph may still be in flight
    size_t lru = 0;
    for (size_t i = 1; i < entries.size(); ++i)
      if (entries[i].used < entries[lru].used) lru = i;
    hipGraphExecDestroy(entries[lru].exec);
    entries.erase(entries.begin() + lru);
  }
  entries.push_back({key, exec, ++tick});
  return hipGraphLaunch(exec, s);
}

void set_error(const std::string& s);
// Separable taps of the Gaussian-weighted window, g(d) = exp(-d^2 / (2 sigma^2)), sigma = R/2,
// d = -R..R (a single tap of 1 for R = 0), into taps[0..2R].
void gaussian_taps(float* taps, int R);
// Flags of the iteration tiles (TW columns x TH rows) of an H x W mask level: 0 = no unmasked
// pixel, 1 = some masked pixels, 2 = no masked pixel; row-major over tile rows.
std::vector<uint8_t> tile_flags(const uint8_t* mask, int H, int W, int TW, int TH);
// Band cut of a tile with masked pixels: rows [y0, e) and columns [c0, c1) of mask m (row
// pitch W), bands of N rows from y0.  Returns the first row and the rows (a multiple of N) from
// the tile's first to its last band that holds an unmasked pixel; the band boundaries stay
// where the tile's are, so the window sums round as in the uncut tile.
void band_cut(const uint8_t* m, int W, int c0, int c1, int y0, int e, int N, int& ty0, int& th);
int default_bands(int H, int W, int R);
int default_tile_variant(long long ntiles);
bool check_params(int H, int W, int levels, int radius, int iters, unsigned flags);
Geometry make_geometry(int H, int W, int levels, int radius, int iters, unsigned flags);
hipError_t enqueue_pair(const Geometry& g, char* ws, const void* I1, const void* I2, float* u,
                        float* v, hipStream_t s, KernelTimer* t);

}  // namespace ofmi
