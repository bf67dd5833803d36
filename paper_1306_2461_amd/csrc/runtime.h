// Plan geometry and the per-pair schedule shared by the plain, batched and session paths.
#pragma once

#include <stddef.h>

#include <string>
#include <vector>

#include "../../include/ofmi.h"
#include "kernels.h"

namespace ofmi {

struct Geometry {
  int L, R, K;
  unsigned flags;
  int H[OF_MAX_LEVELS], W[OF_MAX_LEVELS];
  Elem e0;                          // level-0 frame element type (uint8 or float32)
  Elem ep;                          // element type of pyramid levels >= 1
  size_t off_p1[OF_MAX_LEVELS];     // workspace offsets of the pyramid levels (>= 1)
  size_t off_p2[OF_MAX_LEVELS];
  size_t off_flow[4];               // ping-pong u0, u1, v0, v1 (level-0 size each)
  size_t bytes;
  Elem elem(int l) const;
};

// Optional per-launch event timing (of_plan_set_timing / of_plan_read_timing).
struct KernelTimer {
  struct Rec {
    int kernel;
    hipEvent_t a, b;
    double units, bytes;
  };
  bool on = false;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipError_t begin(hipStream_t s, hipEvent_t* a);
  hipError_t end(hipStream_t s, hipEvent_t a, int kernel, double units, double bytes);
  hipError_t read(int kernel, double* ms, long long* n, double* units, double* bytes);
  ~KernelTimer();
};

void set_error(const std::string& s);
bool check_params(int H, int W, int levels, int radius, int iters, unsigned flags);
Geometry make_geometry(int H, int W, int levels, int radius, int iters, unsigned flags);
hipError_t enqueue_pair(const Geometry& g, char* ws, const void* I1, const void* I2, float* u,
                        float* v, hipStream_t s, KernelTimer* t);

}  // namespace ofmi
