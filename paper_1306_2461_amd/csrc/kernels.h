// Host-side launchers of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "common.h"

namespace ofmi {

enum class Elem : int { U8 = 0, F32 = 1, F16 = 2 };

inline size_t elem_bytes(Elem e) { return e == Elem::U8 ? 1 : (e == Elem::F16 ? 2 : 4); }

// One pyramid reduction of up to two frames of the same geometry (out = reduce(in)).
hipError_t launch_reduce(Elem tin, Elem tout, const void* in1, const void* in2, int H, int W,
                         void* out1, void* out2, int Ho, int Wo, hipStream_t s);

// One fused Gauss-Newton iteration at one level (frames of element type `t`).
hipError_t launch_iter(Elem t, const IterArgs& a, int R, hipStream_t s);

// u = v = 0 over n elements (a fill kernel, safe under stream capture).
hipError_t launch_zero(float* u, float* v, size_t n, hipStream_t s);

}  // namespace ofmi
