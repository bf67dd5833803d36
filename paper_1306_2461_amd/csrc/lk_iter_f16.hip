// Instantiations of the fused iteration kernel for __half frames.
#include "lk_iter_impl.h"

namespace ofmi {

hipError_t launch_iter_f16(const IterArgs& a, int R, hipStream_t s) { return launch_iter_t<__half>(a, R, s); }

}  // namespace ofmi
