// Instantiations of the fused iteration kernel for __half frames.
#include "lk_iter_impl.h"

namespace ofmi {

hipError_t launch_iter_f16(const IterArgs* a, const BatchLaunch* b, int R, int mode, int nb,
                          int variant, hipStream_t s) {
  return launch_iter_t<__half>(a, b, R, mode, nb, variant, s);
}

}  // namespace ofmi
