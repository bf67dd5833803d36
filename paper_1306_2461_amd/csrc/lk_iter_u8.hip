// Instantiations of the fused iteration kernel for uint8_t frames.
#include "lk_iter_impl.h"

namespace ofmi {

hipError_t launch_iter_u8(const IterArgs* a, const BatchLaunch* b, int R, int mode, int nb,
                          int variant, hipStream_t s) {
  return launch_iter_t<uint8_t>(a, b, R, mode, nb, variant, s);
}

}  // namespace ofmi
