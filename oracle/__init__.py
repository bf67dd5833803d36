"""FP64 CPU oracle of the dense pyramidal Lucas-Kanade flow (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package.  It shares no code with the HIP path.
"""
from .lk import (  # noqa: F401
    TAU, bilinear, blur5, box_sum, flow, gaussian_weights, gradients, lk_iteration, mask_pyramid,
    pyr_reduce, pyramid, solve, upsample_flow, warp, window_sum,
)
from .extras import (  # noqa: F401,E402
    bubble_series, bubble_surface, bubble_threshold, levels_for_displacement, local_normalize, running_mean,
)
