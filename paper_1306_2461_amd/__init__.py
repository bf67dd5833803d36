"""MI355X dense pyramidal Lucas-Kanade velocimetry (Gautier & Aider, Sec. 2.4) on HIP.

Python face of the C ABI in ``include/ofmi.h``.  Tensors are ``torch`` CUDA (HIP) tensors;
the library reads and writes them in place on the current torch stream.
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    OF_FLAG_FP16_STORAGE, OF_FLAG_GAUSSIAN_WINDOW, OF_FLAG_GRAPH, OF_FLAG_INPUT_F32, OF_FLAG_NO_GRAPH,
    OF_FLAG_NORMALIZE,
    OF_KERNEL_ITERATE, OF_KERNEL_LEVEL, OF_KERNEL_REDUCE, OF_STAGE_ITERATE, OF_TIMING_LAUNCH,
    OF_TIMING_LEVEL,
    OF_STAGE_REDUCE, OF_TILE_NARROW, OF_TILE_WIDE, OF_TILE_WIDE16, OF_TILE_WIDE16X2, OF_TILE_WIDE32,
    OF_TILE_LEAN32X2, OF_TILE_WIDE32X2, OF_TILE_WIDE_LEAN,
    OfError,
    last_error, load,
)
from .api import Batch, BubbleMonitor, Plan, compute, debug_stage, levels_for, normalize  # noqa: F401
