"""Plan objects over the C ABI (argument marshalling only)."""
from __future__ import annotations

import torch

from . import _binding as B


def _stream_handle(device, stream=None) -> int:
    s = torch.cuda.current_stream(device) if stream is None else stream
    return int(s.cuda_stream)


def _check_frame(t, H, W, dtype, device, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise B.OfError(f"{name} must be a device tensor")
    if t.dtype != dtype or tuple(t.shape) != (H, W) or not t.is_contiguous():
        raise B.OfError(f"{name} must be a contiguous {H}x{W} {dtype} tensor, got "
                        f"{tuple(t.shape)} {t.dtype}")
    if t.device != device:
        raise B.OfError(f"{name} is on {t.device}, plan is on {device}")


class Plan:
    """``of_plan`` for one frame size.

    ``levels`` counts pyramid levels including full resolution, ``radius`` is the window
    radius and ``iters`` the iterations per level (Sec. 2.4, eq. 1).  ``fp16`` stores the
    pyramid levels >= 1 in FP16 (all arithmetic FP32); ``input_f32`` takes float32 frames.
    The workspace is a torch allocation owned by the plan.
    """

    def __init__(self, H, W, levels, radius, iters, fp16=False, input_f32=False, device=None):
        lib = B.load()
        self.H, self.W, self.levels, self.radius, self.iters = H, W, levels, radius, iters
        self.flags = (B.OF_FLAG_FP16_STORAGE if fp16 else 0) | (B.OF_FLAG_INPUT_F32 if input_f32 else 0)
        self.frame_dtype = torch.float32 if input_f32 else torch.uint8
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        nbytes = lib.of_plan_workspace_bytes(H, W, levels, radius, iters, self.flags)
        if nbytes == 0:
            raise B.OfError(f"invalid plan parameters: {B.last_error()}")
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            h = lib.of_plan_create_ex(H, W, levels, radius, iters, self.flags,
                                      self._ws.data_ptr(), nbytes)
        if not h:
            raise B.OfError(f"of_plan_create_ex failed: {B.last_error()}")
        self._h = h
        self.workspace_bytes = nbytes

    def compute(self, I1, I2, u=None, v=None, stream=None):
        """Enqueue the flow of (I1 -> I2) into u, v (allocated if None); returns (u, v)."""
        _check_frame(I1, self.H, self.W, self.frame_dtype, self.device, "I1")
        _check_frame(I2, self.H, self.W, self.frame_dtype, self.device, "I2")
        if u is None:
            u = torch.empty((self.H, self.W), dtype=torch.float32, device=self.device)
        if v is None:
            v = torch.empty((self.H, self.W), dtype=torch.float32, device=self.device)
        _check_frame(u, self.H, self.W, torch.float32, self.device, "u")
        _check_frame(v, self.H, self.W, torch.float32, self.device, "v")
        st = B.load().of_compute(self._h, I1.data_ptr(), I2.data_ptr(), u.data_ptr(),
                                 v.data_ptr(), _stream_handle(self.device, stream))
        B.check(st, "of_compute")
        return u, v

    def set_timing(self, enable: bool):
        """Bracket every kernel launch with hipEvents on its stream (measurement only)."""
        B.check(B.load().of_plan_set_timing(self._h, 1 if enable else 0), "of_plan_set_timing")

    def read_timing(self, kernel: int):
        """(total_ms, launches, units, algorithmic bytes) since the last read; waits on events."""
        return read_timing(self._h, kernel)

    def close(self):
        if getattr(self, "_h", None):
            B.load().of_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def read_timing(handle, kernel: int):
    import ctypes
    ms, n, un, by = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
    B.check(B.load().of_plan_read_timing(handle, kernel, ctypes.byref(ms), ctypes.byref(n),
                                         ctypes.byref(un), ctypes.byref(by)), "of_plan_read_timing")
    return ms.value, n.value, un.value, by.value


def compute(I1, I2, levels, radius, iters, fp16=False):
    """One-shot flow of a frame pair (creates a plan for the pair's size)."""
    H, W = I1.shape
    plan = Plan(H, W, levels, radius, iters, fp16=fp16, input_f32=I1.dtype == torch.float32,
                device=I1.device)
    u, v = plan.compute(I1, I2)
    torch.cuda.current_stream(I1.device).synchronize()
    plan.close()
    return u, v


def debug_stage(plan: Plan, stage: int, level: int, inputs, outputs, stream=None):
    """Run one stage (``OF_STAGE_REDUCE`` / ``OF_STAGE_ITERATE``) on caller tensors."""
    pin, _a = B.ptr_array([t.data_ptr() for t in inputs])
    pout, _b = B.ptr_array([t.data_ptr() for t in outputs])
    st = B.load().of_debug_stage(plan._h, stage, level, pin, pout,
                                 _stream_handle(plan.device, stream))
    B.check(st, "of_debug_stage")
