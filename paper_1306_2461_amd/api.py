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
    pyramid levels >= 1 in FP16 (all arithmetic FP32); ``input_f32`` takes float32 frames;
    ``graph`` replays a captured hipGraph per buffer tuple instead of launching kernels one by
    one (the default, as fast or faster for one stream of pairs);
    ``normalize`` equalises both frames first (eq. 2); ``gaussian_window`` weights the window
    sums by Gaussian taps (sigma = r/2) instead of the unweighted box.
    The workspace is a torch allocation owned by the plan.
    """

    def __init__(self, H, W, levels, radius, iters, fp16=False, input_f32=False, device=None,
                 graph=False, normalize=False, gaussian_window=False):
        lib = B.load()
        self.H, self.W, self.levels, self.radius, self.iters = H, W, levels, radius, iters
        self.flags = ((B.OF_FLAG_FP16_STORAGE if fp16 else 0) | (B.OF_FLAG_INPUT_F32 if input_f32 else 0)
                      | (B.OF_FLAG_GRAPH if graph else 0) | (B.OF_FLAG_NORMALIZE if normalize else 0)
                      | (B.OF_FLAG_GAUSSIAN_WINDOW if gaussian_window else 0))
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

    def compute_raw(self, i1_ptr: int, i2_ptr: int, u_ptr: int, v_ptr: int, stream_handle: int):
        """of_compute on raw device pointers (no Python-side checks; the C side validates)."""
        B.check(B.load().of_compute(self._h, i1_ptr, i2_ptr, u_ptr, v_ptr, stream_handle), "of_compute")

    def config(self):
        import ctypes
        bands = (ctypes.c_int * self.levels)()
        variant = (ctypes.c_int * self.levels)()
        B.check(B.load().of_plan_get_config(self._h, bands, variant), "of_plan_get_config")
        return {"bands": list(bands), "variant": list(variant)}

    def set_config(self, cfg):
        import ctypes
        bands = (ctypes.c_int * self.levels)(*cfg["bands"])
        variant = (ctypes.c_int * self.levels)(*cfg["variant"])
        B.check(B.load().of_plan_set_config(self._h, bands, variant), "of_plan_set_config")

    def autotune(self, I1, I2, u, v, reps=3, stream=None):
        """Pick the fastest launch configuration per level on these buffers; returns it."""
        B.check(B.load().of_plan_autotune(self._h, I1.data_ptr(), I2.data_ptr(), u.data_ptr(), v.data_ptr(),
                                          _stream_handle(self.device, stream), reps), "of_plan_autotune")
        return self.config()

    def set_mask(self, mask, stream=None):
        """Region-of-interest mask (uint8 H x W device tensor, nonzero = compute) or None.
        Masked pixels get zero flow and tiles without unmasked pixels are skipped."""
        if mask is None:
            ptr = None
        else:
            _check_frame(mask, self.H, self.W, torch.uint8, self.device, "mask")
            ptr = mask.data_ptr()
        B.check(B.load().of_plan_set_mask(self._h, ptr, _stream_handle(self.device, stream)),
                "of_plan_set_mask")

    def set_bubble(self, threshold=None, count=None):
        """eq. 3 count in the final iteration against the device scalar ``threshold`` into the
        device uint64 ``count`` (see BubbleMonitor); None removes it."""
        B.check(B.load().of_plan_set_bubble(self._h, None if threshold is None else threshold.data_ptr(),
                                            None if count is None else count.data_ptr()), "of_plan_set_bubble")

    def set_timing(self, enable):
        """Event timing on the launch stream (measurement only): True / OF_TIMING_LAUNCH
        brackets every launch, OF_TIMING_LEVEL each level's iteration launches and the pyramid
        launches as spans; False switches it off."""
        mode = B.OF_TIMING_LAUNCH if enable is True else int(enable)
        B.check(B.load().of_plan_set_timing(self._h, mode), "of_plan_set_timing")

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


def levels_for(dmax: float, H: int, W: int) -> int:
    """Level count from eq. 1 for a largest expected displacement of `dmax` px (host only)."""
    L = int(B.load().of_levels_for_displacement(float(dmax), int(H), int(W)))
    if L < 1:
        raise B.OfError(f"invalid arguments for levels_for: dmax={dmax}, H={H}, W={W}")
    return L


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


class Batch:
    """``of_batch``: many frame pairs of different sizes computed together.

    ``sizes`` is a list of (H, W); all pairs share levels, radius, iterations and flags.
    Each pyramid step and each (level, iteration) phase is one launch over a work list of
    all pairs' tiles; the whole schedule is replayed as a hipGraph per set of buffers.
    """

    def __init__(self, sizes, levels, radius, iters, fp16=False, input_f32=False, device=None,
                 graph=True, gaussian_window=False):
        import ctypes
        lib = B.load()
        self.sizes = [(int(h), int(w)) for h, w in sizes]
        self.n = len(self.sizes)
        self.levels, self.radius, self.iters = levels, radius, iters
        self.flags = ((B.OF_FLAG_FP16_STORAGE if fp16 else 0) | (B.OF_FLAG_INPUT_F32 if input_f32 else 0)
                      | (0 if graph else B.OF_FLAG_NO_GRAPH)
                      | (B.OF_FLAG_GAUSSIAN_WINDOW if gaussian_window else 0))
        self.frame_dtype = torch.float32 if input_f32 else torch.uint8
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self._H = (ctypes.c_int * self.n)(*[h for h, _ in self.sizes])
        self._W = (ctypes.c_int * self.n)(*[w for _, w in self.sizes])
        nbytes = lib.of_batch_workspace_bytes(self.n, self._H, self._W, levels, radius, iters, self.flags)
        if nbytes == 0:
            raise B.OfError(f"invalid batch parameters: {B.last_error()}")
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            h = lib.of_batch_create(self.n, self._H, self._W, levels, radius, iters, self.flags,
                                    self._ws.data_ptr(), nbytes)
        if not h:
            raise B.OfError(f"of_batch_create failed: {B.last_error()}")
        self._h = h
        self.workspace_bytes = nbytes

    def outputs(self):
        """Fresh (us, vs) lists of float32 planes for every pair."""
        us = [torch.empty(s, dtype=torch.float32, device=self.device) for s in self.sizes]
        vs = [torch.empty(s, dtype=torch.float32, device=self.device) for s in self.sizes]
        return us, vs

    def pointer_arrays(self, I1s, I2s, us, vs):
        """ctypes pointer arrays for compute_raw (checks every plane once)."""
        for i, (h, w) in enumerate(self.sizes):
            _check_frame(I1s[i], h, w, self.frame_dtype, self.device, f"I1[{i}]")
            _check_frame(I2s[i], h, w, self.frame_dtype, self.device, f"I2[{i}]")
            _check_frame(us[i], h, w, torch.float32, self.device, f"u[{i}]")
            _check_frame(vs[i], h, w, torch.float32, self.device, f"v[{i}]")
        return tuple(B.ptr_array([t.data_ptr() for t in ts]) for ts in (I1s, I2s, us, vs))

    def compute(self, I1s, I2s, us=None, vs=None, stream=None):
        if us is None or vs is None:
            us, vs = self.outputs()
        arrs = self.pointer_arrays(I1s, I2s, us, vs)
        self.compute_raw(arrs, _stream_handle(self.device, stream))
        return us, vs

    def compute_raw(self, arrs, stream_handle: int):
        """of_batch_compute on pointer arrays from pointer_arrays()."""
        (p1, _a), (p2, _b), (pu, _c), (pv, _d) = arrs
        B.check(B.load().of_batch_compute(self._h, p1, p2, pu, pv, stream_handle), "of_batch_compute")

    def autotune(self, I1s, I2s, us, vs, reps=3, stream=None):
        (p1, _a), (p2, _b), (pu, _c), (pv, _d) = self.pointer_arrays(I1s, I2s, us, vs)
        B.check(B.load().of_batch_autotune(self._h, p1, p2, pu, pv, _stream_handle(self.device, stream), reps),
                "of_batch_autotune")
        return self.config()

    def config(self):
        import ctypes
        bands = (ctypes.c_int * self.levels)()
        grid = (ctypes.c_int * self.levels)()
        variant = (ctypes.c_int * self.levels)()
        B.check(B.load().of_batch_get_config(self._h, bands, grid, variant), "of_batch_get_config")
        return {"bands": list(bands), "grid": list(grid), "variant": list(variant)}

    def set_config(self, cfg):
        """``cfg``: {"bands": [...], "grid": [...], "variant": [...] (optional; -1 = by tile
        count, else one of OF_TILE_NARROW, OF_TILE_WIDE, OF_TILE_WIDE_LEAN)}, one entry per level."""
        import ctypes
        bands = (ctypes.c_int * self.levels)(*cfg["bands"])
        grid = (ctypes.c_int * self.levels)(*cfg["grid"])
        variant = (ctypes.c_int * self.levels)(*cfg.get("variant", [-1] * self.levels))
        B.check(B.load().of_batch_set_config(self._h, bands, grid, variant), "of_batch_set_config")

    def set_masks(self, masks, stream=None):
        """Region-of-interest masks per pair (uint8 device tensors of each pair's size, nonzero =
        compute, or None for an unmasked pair); ``masks=None`` removes them."""
        if masks is None:
            arr = None
        else:
            ptrs = []
            for i, m in enumerate(masks):
                if m is None:
                    ptrs.append(0)
                else:
                    _check_frame(m, self.sizes[i][0], self.sizes[i][1], torch.uint8, self.device, f"mask[{i}]")
                    ptrs.append(m.data_ptr())
            arr, self._mask_keep = B.ptr_array(ptrs)
        B.check(B.load().of_batch_set_masks(self._h, arr, _stream_handle(self.device, stream)),
                "of_batch_set_masks")

    def set_timing(self, enable):
        """As Plan.set_timing."""
        mode = B.OF_TIMING_LAUNCH if enable is True else int(enable)
        B.check(B.load().of_batch_set_timing(self._h, mode), "of_batch_set_timing")

    def read_timing(self, kernel: int):
        import ctypes
        ms, n, un, by = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
        B.check(B.load().of_batch_read_timing(self._h, kernel, ctypes.byref(ms), ctypes.byref(n),
                                              ctypes.byref(un), ctypes.byref(by)), "of_batch_read_timing")
        return ms.value, n.value, un.value, by.value

    def close(self):
        if getattr(self, "_h", None):
            B.load().of_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def normalize(I, radius: int = 5, eps: float = 1.0, out=None, stream=None):
    """Local equalisation of one frame (eq. 2 reading): (I - mean) / (std + eps) over the
    (2r+1)^2 window truncated at the border.  uint8 or float32 in, float32 out."""
    if I.dtype not in (torch.uint8, torch.float32) or not I.is_contiguous() or I.dim() != 2:
        raise B.OfError("normalize takes a contiguous 2-D uint8 or float32 tensor")
    H, W = I.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=I.device)
    flags = B.OF_FLAG_INPUT_F32 if I.dtype == torch.float32 else 0
    B.check(B.load().of_normalize(I.data_ptr(), out.data_ptr(), H, W, radius, float(eps), flags,
                                  _stream_handle(I.device, stream)), "of_normalize")
    return out


class BubbleMonitor:
    """Recirculation-bubble surface of a sequence of fields (Sec. 3.2, eq. 3), on the device.

    Keeps the running time-mean of the streamwise component, the threshold T_v = (min + max)/2
    of the mean of the fields seen so far, the count of vectors at or below it and S_bubble,
    all as device tensors.  ``attach(plan)`` makes the plan's final iteration count the vectors
    at or below the current threshold as it writes them; ``step(u)`` after each field then
    finishes S_bubble for that field and moves the mean and threshold on (``of_bubble_step``).
    Nothing is read back to the host: ``surface`` holds S_bubble of the last field once the
    work on the stream passed to ``step`` has completed."""

    def __init__(self, H, W, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.n = H * W
        self.mean = torch.zeros((H, W), dtype=torch.float32, device=self.device)
        self.threshold = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.count = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.surface = torch.zeros(1, dtype=torch.float32, device=self.device)
        self._work = torch.empty(2, dtype=torch.int32, device=self.device)
        self.t = 0

    def attach(self, plan):
        """Count at or below the threshold inside ``plan``'s final iteration."""
        B.check(B.load().of_plan_set_bubble(plan._h, self.threshold.data_ptr(), self.count.data_ptr()),
                "of_plan_set_bubble")

    def detach(self, plan):
        B.check(B.load().of_plan_set_bubble(plan._h, None, None), "of_plan_set_bubble")

    def step(self, u, stream=None):
        """Finish S_bubble of field u (computed by the attached plan, or any field for t = 0)
        and fold u into the mean; returns the device tensor ``surface``."""
        B.check(B.load().of_bubble_step(self.mean.data_ptr(), u.data_ptr(), self.n, self.t,
                                        self.count.data_ptr(), self.threshold.data_ptr(),
                                        self.surface.data_ptr(), self._work.data_ptr(),
                                        _stream_handle(self.device, stream)), "of_bubble_step")
        self.t += 1
        return self.surface
