"""Table-1 style sweep (Sec. 3.3, Table 1): error and fields/s as functions of the number of
levels n_lev and of iterations per level n_iter, at the paper's region of interest
(1792 x 384, window radius 10, Sec. 2.4).

The paper does not define its error; as its (4, 7) cell reads 0 %, one error here is taken
relative to the (n_lev=4, n_iter=7) field: mean |w - w_ref| / mean |w_ref| in percent, with w
the displacement vector per pixel.  With the synthetic pair's ground truth a second error is
the same ratio against the true field (and its RMS end-point error in px), on the interior
(``margin`` px from the borders).  Fields/s is one field per of_compute call, back to back on
one stream with the inputs resident on the device.  n_lev = 1 is the paper's "n_lev -> 0"
case (no pyramid, Sec. 3.3).
"""
from __future__ import annotations

import time

import torch

from .api import Plan


def _err(u, v, ur, vr, margin=0):
    sl = (slice(margin, u.shape[0] - margin), slice(margin, u.shape[1] - margin))
    u, v, ur, vr = u[sl], v[sl], ur[sl], vr[sl]
    d = torch.sqrt((u - ur) ** 2 + (v - vr) ** 2)
    ref = torch.sqrt(ur ** 2 + vr ** 2).mean()
    return float(100.0 * d.mean() / ref), float(torch.sqrt((d ** 2).mean()))


def table1_sweep(I1, I2, radius=10, levels=(3, 4), iters=range(1, 8), ref=(4, 7), reps=50,
                 device=None, truth=None, margin=24):
    """I1, I2: device uint8 frames; truth: optional (gu, gv) device float tensors.
    Returns {n_lev: {"error_percent": [...], "fields_per_s": [...], and with truth
    "error_vs_truth_percent": [...], "rms_vs_truth_px": [...]}}."""
    H, W = I1.shape
    dev = I1.device if device is None else device
    p = Plan(H, W, ref[0], radius, ref[1], device=dev)
    ur, vr = p.compute(I1, I2)
    torch.cuda.synchronize()
    p.close()
    out = {}
    st = torch.cuda.current_stream().cuda_stream
    for L in levels:
        row = {"error_percent": [], "fields_per_s": []}
        if truth is not None:
            row["error_vs_truth_percent"] = []
            row["rms_vs_truth_px"] = []
        for K in iters:
            p = Plan(H, W, L, radius, K, device=dev)
            u, v = p.compute(I1, I2)
            torch.cuda.synchronize()
            row["error_percent"].append(_err(u, v, ur, vr)[0])
            if truth is not None:
                e, rms = _err(u, v, truth[0], truth[1], margin)
                row["error_vs_truth_percent"].append(e)
                row["rms_vs_truth_px"].append(rms)
            args = (I1.data_ptr(), I2.data_ptr(), u.data_ptr(), v.data_ptr(), st)
            for _ in range(5):
                p.compute_raw(*args)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                p.compute_raw(*args)
            torch.cuda.synchronize()
            row["fields_per_s"].append(reps / (time.perf_counter() - t))
            p.close()
        out[L] = row
    return out
