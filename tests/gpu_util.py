"""Helpers of the GPU tests: device transfer, runs through the C ABI, error reports."""
import sys

import numpy as np


def dev():
    import torch
    return torch.device("cuda", 0)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def announce(msg):
    print(f"[gpu case] {msg}", file=sys.stderr, flush=True)


def gpu_flow(ofmi, I1, I2, levels, radius, iters, fp16=False):
    import torch
    H, W = I1.shape
    announce(f"flow {H}x{W} L={levels} r={radius} K={iters} fp16={fp16} dtype={I1.dtype}")
    plan = ofmi.Plan(H, W, levels, radius, iters, fp16=fp16, input_f32=I1.dtype == np.float32,
                     device=dev())
    u, v = plan.compute(to_dev(I1), to_dev(I2))
    torch.cuda.synchronize()
    out = u.cpu().numpy(), v.cpu().numpy()
    plan.close()
    return out


def flow_error(u, v, ou, ov):
    d = np.maximum(np.abs(u.astype(np.float64) - ou), np.abs(v.astype(np.float64) - ov))
    return d


def report(d, tol):
    n_bad = int((d > tol).sum())
    i = np.unravel_index(int(d.argmax()), d.shape)
    rms = float(np.sqrt((d ** 2).mean()))
    return f"max {d.max():.3e} at {i}, rms {rms:.3e}, {n_bad} px over {tol}"
