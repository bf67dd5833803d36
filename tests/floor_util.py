"""Per-pixel FP32 rounding floor of the oracle's operation order (test infrastructure).

The GPU path computes in FP32 (FP16 storage for the FP16 form) and is compared with the FP64
oracle.  Where a window is nearly singular or the iteration is not contractive (frames whose
content leaves the image, 3x3 windows over several iterations, windows weighted toward clamped
columns), rounding errors of order 1e-7 are amplified, and no FP32 evaluation of the method
can be expected to land within the tolerance of the FP64 result there.  This module measures
how far FP32 evaluations of the oracle's own operation order land, pixel by pixel:

    floor(p) = max over k and over pixels q within the window radius r of p of
               |flow_k(q) - flow_64(q)|   (max over u and v)

where flow_64 is the oracle in float64 and flow_k, k = 1..5, are the oracle run in float32
with split warp coordinates (the form the kernels use) on inputs that give the same result in
exact arithmetic: the frames themselves; the transposed frames (transpose equivariance: the
flow of the transposed pair is the transposed flow with u and v exchanged); the frames plus
37 (the method sees only differences and gradients of intensities); the frames times 3 (the
2x2 solve is invariant to a common intensity scale, and so is its singularity test); and
(3 x frames + 11) transposed.  Each changes which operands meet in every rounding, so the five
runs are five equally valid FP32 rounding orders.  The maximum is also taken over the pixel's
window neighbourhood: an iteration mixes the rounding of every pixel of a window into the
window's centre, so the amplification a sixth rounding order meets at p is sampled better by
the realisations' departures around p than at p alone.  A GPU pixel passes when its error is within
the tolerance, or within the tolerance plus FLOOR_FACTOR times the floor at that pixel; the
GPU tests print how many pixels needed the floor and where.

The per-case floors are stored in tests/golden/floor/<case>.npz by tests/golden/make_floor.py
(which calls only the oracle and the input generators).
"""
from __future__ import annotations

import os

import numpy as np

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
FLOOR_DIR = os.path.join(HERE, "golden", "floor")

# A GPU pixel may depart from the oracle by tol + FLOOR_FACTOR * floor(p).  The five float32
# realisations spread by up to a factor of ~10 among themselves at floor-bound pixels; the GPU
# (FMA contraction, a compensated determinant, reciprocal division, its own summation order)
# is a sixth realisation of the same spread.
FLOOR_FACTOR = 3.0

TOL32 = 1e-3
TOL16 = 2e-2

# Served small streams of the serving tests (H, W), parameters L, r, K.
SERVE_SIZES = [(96, 128), (160, 120), (64, 200)]
SERVE_LRK = (3, 4, 3)


def _r1_inputs():
    I1, I2, _, _ = synth.make_pair("c1", 4)
    return I1[:129, :200].copy(), I2[:129, :200].copy()


def _serve_inputs(s, t):
    def f():
        fr = [x for x, _, _ in synth.stream_frames(s, t + 2, size=SERVE_SIZES[s])]
        return fr[t], fr[t + 1]
    return f


def _c5_640_inputs():
    fr = [x for x, _, _ in synth.stream_frames(0, 2, size=(480, 640))]
    return fr[0], fr[1]


def _pair(name, item):
    def f():
        I1, I2, _, _ = synth.make_pair(name, item)
        return I1, I2
    return f


# name -> (inputs, levels, radius, iters, window, storage, tolerance)
CASES = {
    "c1": (_pair("c1", 0), 3, 4, 4, "box", None, TOL32),
    "c2": (_pair("c2", 0), 4, 8, 4, "box", None, TOL32),
    "c3_fp16": (_pair("c2", 0), 4, 8, 4, "box", np.float16, TOL16),
    "c2_gauss": (_pair("c2", 0), 4, 8, 4, "gauss", None, TOL32),
    "c5_640_fp16": (_c5_640_inputs, 4, 8, 4, "box", np.float16, TOL16),
    "r1_L1_K1": (_r1_inputs, 1, 1, 1, "box", None, TOL32),
    "r1_L1_K3": (_r1_inputs, 1, 1, 3, "box", None, TOL32),
    "r1_L2_K3": (_r1_inputs, 2, 1, 3, "box", None, TOL32),
}
for _s in range(3):
    for _t in range(3):
        CASES[f"serve_{_s}_{_t}"] = (_serve_inputs(_s, _t), *SERVE_LRK, "box", None, TOL32)


def case_inputs(name):
    return CASES[name][0]()


def realisations(I1, I2):
    """(frame 1, frame 2, transposed) triples: five inputs with the same exact flow."""
    a = np.asarray(I1, dtype=np.float64)
    b = np.asarray(I2, dtype=np.float64)
    return [(I1, I2, False), (np.ascontiguousarray(I1.T), np.ascontiguousarray(I2.T), True),
            (a + 37.0, b + 37.0, False), (a * 3.0, b * 3.0, False),
            (np.ascontiguousarray((a * 3.0 + 11.0).T), np.ascontiguousarray((b * 3.0 + 11.0).T), True)]


def ensemble_floor(I1, I2, levels, radius, iters, window="box", storage=None):
    """(floor, flow64): the per-pixel floor (float64 array) and the FP64 oracle flow."""
    from scipy import ndimage
    u, v = oracle.flow(I1, I2, levels, radius, iters, window=window)
    floor = np.zeros(u.shape)
    for f1, f2, tr in realisations(I1, I2):
        uk, vk = oracle.flow(f1, f2, levels, radius, iters, dtype=np.float32, coords="split",
                             window=window, storage=storage)
        if tr:
            uk, vk = vk.T, uk.T
        floor = np.maximum(floor, np.maximum(np.abs(uk - u), np.abs(vk - v)))
    floor = ndimage.maximum_filter(floor, size=2 * radius + 1, mode="nearest")
    return floor, (u, v)


def case_floor(name):
    inp, L, r, K, window, storage, _ = CASES[name]
    I1, I2 = inp()
    return ensemble_floor(I1, I2, L, r, K, window, storage)[0]


def keep_threshold(name):
    """Floors below this are not stored (they are far below the tolerance)."""
    return CASES[name][6] / 50.0


def save_floor(name, floor):
    os.makedirs(FLOOR_DIR, exist_ok=True)
    keep = floor > keep_threshold(name)
    idx = np.flatnonzero(keep).astype(np.int64)
    np.savez(os.path.join(FLOOR_DIR, f"{name}.npz"), shape=np.asarray(floor.shape, dtype=np.int64),
             idx=idx, val=floor.ravel()[idx].astype(np.float64), max=np.float64(floor.max()),
             threshold=np.float64(keep_threshold(name)))


def load_floor(name):
    """Dense floor of a case from its fixture (0 where it was below the storage threshold)."""
    with np.load(os.path.join(FLOOR_DIR, f"{name}.npz"), allow_pickle=False) as z:
        shape = tuple(int(s) for s in z["shape"])
        out = np.zeros(int(np.prod(shape)))
        out[z["idx"]] = z["val"]
        return out.reshape(shape)


def check_all_pixels(d, tol, floor, what=""):
    """Every pixel of the error map d passes at tol or within tol + FLOOR_FACTOR * floor.

    Returns a one-line summary (printed by the tests); raises AssertionError with the worst
    pixels otherwise."""
    assert d.shape == floor.shape, (d.shape, floor.shape)
    over = d > tol
    bound = tol + FLOOR_FACTOR * floor
    bad = d > bound
    locs = np.argwhere(over)
    summary = (f"{what}: max {d.max():.3e} px; {int(over.sum())} of {d.size} px over {tol:g} "
               f"(floor-bound), largest floor there {floor[over].max() if over.any() else 0.0:.3e}")
    if over.any():
        rows, cols = locs[:, 0], locs[:, 1]
        summary += (f", rows {rows.min()}..{rows.max()}, cols {cols.min()}..{cols.max()}, "
                    f"max error/floor {np.max((d[over] - tol) / np.maximum(floor[over], 1e-30)):.2f}")
    if bad.any():
        worst = np.argsort(-(d - bound).ravel())[:8]
        pts = [(int(i // d.shape[1]), int(i % d.shape[1]), float(d.ravel()[i]),
                float(floor.ravel()[i])) for i in worst if bad.ravel()[i]]
        raise AssertionError(f"{summary}; {int(bad.sum())} px beyond tol + {FLOOR_FACTOR} x floor: "
                             f"(row, col, error, floor) {pts}")
    return summary
