"""Particle-image rendering and the displacement fields of the benchmark workloads.

Image model (stands in for the paper's 8-bit laser-sheet particle recordings, Sec. 2.2):

* particle centres uniform over the image extended by a margin
  ``m = ceil(max|D|) + ceil(4 sigma)`` on every side, so borders never run empty;
  count ``round(rho * (W + 2m) * (H + 2m))``;
* each particle is a Gaussian spot ``A exp(-|p - c|^2 / (2 sigma^2))`` point-sampled at
  integer pixel centres, truncated at radius ``ceil(4 sigma)``, amplitude ``A ~ U[150, 255]``,
  spots add on a background of 10;
* i.i.d. ``N(0, 3^2)`` noise per pixel and per frame, then clip to [0, 255], round half to
  even, cast to uint8;
* frame 2 renders the same particles moved by ``D`` evaluated at their frame-1 position;
* ground truth at pixel ``(x, y)`` is ``D(x, y)`` (x = column, y = row, pixel centres at
  integers; u along x, v along y).

Seeds: ``numpy.random.SeedSequence([2461, workload_index, item])`` spawned into independent
streams for positions, amplitudes, noise of frame 1, noise of frame 2 and field parameters.
The number of pyramid levels of every workload satisfies the paper's level rule (eq. 1):
``max|D| / 2**(levels - 1) < 3`` px; :func:`workload` asserts it.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Iterator

import numpy as np

F_STAR = 0.638173  # max of f(s) = (1 - exp(-s^2)) / s, reached at s = 1.120906
BACKGROUND = 10.0
NOISE_STD = 3.0
AMP_LO, AMP_HI = 150.0, 255.0


@dataclasses.dataclass(frozen=True)
class Workload:
    """One benchmark workload: image size, particle model and flow-solver parameters."""

    name: str
    index: int          # seed index of the workload
    H: int
    W: int
    rho: float          # particles per pixel
    sigma: float        # spot radius (px)
    levels: int
    radius: int
    iters: int
    fp16: bool          # frames / pyramid stored in FP16 (FP32 math)
    description: str


WORKLOADS = {
    "c1": Workload("c1", 1, 256, 256, 0.05, 1.0, 3, 4, 4, False,
                   "single pair 256x256, Lamb-Oseen vortex (core 30 px, 3 px) + (0.4,-0.3) px, "
                   "3 levels, r=4, 4 iterations, FP32"),
    "c2": Workload("c2", 2, 1024, 1024, 0.03, 1.2, 4, 8, 4, False,
                   "single pair 1024x1024, tanh shear layer 4+4tanh((y-512)/40) + reverse "
                   "Lamb-Oseen vortex (2 px), 4 levels, r=8, 4 iterations, FP32"),
    "c3": Workload("c3", 2, 1024, 1024, 0.03, 1.2, 4, 8, 4, True,
                   "the 1024x1024 pair with FP16 storage of frames and pyramid"),
    "c4": Workload("c4", 4, 0, 0, 0.03, 1.2, 4, 8, 4, True,
                   "batch of 64 pairs: 16x 512x512, 32x 1024(W)x768(H), 16x 2048x2048; 1-3 "
                   "vortices (max 6 px) + uniform shift U[-1,1]; 4 levels, r=8, 4 iterations, FP16"),
    "c5": Workload("c5", 5, 0, 0, 0.03, 1.2, 4, 8, 4, True,
                   "8 streams of 200 frames, sizes from {640x480, 1024x1024, 2048x2048}, "
                   "shear layer + convecting vortex (max 8 px/frame), Poisson arrivals"),
    "t1": Workload("t1", 6, 384, 1792, 0.03, 1.2, 4, 10, 4, False,
                   "the paper's region of interest 1792(W)x384(H), r=10 (Sec. 2.4, Table 1), "
                   "step shear layer with recirculation, max 10 px"),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def _rngs(index: int, item: int, n: int = 5) -> list[np.random.Generator]:
    ss = np.random.SeedSequence([2461, index, item])
    return [np.random.default_rng(s) for s in ss.spawn(n)]


# --------------------------------------------------------------------------- fields

def lamb_oseen(x, y, cx, cy, rc, V, sign=1.0):
    """Lamb-Oseen vortex displacement with peak tangential displacement ``V`` (px).

    Tangential magnitude ``(V / f*) f(rho / rc)`` with ``f(s) = (1 - exp(-s^2)) / s``;
    direction ``(-(y - cy), x - cx) / rho`` times ``sign``.
    """
    dx = np.asarray(x, dtype=np.float64) - cx
    dy = np.asarray(y, dtype=np.float64) - cy
    rho2 = dx * dx + dy * dy
    s2 = rho2 / (rc * rc)
    with np.errstate(divide="ignore", invalid="ignore"):
        coef = np.where(rho2 > 0, (V / F_STAR) * (-np.expm1(-s2)) * rc / np.where(rho2 > 0, rho2, 1.0),
                        (V / F_STAR) / rc)
    return sign * coef * (-dy), sign * coef * dx


Field = Callable[[np.ndarray, np.ndarray], tuple[np.ndarray, np.ndarray]]


def _grid_max(field: Field, H: int, W: int) -> float:
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    du, dv = field(x, y)
    return float(np.sqrt(du * du + dv * dv).max())


def _field_c1(x, y):
    du, dv = lamb_oseen(x, y, 128.0, 128.0, 30.0, 3.0, +1.0)
    return du + 0.4, dv - 0.3


def _field_c2(x, y):
    su = 4.0 + 4.0 * np.tanh((np.asarray(y, np.float64) - 512.0) / 40.0)
    du, dv = lamb_oseen(x, y, 512.0, 448.0, 40.0, 2.0, -1.0)
    return su + du, dv


def _field_t1(x, y):
    # step shear layer across the region of interest plus a recirculation eddy below it
    y = np.asarray(y, np.float64)
    su = 4.0 + 4.0 * np.tanh((y - 128.0) / 30.0)
    du, dv = lamb_oseen(x, y, 700.0, 220.0, 60.0, 2.0, -1.0)
    return su + du, dv


# --------------------------------------------------------------------------- rendering

def render(xp, yp, amp, H, W, sigma, noise_rng, chunk=40000):
    """Render particles to a uint8 frame (Gaussian spots + background + noise)."""
    R = int(math.ceil(4.0 * sigma))
    off = np.arange(-R, R + 1)
    img = np.zeros(H * W, dtype=np.float64)
    inv2s2 = 1.0 / (2.0 * sigma * sigma)
    for s in range(0, len(xp), chunk):
        px = xp[s:s + chunk]
        py = yp[s:s + chunk]
        pa = amp[s:s + chunk]
        ix = np.rint(px).astype(np.int64)[:, None, None] + off[None, None, :]
        iy = np.rint(py).astype(np.int64)[:, None, None] + off[None, :, None]
        dx = ix - px[:, None, None]
        dy = iy - py[:, None, None]
        r2 = dx * dx + dy * dy
        keep = (r2 <= R * R) & (ix >= 0) & (ix < W) & (iy >= 0) & (iy < H)
        val = pa[:, None, None] * np.exp(-r2 * inv2s2)
        flat = (iy * W + ix)
        flat, val = np.broadcast_arrays(flat, val)
        img += np.bincount(flat[keep], weights=val[keep], minlength=H * W)
    img += BACKGROUND + noise_rng.normal(0.0, NOISE_STD, size=H * W)
    return np.rint(np.clip(img, 0.0, 255.0)).astype(np.uint8).reshape(H, W)


def _particles(rng_pos, rng_amp, H, W, rho, margin):
    n = int(round(rho * (W + 2 * margin) * (H + 2 * margin)))
    xp = rng_pos.uniform(-margin, W + margin, size=n)
    yp = rng_pos.uniform(-margin, H + margin, size=n)
    amp = rng_amp.uniform(AMP_LO, AMP_HI, size=n)
    return xp, yp, amp


def _pair_from_field(field: Field, H, W, rho, sigma, rngs, levels=None):
    dmax = _grid_max(field, H, W)
    if levels is not None:
        assert dmax / 2 ** (levels - 1) < 3.0, "level rule (eq. 1) violated"
    margin = int(math.ceil(dmax)) + int(math.ceil(4.0 * sigma))
    xp, yp, amp = _particles(rngs[0], rngs[1], H, W, rho, margin)
    I1 = render(xp, yp, amp, H, W, sigma, rngs[2])
    du, dv = field(xp, yp)
    I2 = render(xp + du, yp + dv, amp, H, W, sigma, rngs[3])
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    gu, gv = field(x, y)
    return I1, I2, gu, gv, dmax


def make_pair(name: str, item: int = 0):
    """Return ``(I1, I2, gt_u, gt_v)`` for a single-pair workload (c1, c2, c3, t1).

    ``item`` selects a distinct seeded pair of the same workload (the bench rotates items).
    """
    wl = WORKLOADS[name]
    fields = {"c1": _field_c1, "c2": _field_c2, "c3": _field_c2, "t1": _field_t1}
    rngs = _rngs(wl.index, item)
    I1, I2, gu, gv, _ = _pair_from_field(fields[name], wl.H, wl.W, wl.rho, wl.sigma, rngs, wl.levels)
    return I1, I2, gu, gv


def table1_pair(item: int = 0, scale: float = 1.0):
    """Pair at the paper's region of interest (1792x384), used by the Table-1 style sweep.
    ``scale`` multiplies the displacement field (scale 0.25 keeps it under 3 px, where eq. 1
    allows a single level, the paper's "n_lev -> 0" case)."""
    if scale == 1.0:
        return make_pair("t1", item)
    wl = WORKLOADS["t1"]

    def field(x, y):
        du, dv = _field_t1(x, y)
        return scale * du, scale * dv

    rngs = _rngs(wl.index, 1000 + item)
    I1, I2, gu, gv, dmax = _pair_from_field(field, wl.H, wl.W, wl.rho, wl.sigma, rngs)
    return I1, I2, gu, gv


# --------------------------------------------------------------------------- batch (c4)

C4_SIZES = [(512, 512)] * 16 + [(768, 1024)] * 32 + [(2048, 2048)] * 16   # (H, W)


def batch_sizes(n: int = 64):
    """Shuffled (H, W) list of the mixed-size batch; ``n < 64`` takes a prefix."""
    rng = _rngs(4, 1_000_000, 1)[0]
    order = rng.permutation(len(C4_SIZES))
    return [C4_SIZES[i] for i in order][:n]


def _vortex_field(rng, H, W, vmax=6.0):
    nv = int(rng.integers(1, 4))
    cx = rng.uniform(0.15, 0.85, size=nv) * W
    cy = rng.uniform(0.15, 0.85, size=nv) * H
    rc = rng.uniform(0.02, 0.08, size=nv) * min(H, W)
    sg = rng.choice([-1.0, 1.0], size=nv)
    shift = rng.uniform(-1.0, 1.0, size=2)

    def raw(x, y):
        du = np.zeros(np.broadcast(np.asarray(x), np.asarray(y)).shape)
        dv = np.zeros_like(du)
        for i in range(nv):
            a, b = lamb_oseen(x, y, cx[i], cy[i], rc[i], 1.0, sg[i])
            du = du + a
            dv = dv + b
        return du, dv

    scale = vmax / _grid_max(raw, H, W)

    def field(x, y):
        du, dv = raw(x, y)
        return scale * du + shift[0], scale * dv + shift[1]

    return field


def batch_items(n: int = 64, sizes=None):
    """Yield ``(H, W, I1, I2, gt_u, gt_v)`` for the mixed-size batch, pair by pair."""
    wl = WORKLOADS["c4"]
    sizes = batch_sizes(n) if sizes is None else sizes
    for i, (H, W) in enumerate(sizes):
        rngs = _rngs(wl.index, i)
        field = _vortex_field(rngs[4], H, W)
        I1, I2, gu, gv, _ = _pair_from_field(field, H, W, wl.rho, wl.sigma, rngs, wl.levels)
        yield H, W, I1, I2, gu, gv


# --------------------------------------------------------------------------- streams (c5)

C5_SIZES = [(480, 640), (1024, 1024), (2048, 2048)]   # (H, W)


def stream_sizes(n_streams: int = 8):
    rng = _rngs(5, 1_000_000, 1)[0]
    return [C5_SIZES[int(k)] for k in rng.integers(0, len(C5_SIZES), size=n_streams)]


def _stream_raw(H, W, t):
    """Unscaled displacement of stream frame t: a tanh shear layer whose centre line oscillates
    (period 50 frames) plus a Lamb-Oseen vortex convecting downstream."""
    yc = H / 2 + 0.1 * H * math.sin(2 * math.pi * t / 50.0)
    delta = 0.04 * H
    xv = (0.25 * W + 0.5 * t * 4.0) % W
    rc = 0.04 * min(H, W)

    def raw(x, y):
        su = 1.0 + np.tanh((np.asarray(y, np.float64) - yc) / delta)
        du, dv = lamb_oseen(x, y, xv, yc - 0.1 * H, rc, 1.0, -1.0)
        return su + du, dv

    return raw


def stream_scale(H: int, W: int, t: int) -> float:
    """Factor that makes the largest displacement of frame t over the pixel grid 8 px."""
    return 8.0 / _grid_max(_stream_raw(H, W, t), H, W)


def _scaled(raw, scale):
    def field(x, y):
        du, dv = raw(x, y)
        return scale * du, scale * dv

    return field


def stream_field(H: int, W: int, t: int, scale: float | None = None) -> Field:
    """Displacement from stream frame t to frame t + 1 (max 8 px over the grid)."""
    return _scaled(_stream_raw(H, W, t), stream_scale(H, W, t) if scale is None else scale)


def stream_particles(stream: int, n_frames: int, size=None, scales=None):
    """Particle states (x, y, amplitude) of frames 0 .. n_frames-1 of one stream: frame t + 1
    moves every particle of frame t by stream_field(t) at its position; particles leaving the
    extended domain are re-seeded uniformly (a sequential, cheap step).  ``scales``: the
    per-frame scales if already computed (``stream_scale``)."""
    wl = WORKLOADS["c5"]
    H, W = stream_sizes()[stream] if size is None else size
    rngs = _rngs(wl.index, stream)
    margin = 8 + int(math.ceil(4.0 * wl.sigma))
    xp, yp, amp = _particles(rngs[0], rngs[1], H, W, wl.rho, margin)
    out = []
    for t in range(n_frames):
        out.append((xp, yp, amp))
        if t + 1 == n_frames:
            break
        sc = stream_scale(H, W, t) if scales is None else scales[t]
        du, dv = stream_field(H, W, t, sc)(xp, yp)
        xp = xp + du
        yp = yp + dv
        amp = amp.copy()
        gone = (xp < -margin) | (xp >= W + margin) | (yp < -margin) | (yp >= H + margin)
        k = int(gone.sum())
        if k:
            xp[gone] = rngs[4].uniform(-margin, W + margin, size=k)
            yp[gone] = rngs[4].uniform(-margin, H + margin, size=k)
            amp[gone] = rngs[4].uniform(AMP_LO, AMP_HI, size=k)
    return out


def stream_frame(stream: int, t: int, state, size) -> np.ndarray:
    """Render frame t of a stream from its particle state; the noise of every frame has a
    seed of its own, so frames can be rendered in any order or in parallel."""
    wl = WORKLOADS["c5"]
    H, W = size
    xp, yp, amp = state
    noise = np.random.default_rng(np.random.SeedSequence([2461, wl.index, stream, 1, t]))
    return render(xp, yp, amp, H, W, wl.sigma, noise)


def stream_frames(stream: int, n_frames: int = 200, size=None) -> Iterator[tuple[np.ndarray, np.ndarray, np.ndarray]]:
    """Yield ``(frame, gt_u, gt_v)`` of one stream; ``gt`` is the displacement to the next frame."""
    H, W = stream_sizes()[stream] if size is None else size
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    for t, state in enumerate(stream_particles(stream, n_frames, (H, W))):
        gu, gv = stream_field(H, W, t)(x, y)
        yield stream_frame(stream, t, state, (H, W)), gu, gv


def _render_job(args):
    stream, t, state, size = args
    return stream_frame(stream, t, state, size)


def _scale_job(args):
    return stream_scale(*args)


def stream_frames_parallel(stream: int, n_frames: int, size, pool) -> list:
    """The frames of ``stream_frames`` (same bytes), rendered over a process pool (an
    ``Executor``): per-frame scales in parallel, the advection in this process, then the
    renders in parallel.  Ground truth is left out (``stream_field`` gives it per frame)."""
    H, W = size
    scales = list(pool.map(_scale_job, [(H, W, t) for t in range(n_frames)]))
    states = stream_particles(stream, n_frames, size, scales)
    return list(pool.map(_render_job, [(stream, t, st, size) for t, st in enumerate(states)]))
