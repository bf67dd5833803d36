"""FP64 CPU oracle of dense pyramidal iterative Lucas-Kanade optical flow.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import this module; the product path never calls it and shares no code with it.

What it computes follows the paper's description of its optical-flow algorithm (Sec. 2.4):
a dense, window-based, gradient-based method of the Lucas-Kanade family that gives one
displacement vector per pixel; the two images are reduced in size by a factor of 4 in area
level after level into a pyramid; at the coarsest level the displacement starts at zero and
is refined by an iterative Gauss-Newton minimisation of a sum of squared differences over an
interrogation window of radius r; each level's result seeds the next finer level, down to
the full-resolution images.  n_lev (levels, counting full resolution, eq. 1) and n_iter
(iterations per level) are the method's parameters.

The paper leaves the operators themselves unspecified; this oracle fixes them as follows
(every choice is shared by the HIP path):

* pyramid reduce: separable 5-tap binomial [1, 4, 6, 4, 1] / 16, first along rows (y) then
  along columns (x), clamp-to-edge, keep even rows and columns; level sizes ceil(H/2) x ceil(W/2);
* prolongation to a finer level: u <- 2 * bilinear(u_coarse, x/2, y/2), same for v;
* warp: W2(x, y) = bilinear(I2, x + u, y + v), sample coordinates clamped into the image;
* gradients: central differences of the warped frame W2 with clamped neighbours;
* window: unweighted (2r+1)^2 box, truncated at the image border (variant: separable Gaussian
  taps over the same support, ``gaussian_weights``);
* Gauss-Newton step: the residual of every window pixel m is linearised around that pixel's
  own current displacement u(m): W2(m) + grad W2(m) . (d - u(m)) - I1(m), with d the displacement
  sought for the window centre x.  With It(m) = W2(m) - I1(m) - grad W2(m) . u(m), A, B, C, sx,
  sy the window sums of Ix^2, IxIy, Iy^2, Ix It, Iy It and H = [[A, B], [B, C]], the least-squares
  d solves H d = -(sx, sy).  It is computed as an increment from the centre's estimate,
  u(x) + e with H e = -b, b = (sx, sy) + H u(x), which is the same d whenever H is regular and
  keeps the estimate along directions where the window carries no gradient.  T = A + C,
  D = AC - B^2: e by Cramer's rule when D > tau T^2, by the rank-1 pseudo-inverse H / T^2 when
  T > 0, else e = 0; tau = 1e-5;
* iterations are Jacobi (every pixel reads the field of the previous iteration), a fixed
  count per level, no early exit; iters = 0 returns zeros.

``dtype`` exists only for the rounding-floor diagnostic (running the same operation order in
float32); the oracle is the float64 path.
"""
from __future__ import annotations

import numpy as np

TAU = 1e-5
BINOMIAL5 = (1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16)


def bilinear(Z, X, Y):
    """Bilinear sample of plane ``Z[y, x]`` at real coordinates, clamped into the plane."""
    H, W = Z.shape
    dt = Z.dtype
    Xc = np.clip(X, 0, W - 1).astype(dt, copy=False)
    Yc = np.clip(Y, 0, H - 1).astype(dt, copy=False)
    x0 = np.floor(Xc).astype(np.int64)
    y0 = np.floor(Yc).astype(np.int64)
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    a = Xc - x0.astype(dt)
    b = Yc - y0.astype(dt)
    one = dt.type(1)
    return ((one - a) * (one - b) * Z[y0, x0] + a * (one - b) * Z[y0, x1]
            + (one - a) * b * Z[y1, x0] + a * b * Z[y1, x1])


def blur5(P, axis):
    """Binomial [1,4,6,4,1]/16 filter along ``axis`` with clamp-to-edge indices."""
    n = P.shape[axis]
    idx = np.arange(n)
    out = np.zeros_like(P)
    for j, w in zip(range(-2, 3), BINOMIAL5):
        out = out + P.dtype.type(w) * np.take(P, np.clip(idx + j, 0, n - 1), axis=axis)
    return out


def pyr_reduce(P):
    """One pyramid step: blur along y, then along x, then keep even rows and columns."""
    B = blur5(blur5(P, axis=0), axis=1)
    return B[0::2, 0::2].copy()


def pyramid(F, levels, dtype=np.float64, storage=None):
    """Level 0 is the frame itself (converted exactly); level l+1 = pyr_reduce(level l).

    ``storage`` (e.g. ``np.float16``): every level >= 1 is rounded to that type as it is
    produced (and read back exactly), modelling reduced-precision storage of the pyramid for
    the rounding-floor diagnostic; None keeps ``dtype`` throughout."""
    P = [np.asarray(F).astype(dtype)]
    for _ in range(levels - 1):
        nxt = pyr_reduce(P[-1])
        if storage is not None:
            nxt = nxt.astype(storage).astype(dtype)
        P.append(nxt)
    return P


def upsample_flow(uc, H, W):
    """Prolongation of a coarse field to an (H, W) level: 2 * bilinear(uc, x/2, y/2)."""
    dt = uc.dtype
    y, x = np.mgrid[0:H, 0:W]
    return dt.type(2) * bilinear(uc, x.astype(dt) / dt.type(2), y.astype(dt) / dt.type(2))


def bilinear_split(Z, x, y, u, v):
    """The same sample as ``bilinear(Z, x + u, y + v)`` for integer pixel indices x, y, with
    the coordinate kept as an integer base x + floor(u) and a fraction u - floor(u) instead of
    the rounded sum (the sum loses the low bits of u in reduced precision).  A base outside
    [0, W-2] is clamped into the plane with fraction 0, which is where the clamped coordinate
    of ``bilinear`` lands; equal to ``bilinear`` in exact arithmetic."""
    H, W = Z.shape
    dt = Z.dtype
    fu, fv = np.floor(u), np.floor(v)
    bx = x + fu.astype(np.int64)
    by = y + fv.astype(np.int64)
    inx = (bx >= 0) & (bx <= W - 2)
    iny = (by >= 0) & (by <= H - 2)
    a = np.where(inx, u - fu, dt.type(0)).astype(dt, copy=False)
    b = np.where(iny, v - fv, dt.type(0)).astype(dt, copy=False)
    x0 = np.clip(bx, 0, W - 1)
    y0 = np.clip(by, 0, H - 1)
    x1 = np.where(inx, x0 + 1, x0)
    y1 = np.where(iny, y0 + 1, y0)
    one = dt.type(1)
    return ((one - a) * (one - b) * Z[y0, x0] + a * (one - b) * Z[y0, x1]
            + (one - a) * b * Z[y1, x0] + a * b * Z[y1, x1])


def warp(I2, u, v, coords="sum"):
    """W2(x, y) = I2 sampled at (x + u, y + v) with clamped coordinates.

    ``coords``: "sum" forms the sample coordinate x + u (the oracle's definition); "split"
    keeps integer base and fraction apart (``bilinear_split``), used by the reduced-precision
    rounding-floor diagnostic; both are the same function in exact arithmetic."""
    H, W = I2.shape
    dt = I2.dtype
    y, x = np.mgrid[0:H, 0:W]
    if coords == "split":
        return bilinear_split(I2, x, y, u, v)
    if coords != "sum":
        raise ValueError("coords must be 'sum' or 'split'")
    return bilinear(I2, x.astype(dt) + u, y.astype(dt) + v)


def gradients(W2):
    """Central differences along x (columns) and y (rows) with clamped neighbours."""
    H, W = W2.shape
    xi = np.arange(W)
    yi = np.arange(H)
    half = W2.dtype.type(0.5)
    Ix = (W2[:, np.minimum(xi + 1, W - 1)] - W2[:, np.maximum(xi - 1, 0)]) * half
    Iy = (W2[np.minimum(yi + 1, H - 1), :] - W2[np.maximum(yi - 1, 0), :]) * half
    return Ix, Iy


def box_sum(p, r):
    """S(x, y) = sum of p over the in-image part of the (2r+1)^2 window centred on (x, y).

    Written as the double sum over dy of (the sum over dx), outside-image terms being zero.
    """
    H, W = p.shape
    q = np.zeros((H + 2 * r, W + 2 * r), dtype=p.dtype)
    q[r:r + H, r:r + W] = p
    rows = np.zeros((H + 2 * r, W), dtype=p.dtype)
    for dx in range(2 * r + 1):
        rows = rows + q[:, dx:dx + W]
    out = np.zeros((H, W), dtype=p.dtype)
    for dy in range(2 * r + 1):
        out = out + rows[dy:dy + H, :]
    return out


def gaussian_weights(r):
    """Taps of the Gaussian-weighted window variant: g(d) = exp(-d^2 / (2 sigma^2)) for
    d = -r..r with sigma = r / 2 (r = 0: a single tap of weight 1).  The paper's window is the
    unweighted box of radius r; the weighted window is the usual alternative in this family of
    solvers, with the same support, so that the taps at the window edge weigh exp(-2)."""
    if r == 0:
        return np.ones(1)
    d = np.arange(-r, r + 1, dtype=np.float64)
    sigma = r / 2.0
    return np.exp(-d * d / (2.0 * sigma * sigma))


def window_sum(p, r, weights=None):
    """Weighted window sum S(x, y) = sum over the in-image part of the (2r+1)^2 window of
    g[dy] g[dx] p(y + dy, x + dx) (outside-image terms zero), as the double sum over dy of the
    sum over dx.  weights=None is the unweighted box (``box_sum``)."""
    if weights is None:
        return box_sum(p, r)
    g = np.asarray(weights, dtype=p.dtype)
    H, W = p.shape
    q = np.zeros((H + 2 * r, W + 2 * r), dtype=p.dtype)
    q[r:r + H, r:r + W] = p
    rows = np.zeros((H + 2 * r, W), dtype=p.dtype)
    for dx in range(2 * r + 1):
        rows = rows + g[dx] * q[:, dx:dx + W]
    out = np.zeros((H, W), dtype=p.dtype)
    for dy in range(2 * r + 1):
        out = out + g[dy] * rows[dy:dy + H, :]
    return out


def solve(A, B, C, bx, by, tau=TAU):
    """Per-pixel Gauss-Newton increment (du, dv) from the five window sums.

    H = [[A, B], [B, C]], b = [bx, by]; d solves H d = -b when D = AC - B^2 > tau (A+C)^2,
    else d = -(H / T^2) b with T = A + C when T > 0 (rank-1 pseudo-inverse), else d = 0.
    """
    dt = A.dtype
    T = A + C
    D = A * C - B * B
    full = D > dt.type(tau) * T * T
    rank1 = (~full) & (T > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        du_f = -(C * bx - B * by) / D
        dv_f = -(A * by - B * bx) / D
        T2 = T * T
        du_1 = -(A * bx + B * by) / T2
        dv_1 = -(B * bx + C * by) / T2
    zero = dt.type(0)
    du = np.where(full, du_f, np.where(rank1, du_1, zero))
    dv = np.where(full, dv_f, np.where(rank1, dv_1, zero))
    return du, dv


def lk_iteration(I1l, I2l, u, v, r, tau=TAU, weights=None, coords="sum"):
    """One Gauss-Newton iteration at one level: warp, gradients, window sums, solve, update.
    ``weights``: separable window taps (None = unweighted box); ``coords``: see ``warp``."""
    W2 = warp(I2l, u, v, coords)
    Ix, Iy = gradients(W2)
    It = W2 - I1l - Ix * u - Iy * v
    A, B, C, sx, sy = (window_sum(p, r, weights) for p in (Ix * Ix, Ix * Iy, Iy * Iy, Ix * It, Iy * It))
    bx = sx + A * u + B * v
    by = sy + B * u + C * v
    du, dv = solve(A, B, C, bx, by, tau=tau)
    return u + du, v + dv


def mask_pyramid(M, levels):
    """Masks of all levels from a level-0 mask (True = computed): a coarser pixel is computed
    when any of its (up to four) finer pixels is.  Reading of the paper's suggestion to skip
    computation over obstacles and side walls (Sec. 3.3)."""
    out = [np.asarray(M, dtype=bool)]
    for _ in range(levels - 1):
        m = out[-1]
        H, W = m.shape
        ys = np.arange((H + 1) // 2) * 2
        xs = np.arange((W + 1) // 2) * 2
        y1 = np.minimum(ys + 1, H - 1)
        x1 = np.minimum(xs + 1, W - 1)
        out.append(m[np.ix_(ys, xs)] | m[np.ix_(ys, x1)] | m[np.ix_(y1, xs)] | m[np.ix_(y1, x1)])
    return out


def flow(I1, I2, levels, radius, iters, tau=TAU, dtype=np.float64, return_levels=False,
         mask=None, window="box", coords="sum", storage=None):
    """Dense displacement (u, v) in level-0 pixels from frame I1 to frame I2.

    ``levels`` counts the pyramid levels including full resolution (>= 1), ``radius`` is the
    window radius r >= 0 and ``iters`` the Gauss-Newton iterations per level (>= 0).
    ``mask`` (optional, level-0 booleans, True = computed): after every iteration the field is
    set to zero at the pixels the level's mask (``mask_pyramid``) excludes.
    ``window``: "box" (unweighted) or "gauss" (``gaussian_weights``).
    ``coords``: sample coordinates of the warp, "sum" (the definition) or "split" (``warp``).
    ``storage``: reduced-precision storage of pyramid levels >= 1 (``pyramid``), diagnostic only.
    """
    if window not in ("box", "gauss"):
        raise ValueError("window must be 'box' or 'gauss'")
    weights = gaussian_weights(radius) if window == "gauss" else None
    if levels < 1 or radius < 0 or iters < 0:
        raise ValueError("levels >= 1, radius >= 0, iters >= 0 required")
    P1 = pyramid(I1, levels, dtype, storage)
    P2 = pyramid(I2, levels, dtype, storage)
    M = mask_pyramid(mask, levels) if mask is not None else None
    H, W = P1[-1].shape
    u = np.zeros((H, W), dtype=dtype)
    v = np.zeros((H, W), dtype=dtype)
    per_level = []
    for lev in range(levels - 1, -1, -1):
        H, W = P1[lev].shape
        if lev < levels - 1:
            u = upsample_flow(u, H, W)
            v = upsample_flow(v, H, W)
        for _ in range(iters):
            u, v = lk_iteration(P1[lev], P2[lev], u, v, radius, tau, weights, coords)
            if M is not None:
                u = np.where(M[lev], u, 0.0).astype(dtype)
                v = np.where(M[lev], v, 0.0).astype(dtype)
        per_level.append((lev, u.copy(), v.copy()))
    if return_levels:
        return u, v, per_level
    return u, v
