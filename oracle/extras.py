"""FP64 oracle of the steps around the flow: pre-processing, level count, integral quantity.

TEST INFRASTRUCTURE ONLY (same rules as ``oracle.lk``).

* ``local_normalize`` -- the local equalisation applied to raw frames before the flow
  (Sec. 2.4, eq. 2): subtract the local mean and divide by the local standard deviation over a
  window of radius 5.  eq. 2 as printed takes the root of the *negative* of the variance;
  the surrounding text divides by the local standard deviation, which is what is computed:
  sigma = sqrt(mean(I^2) - mean(I)^2), window truncated at the border (means over in-image
  pixels), result (I - mean) / (sigma + eps).
* ``levels_for_displacement`` -- the level rule of eq. 1: the smallest n_lev with
  dmax / 2^(n_lev - 1) < 3 px.
* ``bubble_threshold`` / ``bubble_surface`` -- the recirculation-bubble surface of Sec. 3.2,
  eq. 3: the fraction of vectors whose streamwise component is at or below the threshold
  T_v = (min + max) / 2 of the time-mean streamwise field.  eq. 3's printed denominator is the
  sum of the components; the text describes a ratio to the number of vectors, which is what is
  computed.
* ``bubble_series`` -- eq. 3 over a sequence of fields as a real-time system can evaluate it
  (Sec. 3.2 feeds S_bubble to flow control as fields arrive): the mean field is the running
  time-mean of the fields received so far, and field t is thresholded with T_v of the mean of
  the fields before it (the first field, which has no predecessor, with its own T_v).
"""
from __future__ import annotations

import math

import numpy as np

from .lk import box_sum


def local_normalize(I, radius: int = 5, eps: float = 1.0):
    I = np.asarray(I, dtype=np.float64)
    n = box_sum(np.ones_like(I), radius)
    mean = box_sum(I, radius) / n
    mean2 = box_sum(I * I, radius) / n
    sigma = np.sqrt(np.maximum(mean2 - mean * mean, 0.0))
    return (I - mean) / (sigma + eps)


def levels_for_displacement(dmax: float, limit: float = 3.0) -> int:
    L = 1
    while dmax / 2 ** (L - 1) >= limit:
        L += 1
    return L


def running_mean(mean, x, t: int):
    """Mean of t + 1 fields given the mean of the first t and the next field x."""
    return mean + (np.asarray(x, np.float64) - mean) / (t + 1)


def bubble_threshold(mean_u) -> float:
    m = np.asarray(mean_u, np.float64)
    return 0.5 * (float(m.min()) + float(m.max()))


def bubble_surface(u, threshold: float) -> float:
    u = np.asarray(u)
    return float(np.count_nonzero(u <= threshold)) / u.size


def bubble_series(fields):
    """[S_bubble(t)] of a sequence of streamwise fields: S(0) = bubble_surface(u_0, T_v(u_0));
    S(t) = bubble_surface(u_t, T_v(mean of u_0 .. u_{t-1})) for t >= 1."""
    out = []
    mean = None
    thr = None
    for t, u in enumerate(fields):
        if t == 0:
            mean = running_mean(np.zeros(np.shape(u)), u, 0)
            thr = bubble_threshold(mean)
            out.append(bubble_surface(u, thr))
        else:
            out.append(bubble_surface(u, thr))
            mean = running_mean(mean, u, t)
            thr = bubble_threshold(mean)
    return out


def _check():  # pragma: no cover - documentation of the closed forms used by the pins
    assert levels_for_displacement(2.9) == 1 and math.isclose(0.5 * (1 + 3), 2.0)
