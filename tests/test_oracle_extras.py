"""Pins of the oracle's pre-processing, level rule and bubble surface (no GPU)."""
import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(99)


def _brute_normalize(I, r, eps):
    H, W = I.shape
    out = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            win = I[max(0, y - r):y + r + 1, max(0, x - r):x + r + 1].astype(float).ravel()
            m = win.mean()
            s = np.sqrt(max((win * win).mean() - m * m, 0.0))
            out[y, x] = (I[y, x] - m) / (s + eps)
    return out


@pytest.mark.parametrize("shape,r", [((9, 13), 2), ((20, 17), 5), ((3, 3), 5)])
def test_normalize_brute_force(shape, r):
    I = RNG.integers(0, 256, size=shape).astype(np.uint8)
    np.testing.assert_allclose(oracle.local_normalize(I, r, 1.0), _brute_normalize(I, r, 1.0),
                               rtol=1e-10, atol=1e-10)


def test_normalize_constant_and_affine_invariance():
    assert np.all(oracle.local_normalize(np.full((12, 12), 77.0), 5, 1.0) == 0.0)
    I = RNG.uniform(0, 255, size=(30, 40))
    a = oracle.local_normalize(I, 5, 0.0)
    b = oracle.local_normalize(3.0 * I + 7.0, 5, 0.0)
    np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-9)


def test_normalize_closed_form_on_quadratic():
    # I = x^2, window columns x-5..x+5 (rows constant): mean = x^2 + 10,
    # variance = 40 x^2 + 78 (mean k^2 = 10, var k^2 = 178 - 100), so I~ = -10 / sqrt(40 x^2 + 78)
    y, x = np.mgrid[0:21, 0:31].astype(float)
    n = oracle.local_normalize(x * x, 5, 0.0)
    for xx in (5, 10, 20, 25):
        np.testing.assert_allclose(n[10, xx], -10.0 / np.sqrt(40.0 * xx * xx + 78.0), rtol=1e-9)


def test_level_rule_eq1():
    assert oracle.levels_for_displacement(0.0) == 1
    assert oracle.levels_for_displacement(2.99) == 1
    assert oracle.levels_for_displacement(3.0) == 2
    assert oracle.levels_for_displacement(10.0) == 3        # 10/4 = 2.5 < 3
    assert oracle.levels_for_displacement(12.0) == 4        # 12/4 = 3 is not < 3
    for d in RNG.uniform(0, 100, 50):
        L = oracle.levels_for_displacement(d)
        assert d / 2 ** (L - 1) < 3 and (L == 1 or d / 2 ** (L - 2) >= 3)


def test_bubble_surface_and_threshold():
    mean = np.array([[-2.0, 0.0], [4.0, 6.0]])
    assert oracle.bubble_threshold(mean) == 2.0
    u = np.array([[1.0, 2.0], [2.5, -1.0]])
    assert oracle.bubble_surface(u, 2.0) == 0.75            # 1, 2, -1 are <= 2
    m = np.zeros(3)
    for t, x in enumerate([np.array([1.0, 2, 3]), np.array([3.0, 2, 1]), np.array([2.0, 2, 2])]):
        m = oracle.running_mean(m, x, t)
    np.testing.assert_allclose(m, [2.0, 2.0, 2.0])


def test_bubble_series_causal_threshold():
    """Closed form on constructed fields: field 0 = [0, 1, 2, 3] (T_v = 1.5, S = 2/4);
    field 1 = [4, 4, 4, -4] thresholded with T_v of field 0 (1.5): S = 1/4; the mean becomes
    [2, 2.5, 3, -0.5] (T_v = 1.25); field 2 = [1, 1.25, 1.5, 2] against 1.25: S = 2/4."""
    f = [np.array([0.0, 1, 2, 3]), np.array([4.0, 4, 4, -4]), np.array([1.0, 1.25, 1.5, 2])]
    S = oracle.bubble_series(f)
    assert S == [0.5, 0.25, 0.5]
    # one field alone: its own threshold, as bubble_surface(u, bubble_threshold(u))
    u = np.random.default_rng(3).normal(size=(7, 9))
    assert oracle.bubble_series([u]) == [oracle.bubble_surface(u, oracle.bubble_threshold(u))]
