"""The FP32 rounding-floor diagnostic (tests/floor_util.py) and its committed fixtures."""
import numpy as np
import pytest

import floor_util
import oracle
import synth
from oracle import lk


def test_split_coordinates_equal_summed_coordinates_in_fp64():
    """bilinear_split is the oracle's clamped bilinear sample with the coordinate kept as base
    plus fraction: equal in FP64 (up to rounding of the sum), inside, at and beyond the edges."""
    rng = np.random.default_rng(5)
    Z = rng.random((23, 31)) * 255
    y, x = np.mgrid[0:23, 0:31]
    for scale in (0.3, 4.0, 40.0):
        u = rng.normal(0, scale, size=Z.shape)
        v = rng.normal(0, scale, size=Z.shape)
        a = lk.bilinear(Z, x + u, y + v)
        b = lk.bilinear_split(Z, x, y, u, v)
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-9)
    # integer displacements onto the last row/column and far outside
    for d in (-100.0, -1.0, 0.0, 1.0, 22.0, 30.0, 1e4):
        u = np.full(Z.shape, d)
        np.testing.assert_array_equal(lk.bilinear_split(Z, x, y, u, u), lk.bilinear(Z, x + u, y + u))


def test_storage_rounds_each_level():
    F = np.random.default_rng(6).integers(0, 256, size=(40, 52)).astype(np.uint8)
    P = oracle.pyramid(F, 3, np.float32, storage=np.float16)
    Q = oracle.pyramid(F, 2)
    assert P[0].dtype == np.float32 and np.array_equal(P[0], F.astype(np.float32))
    # level 1 from uint8 is exact in FP32, then rounded once to FP16
    assert np.array_equal(P[1], Q[1].astype(np.float16).astype(np.float32))
    assert np.array_equal(P[2], lk.pyr_reduce(P[1]).astype(np.float16).astype(np.float32))


def test_realisations_have_the_same_exact_flow():
    """The five inputs of the ensemble give the same flow in FP64 (offset and scale invariance,
    transpose equivariance), so their FP32 spread is rounding only."""
    I1, I2, _, _ = synth.make_pair("c1", 0)
    I1, I2 = I1[:96, :120].copy(), I2[:96, :120].copy()
    u, v = oracle.flow(I1, I2, 2, 4, 3)
    for f1, f2, tr in floor_util.realisations(I1, I2):
        uk, vk = oracle.flow(f1, f2, 2, 4, 3)
        if tr:
            uk, vk = vk.T, uk.T
        assert np.abs(uk - u).max() < 1e-9 and np.abs(vk - v).max() < 1e-9


@pytest.mark.parametrize("case", ["c1", "r1_L1_K1", "r1_L1_K3", "r1_L2_K3", "serve_0_0", "serve_1_1",
                                  "serve_2_2"])
def test_committed_floor_reproduces(case):
    """The committed fixture is what the diagnostic computes now (cheap cases)."""
    f = floor_util.case_floor(case)
    g = floor_util.load_floor(case)
    keep = f > floor_util.keep_threshold(case)
    np.testing.assert_allclose(g[keep], f[keep], rtol=1e-6)
    assert np.all(g[~keep] == 0)


def test_every_case_has_a_fixture():
    for name in floor_util.CASES:
        z = floor_util.load_floor(name)
        assert z.ndim == 2 and z.size > 0


def test_floor_is_the_window_maximum_of_the_departures():
    """The stored floor at a pixel is at least every realisation's departure within the
    window radius (checked on a small case against a direct recomputation)."""
    I1, I2 = floor_util.case_inputs("serve_0_0")
    _, L, r, K, _, _, _ = floor_util.CASES["serve_0_0"]
    f, (u, v) = floor_util.ensemble_floor(I1, I2, L, r, K)
    uk, vk = oracle.flow(I1, I2, L, r, K, dtype=np.float32, coords="split")
    dep = np.maximum(np.abs(uk - u), np.abs(vk - v))
    H, W = dep.shape
    for (y, x) in [(0, 0), (50, 60), (H - 1, W - 1), (10, W - 3)]:
        win = dep[max(0, y - r):y + r + 1, max(0, x - r):x + r + 1]
        assert f[y, x] >= win.max()


def test_check_all_pixels_semantics():
    floor = np.zeros((4, 5))
    floor[1, 2] = 0.1
    d = np.full((4, 5), 5e-4)
    d[1, 2] = 0.2                      # within 1e-3 + 3 x 0.1
    s = floor_util.check_all_pixels(d, 1e-3, floor, "t")
    assert "1 of 20 px" in s
    d[0, 0] = 2e-3                     # no floor there
    with pytest.raises(AssertionError):
        floor_util.check_all_pixels(d, 1e-3, floor, "t")
