"""Pins of the FP64 oracle against what the mathematics and the paper fix (no GPU).

Every check compares the oracle with something other than itself: closed forms, brute-force
loops, library routines (scipy / numpy.linalg) or invariants of the method.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from oracle import lk


RNG = np.random.default_rng(12345)


# ------------------------------------------------------------------ warp (bilinear)

def test_warp_identity_bitwise():
    I = RNG.uniform(0, 255, size=(13, 17))
    W2 = lk.warp(I, np.zeros_like(I), np.zeros_like(I))
    assert np.array_equal(W2, I)


@pytest.mark.parametrize("k,l", [(1, 0), (0, -2), (3, 2), (-1, -1)])
def test_warp_integer_shift_is_shifted_copy(k, l):
    I = RNG.uniform(0, 255, size=(20, 24))
    W2 = lk.warp(I, np.full_like(I, float(k)), np.full_like(I, float(l)))
    # interior: W2[y, x] = I[y + l, x + k]
    ys = slice(max(0, -l), 20 - max(0, l))
    xs = slice(max(0, -k), 24 - max(0, k))
    ys2 = slice(ys.start + l, ys.stop + l)
    xs2 = slice(xs.start + k, xs.stop + k)
    assert np.array_equal(W2[ys, xs], I[ys2, xs2])


def test_bilinear_reproduces_bilinear_function():
    H, W = 16, 19
    y, x = np.mgrid[0:H, 0:W].astype(float)
    f = lambda X, Y: 3.0 + 0.7 * X - 1.3 * Y + 0.05 * X * Y  # noqa: E731
    I = f(x, y)
    u = RNG.uniform(-1.5, 1.5, size=(H, W))
    v = RNG.uniform(-1.5, 1.5, size=(H, W))
    W2 = lk.warp(I, u, v)
    X, Y = x + u, y + v
    inside = (X >= 0) & (X <= W - 1) & (Y >= 0) & (Y <= H - 1)
    np.testing.assert_allclose(W2[inside], f(X, Y)[inside], rtol=0, atol=1e-12)


def test_warp_matches_scipy_map_coordinates():
    I = RNG.uniform(0, 255, size=(21, 18))
    u = RNG.uniform(-4, 4, size=I.shape)
    v = RNG.uniform(-4, 4, size=I.shape)
    y, x = np.mgrid[0:21, 0:18].astype(float)
    # clamp-to-edge of the coordinate is what mode='nearest' does for order=1
    ref = ndi.map_coordinates(I, [np.clip(y + v, 0, 20), np.clip(x + u, 0, 17)], order=1, mode="nearest")
    np.testing.assert_allclose(lk.warp(I, u, v), ref, rtol=1e-12, atol=1e-10)


# ------------------------------------------------------------------ box sums

def _brute_box(p, r):
    H, W = p.shape
    out = np.zeros_like(p)
    for y in range(H):
        for x in range(W):
            s = 0.0
            for yy in range(y - r, y + r + 1):
                for xx in range(x - r, x + r + 1):
                    if 0 <= yy < H and 0 <= xx < W:
                        s += p[yy, xx]
            out[y, x] = s
    return out


@pytest.mark.parametrize("shape", [(1, 1), (5, 7), (16, 16), (3, 11)])
@pytest.mark.parametrize("r", [0, 1, 2, 4, 8])
def test_box_sum_brute_force_integer_exact(shape, r):
    p = RNG.integers(-50, 50, size=shape).astype(float)
    assert np.array_equal(lk.box_sum(p, r), _brute_box(p, r))


@pytest.mark.parametrize("r", [1, 3, 6])
def test_box_sum_matches_scipy_uniform_filter(r):
    p = RNG.normal(size=(23, 31))
    ref = ndi.uniform_filter(p, size=2 * r + 1, mode="constant", cval=0.0) * (2 * r + 1) ** 2
    np.testing.assert_allclose(lk.box_sum(p, r), ref, rtol=1e-9, atol=1e-9)


# ------------------------------------------------------------------ pyramid

def test_pyramid_constant_and_sizes():
    for H, W in [(1, 1), (7, 5), (64, 33), (9, 128)]:
        P = lk.pyramid(np.full((H, W), 77, np.uint8), 4)
        h, w = H, W
        for lev in P:
            assert lev.shape == (h, w)
            assert np.all(lev == 77.0)
            h, w = (h + 1) // 2, (w + 1) // 2


def test_pyr_reduce_matches_scipy_correlate():
    F = RNG.integers(0, 256, size=(37, 29)).astype(float)
    k = np.array([1, 4, 6, 4, 1]) / 16.0
    ref = ndi.correlate1d(ndi.correlate1d(F, k, axis=0, mode="nearest"), k, axis=1, mode="nearest")[::2, ::2]
    np.testing.assert_allclose(lk.pyr_reduce(F), ref, rtol=1e-12, atol=1e-12)


def test_pyr_reduce_preserves_bilinear_in_interior():
    y, x = np.mgrid[0:40, 0:44].astype(float)
    F = 5.0 + 2.0 * x - 0.5 * y + 0.01 * x * y
    R = lk.pyr_reduce(F)
    yi, xi = np.mgrid[0:20, 0:22].astype(float)
    expect = 5.0 + 2.0 * (2 * xi) - 0.5 * (2 * yi) + 0.01 * (2 * xi) * (2 * yi)
    np.testing.assert_allclose(R[1:-1, 1:-1], expect[1:-1, 1:-1], rtol=0, atol=1e-10)


def test_pyr_reduce_uint8_is_exact_dyadic():
    # integer weights /16 per axis: level 1 of a uint8 frame is a multiple of 1/256
    F = RNG.integers(0, 256, size=(33, 35)).astype(np.uint8)
    L1 = lk.pyramid(F, 2)[1]
    assert np.array_equal(L1 * 256, np.round(L1 * 256))


# ------------------------------------------------------------------ prolongation

def test_upsample_uniform_and_linear():
    uc = np.full((8, 9), 1.25)
    assert np.all(lk.upsample_flow(uc, 16, 18) == 2.5)
    yc, xc = np.mgrid[0:8, 0:9].astype(float)
    lin = 0.3 * xc - 0.2 * yc + 1.0
    up = lk.upsample_flow(lin, 15, 17)
    y, x = np.mgrid[0:15, 0:17].astype(float)
    expect = 2.0 * (0.3 * x / 2 - 0.2 * y / 2 + 1.0)
    np.testing.assert_allclose(up, expect, rtol=0, atol=1e-12)


# ------------------------------------------------------------------ gradients

def test_gradient_exact_on_quadratic():
    y, x = np.mgrid[0:12, 0:15].astype(float)
    Ix, Iy = lk.gradients(x * x + 3 * y * y)
    np.testing.assert_array_equal(Ix[:, 1:-1], 2 * x[:, 1:-1])
    np.testing.assert_array_equal(Iy[1:-1, :], 6 * y[1:-1, :])


def test_gradient_matches_numpy_gradient_interior():
    Z = RNG.normal(size=(10, 13))
    Ix, Iy = lk.gradients(Z)
    gy, gx = np.gradient(Z)
    np.testing.assert_allclose(Ix[:, 1:-1], gx[:, 1:-1], rtol=1e-14)
    np.testing.assert_allclose(Iy[1:-1, :], gy[1:-1, :], rtol=1e-14)


# ------------------------------------------------------------------ 2x2 solve

def test_solve_cramer_matches_linalg():
    n = 200
    M = RNG.normal(size=(n, 2, 2))
    Hs = M @ np.transpose(M, (0, 2, 1)) + 0.1 * np.eye(2)
    b = RNG.normal(size=(n, 2))
    du, dv = lk.solve(Hs[:, 0, 0], Hs[:, 0, 1], Hs[:, 1, 1], b[:, 0], b[:, 1])
    ref = -np.linalg.solve(Hs, b[..., None])[..., 0]
    np.testing.assert_allclose(du, ref[:, 0], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(dv, ref[:, 1], rtol=1e-10, atol=1e-12)


def test_solve_rank1_matches_pinv_and_zero_branch():
    g = RNG.normal(size=(50, 2))
    w = RNG.uniform(0.5, 3.0, size=50)
    Hs = w[:, None, None] * g[:, :, None] * g[:, None, :]
    b = RNG.normal(size=(50, 2))
    du, dv = lk.solve(Hs[:, 0, 0], Hs[:, 0, 1], Hs[:, 1, 1], b[:, 0], b[:, 1])
    ref = -np.einsum("nij,nj->ni", np.linalg.pinv(Hs), b)
    np.testing.assert_allclose(du, ref[:, 0], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(dv, ref[:, 1], rtol=1e-9, atol=1e-12)
    z = np.zeros(3)
    du, dv = lk.solve(z, z, z, np.ones(3), np.ones(3))
    assert np.all(du == 0) and np.all(dv == 0)


# ------------------------------------------------------------------ one iteration vs least squares

def test_iteration_equals_windowed_least_squares():
    """Independent formulation: per pixel, lstsq of the stacked linearised window residuals."""
    H, W, r = 12, 12, 2
    I1 = ndi.gaussian_filter(RNG.uniform(0, 255, size=(H, W)), 1.0)
    I2 = ndi.gaussian_filter(RNG.uniform(0, 255, size=(H, W)), 1.0)
    u = RNG.uniform(-0.8, 0.8, size=(H, W))
    v = RNG.uniform(-0.8, 0.8, size=(H, W))
    un, vn = lk.lk_iteration(I1, I2, u, v, r)
    W2 = lk.warp(I2, u, v)
    Ix, Iy = lk.gradients(W2)
    for y in range(H):
        for x in range(W):
            rows, rhs = [], []
            for yy in range(max(0, y - r), min(H, y + r + 1)):
                for xx in range(max(0, x - r), min(W, x + r + 1)):
                    g = np.array([Ix[yy, xx], Iy[yy, xx]])
                    # residual W2 + g.(d - u(m)) - I1 = 0  ->  g.d = I1 - W2 + g.u(m)
                    rows.append(g)
                    rhs.append(I1[yy, xx] - W2[yy, xx] + g @ np.array([u[yy, xx], v[yy, xx]]))
            d = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]
            assert abs(un[y, x] - d[0]) < 1e-8 and abs(vn[y, x] - d[1]) < 1e-8, (y, x)


# ------------------------------------------------------------------ whole method

def test_identical_frames_give_zero_flow_bitwise():
    I = RNG.integers(0, 256, size=(40, 52)).astype(np.uint8)
    for L, r, K in [(1, 2, 3), (3, 4, 2), (2, 0, 1)]:
        u, v = oracle.flow(I, I, L, r, K)
        assert np.all(u == 0) and np.all(v == 0)


@pytest.mark.parametrize("K", [1, 3])
def test_linear_ramp_subpixel_shift_exact(K):
    # I1 = 4x, shifted right by 0.25 px: I2(x) = I1(x - 0.25) = 4x - 1, both uint8-exact
    x = np.arange(64, dtype=float)
    I1 = np.tile(4 * x, (40, 1)).astype(np.uint8)
    I2 = np.tile(4 * x - 1, (40, 1)).clip(0).astype(np.uint8)
    r = 3
    u, v = oracle.flow(I1, I2, 1, r, K)
    m = (r + 2) * K + 1
    np.testing.assert_allclose(u[:, m:-m], 0.25, atol=1e-12)
    np.testing.assert_allclose(v[:, m:-m], 0.0, atol=1e-12)


def test_diagonal_ramp_and_aperture_projection():
    y, x = np.mgrid[0:48, 0:48].astype(float)
    I1 = (2 * x + 2 * y).astype(np.uint8)
    I2 = (2 * x + 2 * y - 1).clip(0).astype(np.uint8)   # shift (0.25, 0.25)
    u, v = oracle.flow(I1, I2, 1, 2, 1)
    np.testing.assert_allclose(u[5:-5, 5:-5], 0.25, atol=1e-12)
    np.testing.assert_allclose(v[5:-5, 5:-5], 0.25, atol=1e-12)
    # a vertical shift of an x-ramp is invisible: only the projection on grad I is recovered
    I1 = (4 * x).astype(np.uint8)
    I2 = (4 * x - 2).astype(np.uint8).clip(0)            # shift (0.5, anything)
    u, v = oracle.flow(I1, I2, 1, 2, 1)
    np.testing.assert_allclose(u[5:-5, 5:-5], 0.5, atol=1e-12)
    np.testing.assert_allclose(v[5:-5, 5:-5], 0.0, atol=1e-12)


@pytest.mark.parametrize("levels", [1, 3])
def test_bilinear_intensity_converges_to_shift(levels):
    H, W = 64, 64
    y, x = np.mgrid[0:H, 0:W].astype(float)
    f = lambda X, Y: 50.0 + 2.0 * X + 1.5 * Y + 0.05 * X * Y  # noqa: E731
    d = (0.375, -0.25)
    I1 = f(x, y)
    I2 = f(x - d[0], y - d[1])
    u, v = oracle.flow(I1, I2, levels, 4, 10)
    s = slice(16, -16)
    np.testing.assert_allclose(u[s, s], d[0], atol=1e-10)
    np.testing.assert_allclose(v[s, s], d[1], atol=1e-10)


def test_integer_shift_of_particle_image_converges():
    """Uniform integer shift of a noiseless particle image is an exact fixed point.

    Each update reads the neighbours' estimates inside the window, so what the clamped
    border does reaches r + 1 px further inward per iteration: the checked interior lies
    beyond levels * iters * (r + 1) px from the border.
    """
    from synth.particles import render

    class _NoNoise:
        def normal(self, loc, scale, size):
            return np.zeros(size)

    rng = np.random.default_rng(7)
    H = W = 224
    n = int(0.03 * (W + 24) ** 2)
    xp = rng.uniform(-12, W + 12, n)
    yp = rng.uniform(-12, H + 12, n)
    amp = rng.uniform(150, 255, n)
    I1 = render(xp, yp, amp, H, W, 2.0, _NoNoise()).astype(float)
    I2 = render(xp + 1.0, yp - 1.0, amp, H, W, 2.0, _NoNoise()).astype(float)
    r, K = 4, 16
    u, v = oracle.flow(I1, I2, 1, r, K)
    m = K * (r + 1) + 2
    np.testing.assert_allclose(u[m:-m, m:-m], 1.0, atol=1e-9)
    np.testing.assert_allclose(v[m:-m, m:-m], -1.0, atol=1e-9)


def test_scale_invariance_bitwise():
    I1 = RNG.integers(0, 256, size=(40, 44)).astype(float)
    I2 = np.roll(I1, 1, axis=1)
    u, v = oracle.flow(I1, I2, 2, 3, 3)
    for k in (-3, 4):
        us, vs = oracle.flow(I1 * 2.0 ** k, I2 * 2.0 ** k, 2, 3, 3)
        assert np.array_equal(u, us) and np.array_equal(v, vs)


def test_transpose_equivariance():
    import synth
    I1, I2, _, _ = synth.make_pair("c1", 3)
    I1, I2 = I1[:96, :120], I2[:96, :120]
    u, v = oracle.flow(I1, I2, 2, 4, 3)
    ut, vt = oracle.flow(I1.T.copy(), I2.T.copy(), 2, 4, 3)
    np.testing.assert_allclose(ut, v.T, rtol=0, atol=1e-9)
    np.testing.assert_allclose(vt, u.T, rtol=0, atol=1e-9)


def test_degenerate_parameters():
    I1, I2 = RNG.integers(0, 256, size=(2, 30, 34)).astype(np.uint8)
    u, v = oracle.flow(I1, I2, 3, 4, 0)
    assert u.shape == (30, 34) and np.all(u == 0) and np.all(v == 0)
    # r = 0: the window is one pixel, H = g g^T has rank <= 1 everywhere
    W2 = lk.warp(I2.astype(float), np.zeros((30, 34)), np.zeros((30, 34)))
    Ix, Iy = lk.gradients(W2)
    A, B, C = Ix * Ix, Ix * Iy, Iy * Iy
    assert np.all(A * C - B * B <= lk.TAU * (A + C) ** 2 + 1e-9)
    u, v = oracle.flow(I1, I2, 1, 0, 1)
    g2 = Ix * Ix + Iy * Iy
    It = W2 - I1
    with np.errstate(invalid="ignore", divide="ignore"):
        expect_u = np.where(g2 > 0, -Ix * It / g2, 0.0)
    np.testing.assert_allclose(u, expect_u, atol=1e-12)


def test_iterations_stop_varying():
    """Raising the iteration count makes the field stop varying (Sec. 2.4: n_iter is raised
    until the computed field does not vary); the change per doubling of n_iter shrinks."""
    import synth
    I1, I2, _, _ = synth.make_pair("c1", 1)
    a = oracle.flow(I1, I2, 3, 4, 16)
    b = oracle.flow(I1, I2, 3, 4, 32)
    c = oracle.flow(I1, I2, 3, 4, 64)
    d1 = np.maximum(np.abs(a[0] - b[0]), np.abs(a[1] - b[1]))
    d2 = np.maximum(np.abs(b[0] - c[0]), np.abs(b[1] - c[1]))
    assert d2.max() < 0.6 * d1.max()
    assert np.percentile(d2, 99) < 1e-2


# ------------------------------------------------------------------ Gaussian-weighted window

def test_gaussian_weights_closed_form():
    for r in (1, 4, 8):
        g = lk.gaussian_weights(r)
        assert g.shape == (2 * r + 1,) and g[r] == 1.0
        np.testing.assert_allclose(g, g[::-1], rtol=0, atol=0)
        np.testing.assert_allclose([g[0], g[-1]], np.exp(-2.0), rtol=1e-15)
    assert np.array_equal(lk.gaussian_weights(0), [1.0])


@pytest.mark.parametrize("shape,r", [((7, 9), 2), ((1, 5), 1), ((12, 4), 3), ((5, 5), 0)])
def test_weighted_window_sum_brute_force(shape, r):
    p = RNG.normal(size=shape)
    g = lk.gaussian_weights(r)
    H, W = shape
    ref = np.zeros(shape)
    for y in range(H):
        for x in range(W):
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    if 0 <= y + dy < H and 0 <= x + dx < W:
                        ref[y, x] += g[dy + r] * g[dx + r] * p[y + dy, x + dx]
    np.testing.assert_allclose(lk.window_sum(p, r, g), ref, rtol=1e-12, atol=1e-12)
    # unit taps are the unweighted box, bitwise
    assert np.array_equal(lk.window_sum(p, r, np.ones(2 * r + 1)), lk.box_sum(p, r))


def test_gaussian_iteration_equals_weighted_least_squares():
    """Independent formulation: per pixel, lstsq of the linearised window residuals scaled by
    the square roots of the window weights."""
    H, W, r = 11, 13, 2
    I1 = ndi.gaussian_filter(RNG.uniform(0, 255, size=(H, W)), 1.0)
    I2 = ndi.gaussian_filter(RNG.uniform(0, 255, size=(H, W)), 1.0)
    u = RNG.uniform(-0.8, 0.8, size=(H, W))
    v = RNG.uniform(-0.8, 0.8, size=(H, W))
    g = lk.gaussian_weights(r)
    un, vn = lk.lk_iteration(I1, I2, u, v, r, weights=g)
    W2 = lk.warp(I2, u, v)
    Ix, Iy = lk.gradients(W2)
    for y in range(H):
        for x in range(W):
            rows, rhs = [], []
            for yy in range(max(0, y - r), min(H, y + r + 1)):
                for xx in range(max(0, x - r), min(W, x + r + 1)):
                    s = np.sqrt(g[yy - y + r] * g[xx - x + r])
                    gr = np.array([Ix[yy, xx], Iy[yy, xx]])
                    rows.append(s * gr)
                    rhs.append(s * (I1[yy, xx] - W2[yy, xx] + gr @ np.array([u[yy, xx], v[yy, xx]])))
            d = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]
            assert abs(un[y, x] - d[0]) < 1e-8 and abs(vn[y, x] - d[1]) < 1e-8, (y, x)


def test_gaussian_window_flow_exact_cases():
    I = RNG.integers(0, 256, size=(40, 52)).astype(np.uint8)
    u, v = oracle.flow(I, I, 2, 3, 2, window="gauss")
    assert np.all(u == 0) and np.all(v == 0)
    x = np.arange(64, dtype=float)
    I1 = np.tile(4 * x, (40, 1)).astype(np.uint8)
    I2 = np.tile(4 * x - 1, (40, 1)).clip(0).astype(np.uint8)
    u, v = oracle.flow(I1, I2, 1, 3, 2, window="gauss")
    m = 5 * 2 + 1
    np.testing.assert_allclose(u[:, m:-m], 0.25, atol=1e-12)
    np.testing.assert_allclose(v[:, m:-m], 0.0, atol=1e-12)
    H = W = 64
    yy, xx = np.mgrid[0:H, 0:W].astype(float)
    f = lambda X, Y: 50.0 + 2.0 * X + 1.5 * Y + 0.05 * X * Y  # noqa: E731
    u, v = oracle.flow(f(xx, yy), f(xx - 0.375, yy + 0.25), 2, 4, 10, window="gauss")
    np.testing.assert_allclose(u[16:-16, 16:-16], 0.375, atol=1e-10)
    np.testing.assert_allclose(v[16:-16, 16:-16], -0.25, atol=1e-10)
    with pytest.raises(ValueError):
        oracle.flow(I, I, 1, 2, 1, window="hann")
