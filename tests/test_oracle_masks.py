"""Pins of the oracle's region-of-interest masks and of the eq. 1 level rule as exported by
the C library (no GPU: the level rule is host code)."""
import numpy as np
import pytest

import oracle
import synth


def _brute_mask_pyramid(M, levels):
    out = [M.astype(bool)]
    for _ in range(levels - 1):
        m = out[-1]
        H, W = m.shape
        c = np.zeros(((H + 1) // 2, (W + 1) // 2), dtype=bool)
        for i in range(c.shape[0]):
            for j in range(c.shape[1]):
                c[i, j] = m[2 * i:2 * i + 2, 2 * j:2 * j + 2].any()
        out.append(c)
    return out


@pytest.mark.parametrize("shape", [(9, 13), (16, 16), (1, 7), (5, 1)])
def test_mask_pyramid_brute_force(shape):
    M = np.random.default_rng(5).random(shape) < 0.2
    L = 1 + int(np.floor(np.log2(min(shape))))
    for a, b in zip(oracle.mask_pyramid(M, L), _brute_mask_pyramid(M, L)):
        assert np.array_equal(a, b)


def _crop_pair(n=96, item=3):
    I1, I2, _, _ = synth.make_pair("c1", item)
    return I1[:n, :n + 32], I2[:n, :n + 32]


def test_all_true_mask_is_no_mask():
    I1, I2 = _crop_pair()
    u0, v0 = oracle.flow(I1, I2, 2, 3, 2)
    u1, v1 = oracle.flow(I1, I2, 2, 3, 2, mask=np.ones(I1.shape, bool))
    assert np.array_equal(u0, u1) and np.array_equal(v0, v1)


def test_masked_pixels_are_zero_and_far_pixels_unchanged():
    # Left 30 columns masked.  One level, K = 2, r = 2: an output depends on the field within
    # r + 1 px of it in the previous iteration (window plus gradient stencil), so columns at or
    # beyond 30 + K (r + 1) + 1 see the same inputs as without the mask.
    I1, I2 = _crop_pair()
    M = np.ones(I1.shape, bool)
    M[:, :30] = False
    K, r = 2, 2
    u0, v0 = oracle.flow(I1, I2, 1, r, K)
    u1, v1 = oracle.flow(I1, I2, 1, r, K, mask=M)
    assert np.all(u1[:, :30] == 0) and np.all(v1[:, :30] == 0)
    far = 30 + K * (r + 1) + 1
    assert np.array_equal(u1[:, far:], u0[:, far:]) and np.array_equal(v1[:, far:], v0[:, far:])
    # ... and the mask does change pixels next to its edge (it is not a no-op)
    assert not np.array_equal(u1[:, 30:far], u0[:, 30:far])


def test_mask_far_pixels_two_levels():
    # Two levels: the coarse mask excludes coarse columns < 15, coarse outputs at or beyond
    # 15 + K (r + 1) + 1 are unchanged, the prolongation reads coarse x/2 and x/2 + 1, and the
    # fine iterations add K (r + 1) + 1 more.
    I1, I2 = _crop_pair()
    M = np.ones(I1.shape, bool)
    M[:, :30] = False
    K, r = 2, 2
    u0, v0 = oracle.flow(I1, I2, 2, r, K)
    u1, v1 = oracle.flow(I1, I2, 2, r, K, mask=M)
    coarse_far = 15 + K * (r + 1) + 1
    far = 2 * (coarse_far + 1) + K * (r + 1) + 1
    assert far < I1.shape[1] - 8
    assert np.array_equal(u1[:, far:], u0[:, far:]) and np.array_equal(v1[:, far:], v0[:, far:])
    assert np.all(u1[:, :30] == 0)


@pytest.fixture(scope="module")
def lib():
    import paper_1306_2461_amd as ofmi
    return ofmi.load()


def test_levels_for_displacement_abi_matches_eq1(lib):
    for d in [0.0, 0.5, 2.99, 3.0, 5.9, 6.0, 11.99, 12.0, 47.0, 48.0, 100.0, 1000.0]:
        want = oracle.levels_for_displacement(d)
        assert lib.of_levels_for_displacement(d, 4096, 4096) == want, d
    # capped by the frame: 1 + floor(log2(min(H, W)))
    assert lib.of_levels_for_displacement(1000.0, 64, 300) == 7
    assert lib.of_levels_for_displacement(1000.0, 1, 300) == 1
    for bad in [(-1.0, 10, 10), (float("nan"), 10, 10), (float("inf"), 10, 10), (1.0, 0, 5)]:
        assert lib.of_levels_for_displacement(*bad) == 0
    import paper_1306_2461_amd as ofmi
    assert ofmi.levels_for(10.0, 1024, 1024) == 3   # 10 / 2^2 = 2.5 < 3
    with pytest.raises(ofmi.OfError):
        ofmi.levels_for(-2.0, 10, 10)
