"""Invariants of the seeded particle-image generator (no GPU)."""
import math

import numpy as np
import pytest

import synth
from synth import particles as sp


@pytest.mark.parametrize("name", ["c1", "c2", "t1"])
def test_level_rule_eq1_and_determinism(name):
    wl = synth.workload(name)
    I1, I2, gu, gv = synth.make_pair(name, 0)
    assert I1.dtype == np.uint8 and I1.shape == (wl.H, wl.W) and I2.shape == I1.shape
    dmax = float(np.hypot(gu, gv).max())
    assert dmax / 2 ** (wl.levels - 1) < 3.0          # eq. 1
    J1, J2, _, _ = synth.make_pair(name, 0)
    assert np.array_equal(I1, J1) and np.array_equal(I2, J2)
    K1, _, _, _ = synth.make_pair(name, 1)
    assert not np.array_equal(I1, K1)


def test_c1_c2_peak_displacements():
    _, _, gu, gv = synth.make_pair("c1", 0)
    assert abs(np.hypot(gu, gv).max() - 3.5) < 0.15     # 3 px vortex + (0.4, -0.3)
    _, _, gu, gv = synth.make_pair("c2", 0)
    assert 8.0 < np.hypot(gu, gv).max() < 10.5


def test_lamb_oseen_peak_and_direction():
    r = np.linspace(0.01, 200, 20001)
    du, dv = sp.lamb_oseen(r, np.zeros_like(r), 0.0, 0.0, 30.0, 3.0, +1.0)
    speed = np.hypot(du, dv)
    assert abs(speed.max() - 3.0) < 1e-4
    assert abs(r[speed.argmax()] - 1.120906 * 30.0) < 0.05
    assert np.all(du == 0) and np.all(dv >= 0)          # counter-clockwise for sign +1 on the +x axis


def test_density_amplitude_and_noise():
    rng = np.random.default_rng(0)
    H = W = 128
    xp, yp, amp = sp._particles(rng, rng, H, W, 0.05, 9)
    assert len(xp) == round(0.05 * (W + 18) * (H + 18))
    assert amp.min() >= 150 and amp.max() <= 255
    # no particles: background 10 + N(0, 3) noise, rounded
    img = sp.render(np.zeros(0), np.zeros(0), np.zeros(0), 256, 256, 1.0, np.random.default_rng(1))
    assert abs(img.mean() - 10.0) < 0.05 and abs(img.std() - math.sqrt(9 + 1 / 12)) < 0.05


def test_single_particle_spot_shape():
    class _NoNoise:
        def normal(self, loc, scale, size):
            return np.zeros(size)
    img = sp.render(np.array([10.0]), np.array([12.0]), np.array([200.0]), 24, 24, 1.0, _NoNoise())
    assert img[12, 10] == 210
    assert img[12, 11] == round(10 + 200 * math.exp(-0.5))
    assert img[12, 15] == 10                              # truncated beyond radius 4


def test_batch_and_stream_shapes():
    sizes = sp.batch_sizes()
    assert len(sizes) == 64
    assert sorted(set(sizes)) == [(512, 512), (768, 1024), (2048, 2048)]
    assert sizes.count((512, 512)) == 16 and sizes.count((768, 1024)) == 32
    H, W, I1, I2, gu, gv = next(synth.batch_items(1, sizes=[(96, 128)]))
    assert I1.shape == (96, 128) and np.hypot(gu, gv).max() <= 6.0 + math.sqrt(2) + 1e-9
    frames = list(synth.stream_frames(0, 3, size=(64, 80)))
    assert len(frames) == 3 and frames[0][0].shape == (64, 80)
    assert abs(np.hypot(frames[1][1], frames[1][2]).max() - 8.0) < 1e-6


def test_stream_frames_render_in_parallel_with_the_same_bytes():
    import concurrent.futures as cf
    seq = list(synth.stream_frames(3, 5, size=(72, 90)))
    with cf.ThreadPoolExecutor(3) as ex:
        par = synth.stream_frames_parallel(3, 5, (72, 90), ex)
    assert all(np.array_equal(a[0], b) for a, b in zip(seq, par))
    # ground truth of frame t is the field that moves frame t's particles to frame t + 1
    y, x = np.mgrid[0:72, 0:90].astype(np.float64)
    gu, gv = synth.stream_field(72, 90, 2)(x, y)
    assert np.array_equal(gu, seq[2][1]) and np.array_equal(gv, seq[2][2])
    assert abs(np.hypot(gu, gv).max() - 8.0) < 1e-9
