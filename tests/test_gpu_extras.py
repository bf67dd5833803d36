"""Local equalisation (eq. 2 reading) and bubble-surface statistics (eq. 3) on the GPU."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, dev, flow_error, report, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,r", [((200, 333), 5), ((37, 61), 2), ((64, 64), 16)])
def test_normalize_matches_oracle(gpu_lib, shape, r):
    import torch
    ofmi = gpu_lib
    I1, _, _, _ = synth.make_pair("c1", 3)
    I = np.tile(I1, (2, 2))[:shape[0], :shape[1]].copy()
    announce(f"normalize {shape} r={r}")
    out = ofmi.normalize(to_dev(I), r, 1.0)
    fout = ofmi.normalize(to_dev(I.astype(np.float32) * np.float32(0.5)), r, 0.5)
    torch.cuda.synchronize()
    ref = oracle.local_normalize(I, r, 1.0)
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=2e-6, atol=2e-6)
    np.testing.assert_allclose(fout.cpu().numpy(), ref, rtol=2e-6, atol=2e-6)


def test_plan_with_normalisation_matches_oracle(gpu_lib):
    import torch
    ofmi = gpu_lib
    I1, I2, _, _ = synth.make_pair("c1", 4)
    # an illumination ramp across frame 2 that equalisation removes
    y, x = np.mgrid[0:256, 0:256]
    I2g = np.clip(I2.astype(float) * (0.8 + 0.4 * x / 255.0), 0, 255).astype(np.uint8)
    announce("plan with OF_FLAG_NORMALIZE")
    plan = ofmi.Plan(256, 256, 3, 4, 4, normalize=True, device=dev())
    u, v = plan.compute(to_dev(I1), to_dev(I2g))
    torch.cuda.synchronize()
    ou, ov = oracle.flow(oracle.local_normalize(I1, 5, 1.0), oracle.local_normalize(I2g, 5, 1.0), 3, 4, 4)
    d = flow_error(u.cpu().numpy(), v.cpu().numpy(), ou, ov)
    assert d.max() <= 1e-3, report(d, 1e-3)
    plan.close()


def test_bubble_monitor_matches_oracle(gpu_lib):
    import torch
    ofmi = gpu_lib
    rng = np.random.default_rng(5)
    fields = [rng.normal(2.0, 3.0, size=(70, 90)).astype(np.float32) for _ in range(4)]
    mon = ofmi.BubbleMonitor(70, 90, device=dev())
    mean = np.zeros((70, 90))
    announce("bubble monitor x4")
    for t, f in enumerate(fields):
        s = mon.update(to_dev(f))
        mean = oracle.running_mean(mean, f, t)
        thr = oracle.bubble_threshold(mean)
        np.testing.assert_allclose(mon.mean.cpu().numpy(), mean, rtol=1e-5, atol=1e-5)
        # counts can differ only for values within rounding of the threshold
        near = np.abs(f - thr) < 1e-4
        lo = oracle.bubble_surface(f, thr) - near.mean()
        hi = oracle.bubble_surface(f, thr) + near.mean()
        assert lo - 1e-12 <= s <= hi + 1e-12
