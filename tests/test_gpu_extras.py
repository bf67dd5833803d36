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
    f1 = ofmi.normalize(to_dev(I.astype(np.float32)), r, 1.0)
    torch.cuda.synchronize()
    ref = oracle.local_normalize(I, r, 1.0)
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=2e-6, atol=2e-6)
    np.testing.assert_allclose(fout.cpu().numpy(), ref, rtol=2e-6, atol=2e-6)
    # the 8-bit kernel's exact integer sliding sums equal the float kernel's FP64 sums of the
    # same values, so the two give the same bits
    assert np.array_equal(out.cpu().numpy(), f1.cpu().numpy())


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


def test_bubble_surface_fused_count_matches_oracle(gpu_lib):
    """eq. 3 over a served sequence: the plan's final iteration counts u <= T_v as it writes u
    (threshold and count on the device), of_bubble_step finishes S_bubble and moves the mean and
    threshold on.  Against the oracle's series on the same fields: the mean and threshold agree
    to rounding, and S_bubble exactly up to vectors within rounding of the threshold; against a
    count of the GPU field with the GPU's own threshold, exactly."""
    import torch
    ofmi = gpu_lib
    H, W = 96, 128
    frames = [to_dev(f) for f, _, _ in synth.stream_frames(0, 7, size=(H, W))]
    plan = ofmi.Plan(H, W, 3, 4, 3, device=dev())
    mon = ofmi.BubbleMonitor(H, W, device=dev())
    mon.attach(plan)
    fields, surf, thr_used = [], [], []
    announce("bubble surface over 6 fields")
    for t in range(6):
        thr_used.append(float(mon.threshold.item()))
        u, _ = plan.compute(frames[t], frames[t + 1])
        s = mon.step(u)
        torch.cuda.synchronize()
        fields.append(u.cpu().numpy().astype(np.float64))
        surf.append(float(s.item()))
    ref = oracle.bubble_series(fields)
    mean = np.mean(fields, axis=0)
    np.testing.assert_allclose(mon.mean.cpu().numpy(), mean, rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(float(mon.threshold.item()), oracle.bubble_threshold(mean), rtol=1e-5, atol=1e-5)
    n = H * W
    for t in range(6):
        # exact: the fused count is the count of the written field against the threshold in force
        own = thr_used[t] if t > 0 else float(np.float32(oracle.bubble_threshold(fields[0])))
        if t > 0:
            assert surf[t] == np.float32(np.count_nonzero(fields[t] <= np.float32(own)) / n), t
        # oracle: up to vectors within rounding of its threshold
        m = np.mean(fields[:max(t, 1)], axis=0)
        othr = oracle.bubble_threshold(m)
        near = np.count_nonzero(np.abs(fields[t] - othr) < 1e-4 * max(1.0, abs(othr)))
        assert abs(surf[t] - ref[t]) * n <= near + 0.5, (t, surf[t], ref[t], near)
    mon.detach(plan)
    u0, _ = plan.compute(frames[0], frames[1])
    torch.cuda.synchronize()
    plan.close()
