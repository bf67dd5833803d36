"""Gaussian-weighted window variant (OF_FLAG_GAUSSIAN_WINDOW) against the oracle's weighted
window sums."""
import numpy as np
import pytest

import floor_util
import oracle
import synth
from gpu_util import announce, dev, flow_error, report, to_dev

pytestmark = pytest.mark.gpu


def test_gaussian_single_iteration_stage(gpu_lib):
    import torch
    ofmi = gpu_lib
    I1, I2, gu, gv = synth.make_pair("c1", 11)
    I1, I2 = I1[:150, :170], I2[:150, :170]
    rng = np.random.default_rng(12)
    u = (gu[:150, :170] + rng.normal(0, 0.3, size=(150, 170))).astype(np.float32)
    v = (gv[:150, :170] + rng.normal(0, 0.3, size=(150, 170))).astype(np.float32)
    plan = ofmi.Plan(150, 170, 1, 4, 1, gaussian_window=True, device=dev())
    un = torch.empty((150, 170), dtype=torch.float32, device=dev())
    vn = torch.empty_like(un)
    announce("gaussian window: one iteration 150x170 r=4")
    ofmi.debug_stage(plan, ofmi.OF_STAGE_ITERATE, 0, [to_dev(I1), to_dev(I2), to_dev(u), to_dev(v)], [un, vn])
    torch.cuda.synchronize()
    ou, ov = oracle.lk_iteration(I1.astype(np.float64), I2.astype(np.float64), u.astype(np.float64),
                                 v.astype(np.float64), 4, weights=oracle.gaussian_weights(4))
    d = flow_error(un.cpu().numpy(), vn.cpu().numpy(), ou, ov)
    assert d.max() <= 1e-3, report(d, 1e-3)
    plan.close()


@pytest.mark.parametrize("shape,L,r,K", [((256, 256), 3, 4, 4), ((200, 333), 3, 5, 3), ((67, 45), 2, 12, 2)])
def test_gaussian_window_flow_matches_oracle(gpu_lib, shape, L, r, K):
    import torch
    ofmi = gpu_lib
    I1, I2, _, _ = synth.make_pair("c1", 13)
    H, W = shape
    I1 = np.tile(I1, (2, 2))[:H, :W].copy()
    I2 = np.tile(I2, (2, 2))[:H, :W].copy()
    announce(f"gaussian window flow {shape} L={L} r={r} K={K}")
    plan = ofmi.Plan(H, W, L, r, K, gaussian_window=True, device=dev())
    u, v = plan.compute(to_dev(I1), to_dev(I2))
    torch.cuda.synchronize()
    gu, gv = u.cpu().numpy(), v.cpu().numpy()
    ou, ov = oracle.flow(I1, I2, L, r, K, window="gauss")
    d = flow_error(gu, gv, ou, ov)
    assert d.max() <= 1e-3, report(d, 1e-3)
    # it is a different estimator from the box window
    bu, _ = oracle.flow(I1, I2, L, r, K)
    assert np.abs(bu - ou).max() > 1e-2
    # the narrow-strip variants are box-window only
    for w in (3, 4, 5, 6, 7):
        with pytest.raises(ofmi.OfError):
            plan.set_config({"bands": [1] * L, "variant": [w] * L})
    # tiling and variant independence, bitwise
    for cfg in ({"bands": [1] * L, "variant": [0] * L}, {"bands": [2] * L, "variant": [2] * L}):
        plan.set_config(cfg)
        u2, v2 = plan.compute(to_dev(I1), to_dev(I2))
        torch.cuda.synchronize()
        assert np.array_equal(u2.cpu().numpy(), gu) and np.array_equal(v2.cpu().numpy(), gv), cfg
    plan.close()


def test_gaussian_window_full_size(gpu_lib):
    import torch
    ofmi = gpu_lib
    I1, I2, _, _ = synth.make_pair("c2", 0)
    announce("gaussian window flow 1024x1024 L4 r8 K4")
    plan = ofmi.Plan(1024, 1024, 4, 8, 4, gaussian_window=True, device=dev())
    u, v = plan.compute(to_dev(I1), to_dev(I2))
    torch.cuda.synchronize()
    ou, ov = oracle.flow(I1, I2, 4, 8, 4, window="gauss")
    d = flow_error(u.cpu().numpy(), v.cpu().numpy(), ou, ov)
    # The right edge is the outflow border (displacements up to 8 px to the right): its warp is
    # clamped and the truncated windows, weighted toward the clamped columns, are nearly
    # singular, so FP32 runs of the oracle's own operation order depart from FP64 there by up
    # to 1.5e-3 px.  Every pixel is held to 1e-3 px or, where the committed floor of the pixel
    # says so, to 1e-3 px plus a multiple of that floor.
    print(floor_util.check_all_pixels(d, 1e-3, floor_util.load_floor("c2_gauss"), "gaussian 1024"))
    plan.close()
