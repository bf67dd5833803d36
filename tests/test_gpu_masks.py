"""Region-of-interest masks (tile skipping over obstacles and side walls, Sec. 3.3) on the GPU,
against the oracle's masked flow."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, dev, flow_error, report, to_dev

pytestmark = pytest.mark.gpu


def _obstacle_mask(H, W):
    """A step-like obstacle in the lower left and a side wall along the top."""
    M = np.ones((H, W), dtype=np.uint8)
    M[160:, :80] = 0
    M[:12, :] = 0
    return M


def test_masked_plan_matches_oracle_and_skips_tiles(gpu_lib):
    import torch
    ofmi = gpu_lib
    I1, I2, _, _ = synth.make_pair("c1", 6)
    M = _obstacle_mask(256, 256)
    announce("masked plan 256x256 L3 r4 K4")
    plan = ofmi.Plan(256, 256, 3, 4, 4, device=dev())
    u0, v0 = plan.compute(to_dev(I1), to_dev(I2))
    torch.cuda.synchronize()
    ref0 = (u0.cpu().numpy(), v0.cpu().numpy())
    plan.set_mask(to_dev(M))
    for rep in range(2):                      # two eager runs
        u, v = plan.compute(to_dev(I1), to_dev(I2))
        torch.cuda.synchronize()
        gu, gv = u.cpu().numpy(), v.cpu().numpy()
        assert np.all(gu[M == 0] == 0) and np.all(gv[M == 0] == 0)
        ou, ov = oracle.flow(I1, I2, 3, 4, 4, mask=M.astype(bool))
        d = flow_error(gu, gv, ou, ov)
        assert d.max() <= 1e-3, report(d, 1e-3)
    # other tile widths skip other tiles and give the same bits
    for cfg in ({"bands": [1, 1, 1], "variant": [4, 4, 3]}, {"bands": [4, 2, 1], "variant": [0, 3, 2]},
                {"bands": [1, 2, 1], "variant": [5, 6, 5]}, {"bands": [3, 1, 1], "variant": [7, 7, 6]}):
        plan.set_config(cfg)
        u, v = plan.compute(to_dev(I1), to_dev(I2))
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), gu) and np.array_equal(v.cpu().numpy(), gv), cfg
    # the same plan without the mask again gives the unmasked bits
    plan.set_mask(None)
    u, v = plan.compute(to_dev(I1), to_dev(I2))
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), ref0[0]) and np.array_equal(v.cpu().numpy(), ref0[1])
    plan.close()


def test_all_ones_mask_keeps_bits_and_configs(gpu_lib):
    import torch
    ofmi = gpu_lib
    I1, I2, _, _ = synth.make_pair("c1", 7)
    I1, I2 = I1[:200, :231], I2[:200, :231]
    plan = ofmi.Plan(200, 231, 3, 4, 3, device=dev())
    u0, v0 = plan.compute(to_dev(I1), to_dev(I2))
    torch.cuda.synchronize()
    ref = (u0.cpu().numpy(), v0.cpu().numpy())
    plan.set_mask(to_dev(np.ones((200, 231), np.uint8)))
    for cfg in ({"bands": [1, 1, 1], "variant": [0, 0, 0]}, {"bands": [2, 1, 1], "variant": [1, 2, 1]},
                {"bands": [1, 2, 1], "variant": [4, 3, 4]}, {"bands": [3, 1, 2], "variant": [6, 5, 5]}):
        announce(f"all-ones mask, config {cfg}")
        plan.set_config(cfg)
        u, v = plan.compute(to_dev(I1), to_dev(I2))
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), ref[0]) and np.array_equal(v.cpu().numpy(), ref[1]), cfg
    plan.close()


def test_fully_masked_frame_is_zero(gpu_lib):
    import torch
    ofmi = gpu_lib
    I1, I2, _, _ = synth.make_pair("c1", 8)
    plan = ofmi.Plan(256, 256, 2, 4, 2, device=dev())
    plan.set_mask(to_dev(np.zeros((256, 256), np.uint8)))
    u = torch.full((256, 256), float("nan"), device=dev())
    v = torch.full((256, 256), float("nan"), device=dev())
    announce("fully masked frame")
    plan.compute(to_dev(I1), to_dev(I2), u, v)
    torch.cuda.synchronize()
    assert torch.all(u == 0).item() and torch.all(v == 0).item()
    with pytest.raises(ofmi.OfError):
        plan.set_mask(to_dev(np.ones((255, 256), np.uint8)))
    plan.close()


def test_masked_plan_graph_replay(gpu_lib):
    """A masked plan replaying its captured schedule (OF_FLAG_GRAPH) on fixed buffers equals the
    masked eager plan bitwise, replay after replay with eager work between, and the oracle."""
    import torch
    ofmi = gpu_lib
    I1, I2, _, _ = synth.make_pair("c1", 6)
    M = _obstacle_mask(256, 256)
    d1, d2, dm = to_dev(I1), to_dev(I2), to_dev(M)
    eager = ofmi.Plan(256, 256, 3, 4, 4, device=dev(), graph=False)
    graph = ofmi.Plan(256, 256, 3, 4, 4, device=dev(), graph=True)
    eager.set_mask(dm)
    graph.set_mask(dm)
    ue, ve = eager.compute(d1, d2)
    torch.cuda.synchronize()
    ref = (ue.cpu().numpy(), ve.cpu().numpy())
    ou, ov = oracle.flow(I1, I2, 3, 4, 4, mask=M.astype(bool))
    d = flow_error(ref[0], ref[1], ou, ov)
    assert d.max() <= 1e-3, report(d, 1e-3)
    ug = torch.empty_like(ue)
    vg = torch.empty_like(ve)
    for rep in range(4):
        announce(f"masked plan graph replay {rep}")
        ug.fill_(float("nan"))
        vg.fill_(float("nan"))
        graph.compute(d1, d2, ug, vg)
        eager.compute(d2, d1)                 # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(ug.cpu().numpy(), ref[0]), f"replay {rep}"
        assert np.array_equal(vg.cpu().numpy(), ref[1]), f"replay {rep}"
    eager.close()
    graph.close()
