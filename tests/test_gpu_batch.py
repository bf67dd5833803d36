"""The batched form (one launch per phase over many pairs) against the per-pair path and
the oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, dev, flow_error, report, to_dev

pytestmark = pytest.mark.gpu


def _pairs(sizes, seed_item=0):
    out = []
    for H, W, I1, I2, _, _ in synth.batch_items(len(sizes), sizes=sizes):
        out.append((I1, I2))
    return out


SIZES = [(96, 130), (200, 170), (64, 64), (257, 190), (130, 96)]


def test_batch_equals_per_pair_bitwise_and_oracle(gpu_lib):
    import torch
    ofmi = gpu_lib
    pairs = _pairs(SIZES)
    d1 = [to_dev(p[0]) for p in pairs]
    d2 = [to_dev(p[1]) for p in pairs]
    announce(f"batch {SIZES} L=3 r=4 K=3")
    b = ofmi.Batch(SIZES, 3, 4, 3, device=dev())
    us, vs = b.compute(d1, d2)
    torch.cuda.synchronize()
    for i, (H, W) in enumerate(SIZES):
        plan = ofmi.Plan(H, W, 3, 4, 3, device=dev())
        u, v = plan.compute(d1[i], d2[i])
        torch.cuda.synchronize()
        assert np.array_equal(us[i].cpu().numpy(), u.cpu().numpy()), f"pair {i} u"
        assert np.array_equal(vs[i].cpu().numpy(), v.cpu().numpy()), f"pair {i} v"
        plan.close()
        ou, ov = oracle.flow(pairs[i][0], pairs[i][1], 3, 4, 3)
        d = flow_error(us[i].cpu().numpy(), vs[i].cpu().numpy(), ou, ov)
        assert d.max() <= 1e-3, report(d, 1e-3)
    b.close()


def test_batch_graph_replays_and_configs(gpu_lib):
    import torch
    ofmi = gpu_lib
    pairs = _pairs(SIZES)
    d1 = [to_dev(p[0]) for p in pairs]
    d2 = [to_dev(p[1]) for p in pairs]
    eager = ofmi.Batch(SIZES, 3, 4, 3, device=dev(), graph=False)
    ue, ve = eager.compute(d1, d2)
    torch.cuda.synchronize()
    ref = [(u.cpu().numpy(), v.cpu().numpy()) for u, v in zip(ue, ve)]
    g = ofmi.Batch(SIZES, 3, 4, 3, device=dev(), graph=True)
    us, vs = g.outputs()
    announce("batch graph replays x3")
    for rep in range(3):
        for t in us + vs:
            t.fill_(float("nan"))
        g.compute(d1, d2, us, vs)
        eager.compute(d2, d1)
        torch.cuda.synchronize()
        for i in range(len(SIZES)):
            assert np.array_equal(us[i].cpu().numpy(), ref[i][0]), (rep, i)
            assert np.array_equal(vs[i].cpu().numpy(), ref[i][1]), (rep, i)
    # other tile heights / persistent grids give the same bits
    for bands, grid, var in [([1, 1, 1], [0, 0, 0], [0, 0, 0]), ([2, 4, 8], [256, 512, 8], [1, 1, 1]),
                             ([4, 1, 2], [0, 16, 0], [0, 2, -1]), ([1, 2, 1], [24, 0, 8], [2, 2, 2])]:
        announce(f"batch config bands={bands} grid={grid} variant={var}")
        g.set_config({"bands": bands, "grid": grid, "variant": var})
        assert g.config() == {"bands": bands, "grid": grid, "variant": var}
        g.compute(d1, d2, us, vs)
        torch.cuda.synchronize()
        for i in range(len(SIZES)):
            assert np.array_equal(us[i].cpu().numpy(), ref[i][0]), (bands, grid, var, i)
            assert np.array_equal(vs[i].cpu().numpy(), ref[i][1]), (bands, grid, var, i)
    announce("batch autotune")
    cfg = g.autotune(d1, d2, us, vs, reps=1)
    assert len(cfg["bands"]) == 3
    g.compute(d1, d2, us, vs)
    torch.cuda.synchronize()
    for i in range(len(SIZES)):
        assert np.array_equal(us[i].cpu().numpy(), ref[i][0]), ("autotuned", i)
    g.close()
    eager.close()


def test_batch_fp16_and_zero_iterations(gpu_lib):
    import torch
    ofmi = gpu_lib
    pairs = _pairs(SIZES[:3])
    d1 = [to_dev(p[0]) for p in pairs]
    d2 = [to_dev(p[1]) for p in pairs]
    announce("batch fp16 r=8 L=2 K=2")
    b = ofmi.Batch(SIZES[:3], 2, 8, 2, fp16=True, device=dev())
    us, vs = b.compute(d1, d2)
    torch.cuda.synchronize()
    for i in range(3):
        ou, ov = oracle.flow(pairs[i][0], pairs[i][1], 2, 8, 2)
        d = flow_error(us[i].cpu().numpy(), vs[i].cpu().numpy(), ou, ov)
        assert d.max() <= 2e-2, report(d, 2e-2)
    b.close()
    b0 = ofmi.Batch(SIZES[:2], 2, 4, 0, device=dev())
    us, vs = b0.compute(d1[:2], d2[:2])
    torch.cuda.synchronize()
    assert all(np.all(t.cpu().numpy() == 0) for t in us + vs)
    b0.close()


def test_deep_pyramids_plain_equals_batch_bitwise(gpu_lib):
    """The plain path builds runs of 2 or 3 pyramid levels in one fused launch, the batch one
    level per launch: every level count from 2 to 6 (chains of 2, 3, 3 + 1, 3 + 2 levels), FP32
    and FP16 storage, ragged sizes, gives the same bits."""
    import torch
    ofmi = gpu_lib
    sizes = [(257, 190), (96, 130), (75, 203)]
    pairs = _pairs(sizes)
    d1 = [to_dev(p[0]) for p in pairs]
    d2 = [to_dev(p[1]) for p in pairs]
    for fp16 in (False, True):
        for L in (2, 3, 4, 5, 6):
            announce(f"deep pyramid plain vs batch L={L} fp16={fp16}")
            b = ofmi.Batch(sizes, L, 2, 1, fp16=fp16, device=dev())
            us, vs = b.compute(d1, d2)
            torch.cuda.synchronize()
            for i, (H, W) in enumerate(sizes):
                plan = ofmi.Plan(H, W, L, 2, 1, fp16=fp16, device=dev())
                u, v = plan.compute(d1[i], d2[i])
                torch.cuda.synchronize()
                assert np.array_equal(us[i].cpu().numpy(), u.cpu().numpy()), (L, fp16, i)
                assert np.array_equal(vs[i].cpu().numpy(), v.cpu().numpy()), (L, fp16, i)
                plan.close()
            b.close()
    # a level-1 plane over 2^20 pixels: one staged reduction, then a chain of two from level 1
    big = [(2100, 2090)]
    pairs = _pairs(big)
    d1, d2 = to_dev(pairs[0][0]), to_dev(pairs[0][1])
    for fp16 in (False, True):
        announce(f"pyramid 2100x2090 L=4 plain vs batch fp16={fp16}")
        b = ofmi.Batch(big, 4, 2, 1, fp16=fp16, device=dev())
        us, vs = b.compute([d1], [d2])
        plan = ofmi.Plan(2100, 2090, 4, 2, 1, fp16=fp16, device=dev())
        u, v = plan.compute(d1, d2)
        torch.cuda.synchronize()
        assert np.array_equal(us[0].cpu().numpy(), u.cpu().numpy()), fp16
        assert np.array_equal(vs[0].cpu().numpy(), v.cpu().numpy()), fp16
        plan.close()
        b.close()


def test_thin_frames_plain_equals_batch_bitwise(gpu_lib):
    """Frames 4 pixels high or wide: the fused pyramid launch reaches planes of one row or
    column and the default two-band tiles cover levels shorter than a band; the plain path
    equals the batch bitwise.  (On such frames the method itself runs away to flows of tens to
    hundreds of pixels, the FP64 oracle too, so a 1e-3 px comparison says nothing there.)"""
    import torch
    ofmi = gpu_lib
    sizes = [(4, 37), (37, 4), (9, 9), (5, 131)]
    pairs = _pairs(sizes)
    d1 = [to_dev(p[0]) for p in pairs]
    d2 = [to_dev(p[1]) for p in pairs]
    for L in (2, 3):
        announce(f"thin frames plain vs batch L={L}")
        b = ofmi.Batch(sizes, L, 2, 2, device=dev())
        us, vs = b.compute(d1, d2)
        torch.cuda.synchronize()
        for i, (H, W) in enumerate(sizes):
            plan = ofmi.Plan(H, W, L, 2, 2, device=dev())
            u, v = plan.compute(d1[i], d2[i])
            torch.cuda.synchronize()
            assert np.array_equal(us[i].cpu().numpy(), u.cpu().numpy()), (L, i)
            assert np.array_equal(vs[i].cpu().numpy(), v.cpu().numpy()), (L, i)
            assert np.isfinite(u.cpu().numpy()).all() and np.isfinite(v.cpu().numpy()).all()
            plan.close()
        b.close()
