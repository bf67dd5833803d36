"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: 1e-3 px max-abs over every pixel for the FP32 path, 2e-2 px for FP16 storage;
bit-exact where the arithmetic is exact (pyramid levels 1-2 from uint8, zero flow).
"""
import numpy as np
import pytest

import floor_util
import oracle
import synth
from gpu_util import announce, dev, flow_error, gpu_flow, report, to_dev

pytestmark = pytest.mark.gpu

TOL32 = 1e-3
TOL16 = 2e-2


# ------------------------------------------------------------------ stages

# (2100, 2090): the level-1 plane has more than 2^20 pixels, so the plain path takes the
# LDS-staged reduction kernel instead of the direct one.
@pytest.mark.parametrize("shape,L", [((256, 256), 4), ((97, 131), 4), ((2, 7), 2), ((5, 3), 2),
                                     ((2100, 2090), 2)])
def test_reduce_uint8_exact(gpu_lib, shape, L):
    import torch
    ofmi = gpu_lib
    H, W = shape
    F = np.random.default_rng(1).integers(0, 256, size=shape).astype(np.uint8)
    P = oracle.pyramid(F, L)
    announce(f"reduce uint8 {shape} levels={L}")
    plan = ofmi.Plan(H, W, L, 2, 1, device=dev())
    cur = to_dev(F)
    for lev in range(L - 1):
        h, w = P[lev + 1].shape
        out = torch.empty((h, w), dtype=torch.float32, device=dev())
        ofmi.debug_stage(plan, ofmi.OF_STAGE_REDUCE, lev, [cur], [out])
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        if lev < 2:   # levels 1 and 2 are exact dyadic sums in FP32
            assert np.array_equal(got, P[lev + 1]), f"level {lev + 1}"
        else:
            np.testing.assert_allclose(got, P[lev + 1], rtol=1e-6)
        cur = out
    plan.close()


def test_reduce_float_input_staged(gpu_lib):
    """Float32 frames (rounding matters): the staged kernel against the FP64 reduction."""
    import torch
    ofmi = gpu_lib
    H, W = 2100, 2090
    F = (np.random.default_rng(4).random((H, W)) * 200.0 - 50.0).astype(np.float32)
    P = oracle.pyramid(F.astype(np.float64), 2)
    plan = ofmi.Plan(H, W, 2, 2, 1, input_f32=True, device=dev())
    out = torch.empty(P[1].shape, dtype=torch.float32, device=dev())
    announce("reduce float32 2100x2090 (staged)")
    ofmi.debug_stage(plan, ofmi.OF_STAGE_REDUCE, 0, [to_dev(F)], [out])
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.cpu().numpy().astype(np.float64), P[1], rtol=0, atol=2e-5)
    plan.close()


def test_reduce_fp16_storage(gpu_lib):
    import torch
    ofmi = gpu_lib
    F = np.random.default_rng(2).integers(0, 256, size=(120, 90)).astype(np.uint8)
    P = oracle.pyramid(F, 2)
    plan = ofmi.Plan(120, 90, 2, 2, 1, fp16=True, device=dev())
    out = torch.empty((60, 45), dtype=torch.float16, device=dev())
    announce("reduce fp16 120x90")
    ofmi.debug_stage(plan, ofmi.OF_STAGE_REDUCE, 0, [to_dev(F)], [out])
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), P[1].astype(np.float16))
    plan.close()


@pytest.mark.parametrize("level_dtype", ["uint8", "float32"])
def test_single_iteration_stage(gpu_lib, level_dtype):
    import torch
    ofmi = gpu_lib
    I1, I2, gu, gv = synth.make_pair("c1", 2)
    I1, I2 = I1[:150, :170], I2[:150, :170]
    rng = np.random.default_rng(3)
    u = (gu[:150, :170] + rng.normal(0, 0.3, size=(150, 170))).astype(np.float32)
    v = (gv[:150, :170] + rng.normal(0, 0.3, size=(150, 170))).astype(np.float32)
    if level_dtype == "uint8":
        plan = ofmi.Plan(150, 170, 1, 4, 1, device=dev())
        f1, f2 = I1, I2
    else:
        plan = ofmi.Plan(150, 170, 1, 4, 1, input_f32=True, device=dev())
        f1 = oracle.pyramid(I1, 1)[0].astype(np.float32) * np.float32(0.75)
        f2 = oracle.pyramid(I2, 1)[0].astype(np.float32) * np.float32(0.75)
    un = torch.empty((150, 170), dtype=torch.float32, device=dev())
    vn = torch.empty_like(un)
    announce(f"iterate stage {level_dtype}")
    ofmi.debug_stage(plan, ofmi.OF_STAGE_ITERATE, 0, [to_dev(f1), to_dev(f2), to_dev(u), to_dev(v)], [un, vn])
    torch.cuda.synchronize()
    ou, ov = oracle.lk_iteration(f1.astype(np.float64), f2.astype(np.float64), u.astype(np.float64),
                                 v.astype(np.float64), 4)
    d = flow_error(un.cpu().numpy(), vn.cpu().numpy(), ou, ov)
    assert d.max() <= TOL32, report(d, TOL32)
    plan.close()


# ------------------------------------------------------------------ whole method

def _parity(ofmi, I1, I2, L, r, K, fp16=False, tol=TOL32):
    u, v = gpu_flow(ofmi, I1, I2, L, r, K, fp16=fp16)
    ou, ov = oracle.flow(I1, I2, L, r, K)
    d = flow_error(u, v, ou, ov)
    assert d.max() <= tol, report(d, tol)
    return d


def _floor_case(ofmi, case, fp16=False):
    """Whole-method parity of a floor case on every pixel (tolerance, or tolerance plus the
    committed FP32 floor multiple where the floor says the tolerance is out of reach)."""
    I1, I2 = floor_util.case_inputs(case)
    _, L, r, K, window, _, tol = floor_util.CASES[case]
    u, v = gpu_flow(ofmi, I1, I2, L, r, K, fp16=fp16)
    ou, ov = oracle.flow(I1, I2, L, r, K, window=window)
    d = flow_error(u, v, ou, ov)
    print(floor_util.check_all_pixels(d, tol, floor_util.load_floor(case), case))
    return d


def test_c1_256_fp32(gpu_lib):
    d = _floor_case(gpu_lib, "c1")
    assert d.max() <= TOL32, report(d, TOL32)


def test_c2_1024_fp32_full_size(gpu_lib):
    d = _floor_case(gpu_lib, "c2")
    assert d.max() <= TOL32, report(d, TOL32)


def test_c3_1024_fp16_storage(gpu_lib):
    d = _floor_case(gpu_lib, "c3_fp16", fp16=True)
    print(f"c3 fp16 storage: max {d.max():.3e} rms {np.sqrt((d ** 2).mean()):.3e}")


def test_region_of_interest_r10(gpu_lib):
    I1, I2, _, _ = synth.make_pair("t1", 0)
    _parity(gpu_lib, I1, I2, 4, 10, 3)


@pytest.mark.parametrize("shape,L,r,K", [((200, 333), 3, 5, 3), ((67, 45), 2, 12, 2),
                                         ((129, 257), 4, 3, 2), ((33, 300), 1, 3, 5)])
def test_ragged_sizes(gpu_lib, shape, L, r, K):
    I1, I2, _, _ = synth.make_pair("c1", 4)
    H, W = shape
    big1 = np.tile(I1, (2, 2))[:H, :W].copy()
    big2 = np.tile(I2, (2, 2))[:H, :W].copy()
    _parity(gpu_lib, big1, big2, L, r, K)


@pytest.mark.parametrize("case", ["r1_L1_K1", "r1_L1_K3", "r1_L2_K3"])
def test_radius_one_all_pixels(gpu_lib, case):
    """3x3 windows: one iteration is well within the tolerance everywhere; over several
    iterations the least conditioned windows amplify rounding (an FP32 run of the oracle's own
    operation order departs from FP64 by up to 1.7 px at two levels), so every pixel is held to
    the tolerance or, where the committed FP32 floor of that pixel says no FP32 evaluation can
    get closer, to the tolerance plus a multiple of the floor."""
    I1, I2 = floor_util.case_inputs(case)
    _, L, r, K, _, _, tol = floor_util.CASES[case]
    u, v = gpu_flow(gpu_lib, I1, I2, L, r, K)
    ou, ov = oracle.flow(I1, I2, L, r, K)
    d = flow_error(u, v, ou, ov)
    print(floor_util.check_all_pixels(d, tol, floor_util.load_floor(case), case))
    assert np.all(np.isfinite(u)) and np.all(np.isfinite(v))


def test_identical_frames_zero_bitwise(gpu_lib):
    I1, _, _, _ = synth.make_pair("c1", 5)
    u, v = gpu_flow(gpu_lib, I1, I1, 3, 4, 3)
    assert np.all(u == 0) and np.all(v == 0)


def test_zero_iterations_and_radius_zero(gpu_lib):
    I1, I2, _, _ = synth.make_pair("c1", 6)
    u, v = gpu_flow(gpu_lib, I1, I2, 3, 4, 0)
    assert np.all(u == 0) and np.all(v == 0)
    _parity(gpu_lib, I1[:64, :80].copy(), I2[:64, :80].copy(), 1, 0, 1)


def test_linear_ramp_exact_shift(gpu_lib):
    x = np.arange(64, dtype=float)
    I1 = np.tile(4 * x, (40, 1)).astype(np.uint8)
    I2 = np.tile(4 * x - 1, (40, 1)).clip(0).astype(np.uint8)
    u, v = gpu_flow(gpu_lib, I1, I2, 1, 3, 1)
    np.testing.assert_allclose(u[:, 6:-6], 0.25, atol=1e-6)
    np.testing.assert_allclose(v[:, 6:-6], 0.0, atol=1e-6)


def test_float_input_scale_invariance(gpu_lib):
    I1, I2, _, _ = synth.make_pair("c1", 7)
    f1, f2 = I1.astype(np.float32), I2.astype(np.float32)
    a = gpu_flow(gpu_lib, f1, f2, 3, 4, 3)
    b = gpu_flow(gpu_lib, f1 * np.float32(8), f2 * np.float32(8), 3, 4, 3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_repeat_run_bitwise(gpu_lib):
    I1, I2, _, _ = synth.make_pair("c1", 8)
    a = gpu_flow(gpu_lib, I1, I2, 3, 4, 4)
    b = gpu_flow(gpu_lib, I1, I2, 3, 4, 4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_graph_replay_matches_eager(gpu_lib):
    """Replays of the captured schedule equal eager launches bitwise, replay after replay,
    with eager work and synchronisations in between."""
    import torch
    ofmi = gpu_lib
    I1, I2, _, _ = synth.make_pair("c1", 9)
    d1, d2 = to_dev(I1), to_dev(I2)
    eager = ofmi.Plan(256, 256, 3, 4, 4, device=dev(), graph=False)
    graph = ofmi.Plan(256, 256, 3, 4, 4, device=dev(), graph=True)
    ue, ve = eager.compute(d1, d2)
    torch.cuda.synchronize()
    ref_u, ref_v = ue.cpu().numpy(), ve.cpu().numpy()
    ug = torch.empty_like(ue)
    vg = torch.empty_like(ve)
    announce("graph replay x4 vs eager")
    for rep in range(4):
        ug.fill_(float("nan"))
        vg.fill_(float("nan"))
        graph.compute(d1, d2, ug, vg)
        eager.compute(d2, d1)                 # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(ug.cpu().numpy(), ref_u), f"replay {rep}"
        assert np.array_equal(vg.cpu().numpy(), ref_v), f"replay {rep}"
    eager.close()
    graph.close()


def test_plan_configs_and_autotune_keep_bits(gpu_lib):
    """Tile height and variant change the launch, not the result (window sums are tiling
    independent): every configuration and the autotuned one give the same bits."""
    import torch
    ofmi = gpu_lib
    I1, I2, _, _ = synth.make_pair("c1", 10)
    d1, d2 = to_dev(I1), to_dev(I2)
    plan = ofmi.Plan(256, 256, 3, 4, 3, device=dev())
    u0, v0 = plan.compute(d1, d2)
    torch.cuda.synchronize()
    ref = (u0.cpu().numpy(), v0.cpu().numpy())
    for cfg in ({"bands": [1, 1, 1], "variant": [0, 0, 0]}, {"bands": [8, 4, 2], "variant": [1, 1, 1]},
                {"bands": [2, 8, 1], "variant": [0, 1, 2]}, {"bands": [1, 2, 4], "variant": [2, 2, 2]},
                {"bands": [1, 1, 1], "variant": [3, 4, 4]}, {"bands": [2, 1, 4], "variant": [4, 3, 3]},
                {"bands": [1, 1, 1], "variant": [5, 6, 5]}, {"bands": [2, 3, 1], "variant": [6, 5, 6]},
                {"bands": [4, 1, 8], "variant": [5, 5, 6]}, {"bands": [1, 3, 2], "variant": [7, 7, 5]}):
        announce(f"plan config {cfg}")
        plan.set_config(cfg)
        u, v = plan.compute(d1, d2)
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), ref[0]) and np.array_equal(v.cpu().numpy(), ref[1]), cfg
    for bad in ({"bands": [1, 1, 1], "variant": [0, 8, 0]}, {"bands": [0, 1, 1], "variant": [0, 0, 0]},
                {"bands": [1, 1, 1], "variant": [-1, 0, 0]}):
        with pytest.raises(ofmi.OfError):
            plan.set_config(bad)
    announce("plan autotune")
    cfg = plan.autotune(d1, d2, u0, v0, reps=1)
    u, v = plan.compute(d1, d2)
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), ref[0]) and np.array_equal(v.cpu().numpy(), ref[1]), cfg
    plan.close()


def test_two_band_variants_at_radius_8(gpu_lib):
    """Two bands per pass at the largest radius they take, on a ragged frame (partial strips
    and tiles, odd and even band counts): the same bits as one band per pass and the oracle's
    flow to 1e-3 px; above r = 8 the plan rejects them."""
    import torch
    ofmi = gpu_lib
    I1, I2, _, _ = synth.make_pair("c1", 12)
    I1, I2 = I1[:219, :173].copy(), I2[:219, :173].copy()
    d1, d2 = to_dev(I1), to_dev(I2)
    plan = ofmi.Plan(219, 173, 2, 8, 3, device=dev())
    plan.set_config({"bands": [1, 1], "variant": [1, 3]})
    u0, v0 = plan.compute(d1, d2)
    torch.cuda.synchronize()
    ref = (u0.cpu().numpy(), v0.cpu().numpy())
    ou, ov = oracle.flow(I1, I2, 2, 8, 3)
    d = flow_error(ref[0], ref[1], ou, ov)
    assert d.max() <= 1e-3, report(d, 1e-3)
    for cfg in ({"bands": [1, 1], "variant": [5, 6]}, {"bands": [2, 1], "variant": [6, 5]},
                {"bands": [3, 4], "variant": [5, 5]}, {"bands": [8, 2], "variant": [6, 6]},
                {"bands": [1, 3], "variant": [7, 7]}):
        announce(f"two bands per pass, r=8, config {cfg}")
        plan.set_config(cfg)
        u, v = plan.compute(d1, d2)
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), ref[0]) and np.array_equal(v.cpu().numpy(), ref[1]), cfg
    plan.close()
    big = ofmi.Plan(64, 64, 1, 9, 1, device=dev())
    for w in (5, 6, 7):
        with pytest.raises(ofmi.OfError):
            big.set_config({"bands": [1], "variant": [w]})
    big.set_config({"bands": [1], "variant": [4]})
    big.close()


DEGENERATE = [((1, 1), 1, 0, 2), ((1, 1), 1, 2, 2), ((1, 37), 1, 2, 3), ((29, 1), 1, 3, 3),
              ((2, 3), 2, 1, 2), ((5, 5), 3, 1, 2), ((7, 300), 3, 4, 3), ((300, 7), 3, 4, 3),
              ((3, 64), 2, 8, 2)]


def _crop(H, W):
    I1, I2, _, _ = synth.make_pair("c1", 7)
    I1, I2 = np.tile(I1, (2, 2)), np.tile(I2, (2, 2))
    assert 40 + H <= I1.shape[0] and 50 + W <= I1.shape[1]
    return (np.ascontiguousarray(I1[40:40 + H, 50:50 + W]),
            np.ascontiguousarray(I2[40:40 + H, 50:50 + W]))


@pytest.mark.parametrize("shape,L,r,K", DEGENERATE)
def test_degenerate_shapes_all_pixels(gpu_lib, shape, L, r, K):
    """Single pixels, single rows and columns, frames narrower than one window and pyramids
    down to one-pixel levels: every pixel against the oracle (the windows are truncated at
    the borders and one-row frames have no vertical gradient, so the solve takes its rank-1
    branch), with the FP32 floor computed here on the CPU for these few pixels."""
    I1, I2 = _crop(*shape)
    u, v = gpu_flow(gpu_lib, I1, I2, L, r, K)
    ou, ov = oracle.flow(I1, I2, L, r, K)
    d = flow_error(u, v, ou, ov)
    floor, _ = floor_util.ensemble_floor(I1, I2, L, r, K)
    print(floor_util.check_all_pixels(d, TOL32, floor, f"{shape} L={L} r={r} K={K}"))
    if shape[0] == 1:
        assert np.all(v == 0.0)      # no vertical gradient anywhere: v stays exactly zero
    if shape[1] == 1:
        assert np.all(u == 0.0)


def test_degenerate_shapes_in_one_batch(gpu_lib):
    """The degenerate one-level shapes as one batch: each flow equals its plain path's bits."""
    import torch
    ofmi = gpu_lib
    shapes = [(1, 1), (1, 37), (29, 1), (2, 3), (4, 70)]
    pairs = [_crop(*s) for s in shapes]
    announce("batch of degenerate shapes")
    b = ofmi.Batch(shapes, 1, 2, 3, device=dev())
    us, vs = b.outputs()
    b.compute([to_dev(p[0]) for p in pairs], [to_dev(p[1]) for p in pairs], us, vs)
    torch.cuda.synchronize()
    for i, p in enumerate(pairs):
        pu, pv = gpu_flow(ofmi, p[0], p[1], 1, 2, 3)
        assert np.array_equal(us[i].cpu().numpy(), pu) and np.array_equal(vs[i].cpu().numpy(), pv), shapes[i]
    b.close()


def test_concurrent_plans_on_two_streams(gpu_lib):
    """Two plans driven from two streams at once (their launches interleave on the device, a
    batch of two pairs beside them on a third): every result equals its sequential bits, so
    plans and batches share no hidden device state."""
    import torch
    ofmi = gpu_lib
    pairs = [synth.make_pair("c1", 30 + i)[:2] for i in range(3)]
    d = [(to_dev(p[0]), to_dev(p[1])) for p in pairs]
    announce("two plans and a batch on three streams")
    plans = [ofmi.Plan(256, 256, 3, 4, 4, device=dev()) for _ in range(2)]
    batch = ofmi.Batch([(256, 256), (256, 256)], 3, 4, 4, device=dev())
    ref = []
    for k in range(2):
        u, v = plans[k].compute(*d[k])
        torch.cuda.synchronize()
        ref.append((u.cpu().numpy(), v.cpu().numpy()))
    bu, bv = batch.outputs()
    batch.compute([d[2][0], d[0][0]], [d[2][1], d[0][1]], bu, bv)
    torch.cuda.synchronize()
    bref = [(bu[i].cpu().numpy(), bv[i].cpu().numpy()) for i in range(2)]
    streams = [torch.cuda.Stream(dev()) for _ in range(3)]
    outs = [[(torch.empty((256, 256), device=dev()), torch.empty((256, 256), device=dev()))
             for _ in range(6)] for _ in range(2)]
    bouts = [batch.outputs() for _ in range(6)]
    for rep in range(6):
        for k in range(2):
            plans[k].compute(d[k][0], d[k][1], outs[k][rep][0], outs[k][rep][1], stream=streams[k])
        batch.compute([d[2][0], d[0][0]], [d[2][1], d[0][1]], bouts[rep][0], bouts[rep][1],
                      stream=streams[2])
    torch.cuda.synchronize()
    for rep in range(6):
        for k in range(2):
            u, v = outs[k][rep]
            assert np.array_equal(u.cpu().numpy(), ref[k][0]) and np.array_equal(v.cpu().numpy(), ref[k][1]), (rep, k)
        for i in range(2):
            assert np.array_equal(bouts[rep][0][i].cpu().numpy(), bref[i][0]), (rep, i)
            assert np.array_equal(bouts[rep][1][i].cpu().numpy(), bref[i][1]), (rep, i)
    # the batch's second pair is pair 0, so it also equals plan 0's bits
    assert np.array_equal(bref[1][0], ref[0][0]) and np.array_equal(bref[1][1], ref[0][1])
    for p in plans:
        p.close()
    batch.close()
