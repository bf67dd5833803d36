"""Region-of-interest masks and the Gaussian-weighted window in the batched and served forms:
every result equals the plain per-pair path with the same mask or window, bitwise (window sums
and mask handling do not depend on the tiling), and sampled pairs the oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, dev, flow_error, report, to_dev

pytestmark = pytest.mark.gpu

SIZES = [(160, 200), (96, 128), (256, 256)]
L, R, K = 3, 4, 3


def _pairs():
    out = []
    for i, (H, W) in enumerate(SIZES):
        I1, I2, _, _ = synth.make_pair("c1", 20 + i)
        out.append((np.tile(I1, (2, 2))[:H, :W].copy(), np.tile(I2, (2, 2))[:H, :W].copy()))
    return out


def _mask(H, W, k):
    M = np.ones((H, W), dtype=np.uint8)
    M[H // 2 + k:, :W // 3] = 0          # a step-like obstacle
    M[:6 + k, :] = 0                     # a wall
    return M


def _plain(ofmi, I1, I2, mask=None, gaussian=False, iters=K, fp16=False):
    import torch
    H, W = I1.shape
    plan = ofmi.Plan(H, W, L, R, iters, gaussian_window=gaussian, fp16=fp16, device=dev())
    if mask is not None:
        plan.set_mask(to_dev(mask))
    u, v = plan.compute(to_dev(I1), to_dev(I2))
    torch.cuda.synchronize()
    out = u.cpu().numpy(), v.cpu().numpy()
    plan.close()
    return out


@pytest.mark.parametrize("gaussian,fp16", [(False, False), (True, False), (False, True)])
def test_batch_masks_and_window_equal_plain_path(gpu_lib, gaussian, fp16):
    import torch
    ofmi = gpu_lib
    pairs = _pairs()
    masks = [_mask(*SIZES[0], 0), None, _mask(*SIZES[2], 3)]
    announce(f"batch with masks, gaussian={gaussian}, fp16={fp16}")
    b = ofmi.Batch(SIZES, L, R, K, gaussian_window=gaussian, fp16=fp16, device=dev())
    d1 = [to_dev(p[0]) for p in pairs]
    d2 = [to_dev(p[1]) for p in pairs]
    b.set_masks([None if m is None else to_dev(m) for m in masks])
    for cfg in (None, {"bands": [2, 1, 1], "grid": [0, 16, 0], "variant": [0, 1, 2]},
                {"bands": [1, 3, 2], "grid": [8, 0, 0], "variant": [2, 2, 0]}):
        if cfg is not None:
            b.set_config(cfg)
        us, vs = b.outputs()
        b.compute(d1, d2, us, vs)
        torch.cuda.synchronize()
        for i, (p, m) in enumerate(zip(pairs, masks)):
            pu, pv = _plain(ofmi, p[0], p[1], m, gaussian, fp16=fp16)
            assert np.array_equal(us[i].cpu().numpy(), pu) and np.array_equal(vs[i].cpu().numpy(), pv), (i, cfg)
            if m is not None:
                assert np.all(pu[m == 0] == 0) and np.all(pv[m == 0] == 0)
    ou, ov = oracle.flow(pairs[0][0], pairs[0][1], L, R, K, mask=masks[0].astype(bool),
                         window="gauss" if gaussian else "box")
    d = flow_error(us[0].cpu().numpy(), vs[0].cpu().numpy(), ou, ov)
    tol = 2e-2 if fp16 else 1e-3
    assert d.max() <= tol, report(d, tol)
    # removing the masks gives the unmasked bits again
    b.set_masks(None)
    us, vs = b.outputs()
    b.compute(d1, d2, us, vs)
    torch.cuda.synchronize()
    pu, pv = _plain(ofmi, pairs[2][0], pairs[2][1], None, gaussian, fp16=fp16)
    assert np.array_equal(us[2].cpu().numpy(), pu) and np.array_equal(vs[2].cpu().numpy(), pv)
    b.close()


def test_masked_batch_autotune_keeps_bits(gpu_lib):
    """The autotuner on a masked batch (every candidate rebuilds the active-first tile lists and
    clears the intermediate planes) leaves a configuration whose results equal the plain path's
    with the same masks, bitwise, on the graph path and the eager path alike."""
    import torch
    ofmi = gpu_lib
    pairs = _pairs()
    masks = [_mask(*SIZES[0], 2), _mask(*SIZES[1], 0), None]
    announce("masked batch autotune")
    d1 = [to_dev(p[0]) for p in pairs]
    d2 = [to_dev(p[1]) for p in pairs]
    for graph in (True, False):
        b = ofmi.Batch(SIZES, L, R, K, graph=graph, device=dev())
        b.set_masks([None if m is None else to_dev(m) for m in masks])
        us, vs = b.outputs()
        b.autotune(d1, d2, us, vs, reps=1)
        us, vs = b.outputs()
        for _ in range(2):
            b.compute(d1, d2, us, vs)
        torch.cuda.synchronize()
        for i, (p, m) in enumerate(zip(pairs, masks)):
            pu, pv = _plain(ofmi, p[0], p[1], m)
            assert np.array_equal(us[i].cpu().numpy(), pu) and np.array_equal(vs[i].cpu().numpy(), pv), (graph, i)
        b.close()


@pytest.mark.parametrize("iters,aligned", [(1, False), (K, False), (1, True), (K, True)])
def test_batch_fully_masked_pairs(gpu_lib, iters, aligned):
    """A pair whose mask excludes every pixel has no tile to compute at any level: its flow is
    zero and the other pairs keep the plain path's bits.  With every pair fully masked, no
    iteration launch runs before the final phase, which writes the zeros."""
    import torch
    ofmi = gpu_lib
    pairs = _pairs()
    d1 = [to_dev(p[0]) for p in pairs]
    d2 = [to_dev(p[1]) for p in pairs]
    announce(f"batch with fully masked pairs, iters={iters}, aligned={aligned}")
    b = ofmi.Batch(SIZES, L, R, iters, device=dev())
    # aligned: pair 0 has its first 64-column strip masked out, so at full resolution every
    # tile is all masked or all unmasked (no tile needs the per-pixel mask), at coarser levels not
    m0 = _mask(*SIZES[0], 1)
    if aligned:
        m0 = np.ones(SIZES[0], np.uint8)
        m0[:, :64] = 0
    masks = [m0, np.zeros(SIZES[1], np.uint8), None]
    b.set_masks([None if m is None else to_dev(m) for m in masks])
    for cfg in (None, {"bands": [1, 2, 1], "grid": [8, 0, 16], "variant": [1, 0, 2]}):
        if cfg is not None:
            b.set_config(cfg)
        us, vs = b.outputs()
        for t in us + vs:
            t.fill_(7.0)
        b.compute(d1, d2, us, vs)
        torch.cuda.synchronize()
        for i, (p, m) in enumerate(zip(pairs, masks)):
            pu, pv = _plain(ofmi, p[0], p[1], m, iters=iters)
            assert np.array_equal(us[i].cpu().numpy(), pu) and np.array_equal(vs[i].cpu().numpy(), pv), (i, cfg)
        assert not us[1].any() and not vs[1].any()
    b.set_masks([to_dev(np.zeros(s, np.uint8)) for s in SIZES])
    us, vs = b.outputs()
    for t in us + vs:
        t.fill_(7.0)
    b.compute(d1, d2, us, vs)
    torch.cuda.synchronize()
    assert all(not t.any() for t in us + vs)
    b.close()


def test_served_streams_with_mask_and_window(gpu_lib):
    """Two streams served together with the Gaussian window, one of them masked: each flow
    equals the plain path's with the same window and mask, bitwise."""
    ofmi = gpu_lib
    from paper_1306_2461_amd.serve import GpuExecutor, Server
    sizes = [(96, 128), (160, 120)]
    streams = [[f for f, _, _ in synth.stream_frames(s, 3, size=sizes[s])] for s in range(2)]
    M = _mask(*sizes[0], 1)
    ex = GpuExecutor(L, R, K, device=dev(), keep_on_device=False, gaussian_window=True)
    srv = Server(ex)
    announce("served streams with mask and Gaussian window")
    reqs = {s: [srv.submit(s, streams[s][0])] for s in range(2)}
    srv.drain()
    ex.set_mask(srv.sessions[0], to_dev(M))
    for t in (1, 2):
        for s in range(2):
            reqs[s].append(srv.submit(s, streams[s][t]))
    srv.drain()
    ex.close_all()
    for s in range(2):
        for t in (1, 2):
            pu, pv = _plain(ofmi, streams[s][t - 1], streams[s][t], M if s == 0 else None, True)
            r = reqs[s][t]
            assert r.has_flow and np.array_equal(r.u, pu) and np.array_equal(r.v, pv), (s, t)


def test_served_masks_set_late_full_and_aligned(gpu_lib):
    """Served masks set after unmasked flows (the session's planes held nonzero flow), a fully
    masked stream, a tile-aligned mask (no tile needs the per-pixel mask at full resolution),
    a push of only those two, and a mask removed again: every flow equals the plain path's
    with the same mask, bitwise."""
    ofmi = gpu_lib
    from paper_1306_2461_amd.serve import GpuExecutor, Server
    sizes = [(96, 128), (160, 120), (128, 192)]
    streams = [[f for f, _, _ in synth.stream_frames(s, 5, size=sizes[s])] for s in range(3)]
    aligned = np.ones(sizes[2], np.uint8)
    aligned[:, :64] = 0
    masks = [_mask(*sizes[0], 2), np.zeros(sizes[1], np.uint8), aligned]
    ex = GpuExecutor(L, R, K, device=dev(), keep_on_device=False)
    srv = Server(ex)
    announce("served masks set late, fully masked, tile-aligned, removed")
    # which mask each stream has when frame t is pushed (None = unmasked)
    plan = {1: [None, None, None], 2: masks, 3: [None] + masks[1:], 4: [None] + masks[1:]}
    reqs = {s: [srv.submit(s, streams[s][0])] for s in range(3)}
    srv.drain()
    for t in (1, 2, 3, 4):
        if t == 2:
            for s in range(3):
                ex.set_mask(srv.sessions[s], to_dev(masks[s]))
        if t == 4:
            ex.set_mask(srv.sessions[0], None)
        for s in range(3):
            if t == 3 and s == 0:
                continue
            reqs[s].append((t, srv.submit(s, streams[s][t])))
        srv.drain()
    ex.close_all()
    for s in range(3):
        for t, r in reqs[s][1:]:
            m = plan[t][s]
            prev = t - 1 if not (s == 0 and t == 4) else 2
            pu, pv = _plain(ofmi, streams[s][prev], streams[s][t], m)
            assert r.has_flow and np.array_equal(r.u, pu) and np.array_equal(r.v, pv), (s, t)
            if m is not None:
                assert np.all(r.u[m == 0] == 0) and np.all(r.v[m == 0] == 0)


@pytest.mark.parametrize("bands,variant,gaussian,fp16", [([3, 2, 2], [1, 2, 0], False, False),
                                                         ([2, 3, 1], [2, 1, 1], False, False),
                                                         ([3, 2, 2], [1, 2, 0], True, False),
                                                         ([3, 3, 2], [2, 2, 1], False, True)])
def test_batch_masked_tiles_cut_to_unmasked_rows(gpu_lib, bands, variant, gaussian, fp16):
    """Tiles with masked pixels run only their bands that hold unmasked rows (masked rows cut
    off at the top, at the bottom, and at the frame's bottom edge), and the rows cut off are
    zero-filled in the final phase; tiles at the bottom edge run only the bands the frame
    holds.  Flows equal the plain path's with the same masks, bitwise."""
    import torch
    ofmi = gpu_lib
    pairs = _pairs()
    m0 = np.ones(SIZES[0], np.uint8)      # 160 x 200
    m0[:20] = 0                           # a wall: the first tile row loses its top bands
    m0[40:54, :64] = 0                    # the second tile row of the first strip its bottom
    m0[135:151] = 0                       # the last tile row (at the bottom edge) its top
    m0[60:66, 100:] = 0                   # masked rows inside a tile: nothing cut
    m2 = np.ones(SIZES[2], np.uint8)      # 256 x 256
    m2[90:, :64] = 0
    m2[:, 200:] = 0
    masks = [m0, None, m2]
    announce(f"batch masked tiles cut to unmasked rows, bands={bands}, gaussian={gaussian}, fp16={fp16}")
    d1 = [to_dev(p[0]) for p in pairs]
    d2 = [to_dev(p[1]) for p in pairs]
    b = ofmi.Batch(SIZES, L, R, K, gaussian_window=gaussian, fp16=fp16, device=dev())
    b.set_masks([None if m is None else to_dev(m) for m in masks])
    b.set_config({"bands": bands, "grid": [0, 16, 0], "variant": variant})
    us, vs = b.outputs()
    for t in us + vs:
        t.fill_(7.0)
    b.compute(d1, d2, us, vs)
    torch.cuda.synchronize()
    for i, (p, m) in enumerate(zip(pairs, masks)):
        pu, pv = _plain(ofmi, p[0], p[1], m, gaussian, fp16=fp16)
        assert np.array_equal(us[i].cpu().numpy(), pu) and np.array_equal(vs[i].cpu().numpy(), pv), i
    b.close()


def test_served_masked_tiles_cut_to_unmasked_bands(gpu_lib):
    """A push of 4 Mi full-resolution pixels takes two-band tiles: a served stream's tiles with
    masked pixels then run only their bands with unmasked rows (cut at the top, at the bottom),
    the rows cut off zero-filled in the final phase.  Flows equal the plain path's with the
    same mask, bitwise."""
    ofmi = gpu_lib
    from paper_1306_2461_amd.serve import GpuExecutor, Server
    size = (1024, 2048)                   # two streams: 4 Mi pixels per push
    streams = [[f for f, _, _ in synth.stream_frames(s, 2, size=size)] for s in range(2)]
    M = np.ones(size, np.uint8)
    M[:12] = 0                            # the first tile row loses its top band
    M[99:108, :64] = 0                    # the tile row from row 90 its bottom band, first strip
    M[500:, 1500:] = 0
    ex = GpuExecutor(L, R, K, device=dev(), keep_on_device=False)
    srv = Server(ex)
    announce("served masked tiles cut to unmasked bands")
    for s in range(2):
        srv.submit(s, streams[s][0])
    srv.drain()
    ex.set_mask(srv.sessions[0], to_dev(M))
    reqs = [srv.submit(s, streams[s][1]) for s in range(2)]
    srv.drain()
    ex.close_all()
    for s in range(2):
        pu, pv = _plain(ofmi, streams[s][0], streams[s][1], M if s == 0 else None)
        r = reqs[s]
        assert r.has_flow and np.array_equal(r.u, pu) and np.array_equal(r.v, pv), s
        if s == 0:
            assert np.all(r.u[M == 0] == 0) and np.all(r.v[M == 0] == 0)
