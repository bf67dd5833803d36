"""Serving form on the GPU: resident previous-frame pyramids, multi-stream pushes, budget."""
import numpy as np
import pytest

import floor_util
import oracle
import synth
from gpu_util import announce, dev, flow_error, to_dev

pytestmark = pytest.mark.gpu

SIZES = floor_util.SERVE_SIZES
L, R, K = floor_util.SERVE_LRK


def _streams(n_frames=4):
    return [[f for f, _, _ in synth.stream_frames(s, n_frames, size=SIZES[s])] for s in range(len(SIZES))]


def _run(executor_kw, order):
    """Serve frames in the given (stream, frame index) order; returns {stream: [u,v per pair]}."""
    from paper_1306_2461_amd.serve import GpuExecutor, Server
    ex = GpuExecutor(L, R, K, device=dev(), keep_on_device=False, **executor_kw)
    srv = Server(ex)
    streams = _streams()
    reqs = {}
    for s, t in order:
        reqs.setdefault(s, []).append(srv.submit(s, streams[s][t]))
    srv.drain()
    out = {s: [(r.u, r.v) for r in rs if r.has_flow] for s, rs in reqs.items()}
    ex.close_all()
    return out, streams


def test_alone_equals_mix_equals_plain_and_oracle(gpu_lib):
    """Each served flow equals the same stream served alone and the plain per-pair path on the
    same two frames, bitwise, and the oracle on every pixel: within 1e-3 px, or where these
    small frames move 8 px per frame out of the image and the border windows are so
    ill-conditioned that FP32 runs of the oracle's own operation order depart from FP64 by up
    to 0.08 px, within the tolerance plus a multiple of that committed per-pixel floor."""
    import torch
    ofmi = gpu_lib
    from gpu_util import to_dev
    announce("serving: mix of 3 streams x 4 frames")
    mix, streams = _run({}, [(s, t) for t in range(4) for s in range(3)])
    for s in range(3):
        announce(f"serving: stream {s} alone")
        alone, _ = _run({}, [(s, t) for t in range(4)])
        assert len(mix[s]) == 3 and len(alone[s]) == 3
        H, W = SIZES[s]
        plan = ofmi.Plan(H, W, L, R, K, device=dev())
        for t in range(3):
            assert np.array_equal(mix[s][t][0], alone[s][t][0]), (s, t)
            assert np.array_equal(mix[s][t][1], alone[s][t][1]), (s, t)
            pu, pv = plan.compute(to_dev(streams[s][t]), to_dev(streams[s][t + 1]))
            torch.cuda.synchronize()
            assert np.array_equal(mix[s][t][0], pu.cpu().numpy()), (s, t)
            assert np.array_equal(mix[s][t][1], pv.cpu().numpy()), (s, t)
            ou, ov = oracle.flow(streams[s][t], streams[s][t + 1], L, R, K)
            d = flow_error(mix[s][t][0], mix[s][t][1], ou, ov)
            print(floor_util.check_all_pixels(d, 1e-3, floor_util.load_floor(f"serve_{s}_{t}"),
                                              f"served stream {s} pair {t}"))
        plan.close()


def test_session_budget_and_single_push(gpu_lib):
    import ctypes
    import torch
    ofmi = gpu_lib
    from paper_1306_2461_amd import _binding as B
    lib = B.load()
    per = lib.of_session_bytes(96, 128, L, R, K, 0)
    assert per > 0
    srv = lib.of_server_create(L, R, K, 0, 2 * per)
    a = lib.of_server_open(srv, 96, 128)
    b = lib.of_server_open(srv, 96, 128)
    assert a and b and lib.of_server_resident_bytes(srv) == 2 * per
    assert not lib.of_server_open(srv, 96, 128)
    assert b"budget" in lib.of_last_error()
    assert lib.of_server_close(srv, b) == 0
    c = lib.of_server_open(srv, 96, 128)
    assert c
    frames = _streams()[0]
    d = [torch.from_numpy(f).to(dev()) for f in frames[:2]]
    u = torch.empty((96, 128), dtype=torch.float32, device=dev())
    v = torch.empty_like(u)
    has = ctypes.c_int(-1)
    announce("session push x2")
    st = torch.cuda.current_stream().cuda_stream
    assert lib.of_session_push(a, d[0].data_ptr(), None, None, st, ctypes.byref(has)) == 0
    assert has.value == 0
    assert lib.of_session_push(a, d[1].data_ptr(), u.data_ptr(), v.data_ptr(), st, ctypes.byref(has)) == 0
    torch.cuda.synchronize()
    assert has.value == 1
    ou, ov = oracle.flow(frames[0], frames[1], L, R, K)
    dd = flow_error(u.cpu().numpy(), v.cpu().numpy(), ou, ov)
    print(floor_util.check_all_pixels(dd, 1e-3, floor_util.load_floor("serve_0_0"), "session push"))
    lib.of_server_destroy(srv)


def _long_stream_work(torch, stream, ms_target=60):
    """Finite GPU work queued on `stream` (a few large matrix products) so that calls made
    right after can be seen to return before it completes."""
    a = torch.randn(6144, 6144, device=dev())
    with torch.cuda.stream(stream):
        for _ in range(12):
            a = (a @ a) * 1e-3
    return a


def test_session_entry_points_with_caller_workspace(gpu_lib):
    """of_session_create with torch-owned workspace, of_session_push_many over two sessions and
    of_session_destroy: flows equal the plain path bitwise; the pushes return while earlier work
    on the stream is still running; a full staging ring makes a push return OF_ESTATE (busy)
    without enqueueing anything, and the next push after the ring drains succeeds."""
    import ctypes
    import time

    import torch
    ofmi = gpu_lib
    from paper_1306_2461_amd import _binding as B
    lib = B.load()
    streams = _streams(3)
    sizes = SIZES[:2]
    ws = [torch.empty(lib.of_session_bytes(H, W, L, R, K, 0), dtype=torch.uint8, device=dev()) for H, W in sizes]
    ss = [lib.of_session_create(H, W, L, R, K, 0, w.data_ptr(), w.numel()) for (H, W), w in zip(sizes, ws)]
    assert all(ss), B.last_error()
    assert lib.of_session_resident_bytes(ss[0]) == ws[0].numel()
    sarr = (ctypes.c_void_p * 2)(*ss)
    frames = [[torch.from_numpy(f).to(dev()) for f in streams[s]] for s in range(2)]
    outs = [[(torch.empty(sz, device=dev()), torch.empty(sz, device=dev())) for _ in range(3)] for sz in sizes]
    stream = torch.cuda.Stream()
    st = stream.cuda_stream
    torch.cuda.synchronize()
    keep = []
    for t in range(3):
        if t == 1:
            keep.append(_long_stream_work(torch, stream))
        pf, _a = B.ptr_array([frames[s][t].data_ptr() for s in range(2)])
        pu, _b = B.ptr_array([outs[s][max(t - 1, 0)][0].data_ptr() for s in range(2)])
        pv, _c = B.ptr_array([outs[s][max(t - 1, 0)][1].data_ptr() for s in range(2)])
        has = (ctypes.c_int * 2)()
        t0 = time.perf_counter()
        assert lib.of_session_push_many(ctypes.cast(sarr, B._VPP), 2, pf, pu, pv, has, st) == 0, B.last_error()
        dt = time.perf_counter() - t0
        if t == 1:
            ev = torch.cuda.Event()
            ev.record(stream)
            assert not ev.query(), "the push waited for earlier work on its stream"
            announce(f"push returned in {dt * 1e3:.2f} ms with earlier work still running")
        assert list(has) == ([0, 0] if t == 0 else [1, 1])
    # fill the staging ring behind long work: the push after OF_SERVER_RING in flight is busy
    keep.append(_long_stream_work(torch, stream))
    s0 = ctypes.c_void_p(ss[0])
    has1 = ctypes.c_int()
    statuses = []
    for i in range(10):
        u0, v0 = outs[0][2]
        statuses.append(lib.of_session_push(s0, frames[0][i % 3].data_ptr(), u0.data_ptr(), v0.data_ptr(), st,
                                            ctypes.byref(has1)))
    # pushes succeed until the ring is full (earlier pushes may still hold slots), then busy
    assert B.OF_ESTATE in statuses, statuses
    first_busy = statuses.index(B.OF_ESTATE)
    assert 1 <= first_busy <= 8 and all(x == 0 for x in statuses[:first_busy]), statuses
    assert all(x in (0, B.OF_ESTATE) for x in statuses), statuses
    torch.cuda.synchronize()
    st2 = lib.of_session_push(s0, frames[0][0].data_ptr(), outs[0][2][0].data_ptr(), outs[0][2][1].data_ptr(), st,
                              ctypes.byref(has1))
    assert st2 == 0
    torch.cuda.synchronize()
    for s, (H, W) in enumerate(sizes):
        plan = ofmi.Plan(H, W, L, R, K, device=dev())
        for t in range(2):
            pu_, pv_ = plan.compute(frames[s][t], frames[s][t + 1])
            torch.cuda.synchronize()
            if t == 0:
                assert np.array_equal(outs[s][0][0].cpu().numpy(), pu_.cpu().numpy())
                assert np.array_equal(outs[s][0][1].cpu().numpy(), pv_.cpu().numpy())
            elif s == 1:
                assert np.array_equal(outs[s][1][0].cpu().numpy(), pu_.cpu().numpy())
        plan.close()
    for x in ss:
        lib.of_session_destroy(x)
    del keep


def test_executor_keeps_only_selected_flows(gpu_lib):
    """The request loop over the GPU executor with a keep predicate: kept flows equal the plain
    path bitwise, the others are dropped and their planes reused."""
    import torch
    ofmi = gpu_lib
    from paper_1306_2461_amd.serve import GpuExecutor, Server
    ex = GpuExecutor(L, R, K, device=dev(), keep_on_device=False)
    srv = Server(ex, keep=lambda r: r.stream_id == 1)
    streams = _streams(4)
    reqs = {s: [srv.submit(s, f) for f in streams[s]] for s in range(3)}
    srv.drain()
    ex.close_all()
    for s in range(3):
        assert [r.has_flow for r in reqs[s]] == [False, True, True, True]
        for t in range(1, 4):
            assert (reqs[s][t].u is not None) == (s == 1)
    H, W = SIZES[1]
    plan = ofmi.Plan(H, W, L, R, K, device=dev())
    from gpu_util import to_dev
    pu, pv = plan.compute(to_dev(streams[1][2]), to_dev(streams[1][3]))
    torch.cuda.synchronize()
    assert np.array_equal(reqs[1][3].u, pu.cpu().numpy()) and np.array_equal(reqs[1][3].v, pv.cpu().numpy())
    plan.close()


def test_session_odd_sizes_and_unaligned_frames(gpu_lib):
    """Frames whose byte count is not a multiple of 16 and frame pointers at odd addresses (the
    push copies them with a kernel: 16-byte words where both ends are aligned, bytes
    otherwise): the flows equal the plain path's bits."""
    import ctypes

    import torch
    ofmi = gpu_lib
    from paper_1306_2461_amd import _binding as B
    lib = B.load()
    H, W, Ls, Rs, Ks = 37, 53, 2, 2, 2
    I = [synth.make_pair("c1", 40 + t)[0][:H, :W].copy() for t in range(3)]
    announce("session with odd-size frames at odd addresses")
    ws = torch.empty(lib.of_session_bytes(H, W, Ls, Rs, Ks, 0), dtype=torch.uint8, device=dev())
    s = lib.of_session_create(H, W, Ls, Rs, Ks, 0, ws.data_ptr(), ws.numel())
    assert s, B.last_error()
    # each frame stored one byte into a larger buffer, so its pointer is odd
    bufs = [torch.zeros(H * W + 64, dtype=torch.uint8, device=dev()) for _ in range(3)]
    for b, f in zip(bufs, I):
        b[1:1 + H * W] = torch.from_numpy(f.reshape(-1)).to(dev())
    outs = [(torch.empty((H, W), device=dev()), torch.empty((H, W), device=dev())) for _ in range(3)]
    has = ctypes.c_int()
    st = torch.cuda.current_stream().cuda_stream
    torch.cuda.synchronize()
    for t in range(3):
        assert lib.of_session_push(ctypes.c_void_p(s), bufs[t].data_ptr() + 1, outs[t][0].data_ptr(),
                                   outs[t][1].data_ptr(), st, ctypes.byref(has)) == 0, B.last_error()
        assert has.value == (0 if t == 0 else 1)
    torch.cuda.synchronize()
    lib.of_session_destroy(ctypes.c_void_p(s))
    for t in (1, 2):
        plan = ofmi.Plan(H, W, Ls, Rs, Ks, device=dev())
        pu, pv = plan.compute(to_dev(I[t - 1]), to_dev(I[t]))
        torch.cuda.synchronize()
        assert np.array_equal(outs[t][0].cpu().numpy(), pu.cpu().numpy()), t
        assert np.array_equal(outs[t][1].cpu().numpy(), pv.cpu().numpy()), t
        plan.close()
