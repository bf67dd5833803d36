"""Serving form on the GPU: resident previous-frame pyramids, multi-stream pushes, budget."""
import numpy as np
import pytest

import floor_util
import oracle
import synth
from gpu_util import announce, dev, flow_error

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
