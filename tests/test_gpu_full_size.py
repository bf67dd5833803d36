"""Parity at the full sizes of the batched and served workloads, in the launch configuration
the benchmark times: every result against the plain per-pair path (bitwise; window sums do not
depend on tiling, so any correct launch gives the same bits) and sampled pairs against the FP64
oracle, one pair of each frame size (the oracle takes about 17 s per 2048x2048 pair)."""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import floor_util
import oracle
import synth
from gpu_util import announce, dev, flow_error, report, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL16 = 2e-2


def _gen_c4(i_and_size):
    from synth import particles as P
    i, (H, W) = i_and_size
    wl = P.WORKLOADS["c4"]
    rngs = P._rngs(wl.index, i)
    field = P._vortex_field(rngs[4], H, W)
    I1, I2, _, _, _ = P._pair_from_field(field, H, W, wl.rho, wl.sigma, rngs, wl.levels)
    return I1, I2


def _workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def test_c4_full_batch_against_plain_path_and_oracle(gpu_lib):
    import torch
    ofmi = gpu_lib
    from synth import particles as P
    wl = synth.workload("c4")
    sizes = P.batch_sizes(64)
    announce("c4: generating 64 mixed-size pairs")
    with cf.ProcessPoolExecutor(max_workers=_workers()) as ex:
        pairs = list(ex.map(_gen_c4, list(enumerate(sizes))))
    d1 = [to_dev(p[0]) for p in pairs]
    d2 = [to_dev(p[1]) for p in pairs]
    announce("c4: 64-pair FP16 batch, autotuned, graph replay")
    b = ofmi.Batch(sizes, wl.levels, wl.radius, wl.iters, fp16=True, device=dev())
    us, vs = b.outputs()
    b.autotune(d1, d2, us, vs, reps=1)
    b.compute(d1, d2, us, vs)
    torch.cuda.synchronize()
    got = [(u.cpu().numpy(), v.cpu().numpy()) for u, v in zip(us, vs)]
    b.close()
    plans = {}
    for i, (H, W) in enumerate(sizes):
        if (H, W) not in plans:
            plans[(H, W)] = ofmi.Plan(H, W, wl.levels, wl.radius, wl.iters, fp16=True, device=dev())
        pu, pv = plans[(H, W)].compute(d1[i], d2[i])
        torch.cuda.synchronize()
        assert np.array_equal(got[i][0], pu.cpu().numpy()) and np.array_equal(got[i][1], pv.cpu().numpy()), (i, H, W)
    for p in plans.values():
        p.close()
    sampled = {}
    for i, s in enumerate(sizes):
        sampled.setdefault(s, i)
    for (H, W), i in sampled.items():
        announce(f"c4: oracle on pair {i} ({H}x{W})")
        ou, ov = oracle.flow(pairs[i][0], pairs[i][1], wl.levels, wl.radius, wl.iters)
        d = flow_error(got[i][0], got[i][1], ou, ov)
        assert d.max() <= TOL16, (i, H, W, report(d, TOL16))


def test_c5_served_full_sizes_against_plain_path_and_oracle(gpu_lib):
    import torch
    ofmi = gpu_lib
    from paper_1306_2461_amd.serve import GpuExecutor, Server
    wl = synth.workload("c5")
    sizes = [(480, 640), (1024, 1024), (2048, 2048)]
    announce("c5: generating 3 streams x 3 frames at full sizes")
    streams = [[f for f, _, _ in synth.stream_frames(s, 3, size=sz)] for s, sz in enumerate(sizes)]
    ex = GpuExecutor(wl.levels, wl.radius, wl.iters, fp16=True, device=dev(), keep_on_device=False)
    srv = Server(ex)
    reqs = {}
    for t in range(3):
        for s in range(3):
            reqs.setdefault(s, []).append(srv.submit(s, streams[s][t]))
    announce("c5: serving the mix")
    srv.drain()
    ex.close_all()
    for s, (H, W) in enumerate(sizes):
        flows = [(r.u, r.v) for r in reqs[s] if r.has_flow]
        assert len(flows) == 2
        plan = ofmi.Plan(H, W, wl.levels, wl.radius, wl.iters, fp16=True, device=dev())
        for t in range(2):
            pu, pv = plan.compute(to_dev(streams[s][t]), to_dev(streams[s][t + 1]))
            torch.cuda.synchronize()
            assert np.array_equal(flows[t][0], pu.cpu().numpy()) and np.array_equal(flows[t][1], pv.cpu().numpy()), (s, t)
        plan.close()
    # the oracle on the 640x480 stream, every pixel (its committed FP16-storage floor is far
    # below the tolerance)
    announce("c5: oracle on the 640x480 stream")
    flows = [(r.u, r.v) for r in reqs[0] if r.has_flow]
    ou, ov = oracle.flow(streams[0][0], streams[0][1], wl.levels, wl.radius, wl.iters)
    d = flow_error(flows[0][0], flows[0][1], ou, ov)
    print(floor_util.check_all_pixels(d, TOL16, floor_util.load_floor("c5_640_fp16"), "c5 640x480"))
