#!/usr/bin/env python3
"""Frame pairs/s of dense pyramidal Lucas-Kanade flow at 1024x1024 on one MI355X.

Workload (one step = one frame pair through the whole method): synthetic 1024x1024 uint8
particle images (0.03 particles/px, sigma 1.2 px, shear layer 4 + 4 tanh((y - 512)/40) px plus
a reverse Lamb-Oseen vortex), 4 pyramid levels, window radius 8, 4 iterations per level,
FP32 storage, one of_compute call per pair on one stream.  Inputs rotate over 16 distinct
pairs already resident in HBM.  Also reported: the FP16-storage form of the same workload,
per-pair latency percentiles, the live per-kernel event timing of the fused iteration kernel
against MI355X HBM peak, and the FP64 CPU oracle timed on this host on a bounded sample.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frame pairs/s at 1024² (FP32 vs FP16-stored, % HBM peak); p50/p99 latency"
HBM_PEAK_GBS = 8000.0
WORKLOAD = "c2"


# Launch configuration the plan autotuner settles on for this workload (FP32 and FP16): used by
# the --probe run, which profilers wrap, so that it needs no autotuning launches.
PROBE_CONFIG = {"bands": [4, 1, 1, 1], "variant": [3, 1, 6, 6]}
# One of the configurations the batch autotuner picks for 16 pairs of this workload.
PROBE_BATCH_CONFIG = {"bands": [8, 8, 4, 1], "grid": [512, 0, 512, 512], "variant": [0, 0, 1, 1]}
# Sources of the fused iteration kernel: the HBM traffic recorded in the counter summary is
# used only while they are unchanged.
KERNEL_SOURCES = ["paper_1306_2461_amd/csrc/lk_iter_impl.h", "paper_1306_2461_amd/csrc/common.h",
                  "paper_1306_2461_amd/csrc/lk_iter.hip", "paper_1306_2461_amd/csrc/kernels.h"]
COUNTER_SUMMARY = "profiles/lk_iter_1024_plain_path_counters.md"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    """SHA-256 of the iteration kernel's sources with // comments and blank lines removed (a
    comment edit does not change the kernel the counters measured)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per iteration launch from the committed counter summary (rocprofv3 FETCH_SIZE
    and WRITE_SIZE runs, copy-calibrated), or None when the kernel sources changed since."""
    import re
    try:
        text = open(os.path.join(ROOT, COUNTER_SUMMARY)).read()
    except OSError:
        return None
    m_hash = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    m_val = re.search(r"traffic_bytes_per_launch:\s*([0-9.]+)", text)
    if not m_hash or not m_val or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_val.group(1))


def probe(args):
    """Fixed short run for counter collection: a 256 MiB device copy (calibration of the
    FETCH_SIZE / WRITE_SIZE counters), then 5 plain FP32 pairs (graphs off, so every launch is
    a kernel dispatch of its own) at PROBE_CONFIG, then one 16-pair batch at
    PROBE_BATCH_CONFIG; no timing, no JSON line."""
    import synth
    import torch
    import paper_1306_2461_amd as ofmi
    dev = torch.device("cuda", 0)
    # calibration: a plain copy of 256 MiB (reads and writes 2^28 bytes each)
    src = torch.ones(1 << 26, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    pairs = [synth.make_pair(WORKLOAD, i)[:2] for i in range(4)]
    d1 = [torch.from_numpy(p[0]).to(dev) for p in pairs]
    d2 = [torch.from_numpy(p[1]).to(dev) for p in pairs]
    wl = synth.workload(WORKLOAD)
    plan = ofmi.Plan(wl.H, wl.W, wl.levels, wl.radius, wl.iters, device=dev, graph=False)
    plan.set_config(PROBE_CONFIG)
    u, v = plan.compute(d1[0], d2[0])
    for i in range(4):
        plan.compute(d1[i], d2[i], u, v)
    torch.cuda.synchronize()
    log(f"probe: plain path done, kernel sources {kernel_source_hash()}")
    plan.close()
    b = ofmi.Batch([(wl.H, wl.W)] * 16, wl.levels, wl.radius, wl.iters, device=dev, graph=False)
    b.set_config(PROBE_BATCH_CONFIG)
    bu, bv = b.outputs()
    b.compute([d1[i % 4] for i in range(16)], [d2[i % 4] for i in range(16)], bu, bv)
    torch.cuda.synchronize()
    log("probe: 16-pair batch done")
    b.close()


def _gen(i):
    import synth
    I1, I2, _, _ = synth.make_pair(WORKLOAD, i)
    return I1, I2


def _oracle_pair(args):
    os.environ["OMP_NUM_THREADS"] = "1"
    import oracle
    I1, I2, L, r, K = args
    t = time.perf_counter()
    oracle.flow(I1, I2, L, r, K)
    return time.perf_counter() - t


def cpu_baseline(pairs, L, r, K, n_pairs, workers):
    """The FP64 oracle on `n_pairs` pairs over a pool of `workers` processes (no GPU touched)."""
    jobs = [(pairs[i % len(pairs)][0], pairs[i % len(pairs)][1], L, r, K) for i in range(n_pairs)]
    t = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        per = list(ex.map(_oracle_pair, jobs))
    wall = time.perf_counter() - t
    return {"value": n_pairs / wall, "unit": "frame pairs/s", "cores": workers, "kind": "oracle",
            "sample": f"{n_pairs} distinct 1024x1024 pairs of the bench workload, FP64 numpy oracle, "
                      f"one pair per worker process ({workers} processes, 1 thread each); "
                      f"mean single-pair time {sum(per) / len(per):.2f} s",
            "cpu_seconds": round(sum(per), 2)}


def _ptrs(d1, d2, us, vs):
    return [(a.data_ptr(), b.data_ptr(), u.data_ptr(), v.data_ptr()) for a, b, u, v in zip(d1, d2, us, vs)]


def time_plan(torch, plan, d1, d2, us, vs, steps, warmup):
    """Enqueue `steps` pairs back to back on the current stream (pointers resident in HBM)."""
    ptrs = _ptrs(d1, d2, us, vs)
    n = len(ptrs)
    st = torch.cuda.current_stream().cuda_stream
    for i in range(warmup):
        plan.compute_raw(*ptrs[i % n], st)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(steps):
        plan.compute_raw(*ptrs[i % n], st)
    torch.cuda.synchronize()
    return time.perf_counter() - t


def latency(torch, plan, d1, d2, us, vs, n_calls):
    """Host-observed per-pair latency: enqueue one pair, wait for it, repeat."""
    ptrs = _ptrs(d1, d2, us, vs)
    n = len(ptrs)
    stream = torch.cuda.current_stream()
    st = stream.cuda_stream
    out = []
    for i in range(n_calls):
        t = time.perf_counter()
        plan.compute_raw(*ptrs[i % n], st)
        stream.synchronize()
        out.append((time.perf_counter() - t) * 1e3)
    out.sort()
    return {"p50_ms": round(out[len(out) // 2], 4), "p99_ms": round(out[min(len(out) - 1, int(0.99 * len(out)))], 4)}


def _gen_c4(i_and_size):
    import synth
    i, size = i_and_size
    H, W, I1, I2, _, _ = next(synth.batch_items(1, sizes=[size]))
    return I1, I2


def _gen_stream(args):
    import synth
    sid, n, size = args
    return [f for f, _, _ in synth.stream_frames(sid, n, size=size)]


def bench_batched(torch, ofmi, dev, pairs, wl, fp16, reps, tag):
    """The 1024x1024 workload as one batch of all resident pairs per graph replay."""
    n = len(pairs)
    b = ofmi.Batch([(wl.H, wl.W)] * n, wl.levels, wl.radius, wl.iters, fp16=fp16, device=dev)
    d1 = [torch.from_numpy(p[0]).to(dev) for p in pairs]
    d2 = [torch.from_numpy(p[1]).to(dev) for p in pairs]
    us, vs = b.outputs()
    cfg = b.autotune(d1, d2, us, vs, reps=2)
    arrs = b.pointer_arrays(d1, d2, us, vs)
    st = torch.cuda.current_stream().cuda_stream
    for _ in range(3):
        b.compute_raw(arrs, st)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        b.compute_raw(arrs, st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    b.set_timing(True)
    b.compute(d1, d2, us, vs)
    torch.cuda.synchronize()
    it = b.read_timing(ofmi.OF_KERNEL_ITERATE)
    b.read_timing(ofmi.OF_KERNEL_REDUCE)
    b.set_timing(False)
    b.close()
    ach = it[3] / it[0] / 1e6 if it[0] > 0 else 0.0
    log(f"batched {tag}: {n * reps / el:.1f} pairs/s ({el / reps * 1e3:.3f} ms per batch of {n}), "
        f"iterate {ach:.0f} GB/s, config {cfg}")
    return {"value": round(n * reps / el, 3), "unit": "frame pairs/s", "pairs_per_batch": n,
            "ms_per_batch": round(el / reps * 1e3, 4), "config": cfg,
            "iterate_achieved_GBs": round(ach, 1), "iterate_frac_hbm": round(ach / HBM_PEAK_GBS, 4),
            "iterate_avg_launch_us": round(it[0] / max(it[1], 1) * 1e3, 3)}


def bench_c4(torch, ofmi, dev, workers, reps):
    """64 mixed-size pairs (16x 512^2, 32x 1024x768, 16x 2048^2), FP16 storage, one replay per batch."""
    import synth
    wl = synth.workload("c4")
    sizes = synth.particles.batch_sizes(64)
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        pairs = list(ex.map(_gen_c4, list(enumerate(sizes))))
    b = ofmi.Batch(sizes, wl.levels, wl.radius, wl.iters, fp16=True, device=dev)
    d1 = [torch.from_numpy(p[0]).to(dev) for p in pairs]
    d2 = [torch.from_numpy(p[1]).to(dev) for p in pairs]
    us, vs = b.outputs()
    cfg = b.autotune(d1, d2, us, vs, reps=1)
    arrs = b.pointer_arrays(d1, d2, us, vs)
    st = torch.cuda.current_stream().cuda_stream
    b.compute_raw(arrs, st)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        b.compute_raw(arrs, st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    b.set_timing(True)
    b.compute(d1, d2, us, vs)
    torch.cuda.synchronize()
    it = b.read_timing(ofmi.OF_KERNEL_ITERATE)
    rd = b.read_timing(ofmi.OF_KERNEL_REDUCE)
    b.set_timing(False)
    b.close()
    alg = it[3] + rd[3]
    ach = it[3] / it[0] / 1e6 if it[0] > 0 else 0.0
    log(f"c4: {64 * reps / el:.1f} pairs/s, {el / reps * 1e3:.2f} ms per batch, iterate {ach:.0f} GB/s")
    return {"value": round(64 * reps / el, 3), "unit": "frame pairs/s", "ms_per_batch": round(el / reps * 1e3, 3),
            "algorithmic_GB_per_batch": round(alg / 1e9, 3),
            "effective_frac_hbm": round(alg / (el / reps) / 1e9 / HBM_PEAK_GBS, 4),
            "iterate_achieved_GBs": round(ach, 1), "iterate_frac_hbm": round(ach / HBM_PEAK_GBS, 4),
            "config": cfg}


def bench_masked(torch, ofmi, dev, d1, d2, us, vs, wl, steps, warmup, unmasked_value):
    """Plain FP32 path with a region-of-interest mask: a step-like obstacle over the lower-left
    quarter and 64-row side walls top and bottom (the masking lever of Sec. 3.3)."""
    import numpy as np
    M = np.ones((wl.H, wl.W), dtype=np.uint8)
    M[wl.H // 2:, :wl.W // 2] = 0
    M[:64, :] = 0
    M[-64:, :] = 0
    plan = ofmi.Plan(wl.H, wl.W, wl.levels, wl.radius, wl.iters, device=dev)
    plan.set_mask(torch.from_numpy(M).to(dev))
    tuned = plan.autotune(d1[0], d2[0], us[0], vs[0], reps=3)
    el = time_plan(torch, plan, d1, d2, us, vs, steps, warmup)
    plan.close()
    value = steps / el
    log(f"masked: {value:.1f} pairs/s with {M.mean():.3f} of the frame unmasked, config {tuned}")
    return {"value": round(value, 3), "unit": "frame pairs/s", "unmasked_fraction": round(float(M.mean()), 4),
            "speedup_vs_unmasked": round(value / unmasked_value, 3), "config": tuned,
            "mask": "lower-left quarter (step) and 64-row walls top and bottom excluded"}


def bench_gaussian(torch, ofmi, dev, d1, d2, us, vs, wl, steps, warmup, box_value):
    """Plain FP32 path with the Gaussian-weighted window (OF_FLAG_GAUSSIAN_WINDOW)."""
    plan = ofmi.Plan(wl.H, wl.W, wl.levels, wl.radius, wl.iters, gaussian_window=True, device=dev)
    tuned = plan.autotune(d1[0], d2[0], us[0], vs[0], reps=3)
    el = time_plan(torch, plan, d1, d2, us, vs, steps, warmup)
    plan.close()
    value = steps / el
    log(f"gaussian window: {value:.1f} pairs/s, config {tuned}")
    return {"value": round(value, 3), "unit": "frame pairs/s", "vs_box_window": round(value / box_value, 3),
            "config": tuned}


def bench_serving(torch, ofmi, dev, workers, frames_per_stream):
    """8 streams (sizes from {640x480, 1024^2, 2048^2}), Poisson arrivals at 250 frames/s each."""
    import synth
    from paper_1306_2461_amd.serve import GpuExecutor, Server, poisson_arrivals
    wl = synth.workload("c5")
    sizes = synth.particles.stream_sizes(8)
    with cf.ProcessPoolExecutor(max_workers=min(8, workers)) as ex:
        streams = list(ex.map(_gen_stream, [(s, frames_per_stream, sizes[s]) for s in range(8)]))
    arrivals = poisson_arrivals(streams, 250.0)
    exe = GpuExecutor(wl.levels, wl.radius, wl.iters, fp16=True, budget_bytes=8 << 30, device=dev)
    warm = Server(exe)                       # opens sessions, builds first pyramids, warms up
    for sid in range(8):
        for f in streams[sid][:2]:
            warm.submit(sid, f)
    warm.drain()
    for sid in range(8):
        warm.close_stream(sid)
    srv = Server(exe)
    st = srv.replay(arrivals, realtime=True)
    exe.close_all()
    st = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}
    st.update({"streams": [f"{w}x{h}" for h, w in sizes], "frames_per_stream": frames_per_stream,
               "offered_frames_per_s": 2000})
    log(f"serving: {st}")
    return st


def kernel_timing(torch, ofmi, plan, d1, d2, us, vs, steps):
    """Average duration of each kernel from hipEvents recorded around its launches."""
    n = len(d1)
    plan.set_timing(True)
    for i in range(steps):
        plan.compute(d1[i % n], d2[i % n], us[i % n], vs[i % n])
    torch.cuda.synchronize()
    it = plan.read_timing(ofmi.OF_KERNEL_ITERATE)
    rd = plan.read_timing(ofmi.OF_KERNEL_REDUCE)
    plan.set_timing(False)
    return it, rd


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--pairs", type=int, default=16, help="distinct resident pairs rotated over")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--cpu-pairs", type=int, default=8)
    ap.add_argument("--no-extra", action="store_true", help="skip the batched, mixed-batch and serving runs")
    ap.add_argument("--serve-frames", type=int, default=24)
    ap.add_argument("--c4-only", action="store_true",
                    help="only the 64-pair mixed batch (for profilers): autotune, 3 timed replays, no JSON line")
    ap.add_argument("--probe", action="store_true",
                    help="short fixed run for profilers (4 plain pairs), no timing, no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); pairs are "
              "independent, so a multi-GPU run would deal pairs to GPUs with no exchange", file=sys.stderr)
        sys.exit(2)

    if args.probe:
        probe(args)
        return
    if args.c4_only:
        import torch
        import paper_1306_2461_amd as ofmi
        ofmi.load()
        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        bench_c4(torch, ofmi, dev, max(1, min(16, len(os.sched_getaffinity(0)))), 3)
        return

    import numpy as np
    import synth
    wl = synth.workload(WORKLOAD)
    L, r, K = wl.levels, wl.radius, wl.iters
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    t = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=min(workers, args.pairs)) as ex:
        pairs = list(ex.map(_gen, range(args.pairs)))
    log(f"generated {len(pairs)} pairs in {time.perf_counter() - t:.1f} s")

    cpu = None
    if not args.no_cpu_baseline:
        n_cpu = min(args.cpu_pairs, workers)
        cpu = cpu_baseline(pairs, L, r, K, args.cpu_pairs, n_cpu)
        log(f"cpu baseline: {cpu['value']:.3f} pairs/s on {cpu['cores']} processes")

    import torch
    import paper_1306_2461_amd as ofmi
    ofmi.load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    d1 = [torch.from_numpy(p[0]).to(dev) for p in pairs]
    d2 = [torch.from_numpy(p[1]).to(dev) for p in pairs]
    us = [torch.empty((wl.H, wl.W), dtype=torch.float32, device=dev) for _ in pairs]
    vs = [torch.empty((wl.H, wl.W), dtype=torch.float32, device=dev) for _ in pairs]
    torch.cuda.synchronize()

    results = {}
    for tag, fp16 in (("fp32", False), ("fp16", True)):
        plan = ofmi.Plan(wl.H, wl.W, L, r, K, fp16=fp16, device=dev)
        tuned = plan.autotune(d1[0], d2[0], us[0], vs[0], reps=3)
        log(f"{tag}: autotuned launch configuration {tuned}")
        el = time_plan(torch, plan, d1, d2, us, vs, args.steps, args.warmup)
        lat = latency(torch, plan, d1, d2, us, vs, min(200, args.steps))
        it, rd = kernel_timing(torch, ofmi, plan, d1, d2, us, vs, min(100, args.steps))
        err = None
        if not args.no_parity:
            import oracle
            plan.compute(d1[0], d2[0], us[0], vs[0])
            torch.cuda.synchronize()
            ou, ov = oracle.flow(pairs[0][0], pairs[0][1], L, r, K)
            err = float(max(np.abs(us[0].cpu().numpy() - ou).max(), np.abs(vs[0].cpu().numpy() - ov).max()))
        graphed = None
        if tag == "fp32":
            pg = ofmi.Plan(wl.H, wl.W, L, r, K, fp16=fp16, device=dev, graph=True)
            pg.set_config(tuned)
            graphed = args.steps / time_plan(torch, pg, d1, d2, us, vs, args.steps, args.warmup)
            pg.close()
        results[tag] = {"el": el, "lat": lat, "it": it, "rd": rd, "err": err, "graphed": graphed,
                        "cfg": tuned}
        plan.close()
        log(f"{tag}: {args.steps / el:.1f} pairs/s, {el / args.steps * 1e3:.4f} ms/pair, "
            f"latency {lat}, iterate kernel avg {it[0] / max(it[1], 1) * 1e3:.2f} us over {it[1]} launches, "
            f"max |err| {err}")

    extra = {}
    if not args.no_extra:
        for name, fn in (("batched_1024_fp32", lambda: bench_batched(torch, ofmi, dev, pairs, wl, False, 20, "fp32")),
                         ("batched_1024_fp16", lambda: bench_batched(torch, ofmi, dev, pairs, wl, True, 20, "fp16")),
                         ("mixed_batch_64", lambda: bench_c4(torch, ofmi, dev, workers, 5)),
                         ("gaussian_window_1024_fp32", lambda: bench_gaussian(torch, ofmi, dev, d1, d2, us, vs, wl,
                                                                             args.steps, args.warmup,
                                                                             args.steps / results["fp32"]["el"])),
                         ("masked_1024_fp32", lambda: bench_masked(torch, ofmi, dev, d1, d2, us, vs, wl,
                                                                   args.steps, args.warmup,
                                                                   args.steps / results["fp32"]["el"])),
                         ("serving_8_streams", lambda: bench_serving(torch, ofmi, dev, workers, args.serve_frames))):
            try:
                extra[name] = fn()
            except Exception as e:  # report, keep the main line
                extra[name] = {"error": repr(e)}
                log(f"{name} failed: {e!r}")

    r32 = results["fp32"]
    ms_it, n_it, units_it, bytes_it = r32["it"]
    achieved = bytes_it / ms_it / 1e6 if ms_it > 0 else 0.0
    line = {
        "metric": METRIC,
        "value": round(args.steps / r32["el"], 3),
        "unit": "frame pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["el"] / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1024x1024 uint8 particle-image pair, 4 levels, radius 8, 4 iterations/level, "
                               "FP32 plain per-pair path (one of_compute per pair, one stream)",
                   "H": wl.H, "W": wl.W, "levels": L, "radius": r, "iters": K,
                   "distinct_pairs": args.pairs, "launch_config": r32["cfg"]},
        "latency_ms": r32["lat"],
        "graph_replay_value": round(r32["graphed"], 3),
        "max_abs_err_px": r32["err"],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "kernel": "lk_iter (fused iteration)", "launches": n_it,
                     "avg_launch_us": round(ms_it / max(n_it, 1) * 1e3, 3),
                     "bytes_per_launch": round(bytes_it / max(n_it, 1))},
        "fp16": {"value": round(args.steps / results["fp16"]["el"], 3),
                 "ms_per_step": round(results["fp16"]["el"] / args.steps * 1e3, 5),
                 "latency_ms": results["fp16"]["lat"], "max_abs_err_px": results["fp16"]["err"],
                 "iterate_avg_launch_us": round(results["fp16"]["it"][0] / max(results["fp16"]["it"][1], 1) * 1e3, 3)},
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
