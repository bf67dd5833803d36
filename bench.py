#!/usr/bin/env python3
"""Frame pairs/s of dense pyramidal Lucas-Kanade flow at 1024x1024 on one MI355X.

Workload (one step = one frame pair through the whole method): synthetic 1024x1024 uint8
particle images (0.03 particles/px, sigma 1.2 px, shear layer 4 + 4 tanh((y - 512)/40) px plus
a reverse Lamb-Oseen vortex), 4 pyramid levels, window radius 8, 4 iterations per level,
FP32 storage, one of_compute call per pair on one stream.  Inputs rotate over 16 distinct
pairs already resident in HBM.  Also reported, in the same JSON line: the FP16-storage form,
the 256x256 workload (3 levels, r = 4), per-pair latency percentiles, the fused iteration
kernel per level against MI355X HBM peak (hipEvent spans on the launch stream), parity with
the FP64 oracle and accuracy against the generator's ground truth, the batched and mixed-size
forms, the Gaussian window and masks, the served streams, and the FP64 CPU oracle timed on
this host's cores.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import gc
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frame pairs/s at 1024² (FP32 vs FP16-stored, % HBM peak); p50/p99 latency"
HBM_PEAK_GBS = 8000.0
WORKLOAD = "c2"

# Launch configurations the plan autotuner settles on for this workload (level 0: wide strips of
# 4 bands, 64 or 32 columns): used by the --probe run, which profilers wrap, so that it needs
# no autotuning launches.
PROBE_CONFIGS = [{"bands": [4, 1, 1, 1], "variant": [1, 1, 6, 6]},
                 {"bands": [4, 1, 1, 1], "variant": [3, 1, 6, 6]}]
# The configuration the batch autotuner picked for 16 masked pairs of this workload (masked probe).
MASK_PROBE_CONFIG = {"bands": [8, 4, 2, 1], "grid": [0, 2048, 2048, 2048], "variant": [2, 2, 2, 1]}
# One of the configurations the batch autotuner picks for 16 pairs of this workload.
PROBE_BATCH_CONFIG = {"bands": [16, 8, 2, 1], "grid": [2048, 512, 1024, 512], "variant": [2, 2, 2, 1]}
# Sources of the fused iteration kernel: the HBM traffic recorded in the counter summary is
# used only while they are unchanged.
KERNEL_SOURCES = ["paper_1306_2461_amd/csrc/lk_iter_impl.h", "paper_1306_2461_amd/csrc/common.h",
                  "paper_1306_2461_amd/csrc/lk_iter.hip", "paper_1306_2461_amd/csrc/kernels.h"]
COUNTER_SUMMARY = "profiles/lk_iter_1024_plain_path_counters.md"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# --------------------------------------------------------------------------- host helpers

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


def measured_traffic(variant):
    """HBM bytes per level-0 iteration launch of tile variant `variant` from the committed
    counter summary (rocprofv3 FETCH_SIZE and WRITE_SIZE runs, copy-calibrated), or None when
    the kernel sources changed since the counters were taken or that variant was not
    profiled."""
    import re
    try:
        text = open(os.path.join(ROOT, COUNTER_SUMMARY)).read()
    except OSError:
        return None
    m_hash = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    m_val = re.search(rf"level0_traffic_bytes_per_launch\[variant {variant}\]:\s*([0-9.]+)", text)
    if not m_hash or not m_val or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_val.group(1))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _noop(x):
    return x


def pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(q * len(xs)))]


def err_stats(u, v, ou, ov):
    """max-abs and RMS (over both components) of a flow against a reference, in px."""
    import numpy as np
    du = u.astype(np.float64) - ou
    dv = v.astype(np.float64) - ov
    return {"max_abs_px": float(max(np.abs(du).max(), np.abs(dv).max())),
            "rms_px": float(np.sqrt(0.5 * ((du ** 2).mean() + (dv ** 2).mean())))}


def truth_stats(u, v, gu, gv, margin):
    """Method accuracy against the generator's ground-truth field on the interior (pixels at
    least `margin` px from every border): RMS and max of the end-point error."""
    import numpy as np
    sl = (slice(margin, -margin), slice(margin, -margin))
    e = np.hypot(u[sl].astype(np.float64) - gu[sl], v[sl].astype(np.float64) - gv[sl])
    return {"rms_px": float(np.sqrt((e ** 2).mean())), "max_px": float(e.max()), "interior_margin_px": margin}


def floor_max(case):
    """Largest committed FP32 rounding floor of a parity case (tests/golden/floor), or None."""
    import numpy as np
    try:
        with np.load(os.path.join(ROOT, "tests", "golden", "floor", f"{case}.npz"), allow_pickle=False) as z:
            return float(z["max"])
    except OSError:
        return None


# --------------------------------------------------------------------------- CPU workers
# (forked before the GPU is touched; they run numpy only)

def _gen(args):
    import synth
    name, i = args
    I1, I2, gu, gv = synth.make_pair(name, i)
    return I1, I2, gu.astype("float32"), gv.astype("float32")


def _gen_c4(i_and_size):
    from synth import particles as P
    i, (H, W) = i_and_size
    wl = P.WORKLOADS["c4"]
    rngs = P._rngs(wl.index, i)
    field = P._vortex_field(rngs[4], H, W)
    I1, I2, gu, gv, _ = P._pair_from_field(field, H, W, wl.rho, wl.sigma, rngs, wl.levels)
    return I1, I2, gu.astype("float32"), gv.astype("float32")


def _oracle_job(args):
    """The FP64 oracle on one pair, one thread; returns (flow as float32, seconds)."""
    import numpy as np
    import oracle
    I1, I2, L, r, K = args
    t = time.perf_counter()
    u, v = oracle.flow(I1, I2, L, r, K)
    return u.astype(np.float32), v.astype(np.float32), time.perf_counter() - t


def _floor_job(args):
    """One float32 realisation of the oracle's operation order (tests/floor_util.py) of a pair:
    its per-pixel departure from the FP64 flow is a sample of the rounding floor."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import floor_util
    import oracle
    I1, I2, L, r, K, k, storage, ou, ov = args
    f1, f2, tr = floor_util.realisations(I1, I2)[k]
    uk, vk = oracle.flow(f1, f2, L, r, K, dtype=np.float32, coords="split", storage=storage)
    if tr:
        uk, vk = vk.T, uk.T
    return np.maximum(np.abs(uk - ou), np.abs(vk - ov)).astype(np.float32)


def floor_stats(pool, pairs, flows, gpu, L, r, K, tol, storage):
    """Per-pixel parity of GPU flows against the oracle with the FP32 rounding floor of each
    pair (five float32 realisations, window-dilated, as the GPU tests use): pixels over the
    tolerance, and whether each is within tol + 3 x floor."""
    import numpy as np
    from scipy import ndimage
    jobs = [(p[0], p[1], L, r, K, k, storage, f[0].astype(np.float64), f[1].astype(np.float64))
            for p, f in zip(pairs, flows) for k in range(5)]
    deps = list(pool.map(_floor_job, jobs))
    over = bound = 0
    worst = 0.0
    for i, ((u, v), f) in enumerate(zip(gpu, flows)):
        fl = np.max(deps[5 * i:5 * i + 5], axis=0)
        fl = ndimage.maximum_filter(fl, size=2 * r + 1, mode="nearest").astype(np.float64)
        d = np.maximum(np.abs(u - f[0].astype(np.float64)), np.abs(v - f[1].astype(np.float64)))
        o = d > tol
        over += int(o.sum())
        bound += int((d > tol + 3.0 * fl).sum())
        if o.any():
            worst = max(worst, float(np.max((d[o] - tol) / np.maximum(fl[o], 1e-30))))
    return {"px_over_tolerance": over, "px_beyond_tol_plus_3x_floor": bound,
            "max_excess_over_floor": round(worst, 3)}


def cpu_pool(pool, workers, pairs, L, r, K):
    """The oracle over `pairs` [(I1, I2), ...] on the pool, longest first; returns the flows in
    input order, the wall time and the per-pair CPU times."""
    order = sorted(range(len(pairs)), key=lambda i: -pairs[i][0].size)
    t = time.perf_counter()
    res = list(pool.map(_oracle_job, [(pairs[i][0], pairs[i][1], L, r, K) for i in order]))
    wall = time.perf_counter() - t
    out = [None] * len(pairs)
    for i, rr in zip(order, res):
        out[i] = rr
    return out, wall


# --------------------------------------------------------------------------- GPU timing

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
    return {"p50_ms": round(pct(out, 0.5), 4), "p99_ms": round(pct(out, 0.99), 4)}


def level_timing(torch, ofmi, obj, run, levels, n_runs):
    """Per-level span timing (OF_TIMING_LEVEL): one hipEvent pair around each level's K
    iteration launches and one around the pyramid launches, on the launch stream, with the
    host enqueueing ahead of the GPU.  Returns [(level, ms, launches, units, bytes)] and the
    pyramid record."""
    obj.set_timing(ofmi.OF_TIMING_LEVEL)
    for i in range(n_runs):
        run(i)
    torch.cuda.synchronize()
    lv = [(l,) + tuple(obj.read_timing(ofmi.OF_KERNEL_LEVEL(l))) for l in range(levels)]
    rd = obj.read_timing(ofmi.OF_KERNEL_REDUCE)
    obj.read_timing(ofmi.OF_KERNEL_ITERATE)
    obj.set_timing(False)
    return lv, rd


def roofline_from_levels(lv, sizes, frame_bytes):
    """Per-level table and the dominant level (largest share of the iteration time)."""
    total = sum(r[1] for r in lv)
    per = []
    for (l, ms, n, units, by), (H, W) in zip(lv, sizes):
        avg_us = ms / max(n, 1) * 1e3
        gbs = by / ms / 1e6 if ms > 0 else 0.0
        per.append({"level": l, "H": H, "W": W, "frame_bytes_per_px": frame_bytes[l],
                    "launches": n, "avg_launch_us": round(avg_us, 3),
                    "bytes_per_launch": round(by / max(n, 1)), "achieved_GBs": round(gbs, 1),
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "time_share": round(ms / total, 4) if total else 0})
    dom = max(per, key=lambda p: p["time_share"])
    return per, dom


# --------------------------------------------------------------------------- forms

def bench_plain(torch, ofmi, dev, wl, d1, d2, us, vs, fp16, steps, warmup, tag):
    plan = ofmi.Plan(wl.H, wl.W, wl.levels, wl.radius, wl.iters, fp16=fp16, device=dev)
    tuned = plan.autotune(d1[0], d2[0], us[0], vs[0], reps=3)
    el = time_plan(torch, plan, d1, d2, us, vs, steps, warmup)
    lat = latency(torch, plan, d1, d2, us, vs, min(200, max(steps, 50)))
    n = len(d1)
    lv, rd = level_timing(torch, ofmi, plan, lambda i: plan.compute(d1[i % n], d2[i % n], us[i % n], vs[i % n]),
                          wl.levels, max(50, min(steps, 200)))
    sizes = [(wl.H, wl.W)]
    for _ in range(wl.levels - 1):
        sizes.append(((sizes[-1][0] + 1) // 2, (sizes[-1][1] + 1) // 2))
    fb = [1] + [2 if fp16 else 4] * (wl.levels - 1)
    per, dom = roofline_from_levels(lv, sizes, fb)
    log(f"{tag}: {steps / el:.1f} pairs/s, {el / steps * 1e3:.4f} ms/pair, latency {lat}, config {tuned}, "
        f"levels " + ", ".join(f"L{p['level']} {p['avg_launch_us']} us {p['frac']:.3f}" for p in per))
    return plan, {"el": el, "lat": lat, "cfg": tuned, "per_level": per, "dominant": dom,
                  "pyramid": {"launches": rd[1], "avg_launch_us": round(rd[0] / max(rd[1], 1) * 1e3, 3),
                              "achieved_GBs": round(rd[3] / rd[0] / 1e6, 1) if rd[0] > 0 else 0.0}}


def bench_c1(torch, ofmi, dev, pairs, oracle_flow, steps, warmup):
    """The 256x256 workload (3 levels, r = 4, 4 iterations, FP32 plain path)."""
    import synth
    wl = synth.workload("c1")
    d1 = [torch.from_numpy(p[0]).to(dev) for p in pairs]
    d2 = [torch.from_numpy(p[1]).to(dev) for p in pairs]
    us = [torch.empty((wl.H, wl.W), dtype=torch.float32, device=dev) for _ in pairs]
    vs = [torch.empty((wl.H, wl.W), dtype=torch.float32, device=dev) for _ in pairs]
    plan = ofmi.Plan(wl.H, wl.W, wl.levels, wl.radius, wl.iters, device=dev)
    tuned = plan.autotune(d1[0], d2[0], us[0], vs[0], reps=3)
    el = time_plan(torch, plan, d1, d2, us, vs, steps, warmup)
    lat = latency(torch, plan, d1, d2, us, vs, min(200, max(steps, 50)))
    plan.compute(d1[0], d2[0], us[0], vs[0])
    torch.cuda.synchronize()
    u, v = us[0].cpu().numpy(), vs[0].cpu().numpy()
    plan.close()
    ou, ov, osec = oracle_flow
    out = {"value": round(steps / el, 3), "unit": "frame pairs/s", "ms_per_step": round(el / steps * 1e3, 5),
           "latency_ms": lat, "config": {"workload": "256x256 uint8 particle pair, 3 levels, radius 4, 4 iterations, "
                                                     "FP32 plain per-pair path", "launch_config": tuned},
           "parity": dict(err_stats(u, v, ou, ov), tolerance_px=1e-3, fp32_floor_max_px=floor_max("c1")),
           "accuracy_vs_truth": truth_stats(u, v, pairs[0][2], pairs[0][3], wl.radius + 4 + 2),
           "cpu_oracle_single_pair_s": round(osec, 4)}
    log(f"c1: {out['value']:.1f} pairs/s, latency {lat}, parity {out['parity']}")
    return out


def bench_batched(torch, ofmi, dev, d1, d2, wl, fp16, reps, tag):
    """The 1024x1024 workload as one batch of all resident pairs per graph replay."""
    n = len(d1)
    b = ofmi.Batch([(wl.H, wl.W)] * n, wl.levels, wl.radius, wl.iters, fp16=fp16, device=dev)
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
    lv, _ = level_timing(torch, ofmi, b, lambda i: b.compute(d1, d2, us, vs), wl.levels, 3)
    b.close()
    l0 = lv[0]
    ach = l0[4] / l0[1] / 1e6 if l0[1] > 0 else 0.0
    log(f"batched {tag}: {n * reps / el:.1f} pairs/s ({el / reps * 1e3:.3f} ms per batch of {n}), "
        f"level 0 {ach:.0f} GB/s, config {cfg}")
    return {"value": round(n * reps / el, 3), "unit": "frame pairs/s", "pairs_per_batch": n,
            "ms_per_batch": round(el / reps * 1e3, 4), "config": cfg,
            "level0_achieved_GBs": round(ach, 1), "level0_frac_hbm": round(ach / HBM_PEAK_GBS, 4),
            "level0_avg_launch_us": round(l0[1] / max(l0[2], 1) * 1e3, 3)}


def bench_c4(torch, ofmi, dev, pool, workers, reps, with_cpu=True):
    """64 mixed-size pairs (16x 512^2, 32x 1024x768, 16x 2048^2), FP16 storage, one replay per
    batch; the plain per-pair path on the same 64 pairs; the oracle over all 64 pairs on the
    host pool (parity of every pair and the CPU baseline)."""
    import numpy as np
    import synth
    wl = synth.workload("c4")
    sizes = synth.particles.batch_sizes(64)
    t = time.perf_counter()
    pairs = list(pool.map(_gen_c4, list(enumerate(sizes))))
    log(f"c4: generated 64 pairs in {time.perf_counter() - t:.1f} s")
    cpu = None
    if with_cpu:
        flows, wall = cpu_pool(pool, workers, [(p[0], p[1]) for p in pairs], wl.levels, wl.radius, wl.iters)
        cpu = {"value": round(64 / wall, 4), "unit": "frame pairs/s", "cores": workers, "kind": "oracle",
               "sample": "all 64 pairs of the mixed batch, FP64 numpy oracle, one pair per worker process at a time, "
                         "longest first", "cpu_seconds": round(sum(f[2] for f in flows), 2), "wall_s": round(wall, 2)}
        log(f"c4: oracle pool {cpu['value']} pairs/s on {workers} processes")
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
    got = [(u.cpu().numpy(), v.cpu().numpy()) for u, v in zip(us, vs)]
    lv, rd = level_timing(torch, ofmi, b, lambda i: b.compute(d1, d2, us, vs), wl.levels, 2)
    b.close()
    alg = sum(r[4] for r in lv) / 2 + rd[3] / 2
    l0 = lv[0]
    ach = l0[4] / l0[1] / 1e6 if l0[1] > 0 else 0.0
    it_ms = sum(r[1] for r in lv)
    it_ach = sum(r[4] for r in lv) / it_ms / 1e6 if it_ms > 0 else 0.0
    # the plain per-pair path on the same 64 pairs (one plan per size, autotuned)
    plans = {}
    for i, s in enumerate(sizes):
        if s not in plans:
            p = ofmi.Plan(s[0], s[1], wl.levels, wl.radius, wl.iters, fp16=True, device=dev)
            p.autotune(d1[i], d2[i], us[i], vs[i], reps=2)
            plans[s] = p
    ptr = _ptrs(d1, d2, us, vs)
    for i, s in enumerate(sizes):
        plans[s].compute_raw(*ptr[i], st)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        for i, s in enumerate(sizes):
            plans[s].compute_raw(*ptr[i], st)
    torch.cuda.synchronize()
    el_plain = time.perf_counter() - t
    for p in plans.values():
        p.close()
    out = {"value": round(64 * reps / el, 3), "unit": "frame pairs/s", "ms_per_batch": round(el / reps * 1e3, 3),
           "plain_path_value": round(64 * reps / el_plain, 3),
           "speedup_vs_plain_path": round(el_plain / el, 3),
           "algorithmic_GB_per_batch": round(alg / 1e9, 3),
           "effective_frac_hbm": round(alg / (el / reps) / 1e9 / HBM_PEAK_GBS, 4),
           "iterate_achieved_GBs": round(it_ach, 1), "iterate_frac_hbm": round(it_ach / HBM_PEAK_GBS, 4),
           "level0_achieved_GBs": round(ach, 1), "level0_frac_hbm": round(ach / HBM_PEAK_GBS, 4),
           "level0_avg_launch_us": round(l0[1] / max(l0[2], 1) * 1e3, 3), "config": cfg}
    # accuracy against ground truth, per pair, interior
    tr = [truth_stats(g[0], g[1], p[2], p[3], wl.radius + 7 + 2) for g, p in zip(got, pairs)]
    out["accuracy_vs_truth"] = {"rms_px_mean": round(float(np.mean([x["rms_px"] for x in tr])), 5),
                                "max_px": round(max(x["max_px"] for x in tr), 4), "interior_margin_px": wl.radius + 9}
    if cpu is not None:
        es = [err_stats(g[0], g[1], f[0].astype(np.float64), f[1].astype(np.float64)) for g, f in zip(got, flows)]
        out["parity"] = {"pairs": 64, "max_abs_px": max(e["max_abs_px"] for e in es),
                         "rms_px_max_over_pairs": max(e["rms_px"] for e in es), "tolerance_px": 2e-2,
                         "reference": "FP64 oracle rounded to float32"}
        out["cpu_baseline"] = cpu
    log(f"c4: {out['value']:.1f} pairs/s (plain path {out['plain_path_value']:.1f}), level 0 {ach:.0f} GB/s, "
        f"parity {out.get('parity')}")
    return out


def step_mask(H, W):
    """Region-of-interest mask of the masked runs: a step-like obstacle over the lower-left
    quarter and 64-row side walls top and bottom excluded (uint8, 1 = computed)."""
    import numpy as np
    M = np.ones((H, W), dtype=np.uint8)
    M[H // 2:, :W // 2] = 0
    M[:64, :] = 0
    M[-64:, :] = 0
    return M


def bench_masked(torch, ofmi, dev, d1, d2, us, vs, wl, steps, warmup, unmasked_value,
                 unmasked_batch_value=None):
    """Plain FP32 path with a region-of-interest mask: a step-like obstacle over the lower-left
    quarter and 64-row side walls top and bottom (the masking lever of Sec. 3.3); then the same
    mask on every pair of the 16-pair batch, where skipped tiles free the device for the rest."""
    M = step_mask(wl.H, wl.W)
    plan = ofmi.Plan(wl.H, wl.W, wl.levels, wl.radius, wl.iters, device=dev)
    plan.set_mask(torch.from_numpy(M).to(dev))
    tuned = plan.autotune(d1[0], d2[0], us[0], vs[0], reps=3)
    el = time_plan(torch, plan, d1, d2, us, vs, steps, warmup)
    plan.close()
    value = steps / el
    log(f"masked: {value:.1f} pairs/s with {M.mean():.3f} of the frame unmasked, config {tuned}")
    out = {"value": round(value, 3), "unit": "frame pairs/s", "unmasked_fraction": round(float(M.mean()), 4),
           "speedup_vs_unmasked": round(value / unmasked_value, 3), "config": tuned,
           "mask": "lower-left quarter (step) and 64-row walls top and bottom excluded"}
    n = len(d1)
    b = ofmi.Batch([(wl.H, wl.W)] * n, wl.levels, wl.radius, wl.iters, device=dev)
    dm = torch.from_numpy(M).to(dev)
    b.set_masks([dm] * n)
    bu, bv = b.outputs()
    bcfg = b.autotune(d1, d2, bu, bv, reps=2)
    arrs = b.pointer_arrays(d1, d2, bu, bv)
    st = torch.cuda.current_stream().cuda_stream
    for _ in range(3):
        b.compute_raw(arrs, st)
    torch.cuda.synchronize()
    reps = 20
    t = time.perf_counter()
    for _ in range(reps):
        b.compute_raw(arrs, st)
    torch.cuda.synchronize()
    bval = n * reps / (time.perf_counter() - t)
    b.close()
    log(f"masked batch of {n}: {bval:.1f} pairs/s, config {bcfg}")
    out["batched"] = {"value": round(bval, 3), "pairs_per_batch": n, "config": bcfg}
    if unmasked_batch_value:
        out["batched"]["speedup_vs_unmasked_batch"] = round(bval / unmasked_batch_value, 3)
    return out


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


def bench_serving(torch, ofmi, dev, pool, workers, frames_per_stream, with_cpu=True, max_inflight=2):
    """8 streams (sizes from {640x480, 1024^2, 2048^2}), Poisson arrivals at 250 frames/s each,
    replayed in real time; one sampled pair per stream checked against the oracle."""
    import numpy as np
    import synth
    from paper_1306_2461_amd.serve import GpuExecutor, Server, poisson_arrivals
    wl = synth.workload("c5")
    sizes = synth.particles.stream_sizes(8)
    t = time.perf_counter()
    streams = [synth.stream_frames_parallel(s, frames_per_stream, sizes[s], pool) for s in range(8)]
    log(f"serving: generated 8 x {frames_per_stream} frames in {time.perf_counter() - t:.1f} s")
    # frames arrive in pinned host memory, as from a camera driver's DMA buffers (one pinned block
    # per stream); the executor copies them to the device on its copy stream
    pinned = []
    for s in range(8):
        blk = torch.empty((frames_per_stream,) + sizes[s], dtype=torch.uint8, pin_memory=True)
        blk.numpy()[...] = np.stack(streams[s])
        pinned.append([blk[t] for t in range(frames_per_stream)])
    arrivals = poisson_arrivals(pinned, 250.0)
    exe = GpuExecutor(wl.levels, wl.radius, wl.iters, fp16=True, budget_bytes=8 << 30, device=dev)
    # warm-up: the first 48 frames of every stream replayed in real time through the same
    # executor (opens sessions, fills its frame and plane pools, runs every launch shape once);
    # results are not kept, so their planes go back to the pools.  Without it the timed run's
    # first pushes and first pool growth land in its tail.
    warm = Server(exe, keep=lambda r: False, max_inflight=max_inflight)
    warm.replay(poisson_arrivals([p[:48] for p in pinned], 250.0, seed=2462), realtime=True)
    for sid in range(8):
        warm.close_stream(sid)
    # sampled pairs: the flow of frames (ts-1, ts) of every stream is kept; every other result
    # is only timed and its output planes go back to the executor's pool
    ts = frames_per_stream // 2
    srv = Server(exe, keep=lambda r: r.frame is pinned[r.stream_id][ts], max_inflight=max_inflight)
    for sid in range(8):                     # sessions open before the first frame arrives
        srv.open_stream(sid, sizes[sid])
    gc.collect()
    st = srv.replay(arrivals, realtime=True)
    sampled = []
    for r in srv.done:
        if r.has_flow and r.u is not None:
            u = r.u.cpu().numpy() if hasattr(r.u, "cpu") else r.u
            v = r.v.cpu().numpy() if hasattr(r.v, "cpu") else r.v
            sampled.append((r.stream_id, ts - 1, u, v))
    sampled.sort(key=lambda x: x[0])
    exe.close_all()
    st = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}
    st.update({"streams": [f"{w}x{h}" for h, w in sizes], "frames_per_stream": frames_per_stream,
               "offered_frames_per_s": 2000})
    if with_cpu and sampled:
        jobs = [(streams[sid][t0], streams[sid][t0 + 1]) for sid, t0, _, _ in sampled]
        flows, wall = cpu_pool(pool, workers, jobs, wl.levels, wl.radius, wl.iters)
        es = [err_stats(u, v, f[0].astype(np.float64), f[1].astype(np.float64))
              for (_, _, u, v), f in zip(sampled, flows)]
        y = {}
        tr = []
        for sid, t0, u, v in sampled:
            H, W = sizes[sid]
            if (H, W) not in y:
                y[(H, W)] = np.mgrid[0:H, 0:W].astype(np.float64)
            gu, gv = synth.stream_field(H, W, t0)(y[(H, W)][1], y[(H, W)][0])
            tr.append(truth_stats(u, v, gu, gv, wl.radius + 8 + 2))
        st["parity"] = {"pairs": len(sampled), "max_abs_px": max(e["max_abs_px"] for e in es),
                        "rms_px_max_over_pairs": max(e["rms_px"] for e in es), "tolerance_px": 2e-2}
        import numpy as np
        st["parity"].update(floor_stats(pool, jobs, flows, [(u, v) for _, _, u, v in sampled], wl.levels,
                                        wl.radius, wl.iters, 2e-2, np.float16))
        st["accuracy_vs_truth"] = {"rms_px_mean": round(float(np.mean([x["rms_px"] for x in tr])), 5),
                                   "max_px": round(max(x["max_px"] for x in tr), 4)}
        st["cpu_baseline"] = {"value": round(len(jobs) / wall, 4), "unit": "frame pairs/s", "cores": workers,
                              "kind": "oracle", "sample": f"{len(jobs)} served pairs, one per stream (frames "
                                                          f"{ts - 1}->{ts}), FP64 numpy oracle",
                              "cpu_seconds": round(sum(f[2] for f in flows), 2)}
    log(f"serving: {st}")
    return st


def bench_table1(torch, dev, pool):
    """Table 1's experiment in shape (Sec. 3.3): the paper's region of interest 1792x384, r = 10,
    n_lev in {1, 3, 4}, n_iter 1..7; fields/s, error against the (4, 7) field and against the
    ground truth (interior), FP32 plain path with default launch configuration."""
    import numpy as np
    from paper_1306_2461_amd.sweep import table1_sweep
    I1, I2, gu, gv = pool.submit(_gen, ("t1", 0)).result()
    res = table1_sweep(torch.from_numpy(I1).to(dev), torch.from_numpy(I2).to(dev), levels=(1, 3, 4),
                       reps=50, truth=(torch.from_numpy(np.ascontiguousarray(gu)).to(dev),
                                       torch.from_numpy(np.ascontiguousarray(gv)).to(dev)))
    out = {"workload": "1792x384 uint8 particle pair (step shear layer + eddy, max 10 px), r = 10, FP32",
           "n_iter": list(range(1, 8))}
    for L, row in res.items():
        out[f"n_lev_{L}"] = {k: [round(x, 4) for x in v] for k, v in row.items()}
    log("table1: " + ", ".join(f"L{L} fields/s {[round(x) for x in r['fields_per_s']]}" for L, r in res.items()))
    return out


def probe(args):
    """Fixed short run for counter collection: a 256 MiB device copy (calibration of the
    FETCH_SIZE / WRITE_SIZE counters), then 5 plain FP32 pairs (eager launches, so every launch
    is a kernel dispatch of its own) at each of PROBE_CONFIGS, then one 16-pair batch at
    PROBE_BATCH_CONFIG; no timing, no JSON line."""
    import synth
    import torch
    import paper_1306_2461_amd as ofmi
    dev = torch.device("cuda", 0)
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
    for cfg in PROBE_CONFIGS:
        plan.set_config(cfg)
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


def masked_probe(args):
    """Fixed run for a kernel trace of masked batches: the 16-pair 1024x1024 batch at
    MASK_PROBE_CONFIG without masks, then with step_mask on every pair; 3 warm-up and 10
    timed graph replays each; no JSON line."""
    import synth
    import torch
    import paper_1306_2461_amd as ofmi
    dev = torch.device("cuda", 0)
    wl = synth.workload(WORKLOAD)
    pairs = [synth.make_pair(WORKLOAD, i)[:2] for i in range(16)]
    d1 = [torch.from_numpy(p[0]).to(dev) for p in pairs]
    d2 = [torch.from_numpy(p[1]).to(dev) for p in pairs]
    dm = torch.from_numpy(step_mask(wl.H, wl.W)).to(dev)
    for masked in (False, True):
        b = ofmi.Batch([(wl.H, wl.W)] * 16, wl.levels, wl.radius, wl.iters, device=dev)
        if masked:
            b.set_masks([dm] * 16)
        b.set_config(MASK_PROBE_CONFIG)
        us, vs = b.outputs()
        arrs = b.pointer_arrays(d1, d2, us, vs)
        st = torch.cuda.current_stream().cuda_stream
        for _ in range(3):
            b.compute_raw(arrs, st)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(10):
            b.compute_raw(arrs, st)
        torch.cuda.synchronize()
        log(f"masked probe: masks={masked}: {160 / (time.perf_counter() - t):.1f} pairs/s")
        b.close()


# --------------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--pairs", type=int, default=16, help="distinct resident pairs rotated over")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the c1, batched, mixed-batch, window, mask "
                                                            "and serving runs")
    ap.add_argument("--main-only", action="store_true",
                    help="only the 1024x1024 FP32 and FP16 plain-path measurements (for profilers)")
    ap.add_argument("--serve-frames", type=int, default=200)
    ap.add_argument("--c4-only", action="store_true",
                    help="only the 64-pair mixed batch (for profilers): autotune, 3 timed replays, no JSON line")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the 8-stream serving run (for profilers): no CPU baseline, no JSON line")
    ap.add_argument("--masked-probe", action="store_true",
                    help="fixed run for profilers: the 16-pair batch without and with masks, no JSON line")
    ap.add_argument("--probe", action="store_true",
                    help="short fixed run for profilers (5 plain pairs, one batch), no timing, no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); pairs are "
              "independent, so a multi-GPU run would deal pairs to GPUs with no exchange", file=sys.stderr)
        sys.exit(2)
    if args.probe:
        probe(args)
        return
    if args.masked_probe:
        masked_probe(args)
        return
    if args.main_only:
        args.no_extra = True
        args.no_cpu_baseline = True
        args.no_parity = True

    import numpy as np
    import synth
    workers = host_workers()
    # Worker processes are forked now, before anything touches the GPU, and reused throughout.
    pool = cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork"))
    list(pool.map(_noop, range(workers)))

    if args.c4_only:
        import torch
        import paper_1306_2461_amd as ofmi
        ofmi.load()
        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        bench_c4(torch, ofmi, dev, pool, workers, 3, with_cpu=False)
        pool.shutdown()
        return
    if args.serve_only:
        import torch
        import paper_1306_2461_amd as ofmi
        ofmi.load()
        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        bench_serving(torch, ofmi, dev, pool, workers, args.serve_frames, with_cpu=False)
        pool.shutdown()
        return

    wl = synth.workload(WORKLOAD)
    L, r, K = wl.levels, wl.radius, wl.iters
    t = time.perf_counter()
    pairs = list(pool.map(_gen, [(WORKLOAD, i) for i in range(args.pairs)]))
    c1_pairs = [] if args.no_extra else list(pool.map(_gen, [("c1", i) for i in range(16)]))
    log(f"generated {len(pairs)} + {len(c1_pairs)} pairs in {time.perf_counter() - t:.1f} s")

    # CPU baseline (the oracle on this host's cores) and the oracle flows for parity
    cpu = None
    oracle_c2 = None
    oracle_c1 = None
    if not args.no_cpu_baseline or not args.no_parity:
        n_cpu = workers if not args.no_cpu_baseline else 1
        flows, wall = cpu_pool(pool, workers, [(p[0], p[1]) for p in pairs[:n_cpu]], L, r, K)
        oracle_c2 = flows[0]
        if not args.no_cpu_baseline:
            cpu = {"value": round(n_cpu / wall, 4), "unit": "frame pairs/s", "cores": workers, "kind": "oracle",
                   "sample": f"{n_cpu} distinct 1024x1024 pairs of the bench workload, FP64 numpy oracle, one pair "
                             f"per worker process ({workers} processes, 1 thread each)",
                   "single_pair_s": round(float(np.mean([f[2] for f in flows])), 3),
                   "cpu_seconds": round(sum(f[2] for f in flows), 2), "cpu_model": cpu_model()}
            log(f"cpu baseline: {cpu['value']:.3f} pairs/s on {workers} processes ({cpu['cpu_model']})")
        if c1_pairs:
            oracle_c1 = cpu_pool(pool, workers, [(c1_pairs[0][0], c1_pairs[0][1])], 3, 4, 4)[0][0]

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
    margin = r + 10 + 2
    for tag, fp16 in (("fp32", False), ("fp16", True)):
        plan, res = bench_plain(torch, ofmi, dev, wl, d1, d2, us, vs, fp16, args.steps, args.warmup, tag)
        plan.compute(d1[0], d2[0], us[0], vs[0])
        torch.cuda.synchronize()
        u, v = us[0].cpu().numpy(), vs[0].cpu().numpy()
        res["truth"] = truth_stats(u, v, pairs[0][2], pairs[0][3], margin)
        if oracle_c2 is not None:
            res["parity"] = err_stats(u, v, oracle_c2[0].astype(np.float64), oracle_c2[1].astype(np.float64))
        if tag == "fp32":
            pg = ofmi.Plan(wl.H, wl.W, L, r, K, fp16=fp16, device=dev, graph=True)
            pg.set_config(res["cfg"])
            res["graphed"] = args.steps / time_plan(torch, pg, d1, d2, us, vs, args.steps, args.warmup)
            pg.close()
        plan.close()
        results[tag] = res

    extra = {}
    if not args.no_extra:
        v32 = args.steps / results["fp32"]["el"]
        runs = (("c1_256_fp32", lambda: bench_c1(torch, ofmi, dev, c1_pairs, oracle_c1, args.steps, args.warmup)),
                ("batched_1024_fp32", lambda: bench_batched(torch, ofmi, dev, d1, d2, wl, False, 20, "fp32")),
                ("batched_1024_fp16", lambda: bench_batched(torch, ofmi, dev, d1, d2, wl, True, 20, "fp16")),
                ("mixed_batch_64", lambda: bench_c4(torch, ofmi, dev, pool, workers, 5, not args.no_cpu_baseline)),
                ("table1_sweep", lambda: bench_table1(torch, dev, pool)),
                ("gaussian_window_1024_fp32", lambda: bench_gaussian(torch, ofmi, dev, d1, d2, us, vs, wl,
                                                                     args.steps, args.warmup, v32)),
                ("masked_1024_fp32", lambda: bench_masked(torch, ofmi, dev, d1, d2, us, vs, wl, args.steps,
                                                          args.warmup, v32,
                                                          extra.get("batched_1024_fp32", {}).get("value"))),
                ("serving_8_streams", lambda: bench_serving(torch, ofmi, dev, pool, workers, args.serve_frames,
                                                            not args.no_cpu_baseline)))
        for name, fn in runs:
            try:
                extra[name] = fn()
            except Exception as e:  # report, keep the main line
                extra[name] = {"error": repr(e)}
                log(f"{name} failed: {e!r}")
    pool.shutdown()

    r32, r16 = results["fp32"], results["fp16"]
    dom = r32["dominant"]
    traffic = measured_traffic(r32["cfg"]["variant"][0]) if dom["level"] == 0 else None
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
        "parity": dict(r32.get("parity", {}), tolerance_px=1e-3, fp32_floor_max_px=floor_max("c2")),
        "accuracy_vs_truth": r32["truth"],
        "roofline": {"bound": "hbm", "achieved": dom["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom["frac"], "traffic": traffic,
                     "kernel": f"lk_iter_strip, level {dom['level']} ({dom['H']}x{dom['W']}, "
                               f"{'uint8' if dom['level'] == 0 else 'float32'} frames), the largest share of the "
                               f"iteration time",
                     "avg_launch_us": dom["avg_launch_us"], "bytes_per_launch": dom["bytes_per_launch"],
                     "launches": dom["launches"],
                     "timing": "one hipEvent pair around each level's 4 back-to-back iteration launches on the launch "
                               "stream, host enqueueing ahead; algorithmic bytes = pixels x (2 frame elements + 16 B)",
                     "per_level": r32["per_level"], "pyramid": r32["pyramid"]},
        "fp16": {"value": round(args.steps / r16["el"], 3),
                 "ms_per_step": round(r16["el"] / args.steps * 1e3, 5),
                 "speedup_vs_fp32": round(r32["el"] / r16["el"], 4),
                 "latency_ms": r16["lat"],
                 "parity": dict(r16.get("parity", {}), tolerance_px=2e-2, fp16_floor_max_px=floor_max("c3_fp16")),
                 "accuracy_vs_truth": r16["truth"],
                 "per_level": r16["per_level"], "launch_config": r16["cfg"]},
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
