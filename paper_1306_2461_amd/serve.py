"""Serving loop: frame-stream requests, admission by HBM budget, continuous batching.

Frames of many streams arrive over time (the paper's real-time setting, Sec. 2.2 and Sec. 2.4:
each new camera frame yields one field).  ``Server`` keeps a queue of requests; every
``step`` takes the oldest pending frame of each admitted stream (at most one frame per stream
per push, so a stream's frames stay in order) and launches them together through an executor.
Requests that arrive while earlier pushes run on the device join the next push (continuous
batching); their work overlaps on the device stream.  Streams are admitted when their
resident memory fits the HBM budget; a stream that can never fit is rejected.  Completion is
observed by polling the pushes' events; each request records arrival and completion times.

Executors implement ``open(H, W) -> handle`` (raising ``BudgetExceeded``),
``session_bytes(H, W)``, ``budget``, ``close(handle)``,
``submit([(handle, frame)], keep) -> token`` (raising ``Busy`` when it cannot take a push now),
``ready(token) -> bool``, ``wait(token)`` and ``finish(token) -> [(u, v, has_flow)]``.
``GpuExecutor`` runs the HIP library (``of_server_*``).
"""
from __future__ import annotations

import collections
import dataclasses
import gc
import time
from typing import Any

import numpy as np


class BudgetExceeded(RuntimeError):
    """Opening a stream would exceed the executor's HBM budget."""


class Busy(RuntimeError):
    """The executor holds as many pushes in flight as it can stage; retry after one completes."""


@dataclasses.dataclass
class Request:
    stream_id: int
    frame: Any
    t_arrival: float
    t_launch: float | None = None
    t_done: float | None = None
    has_flow: bool | None = None
    u: Any = None
    v: Any = None
    error: str | None = None

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival


class Server:
    """Continuous-batching request loop over an executor."""

    def __init__(self, executor, max_batch: int = 64, clock=time.perf_counter, keep=None,
                 max_inflight: int | None = 2):
        """``keep(request) -> bool`` selects the requests whose flow is kept (default: all);
        the others are only timed, and their output planes go back to the executor's pool.
        ``max_inflight`` bounds the pushes in flight (None: as many as the executor stages).
        While the bound is reached, arriving frames wait on the host and join one larger push
        instead of queueing on the device as many small ones: the default, one push running
        and one queued behind it, keeps the device busy and turns bursts into batches."""
        self.ex = executor
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.clock = clock
        self.keep = keep
        self.pending: collections.deque[Request] = collections.deque()
        self.inflight: collections.deque = collections.deque()
        self.sessions: dict[int, Any] = {}
        self.sizes: dict[int, tuple] = {}
        self.done: list[Request] = []
        self.rejected: list[Request] = []
        self.admission_log: list[tuple] = []
        self.busy = False

    # ------------------------------------------------------------------ requests
    def submit(self, stream_id: int, frame, t_arrival: float | None = None) -> Request:
        shape = tuple(frame.shape)
        if stream_id in self.sizes and self.sizes[stream_id] != shape:
            req = Request(stream_id, frame, self.clock() if t_arrival is None else t_arrival)
            req.error = f"frame size {shape} differs from the stream's {self.sizes[stream_id]}"
            self.rejected.append(req)
            return req
        self.sizes.setdefault(stream_id, shape)
        req = Request(stream_id, frame, self.clock() if t_arrival is None else t_arrival)
        self.pending.append(req)
        return req

    def close_stream(self, stream_id: int):
        """Closes a stream's session once its pushes are done; frees its budget."""
        self.drain(stream_id)
        h = self.sessions.pop(stream_id, None)
        if h is not None:
            self.ex.close(h)
            self.admission_log.append((self.clock(), "close", stream_id))

    # ------------------------------------------------------------------ loop
    def _admit(self, req: Request):
        h = self._open(req.stream_id, tuple(req.frame.shape))
        if h == "reject":
            H, W = req.frame.shape
            req.error = (f"stream needs {self.ex.session_bytes(H, W)} bytes, more than the whole "
                         f"budget {self.ex.budget}")
        return h

    def _open(self, stream_id: int, shape: tuple):
        h = self.sessions.get(stream_id)
        if h is not None:
            return h
        H, W = shape
        need = self.ex.session_bytes(H, W)
        if self.ex.budget and need > self.ex.budget:
            return "reject"
        try:
            h = self.ex.open(H, W)
        except BudgetExceeded:
            return None
        self.sessions[stream_id] = h
        self.admission_log.append((self.clock(), "open", stream_id))
        return h

    def open_stream(self, stream_id: int, shape: tuple) -> bool:
        """Admits a stream before its first frame arrives, so that opening its session (which
        may allocate) stays out of the request path; False if the budget has no room now."""
        shape = tuple(shape)
        if self.sizes.setdefault(stream_id, shape) != shape:
            raise ValueError(f"stream {stream_id} has frames of size {self.sizes[stream_id]}")
        h = self._open(stream_id, shape)
        if h == "reject":
            raise BudgetExceeded(f"stream {stream_id} of size {shape} can never fit the budget")
        return h is not None

    def step(self) -> int:
        """Launch one push with the oldest pending frame of every admitted stream."""
        self.busy = self.max_inflight is not None and len(self.inflight) >= self.max_inflight
        if self.busy:
            return 0
        batch, seen, keep = [], set(), collections.deque()
        while self.pending:
            req = self.pending.popleft()
            if req.stream_id in seen or len(batch) >= self.max_batch:
                keep.append(req)
                continue
            h = self._admit(req)
            if h == "reject":
                self.rejected.append(req)
                continue
            seen.add(req.stream_id)          # later frames of this stream wait for a later push
            if h is None:
                keep.append(req)             # waits for budget
                continue
            batch.append((h, req))
        self.pending = keep
        if not batch:
            return 0
        keep = [True if self.keep is None else bool(self.keep(r)) for _, r in batch]
        try:
            token = self.ex.submit([(h, r.frame) for h, r in batch], keep)
        except Busy:
            # nothing was pushed: the requests go back in front, in order, and wait for a
            # push in flight to complete
            self.pending.extendleft(reversed([r for _, r in batch]))
            self.busy = True
            return 0
        t = self.clock()
        for _, r in batch:
            r.t_launch = t
        self.inflight.append((token, [r for _, r in batch]))
        return len(batch)

    def poll(self) -> int:
        """Complete finished pushes in launch order; returns the number completed."""
        n = 0
        while self.inflight and self.ex.ready(self.inflight[0][0]):
            token, reqs = self.inflight.popleft()
            t = self.clock()
            for r, (u, v, has) in zip(reqs, self.ex.finish(token)):
                r.t_done, r.u, r.v, r.has_flow = t, u, v, bool(has)
                self.done.append(r)
                n += 1
        return n

    def drain(self, stream_id: int | None = None):
        """Run until no request (of `stream_id`, or at all) is pending or in flight."""
        def busy():
            if stream_id is None:
                return bool(self.pending or self.inflight)
            return any(r.stream_id == stream_id for r in self.pending) or any(
                r.stream_id == stream_id for _, rs in self.inflight for r in rs)
        while busy():
            launched = self.step()
            if not self.poll() and not launched:
                if self.inflight:
                    self.ex.wait(self.inflight[0][0])
                elif self.pending:
                    raise RuntimeError("pending requests cannot be admitted (HBM budget)")

    def replay(self, arrivals, realtime: bool = True):
        """Serve (t, stream_id, frame) arrivals (sorted by t), optionally paced in real time.

        Returns per-pair latency percentiles and throughput over the flows computed.  The
        garbage collector is paused while the loop runs (its pauses would land in the tail)."""
        gc_on = gc.isenabled()
        gc.disable()
        try:
            self._replay(arrivals, realtime)
        finally:
            if gc_on:
                gc.enable()
        return self.stats()

    def _replay(self, arrivals, realtime):
        t0 = self.clock()
        i = 0
        while i < len(arrivals) or self.pending or self.inflight:
            now = self.clock() - t0
            while i < len(arrivals) and (not realtime or arrivals[i][0] <= now):
                ta, sid, frame = arrivals[i]
                self.submit(sid, frame, t0 + ta if realtime else self.clock())
                i += 1
            launched = self.step() if self.pending else 0
            completed = self.poll()
            if not launched and not completed:
                if self.inflight and (i >= len(arrivals) or not realtime or (self.busy and self.pending)):
                    self.ex.wait(self.inflight[0][0])
                elif realtime and i < len(arrivals):
                    time.sleep(max(0.0, min(2e-4, arrivals[i][0] - (self.clock() - t0))))
                elif self.pending and not self.inflight:
                    raise RuntimeError("pending requests cannot be admitted (HBM budget)")

    def stats(self):
        flows = [r for r in self.done if r.has_flow]
        lat = sorted(r.latency for r in flows)
        out = {"requests": len(self.done), "flows": len(flows), "rejected": len(self.rejected)}
        if lat:
            def q(xs, f):
                xs = sorted(xs)
                return 1e3 * xs[min(len(xs) - 1, int(f * len(xs)))]
            out["p50_ms"] = q(lat, 0.5)
            out["p99_ms"] = q(lat, 0.99)
            # where the time goes: waiting for a push (arrival -> launch) and on the device
            # (launch -> completion seen by the host)
            wait = [r.t_launch - r.t_arrival for r in flows]
            run = [r.t_done - r.t_launch for r in flows]
            out["queue_p50_ms"], out["queue_p99_ms"] = q(wait, 0.5), q(wait, 0.99)
            out["device_p50_ms"], out["device_p99_ms"] = q(run, 0.5), q(run, 0.99)
            by_size = {}
            for r in flows:
                by_size.setdefault("x".join(str(d) for d in reversed(r.frame.shape)), []).append(r.latency)
            out["p99_ms_by_size"] = {k: q(v, 0.99) for k, v in sorted(by_size.items())}
            t_first = min(r.t_arrival for r in self.done)
            t_last = max(r.t_done for r in flows)
            out["pairs_per_s"] = len(flows) / max(t_last - t_first, 1e-9)
        return out


class GpuExecutor:
    """Executor over the HIP server ABI (``of_server_*``) on one device.

    Session memory is a torch allocation per stream (``of_server_open_ex``).  A push stages each
    frame into a pinned host buffer and copies it to a device staging frame on a copy stream;
    the compute stream waits for that copy (an event) and runs the push, so frame uploads
    overlap the kernels of earlier pushes.  Output planes come from per-shape pools; planes of
    results that are not kept go back to their pool when the push completes.  At most
    ``OF_SERVER_RING`` pushes are in flight; beyond that ``submit`` raises ``Busy``.
    """

    RING = 8   # OF_SERVER_RING

    def __init__(self, levels, radius, iters, fp16=False, budget_bytes=0, device=None,
                 keep_on_device=True, gaussian_window=False):
        import torch

        from . import _binding as B
        self.torch = torch
        self.B = B
        self.lib = B.load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.levels, self.radius, self.iters = levels, radius, iters
        self.flags = ((B.OF_FLAG_FP16_STORAGE if fp16 else 0)
                      | (B.OF_FLAG_GAUSSIAN_WINDOW if gaussian_window else 0))
        self.budget = int(budget_bytes)
        self.keep_on_device = keep_on_device
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(self.device)
            self.copy_stream = torch.cuda.Stream(self.device)
            h = self.lib.of_server_create(levels, radius, iters, self.flags, self.budget)
        if not h:
            raise B.OfError(f"of_server_create failed: {B.last_error()}")
        self._h = h
        self._ws: dict[int, Any] = {}
        self._host: dict[tuple, list] = collections.defaultdict(list)      # pinned frames
        self._dev: dict[tuple, list] = collections.defaultdict(list)       # device frames
        self._planes: dict[tuple, list] = collections.defaultdict(list)    # output planes
        self._events: collections.deque = collections.deque()              # pushes in flight

    def session_bytes(self, H, W):
        return int(self.lib.of_session_bytes(H, W, self.levels, self.radius, self.iters, self.flags))

    def open(self, H, W):
        torch = self.torch
        nbytes = self.session_bytes(H, W)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            s = self.lib.of_server_open_ex(self._h, H, W, ws.data_ptr(), nbytes)
        if not s:
            msg = self.B.last_error()
            if "budget" in msg:
                raise BudgetExceeded(msg)
            raise self.B.OfError(f"of_server_open_ex failed: {msg}")
        self._ws[s] = ws
        return s

    def set_mask(self, handle, mask):
        """Region-of-interest mask of one open stream (uint8 device tensor, nonzero = compute) or
        None."""
        self.B.check(self.lib.of_session_set_mask(handle, None if mask is None else mask.data_ptr(),
                                                  self.stream.cuda_stream), "of_session_set_mask")

    def close(self, handle):
        self.B.check(self.lib.of_server_close(self._h, handle), "of_server_close")
        self._ws.pop(handle, None)

    def resident_bytes(self):
        return int(self.lib.of_server_resident_bytes(self._h))

    @staticmethod
    def _take(pool, make):
        return pool.pop() if pool else make()

    def submit(self, items, keep=None):
        import ctypes
        torch = self.torch
        n = len(items)
        keep = [True] * n if keep is None else list(keep)
        while self._events and self._events[0].query():
            self._events.popleft()
        if len(self._events) >= self.RING:
            raise Busy("every staging slot holds a push in flight")
        hosts, devs, us, vs, producer = [], [], [], [], []
        with torch.cuda.stream(self.copy_stream):
            for _, f in items:
                shape = tuple(f.shape)
                db = self._take(self._dev[shape], lambda: torch.empty(shape, dtype=torch.uint8, device=self.device))
                if isinstance(f, torch.Tensor) and f.is_pinned():
                    hb = f            # a producer's pinned frame is copied as is (kept until done)
                    producer.append(hb)
                else:
                    hb = self._take(self._host[shape], lambda: torch.empty(shape, dtype=torch.uint8, pin_memory=True))
                    hb.numpy()[...] = f
                    hosts.append(hb)
                db.copy_(hb, non_blocking=True)
                devs.append(db)
        copied = torch.cuda.Event()
        copied.record(self.copy_stream)
        for _, f in items:
            shape = tuple(f.shape)
            mk = lambda: torch.empty(shape, dtype=torch.float32, device=self.device)  # noqa: E731
            us.append(self._take(self._planes[shape], mk))
            vs.append(self._take(self._planes[shape], mk))
        self.stream.wait_event(copied)
        sess = (ctypes.c_void_p * n)(*[h for h, _ in items])
        pf, _a = self.B.ptr_array([t.data_ptr() for t in devs])
        pu, _b = self.B.ptr_array([t.data_ptr() for t in us])
        pv, _c = self.B.ptr_array([t.data_ptr() for t in vs])
        has = (ctypes.c_int * n)()
        st = self.lib.of_server_push(self._h, ctypes.cast(sess, self.B._VPP), n, pf, pu, pv, has,
                                     self.stream.cuda_stream)
        if st == self.B.OF_ESTATE:
            self._give_back(hosts, devs, us, vs)
            raise Busy(self.B.last_error())
        self.B.check(st, "of_server_push")
        ev = torch.cuda.Event()
        ev.record(self.stream)
        self._events.append(ev)
        return {"event": ev, "us": us, "vs": vs, "has": list(has), "keep": keep,
                "frames": (hosts, devs), "producer": producer}

    def _give_back(self, hosts, devs, us, vs):
        for t in hosts:
            self._host[tuple(t.shape)].append(t)
        for t in devs:
            self._dev[tuple(t.shape)].append(t)
        for t in list(us) + list(vs):
            self._planes[tuple(t.shape)].append(t)

    def ready(self, token):
        return token["event"].query()

    def wait(self, token):
        token["event"].synchronize()

    def finish(self, token):
        hosts, devs = token["frames"]
        out, back_u, back_v = [], [], []
        for u, v, has, k in zip(token["us"], token["vs"], token["has"], token["keep"]):
            if not has or not k:
                out.append((None, None, has))
                back_u.append(u)
                back_v.append(v)
            elif self.keep_on_device:
                out.append((u, v, 1))
            else:
                out.append((u.cpu().numpy(), v.cpu().numpy(), 1))
                back_u.append(u)
                back_v.append(v)
        self._give_back(hosts, devs, back_u, back_v)
        return out

    def close_all(self):
        if getattr(self, "_h", None):
            self.lib.of_server_destroy(self._h)
            self._h = None
            self._ws.clear()

    def __del__(self):
        try:
            self.close_all()
        except Exception:
            pass


def poisson_arrivals(streams, rate_per_stream: float, seed: int = 2461):
    """Merge per-stream frame lists into (t, stream, frame) arrivals, each stream an
    independent Poisson process of the given rate (frames of a stream keep their order)."""
    rng = np.random.default_rng(seed)
    out = []
    for sid, frames in enumerate(streams):
        t = 0.0
        for f in frames:
            t += rng.exponential(1.0 / rate_per_stream)
            out.append((t, sid, f))
    out.sort(key=lambda a: a[0])
    return out
