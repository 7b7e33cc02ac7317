"""Serving form: continuous batching of moment requests on one GPU.

Requests arrive over time (frames of mixed sizes and orders).  The scheduler
admits them in arrival order as device memory (an HBM byte budget) and launch
slots free up, groups admitted requests that share a plan into one launch,
and spreads launches over several HIP streams so that the work of requests
admitted at different times overlaps on the device.  Plans (radial tables
and projection operands) stay resident.  Latency = completion time - arrival
time, where completion means the moments are back in host memory.

The policy (`Scheduler`) is device-agnostic: `GpuDevice` runs it on the
library, `FakeDevice` + `FakeClock` run it on the CPU for tests.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    t_arrival: float
    H: int
    W: int
    nmax: int
    frame: object = None          # host frame (numpy float32, pinned torch tensor, ...)
    t_admit: float = math.nan
    t_done: float = math.nan
    result: object = None
    nbytes: int = 0
    status: str = "waiting"       # then "done", "timeout" (expired in the queue) or "busy" (queue full)
    # device-side time of the request's launch (seconds; GpuDevice only): the
    # host-to-device copy, the moment computation, the device-to-host copy
    t_h2d: float = math.nan
    t_compute: float = math.nan
    t_d2h: float = math.nan


@dataclass
class Launch:
    key: tuple
    reqs: list
    nbytes: int
    handle: object = None
    t_launch: float = 0.0


class SchedulerBusy(RuntimeError):
    """The waiting queue is full (the request was not queued)."""


class Scheduler:
    """FIFO admission under a byte budget and an in-flight launch cap; admitted
    requests with the same plan key are launched together (up to max_batch).

    max_waiting bounds the queue (submit raises SchedulerBusy when it is
    full); a request that waits longer than timeout_s is dropped with status
    "timeout" (in `expired`).  set_budget changes the byte budget at run time
    (down to 0, e.g. while other work holds the memory); requests larger than
    the budget given at construction are refused at submit."""

    def __init__(self, device, budget_bytes: int, max_inflight: int = 8, max_batch: int = 16,
                 max_waiting: int | None = None, timeout_s: float | None = None):
        self.dev = device
        self.budget_cap = int(budget_bytes)
        self.budget = self.budget_cap
        self.max_inflight = max_inflight
        self.max_batch = max_batch
        self.max_waiting = max_waiting
        self.timeout_s = timeout_s
        self.waiting = collections.deque()
        self.inflight: list[Launch] = []
        self.used = 0
        self.peak_used = 0
        self.done: list[Request] = []
        self.expired: list[Request] = []

    def set_budget(self, budget_bytes: int):
        self.budget = max(0, min(int(budget_bytes), self.budget_cap))

    def submit(self, req: Request):
        req.nbytes = self.dev.request_bytes(req)
        if req.nbytes > self.budget_cap:
            raise ValueError(f"request {req.rid} needs {req.nbytes} bytes, more than the whole budget")
        if self.max_waiting is not None and len(self.waiting) >= self.max_waiting:
            req.status = "busy"
            raise SchedulerBusy(f"request {req.rid}: {len(self.waiting)} requests already waiting")
        self.waiting.append(req)

    def _expire(self, now: float):
        if self.timeout_s is None:
            return
        keep = collections.deque()
        for r in self.waiting:
            if now - r.t_arrival > self.timeout_s:
                r.status = "timeout"
                r.t_done = now
                self.expired.append(r)
            else:
                keep.append(r)
        self.waiting = keep

    def _admit(self, now: float):
        # head-of-line FIFO: admit from the front while it fits; gather requests
        # of the same plan from the admitted prefix into one launch
        admitted = []
        room = (self.max_inflight - len(self.inflight)) * self.max_batch
        while self.waiting and len(admitted) < room:
            r = self.waiting[0]
            if self.used + r.nbytes > self.budget:
                break
            self.waiting.popleft()
            self.used += r.nbytes
            self.peak_used = max(self.peak_used, self.used)
            r.t_admit = now
            admitted.append(r)
        groups = collections.OrderedDict()
        for r in admitted:
            groups.setdefault(self.dev.plan_key(r), []).append(r)
        out = []
        for key, rs in groups.items():
            for i in range(0, len(rs), self.max_batch):
                chunk = rs[i:i + self.max_batch]
                out.append(Launch(key=key, reqs=chunk, nbytes=sum(r.nbytes for r in chunk)))
        return out

    def step(self, now: float):
        """Retire finished launches, drop expired requests, then admit and
        launch what fits."""
        still = []
        for ln in self.inflight:
            if self.dev.is_done(ln):
                self.dev.finish(ln)
                for r in ln.reqs:
                    r.t_done = now  # completion observed at this poll
                    r.status = "done"
                    self.done.append(r)
                self.used -= ln.nbytes
            else:
                still.append(ln)
        self.inflight = still
        self._expire(now)
        if len(self.inflight) < self.max_inflight:
            for ln in self._admit(now):
                ln.t_launch = now
                self.dev.launch(ln)
                self.inflight.append(ln)

    def idle(self):
        return not self.waiting and not self.inflight


def run_stream(requests, scheduler: Scheduler, clock=time.perf_counter, sleep=None, idle_sleep=None,
               rejected=None):
    """Replay `requests` (t_arrival in seconds from the start) through the
    scheduler in real (or fake) time.  Returns the completed requests with
    t_admit / t_done on the same time axis as t_arrival.

    The loop polls without pausing while work is queued or in flight (a
    completion is seen within one poll); `sleep` (no argument) is called
    after every poll if given.  With nothing queued or in flight,
    `idle_sleep(seconds)` (e.g. time.sleep) is called until shortly before
    the next arrival, when that is more than 0.5 ms away.  Requests refused
    because the queue is full get status "busy" and go to `rejected` (a
    list) when given, else the SchedulerBusy propagates."""
    pending = collections.deque(sorted(requests, key=lambda r: r.t_arrival))
    start = clock()
    while pending or not scheduler.idle():
        now = clock() - start
        while pending and pending[0].t_arrival <= now:
            r = pending.popleft()
            try:
                scheduler.submit(r)
            except SchedulerBusy:
                if rejected is None:
                    raise
                r.t_done = now
                rejected.append(r)
        scheduler.step(now)
        if sleep is not None:
            sleep()
        if idle_sleep is not None and scheduler.idle() and pending:
            gap = pending[0].t_arrival - (clock() - start)
            if gap > 5e-4:
                idle_sleep(gap - 2e-4)
    return scheduler.done


def _percentiles(lat):
    return dict(count=int(lat.size), p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), p999_ms=float(np.percentile(lat, 99.9) * 1e3),
                mean_ms=float(lat.mean() * 1e3))


def latency_stats(done, warmup_s: float = 0.0, by_size: bool = False):
    """Latency percentiles over the requests that arrived after warmup_s;
    images_per_s counts every completed request over the whole span.  With
    by_size, also per frame size ("HxW")."""
    kept = [r for r in done if r.t_arrival >= warmup_s]
    if not kept:
        return {}
    lat = np.array([r.t_done - r.t_arrival for r in kept])
    span = max(r.t_done for r in done) - min(r.t_arrival for r in done)
    out = _percentiles(lat)
    out["images_per_s"] = float(len(done) / span) if span > 0 else 0.0
    # where the time goes: waiting for admission (host queue), then from the
    # launch to the observed completion, split on the device (when measured)
    # into the copies and the computation; "other" is the rest of that span
    # (the launch calls, waits between the streams, the polling loop)
    queue = np.array([r.t_admit - r.t_arrival for r in kept])
    served = np.array([r.t_done - r.t_admit for r in kept])
    parts = {"queue": queue, "launch_to_done": served}
    dev = np.array([[r.t_h2d, r.t_compute, r.t_d2h] for r in kept])
    if np.all(np.isfinite(dev)):
        parts.update(h2d=dev[:, 0], compute=dev[:, 1], d2h=dev[:, 2], other=served - dev.sum(axis=1))
    out["split_ms"] = {k: {"mean": float(v.mean() * 1e3), "p99": float(np.percentile(v, 99) * 1e3)}
                       for k, v in parts.items()}
    tail = lat >= np.percentile(lat, 99)
    out["split_ms_p99_tail"] = {k: float(v[tail].mean() * 1e3) for k, v in parts.items()}
    if by_size:
        sizes = collections.defaultdict(list)
        for r in kept:
            sizes[f"{r.H}x{r.W}"].append(r.t_done - r.t_arrival)
        out["by_size"] = {k: _percentiles(np.array(v)) for k, v in sorted(sizes.items())}
    return out


# --------------------------------------------------------------------------
# Devices
# --------------------------------------------------------------------------
class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt=1e-5):
        self.t += dt


class FakeDevice:
    """Completes a launch a fixed time per request after it starts; used to
    test the scheduling policy on the CPU."""

    def __init__(self, clock: FakeClock, bytes_per_pixel: int = 12, service_s_per_mpix: float = 1e-4):
        self.clock = clock
        self.bpp = bytes_per_pixel
        self.svc = service_s_per_mpix
        self.launched = []

    def request_bytes(self, r: Request) -> int:
        return self.bpp * r.H * r.W

    def plan_key(self, r: Request):
        return (r.H, r.W, r.nmax)

    def launch(self, ln: Launch):
        dur = sum(self.svc * r.H * r.W / 1e6 for r in ln.reqs)
        ln.handle = self.clock() + dur
        self.launched.append(ln)

    def is_done(self, ln: Launch) -> bool:
        return self.clock() >= ln.handle

    def finish(self, ln: Launch):
        for r in ln.reqs:
            r.result = ("done", r.rid)


class GpuDevice:
    """Runs launches on the library: pinned host frames -> device (copy
    stream), the moments on one of several compute streams, moments ->
    pinned host buffers (copy stream); an event marks completion.

    mode "per_plan": a launch holds requests of one plan and runs zm_moments
    on their stacked frames.  mode "persistent": a launch holds the admitted
    requests of any plans (frame sizes and orders mixed) and runs them as one
    persistent kernel over a (frame, ring tile) work queue
    (zm_moments_batch_async, no host wait)."""

    def __init__(self, dtype: str = "f32", n_streams: int = 4, plans=None, mode: str = "per_plan"):
        import torch

        import paper_2304_14492_amd as zm
        if mode not in ("per_plan", "persistent"):
            raise ValueError(f"unknown mode {mode!r}")
        self.mode = mode
        self.zm = zm
        self.torch = torch
        self.dtype = dtype
        self.plans = dict(plans or {})
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.copy_in = torch.cuda.Stream()
        self.copy_out = torch.cuda.Stream()
        self.rr = 0
        self._events = []  # timing events of retired launches, reused

    def plan(self, H, W, nmax):
        key = (H, W, nmax)
        if key not in self.plans:
            self.plans[key] = self.zm.Plan(nmax, H, W, dtype=self.dtype)
        return self.plans[key]

    def plan_key(self, r: Request):
        # the persistent form takes any mix of plans in one launch
        return () if self.mode == "persistent" else (r.H, r.W, r.nmax)

    def request_bytes(self, r: Request) -> int:
        p = self.plan(r.H, r.W, r.nmax)
        return 4 * r.H * r.W + p.workspace_size(1) + 8 * p.num_moments

    def launch(self, ln: Launch):
        if self.mode == "persistent":
            return self._launch_persistent(ln)
        torch = self.torch
        H, W, nmax = ln.key
        p = self.plan(H, W, nmax)
        B = len(ln.reqs)
        cs = self.streams[self.rr % len(self.streams)]
        self.rr += 1
        frames = torch.empty(B, H, W, dtype=torch.float32, device="cuda")
        ws = p.workspace(B)
        Z = torch.empty(B, p.num_moments, 2, dtype=torch.float32, device="cuda")
        host_out = torch.empty(B, p.num_moments, 2, dtype=torch.float32, pin_memory=True)
        ev = self._events.pop() if self._events else [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        with torch.cuda.stream(self.copy_in):
            ev[0].record(self.copy_in)
            for i, r in enumerate(ln.reqs):
                frames[i].copy_(r.frame, non_blocking=True)
            ev[1].record(self.copy_in)
        cs.wait_event(ev[1])
        ev[2].record(cs)
        p.moments(frames, out=Z, workspace=ws, stream=cs)
        ev[3].record(cs)
        self.copy_out.wait_event(ev[3])
        with torch.cuda.stream(self.copy_out):
            ev[4].record(self.copy_out)
            host_out.copy_(Z, non_blocking=True)
            ev[5].record(self.copy_out)
        ev_done = ev[5]
        # keep device buffers alive until the launch retires
        frames.record_stream(self.copy_in)
        frames.record_stream(cs)
        Z.record_stream(cs)
        Z.record_stream(self.copy_out)
        ws.record_stream(cs)
        ln.handle = (ev_done, frames, ws, Z, host_out, ev)

    def _launch_persistent(self, ln: Launch):
        torch = self.torch
        cs = self.streams[self.rr % len(self.streams)]
        self.rr += 1
        plans = [self.plan(r.H, r.W, r.nmax) for r in ln.reqs]
        frames = [torch.empty(r.H, r.W, dtype=torch.float32, device="cuda") for r in ln.reqs]
        outs = [torch.empty(p.num_moments, 2, dtype=torch.float32, device="cuda") for p in plans]
        host_out = [torch.empty(p.num_moments, 2, dtype=torch.float32, pin_memory=True) for p in plans]
        ev = self._events.pop() if self._events else [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        with torch.cuda.stream(self.copy_in):
            ev[0].record(self.copy_in)
            for f, r in zip(frames, ln.reqs):
                f.copy_(r.frame, non_blocking=True)
            ev[1].record(self.copy_in)
        cs.wait_event(ev[1])
        ev[2].record(cs)
        bl = self.zm.BatchLaunch(plans, frames, outs, stream=cs)
        ev[3].record(cs)
        self.copy_out.wait_event(ev[3])
        with torch.cuda.stream(self.copy_out):
            ev[4].record(self.copy_out)
            for h, z in zip(host_out, outs):
                h.copy_(z, non_blocking=True)
            ev[5].record(self.copy_out)
        for f in frames:
            f.record_stream(self.copy_in)
        for z in outs:
            z.record_stream(self.copy_out)
        ln.handle = (ev[5], frames, bl, outs, host_out, ev)

    def is_done(self, ln: Launch) -> bool:
        return ln.handle[0].query()

    def finish(self, ln: Launch):
        host_out, ev = ln.handle[4], ln.handle[5]
        if self.mode == "persistent":
            ln.handle[2].check()  # the run's error flag, back in its staging buffer
        h2d = ev[0].elapsed_time(ev[1]) / 1e3
        comp = ev[2].elapsed_time(ev[3]) / 1e3
        d2h = ev[4].elapsed_time(ev[5]) / 1e3
        for i, r in enumerate(ln.reqs):
            r.result = host_out[i]
            r.t_h2d, r.t_compute, r.t_d2h = h2d, comp, d2h
        self._events.append(ev)
        ln.handle = None

    def warm(self, keys):
        """Create the resident plans for these (H, W, nmax) keys up front."""
        for H, W, nmax in keys:
            self.plan(H, W, nmax)


_FRAME_POOL: dict = {}


def make_requests(count: int, qps: float, seed: int = 5, pool_per_size: int = 3, pin: bool = True):
    """Poisson stream (synth.request_stream); frames come from a pool of
    `pool_per_size` seeded frames per size (request seed mod pool), kept for
    later calls in this process."""
    import synth
    from synth.frames import FrameSpec
    stream = synth.request_stream(count, qps, seed=seed)
    pool = _FRAME_POOL.setdefault(pin, {})
    reqs = []
    for i, (t, H, W, nmax, fseed) in enumerate(stream):
        k = (H, W, fseed % pool_per_size)
        if k not in pool:
            f = synth.make_frame(FrameSpec(H, W, blobs=16, polygons=8, noise=False, zero_outside=False),
                                 seed=5000 + fseed % pool_per_size)
            if pin:
                import torch
                pool[k] = torch.from_numpy(f).pin_memory()
            else:
                pool[k] = f
        reqs.append(Request(rid=i, t_arrival=t, H=H, W=W, nmax=nmax, frame=pool[k]))
    return reqs
