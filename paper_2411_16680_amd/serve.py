"""Request loop for novel-view serving: continuous admission of requests,
each rendered by the paper's whole per-frame method on a fresh layered
depth map (the paper makes and discards an LDM per frame, Sec. 3; 30
frames/s is its real-time target, Sec. 1).

A request names a resident scene (input cameras, encoded feature pyramid
and input images), an output size and a novel camera.  Its work is one
frame: the ray-direction encoding of the scene's pyramid for its camera, the
learned initialisation, the chained Update & Fuse steps of the network
(collapse, upsampling, decode, attention, residual CNN blocks), the blend
weights of the last attention and the final render at the requested size --
all in libquark.

Scheduling:
  * Requests are admitted first come, first served as they arrive -- no
    batch boundary: a request starts as soon as it fits.
  * Admission is bounded by an HBM budget: a request reserves the bytes of
    its frame's buffers; if the head of the queue does not fit, it waits for
    completions (head-of-line order is kept); a request that could never fit
    is rejected.
  * The requests admitted at one poll form a batch: each Update & Fuse step
    of all of them is one launch (qk_batch_update_fuse), the other kernels
    run per request.  Batches go round-robin onto a few HIP streams (default
    priority), each with its own libquark context, so batches overlap on the
    device.  A request's result does not depend on what else runs: the
    forward kernels have no atomics, every request owns its buffers, and a
    batched step equals the request's own step bit for bit.
  * Failures are per request (a rejected argument, an unknown scene, a
    missed deadline, a cancellation); the loop keeps going.

The loop is written against an ``Executor`` (launch / done / release) and a
clock, so its policy is tested on the CPU with a fake executor and a fake
clock; ``GpuExecutor`` is the device implementation.
"""

from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Deque, Dict, List, Optional

import numpy as np

from . import lib, runner, synth

QUEUED, RUNNING, DONE, FAILED, REJECTED, CANCELLED = (
    "queued", "running", "done", "failed", "rejected", "cancelled")


@dataclass
class Job:
    req: synth.ServeRequest
    deadline: Optional[float] = None         # seconds after arrival, or None
    status: str = QUEUED
    error: str = ""
    bytes: int = 0
    t_start: float = math.nan
    t_done: float = math.nan
    handle: object = None
    rgb: object = None
    frame: object = None

    @property
    def latency(self) -> float:
        return self.t_done - self.req.arrival

    @property
    def missed(self) -> bool:
        return self.deadline is not None and self.status == DONE and self.latency > self.deadline


class Executor:
    """Device side of the loop."""

    def bytes_needed(self, req: synth.ServeRequest) -> int:
        raise NotImplementedError

    def launch(self, job: Job):
        """Enqueue the request's work; returns a handle.  Raises on a request
        that cannot run (the loop marks it failed)."""
        raise NotImplementedError

    def launch_batch(self, jobs: List[Job]) -> list:
        """Enqueue several requests admitted together; returns, per job, its
        handle or the exception that stopped it."""
        out = []
        for job in jobs:
            try:
                out.append(self.launch(job))
            except Exception as e:                 # per-request failure
                out.append(e)
        return out

    def done(self, handle) -> bool:
        raise NotImplementedError

    def release(self, job: Job, handle) -> None:
        pass


def request_bytes(req: synth.ServeRequest, V: int = 8, steps=synth.QUARK_STEPS, C: int = 32,
                  feat_hw=synth.QUARK_FEAT_HW, elem: int = 2) -> int:
    """HBM a request holds while it runs: its frame's buffers -- the
    ray-encoded copy of the pyramid, per step the volumes (input
    transitions, update output, residual block output, elem bytes per
    feature) and float32 depth / alpha planes (input and output), the
    initial volume, the last step's blend logits (V per layer-pixel) and the
    final logits, and the float32 RGB, alpha and depth of the output."""
    total = sum(h * w * C * elem for h, w in feat_hw) * V
    for i, st in enumerate(steps):
        n = st.L * st.H * st.W
        vols = 1 + (i > 0 and st.upsample) + (i > 0 and st.collapse) + bool(st.conv)
        if i > 0 and st.collapse:            # collapsed, before upsampling
            vols -= 1
            total += n // (4 if st.upsample else 1) * C * elem
        total += vols * n * C * elem + 4 * n * 4
    s0, last = steps[0], steps[-1]
    total += s0.L * s0.H * s0.W * C * elem
    total += last.L * last.H * last.W * (V + 2) * 4
    total += req.width * req.height * (3 + 2) * 4
    return total


class Server:
    def __init__(self, executor: Executor, budget_bytes: int,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.clock = clock
        self.queue: Deque[Job] = collections.deque()
        self.running: List[Job] = []
        self.jobs: Dict[int, Job] = {}
        self.used = 0
        self.t0 = None

    def now(self) -> float:
        """Seconds since the loop started (request arrivals use this origin)."""
        return self.clock() - self.t0

    def start(self):
        self.t0 = self.clock()

    def submit(self, req: synth.ServeRequest, deadline: Optional[float] = None) -> Job:
        job = Job(req, deadline)
        self.jobs[req.rid] = job
        self.queue.append(job)
        return job

    def cancel(self, rid: int) -> bool:
        """Cancel a request that has not started."""
        job = self.jobs.get(rid)
        if job is None or job.status != QUEUED:
            return False
        self.queue.remove(job)
        job.status = CANCELLED
        return True

    def step(self) -> None:
        """Retire finished requests, then admit what fits."""
        now = self.now()
        still = []
        for job in self.running:
            if self.ex.done(job.handle):
                job.t_done = now
                job.status = DONE
                self.ex.release(job, job.handle)
                job.handle = None
                self.used -= job.bytes
            else:
                still.append(job)
        self.running = still
        batch = []
        while self.queue:
            job = self.queue[0]
            if job.req.arrival > now:
                break
            need = self.ex.bytes_needed(job.req)
            if need > self.budget:
                self.queue.popleft()
                job.status = REJECTED
                job.error = f"needs {need} bytes, budget {self.budget}"
                continue
            if self.used + need > self.budget:
                break                                  # wait for completions
            self.queue.popleft()
            job.bytes = need
            job.t_start = now
            self.used += need                          # reserved at admission
            batch.append(job)
        if batch:
            for job, h in zip(batch, self.ex.launch_batch(batch)):
                if isinstance(h, Exception):           # per-request failure
                    job.status = FAILED
                    job.error = str(h)
                    self.used -= job.bytes
                    continue
                job.handle = h
                job.status = RUNNING
                self.running.append(job)

    def idle(self) -> bool:
        return not self.queue and not self.running

    def next_arrival(self) -> Optional[float]:
        return self.queue[0].req.arrival if self.queue else None

    def run(self, requests: List[synth.ServeRequest], deadline: Optional[float] = None,
            sleep: Callable[[float], None] = time.sleep, poll: float = 5e-5) -> List[Job]:
        """Serve ``requests`` (sorted by arrival, times relative to the start)
        to completion.  Waits for arrivals with ``sleep``; while requests run
        it polls every ``poll`` seconds."""
        for r in sorted(requests, key=lambda r: r.arrival):
            self.submit(r, deadline)
        self.start()
        while not self.idle():
            self.step()
            if self.idle():
                break
            if not self.running:
                nxt = self.next_arrival()
                wait = nxt - self.now() if nxt is not None else poll
                if wait > 0:
                    sleep(min(wait, 0.5))
            else:
                sleep(poll)
        return [self.jobs[r.rid] for r in requests]


def summarize(jobs: List[Job], slo: float = 1.0 / 30.0) -> dict:
    done = [j for j in jobs if j.status == DONE]
    lat = np.array([j.latency for j in done]) * 1e3
    span = (max(j.t_done for j in done) - min(j.req.arrival for j in done)) if done else 0.0
    out = {"requests": len(jobs), "done": len(done),
           "failed": sum(j.status == FAILED for j in jobs),
           "rejected": sum(j.status == REJECTED for j in jobs),
           "cancelled": sum(j.status == CANCELLED for j in jobs),
           "deadline_missed": sum(j.missed for j in jobs)}
    if len(done):
        out.update({"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                    "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
                    "throughput_rps": len(done) / span if span > 0 else math.nan,
                    "frac_under_slo": float(np.mean(lat <= slo * 1e3)), "slo_ms": slo * 1e3})
    return out


# ----------------------------------------------------------------------------
# Device executor
# ----------------------------------------------------------------------------

@dataclass
class FrameScene:
    """What a frame reads of its scene and request (``runner.run_pipelines``)."""
    in_cams: list
    novel: object
    near: float
    far: float
    steps: list
    dtype: str = "bf16"


class GpuExecutor(Executor):
    """Runs requests' frames through libquark, a batch of requests admitted
    together at a time, batches round-robin over ``n_streams`` HIP streams
    (default priority), one libquark context per stream.  Scenes' pyramids
    and images stay resident (``resident[scene_id] = (pyramid, images)``);
    the network's weights are on the device once; each request's frame
    buffers come from torch's caching allocator on its batch's stream (no
    device allocation once warm)."""

    MAX_BATCH = 64

    def __init__(self, scenes: Dict[int, synth.ServeScene], resident: Dict[int, tuple],
                 model: synth.ServeModel, *, n_streams: int = 4, attn_form: str = "auto",
                 device: int = 0, keep_frames: bool = False):
        import torch
        self.torch = torch
        self.scenes = scenes
        self.resident = resident
        self.model = model
        self.attn_form = attn_form
        dev = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(n_streams)]
        self.ctxs = [lib.Context(device) for _ in range(n_streams)]
        for c in self.ctxs:                # the network's weights do not change while serving
            c.weights_static(True)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
        self.w = [{k: t(v) for k, v in wl.items()} for wl in model.weights]
        self.cw = [None if c is None else tuple(t(a) for a in c) for c in model.collapse_w]
        self.kw = [None if c is None else tuple(t(a) for a in c) for c in model.conv_w]
        self.Wr = [t(w) for w in model.Wr]
        self.f0 = t(model.f0)
        self.dev = dev
        self.keep_frames = keep_frames
        self.rr = 0

    def bytes_needed(self, req):
        sc = self.scenes.get(req.scene_id)
        m = self.model
        return request_bytes(req, V=sc.V if sc is not None else 8, steps=m.steps, C=m.C,
                             feat_hw=sc.feat_hw if sc is not None else synth.QUARK_FEAT_HW)

    def launch(self, job: Job):
        return self.launch_batch([job])[0]

    def launch_batch(self, jobs: List[Job]) -> list:
        out = []
        ok = []
        for job in jobs:
            if job.req.scene_id not in self.scenes:
                out.append(lib.QuarkError(lib.QK_EINVAL, f"unknown scene {job.req.scene_id}"))
            else:
                out.append(None)
                ok.append(job)
        for k in range(0, len(ok), self.MAX_BATCH):
            part = ok[k:k + self.MAX_BATCH]
            try:
                handles = self._run(part)
            except Exception as e:               # the library refused the batch
                handles = [e] * len(part)
            for job, h in zip(part, handles):
                out[jobs.index(job)] = h
        return out

    def _run(self, jobs: List[Job]) -> list:
        torch = self.torch
        m = self.model
        i = self.rr
        self.rr = (self.rr + 1) % len(self.streams)
        s, ctx = self.streams[i], self.ctxs[i]
        frames = []
        with torch.cuda.stream(s):
            for job in jobs:
                req = job.req
                sc = self.scenes[req.scene_id]
                pyr, images = self.resident[req.scene_id]
                dp = runner.make_device_pipeline(m.steps, m.C, pyr, self.w, self.cw, self.kw,
                                                 self.Wr, self.f0, images,
                                                 (req.height, req.width), "bf16", self.dev)
                frames.append((FrameScene(sc.in_cams, req.novel, m.near, m.far, m.steps),
                               m.low_hw, dp))
            runner.run_pipelines(ctx, frames, attn_form=self.attn_form, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        handles = []
        for job, (_, _, dp) in zip(jobs, frames):
            job.rgb = dp.rgb
            handles.append((ev, dp))
        return handles

    def done(self, handle) -> bool:
        return handle[0].query()

    def release(self, job: Job, handle) -> None:
        if self.keep_frames:
            job.frame = handle[1]
        else:
            job.rgb = None


# ----------------------------------------------------------------------------
# Fake executor (CPU tests of the loop's policy)
# ----------------------------------------------------------------------------

class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self) -> float:
        return self.t

    def sleep(self, dt: float) -> None:
        self.t += max(dt, 1e-6)


class FakeExecutor(Executor):
    """Completes each request ``cost(req)`` seconds of fake time after its
    launch, ``concurrency`` at a time (later ones queue behind)."""

    def __init__(self, clock: FakeClock, cost: Callable[[synth.ServeRequest], float],
                 bytes_fn: Callable[[synth.ServeRequest], int] = request_bytes,
                 fail_on: Callable[[synth.ServeRequest], bool] = lambda r: False,
                 concurrency: int = 1):
        self.clock = clock
        self.cost = cost
        self.bytes_fn = bytes_fn
        self.fail_on = fail_on
        self.lanes = [0.0] * concurrency
        self.launched: List[int] = []

    def bytes_needed(self, req):
        return self.bytes_fn(req)

    def launch(self, job: Job):
        if self.fail_on(job.req):
            raise lib.QuarkError(lib.QK_ESHAPE, "rejected by the library")
        i = int(np.argmin(self.lanes))
        t_end = max(self.lanes[i], self.clock()) + self.cost(job.req)
        self.lanes[i] = t_end
        self.launched.append(job.req.rid)
        return t_end

    def done(self, handle) -> bool:
        return self.clock() >= handle
