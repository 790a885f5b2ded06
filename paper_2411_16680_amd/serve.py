"""Request loop for novel-view serving: continuous admission of requests,
each rendered by a fresh layered depth map (the paper makes and discards an
LDM per frame, Sec. 3; 30 frames/s is its real-time target, Sec. 1).

A request names a resident scene (input cameras and its encoded feature
pyramid), an output size and a novel camera.  Its work is one learned
initialisation plus one Update & Fuse step per pyramid level (independent
per-level states), the finest level composited to RGB -- all in libquark.

Scheduling:
  * Requests are admitted first come, first served as they arrive -- no
    batch boundary: a request starts as soon as it fits.
  * Admission is bounded by an HBM budget: a request reserves the bytes of
    its LDMs and output; if the head of the queue does not fit, it waits for
    completions (head-of-line order is kept); a request that could never fit
    is rejected.
  * Admitted requests go round-robin onto a few HIP streams (default
    priority), each with its own libquark context, so requests overlap on
    the device.  A request's result does not depend on what else runs: the
    forward kernels have no atomics and every request owns its buffers.
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

from . import lib, synth

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

    def done(self, handle) -> bool:
        raise NotImplementedError

    def release(self, job: Job, handle) -> None:
        pass


def request_bytes(req: synth.ServeRequest, ldm_bytes_per_elem: int = 2) -> int:
    """HBM a request holds while it runs: per level an LDM of
    L x H x W x C features plus depth and alpha (float32), and the float32
    RGB output."""
    total = req.width * req.height * 3 * 4
    for k, C, L in synth.SERVE_LEVELS:
        n = L * (req.height // k) * (req.width // k)
        total += n * (C * ldm_bytes_per_elem + 8)
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
            try:
                job.handle = self.ex.launch(job)
            except Exception as e:                     # per-request failure
                job.status = FAILED
                job.error = str(e)
                continue
            job.status = RUNNING
            self.used += need
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

class GpuExecutor(Executor):
    """Runs requests through libquark on ``n_streams`` HIP streams (default
    priority), one libquark context per stream.  Scenes' pyramids stay
    resident; each request's LDMs and RGB are allocated on its stream from
    torch's caching allocator (no device allocation once warm)."""

    def __init__(self, scenes: Dict[int, synth.ServeScene], pyramids: Dict[int, list],
                 model: synth.ServeModel, *, n_streams: int = 4, attn_form: str = "folded",
                 device: int = 0, keep_rgb: bool = False):
        import torch
        self.torch = torch
        self.scenes = scenes
        self.pyr = pyramids
        self.model = model
        self.attn_form = attn_form
        dev = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(n_streams)]
        self.ctxs = [lib.Context(device) for _ in range(n_streams)]
        self.w = [{k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(dev)
                   for k, v in wl.items()} for wl in model.weights]
        self.f0 = [torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).to(dev)
                   for f in model.f0]
        self.dev = dev
        self.keep_rgb = keep_rgb
        self.rr = 0

    def bytes_needed(self, req):
        return request_bytes(req)

    def launch(self, job: Job):
        torch = self.torch
        req = job.req
        sc = self.scenes.get(req.scene_id)
        if sc is None:
            raise lib.QuarkError(lib.QK_EINVAL, f"unknown scene {req.scene_id}")
        i = self.rr
        self.rr = (self.rr + 1) % len(self.streams)
        s, ctx = self.streams[i], self.ctxs[i]
        m = self.model
        with torch.cuda.stream(s):
            rgb = torch.empty((req.height, req.width, 3), device=self.dev, dtype=torch.float32)
            bufs = []
            for li, (k, C, L) in enumerate(synth.SERVE_LEVELS):
                H, W = req.height // k, req.width // k
                F = torch.empty((L, H, W, C), device=self.dev, dtype=torch.bfloat16)
                d = torch.empty((L, H, W), device=self.dev, dtype=torch.float32)
                a = torch.empty((L, H, W), device=self.dev, dtype=torch.float32)
                bufs.append((F, d, a))
                lib.ldm_init(ctx, self.f0[li], m.near, m.far, (F, d, a), stream=s)
                last = li == len(synth.SERVE_LEVELS) - 1
                lib.update_fuse(ctx, sc.in_cams, self.pyr[req.scene_id][li], req.novel, m.near,
                                m.far, self.w[li], (F, d, a), (F, d, a), precision="bf16",
                                attn_form=self.attn_form, mode="residual",
                                rgb_out=rgb if last else None, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        job.rgb = rgb
        return (ev, bufs)

    def done(self, handle) -> bool:
        return handle[0].query()

    def release(self, job: Job, handle) -> None:
        handle[1].clear()              # LDMs go back to the stream's cache
        if not self.keep_rgb:
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
