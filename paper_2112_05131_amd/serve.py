"""Novel-view serving with continuous batching over resident scenes.

Scenes (Grid objects, one SH storage type) stay resident on the device.
Requests (scene, camera pose, focal length, width, height) arrive at any time
and wait in a FIFO queue.  Whenever a stream of the pool is idle, every queued
request that fits the HBM admission budget joins one batch, which is rendered
by a single persistent launch of plx_render_views on that stream.  A batch
never waits for earlier batches: requests that arrive while others are on the
device are admitted as streams and budget free up, and their work overlaps with
the running launches.  Completion is observed through a per-batch event;
latency = completion time - arrival time (host monotonic clock).
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B
from .grid import Grid


@dataclass
class Request:
    scene: int
    c2w: np.ndarray  # [3, 4] float64
    focal: float
    width: int
    height: int
    t_arrival: float = 0.0
    t_launch: float = 0.0
    t_done: float = 0.0
    rgb: torch.Tensor | None = None  # [H, W, 3] float32 (device), set on launch
    done: bool = False

    @property
    def n_pixels(self) -> int:
        return self.width * self.height

    @property
    def out_bytes(self) -> int:
        return 12 * self.n_pixels

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclass
class _Batch:
    requests: list
    stream: torch.cuda.Stream
    event: torch.cuda.Event
    out: torch.Tensor
    bytes: int


class Server:
    """Continuous-batching render server.

    hbm_budget: bytes of output buffers admitted at once (queued requests wait
    beyond it); max_batch_pixels: pixels per launch (a request larger than it
    runs alone), so that no launch, whose requests all complete together,
    grows long; n_streams: launches in flight at once; max_batch: requests per
    launch."""

    def __init__(self, scenes: list[Grid], hbm_budget: int = 512 << 20, n_streams: int = 4,
                 max_batch: int = 64, background=(1.0, 1.0, 1.0), keep_outputs: bool = True,
                 max_batch_pixels: int | None = 1 << 21):
        self.keep_outputs = keep_outputs
        if not scenes:
            raise ValueError("need at least one scene")
        dt = scenes[0].sh_dtype
        if any(s.sh_dtype != dt for s in scenes):
            raise ValueError("scenes must share one SH storage type")
        self.scenes = scenes
        self.table = B.SceneTable(scenes)  # resident descriptors, written once
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch)
        self.max_batch_pixels = max_batch_pixels
        self.bg = tuple(background)
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.queues = [B.views_queue(scenes[0].device) for _ in range(n_streams)]
        for st in self.streams:
            st.wait_stream(torch.cuda.current_stream())  # the table and queues are written
        self.queue: deque[Request] = deque()
        self.inflight: list[_Batch] = []
        self.in_use = 0
        self.peak_in_use = 0
        self.completed: list[Request] = []

    def submit(self, req: Request, now: float | None = None) -> Request:
        if req.out_bytes > self.budget:
            raise ValueError("request larger than the HBM admission budget")
        if not 0 <= req.scene < len(self.scenes):
            raise ValueError("unknown scene")
        req.t_arrival = time.perf_counter() if now is None else now
        self.queue.append(req)
        return req

    def _idle_streams(self):
        busy = {id(b.stream) for b in self.inflight}
        return [i for i, s in enumerate(self.streams) if id(s) not in busy]

    def pump(self):
        """Launches queued requests on idle streams while the budget allows."""
        for si in self._idle_streams():
            if not self.queue:
                return
            batch, nbytes, npix = [], 0, 0
            while (self.queue and len(batch) < self.max_batch
                   and self.in_use + nbytes + self.queue[0].out_bytes <= self.budget
                   and (not batch or self.max_batch_pixels is None
                        or npix + self.queue[0].n_pixels <= self.max_batch_pixels)):
                r = self.queue.popleft()
                batch.append(r)
                nbytes += r.out_bytes
                npix += r.n_pixels
            if not batch:
                return  # head of the queue waits for budget
            self._launch(batch, nbytes, si)

    def _launch(self, batch, nbytes, si):
        stream = self.streams[si]
        npix = sum(r.n_pixels for r in batch)
        with torch.cuda.stream(stream):
            out = torch.empty(npix * 3, dtype=torch.float32, device=self.scenes[0].device)
            views, off = [], 0
            for r in batch:
                v = B.PlxView()
                v.c2w[:] = [float(x) for x in np.asarray(r.c2w, np.float64).reshape(12)]
                v.focal = float(r.focal)
                v.width, v.height, v.scene, v.reserved = r.width, r.height, r.scene, 0
                v.out_offset = off
                r.rgb = out[3 * off:3 * (off + r.n_pixels)].view(r.height, r.width, 3)
                off += r.n_pixels
                views.append(v)
            t = time.perf_counter()
            B.plx_render_views(self.table, views, out, self.queues[si], self.bg, stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        for r in batch:
            r.t_launch = t
        self.in_use += nbytes
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        self.inflight.append(_Batch(batch, stream, ev, out, nbytes))

    def poll(self) -> int:
        """Completes finished batches; returns the number of requests done."""
        n = 0
        still = []
        for b in self.inflight:
            if b.event.query():
                t = time.perf_counter()
                for r in b.requests:
                    r.t_done = t
                    r.done = True
                    if not self.keep_outputs:
                        r.rgb = None
                    self.completed.append(r)
                n += len(b.requests)
                self.in_use -= b.bytes
            else:
                still.append(b)
        self.inflight = still
        return n

    def drain(self):
        while self.queue or self.inflight:
            self.pump()
            self.poll()


RESOLUTIONS = ((200, 200), (400, 400), (800, 800), (1280, 720), (1920, 1080))


def random_requests(n: int, n_scenes: int, seed: int, radius: float = 2.0, fov_deg: float = 45.0,
                    resolutions=RESOLUTIONS) -> list[Request]:
    """Requests with uniform scene, resolution and pose on the view sphere."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        v = rng.normal(size=3)
        c = radius * v / np.linalg.norm(v)
        fwd = -c / np.linalg.norm(c)
        up = np.array([0.0, 0.0, 1.0]) if abs(fwd[2]) < 0.99 else np.array([0.0, 1.0, 0.0])
        right = np.cross(fwd, up)
        right /= np.linalg.norm(right)
        tup = np.cross(right, fwd)
        c2w = np.stack([right, tup, -fwd, c], axis=1)
        w, h = resolutions[int(rng.integers(len(resolutions)))]
        focal = 0.5 * w / math.tan(0.5 * math.radians(fov_deg))
        out.append(Request(int(rng.integers(n_scenes)), c2w, focal, w, h))
    return out


def run_load(server: Server, requests: list[Request], rate_hz: float | None, seed: int = 0):
    """Plays the requests against the server: Poisson arrivals at rate_hz, or
    all at t=0 (rate_hz None).  Returns (latencies [s], wall time [s])."""
    rng = np.random.default_rng(seed)
    if rate_hz:
        gaps = rng.exponential(1.0 / rate_hz, size=len(requests))
        offsets = np.cumsum(gaps) - gaps[0]
    else:
        offsets = np.zeros(len(requests))
    t0 = time.perf_counter()
    i = 0
    done0 = len(server.completed)
    while i < len(requests) or server.queue or server.inflight:
        now = time.perf_counter()
        while i < len(requests) and t0 + offsets[i] <= now:
            server.submit(requests[i], now=t0 + offsets[i])
            i += 1
        server.pump()
        server.poll()
    wall = time.perf_counter() - t0
    lat = np.array([r.latency for r in server.completed[done0:]])
    return lat, wall
