"""Continuous-batching render server (forward only) over libdarb.

Scenes stay resident in HBM.  A request (scene, camera, W x H) runs as one
replay of a captured HIP graph of preprocess (camera read from a device
buffer) -> bin/sort (no host readback) -> raster forward on a *render slot*:
buffers sized for its (scene, W, H) key, a device camera buffer and a stream
of its own.

Admission is by memory: a request starts when an idle slot of its key exists,
or when a new slot fits in the memory budget (idle slots of other keys are
freed, least recently used first, to make room); otherwise it waits, first in
first out.  Requests that arrive while others run are admitted as slots and
memory free up, and their graphs run concurrently on separate streams.  The
instance count K is decided on the device before any instance is written, so a
too-small capacity only sets a flag; the server checks it at completion,
renders that request again outside the graph with a larger capacity, and
re-captures the slot.

The scheduling core (:class:`Scheduler`) takes a slot factory, so the policy can
be exercised without a GPU.
"""
from __future__ import annotations

import math
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float  # seconds from the start of the run
    scene: int
    camera: dict

    @property
    def key(self):
        return (self.scene, int(self.camera["width"]), int(self.camera["height"]))

    @property
    def pixels(self) -> int:
        return int(self.camera["width"]) * int(self.camera["height"])


@dataclass
class Result:
    rid: int
    key: tuple
    arrival: float
    start: float
    end: float
    pixels: int
    retried: bool = False
    image: object = None
    work: tuple | None = None  # (K, N_v) of the render, when the slot reports them

    @property
    def latency(self) -> float:
        return self.end - self.arrival


@dataclass
class Stats:
    n: int
    p50_ms: float
    p99_ms: float
    mean_ms: float
    max_ms: float
    mpix_per_s: float
    req_per_s: float
    wall_s: float
    retries: int
    peak_slots: int
    peak_bytes: int
    evictions: int
    peak_inflight: int = 0
    extra: dict = field(default_factory=dict)

    def as_dict(self):
        d = dict(self.__dict__)
        d.pop("extra")
        d.update(self.extra)
        return d


def summarize(results, wall_s, retries, peak_slots, peak_bytes, evictions, peak_inflight=0) -> Stats:
    lat = np.array([r.latency for r in results]) * 1e3
    pix = sum(r.pixels for r in results)
    return Stats(n=len(results), p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                 mean_ms=float(lat.mean()), max_ms=float(lat.max()), mpix_per_s=pix / wall_s / 1e6,
                 req_per_s=len(results) / wall_s, wall_s=wall_s, retries=retries, peak_slots=peak_slots,
                 peak_bytes=peak_bytes, evictions=evictions, peak_inflight=peak_inflight)


class Scheduler:
    """FIFO admission by memory over slots made by ``factory``.

    ``factory(key, capacity_hint)`` returns a slot with attributes ``key``,
    ``nbytes`` and methods ``launch(request)``, ``poll() -> bool`` (finished),
    ``finish() -> (ok, K)`` (ok False when the capacity overflowed; then K is
    the count needed), ``rerun(request, K)`` (blocking re-render with room for K)
    and ``free()``.  ``need(key)`` estimates a new slot's bytes.
    """

    def __init__(self, factory, need, mem_budget: int, max_slots: int = 8, clock=time.perf_counter,
                 sleep=time.sleep, max_inflight: int | None = None):
        self.factory = factory
        self.need = need
        self.budget = int(mem_budget)
        self.max_slots = int(max_slots)
        self.max_inflight = int(max_inflight) if max_inflight is not None else self.max_slots
        self.lookahead = 64  # queued requests considered per admission round
        self.clock = clock
        self.sleep = sleep
        self.idle = OrderedDict()  # key -> list of idle slots (LRU order of keys)
        self.busy = []              # (slot, request, start)
        self.key_slots = {}         # key -> slots of that key (idle or busy)
        self.mem_used = 0
        self.n_slots = 0
        self.peak_slots = 0
        self.peak_bytes = 0
        self.evictions = 0
        self.retries = 0

    def _evict_for(self, need_bytes: int, keep_key) -> bool:
        for key in list(self.idle.keys()):
            if self.mem_used + need_bytes <= self.budget and self.n_slots < self.max_slots:
                break
            if key == keep_key:
                continue
            while self.idle[key] and (self.mem_used + need_bytes > self.budget or self.n_slots >= self.max_slots):
                s = self.idle[key].pop()
                self.mem_used -= s.nbytes
                self.n_slots -= 1
                self.key_slots[key] -= 1
                self.evictions += 1
                s.free()
            if not self.idle[key]:
                del self.idle[key]
        return self.mem_used + need_bytes <= self.budget and self.n_slots < self.max_slots

    def acquire(self, req: Request):
        key = req.key
        lst = self.idle.get(key)
        if lst:
            self.idle.move_to_end(key)
            return lst.pop()
        need = self.need(key)
        if need > self.budget:
            raise MemoryError(f"request key {key} needs {need} bytes, above the budget {self.budget}")
        fits = self.mem_used + need <= self.budget and self.n_slots < self.max_slots
        if not fits and self.key_slots.get(key, 0) > 0:
            return None  # wait for a slot of this key rather than evict another key's
        if not self._evict_for(need, key):
            return None
        s = self.factory(key, None)
        self.mem_used += s.nbytes
        self.n_slots += 1
        self.key_slots[key] = self.key_slots.get(key, 0) + 1
        self.peak_slots = max(self.peak_slots, self.n_slots)
        self.peak_bytes = max(self.peak_bytes, self.mem_used)
        return s

    def release(self, s):
        self.idle.setdefault(s.key, []).append(s)
        self.idle.move_to_end(s.key)

    def run(self, requests, keep_images: bool = False, poll_sleep: float = 20e-6):
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue = deque()
        results = []
        # statistics of this run only
        retries0, evictions0 = self.retries, self.evictions
        self.peak_slots, self.peak_bytes = self.n_slots, self.mem_used
        peak_inflight = 0
        t0 = self.clock()
        while pending or queue or self.busy:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            progressed = False
            # admission: the oldest waiting request that can get a slot, looking past
            # requests that wait for a busy slot of their key (order kept per key)
            i = 0
            blocked = set()
            while i < min(len(queue), self.lookahead) and len(self.busy) < self.max_inflight:
                r = queue[i]
                s = None if r.key in blocked else self.acquire(r)
                if s is None:
                    blocked.add(r.key)
                    i += 1
                    continue
                del queue[i]
                s.launch(r)
                self.busy.append((s, r, self.clock() - t0))
                peak_inflight = max(peak_inflight, len(self.busy))
                progressed = True
            still = []
            for s, req, start in self.busy:
                if s.poll():
                    ok, K = s.finish()
                    retried = False
                    if not ok:
                        self.retries += 1
                        retried = True
                        old = s.nbytes
                        s.rerun(req, K)
                        self.mem_used += s.nbytes - old
                        self.peak_bytes = max(self.peak_bytes, self.mem_used)
                    end = self.clock() - t0
                    results.append(Result(req.rid, req.key, req.arrival, start, end, req.pixels, retried,
                                          s.image_copy() if keep_images else None,
                                          s.counts() if hasattr(s, "counts") else None))
                    self.release(s)
                    progressed = True
                else:
                    still.append((s, req, start))
            self.busy = still
            if not progressed:
                if not self.busy and not queue and pending:
                    self.sleep(max(0.0, min(pending[0].arrival - (self.clock() - t0), 1e-3)))
                else:
                    self.sleep(poll_sleep)
        wall = max(r.end for r in results) - min(r.arrival for r in results) if results else 0.0
        return results, summarize(results, max(wall, 1e-9), self.retries - retries0, self.peak_slots,
                                  self.peak_bytes, self.evictions - evictions0, peak_inflight)


# ---------------------------------------------------------------------------
# GPU slots
# ---------------------------------------------------------------------------

def _round16(n: int) -> int:
    return (n + 15) // 16 * 16


class RenderSlot:
    """Buffers, device camera, stream and captured graph of one (scene, W, H) key."""

    def __init__(self, server, key, capacity: int):
        import torch

        from . import native, pipeline

        self.torch, self.native, self.pipeline = torch, native, pipeline
        self.server = server
        self.key = key
        scene_id, W, H = key
        self.splats = server.scenes[scene_id]
        self.n = int(self.splats["means"].shape[1])
        self.W, self.H = W, H
        self.stream = torch.cuda.Stream()
        self.cam_dev = torch.zeros(_round16(native.CAMERA_NBYTES), dtype=torch.uint8, device="cuda")
        self.cam_host = torch.zeros(_round16(native.CAMERA_NBYTES), dtype=torch.uint8, pin_memory=True)
        self.ovf_host = torch.zeros(4, dtype=torch.int32, pin_memory=True)
        self.k_host = torch.zeros(2, dtype=torch.int64, pin_memory=True)
        self.done = torch.cuda.Event()
        self._alloc(capacity)

    def _alloc(self, capacity: int):
        torch, pipeline = self.torch, self.pipeline
        self.graph = None
        self.frame = None
        self.frame = pipeline.alloc_frame(self.n, self.W, self.H, capacity, "cuda", dcolor=False)
        self.nbytes = self.server.slot_bytes(self.n, self.W, self.H, capacity)
        self._capture()

    def _enqueue(self):
        native, fr, srv = self.native, self.frame, self.server
        native.darb_preprocess_cam_dev(self.cam_dev, self.W, self.H, srv.kernel, self.n, self.splats, fr.proj)
        native.darb_bin_sort(fr.proj, self.n, self.W, self.H, fr.capacity, fr.ws, None, fr.vals, fr.ranges, fr.k_dev,
                             fr.overflow)
        native.darb_raster_fwd(fr.proj, self.n, fr.vals, fr.ranges, fr.overflow, self.W, self.H, srv.kernel, srv.opts,
                               fr.image, fr.final_T, fr.last, None)

    def _capture(self):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            self._enqueue()  # warm-up outside the graph
        self.stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=self.stream):
            self._enqueue()
        self.graph = g

    def _write_camera(self, cam: dict):
        b = np.frombuffer(self.native.camera_bytes(cam), dtype=np.uint8)
        self.cam_host.numpy()[: len(b)] = b

    def launch(self, req: Request):
        torch = self.torch
        self._write_camera(req.camera)
        with torch.cuda.stream(self.stream):
            self.cam_dev.copy_(self.cam_host, non_blocking=True)
            self.graph.replay()
            self.ovf_host[0:1].copy_(self.frame.overflow[0:1], non_blocking=True)
            self.k_host.copy_(self.frame.k_dev[0:2], non_blocking=True)
            self.done.record(self.stream)

    def poll(self) -> bool:
        return self.done.query()

    def finish(self):
        return int(self.ovf_host[0]) == 0, int(self.k_host[0])

    def counts(self):
        """(K, N_v) of the last completed render."""
        return int(self.k_host[0]), int(self.k_host[1])

    def rerun(self, req: Request, K: int):
        """Capacity overflow: grow, re-capture, render again (blocking)."""
        self.server.cap_hint[self.key] = max(self.server.cap_hint.get(self.key, 0), K)
        self._alloc(int(K * self.server.k_margin) + 4096)
        self.launch(req)
        self.done.synchronize()

    def image_copy(self):
        # copied on the slot's stream, so the slot's next replay cannot overwrite
        # the image before the copy has read it; returned ready to use
        with self.torch.cuda.stream(self.stream):
            img = self.frame.image.clone()
        self.stream.synchronize()
        return img

    def free(self):
        self.graph = None
        self.frame = None


class RenderServer:
    """Scenes resident on the GPU + a :class:`Scheduler` of :class:`RenderSlot`s."""

    def __init__(self, scenes: list, kernel, opts: dict | None = None, mem_budget: int = 24 << 30,
                 max_slots: int = 8, k_margin: float = 1.5, n_probe: int = 4, max_inflight: int | None = None):
        from . import pipeline

        self.scenes = scenes
        self.kernel = kernel
        self.opts = opts or pipeline.DEFAULT_OPTS
        self.k_margin = k_margin
        self.n_probe = n_probe
        self.cap_hint = {}
        self.sched = Scheduler(self._make_slot, self._need, mem_budget, max_slots, max_inflight=max_inflight)

    @staticmethod
    def slot_bytes(n: int, W: int, H: int, capacity: int) -> int:
        from . import native

        return (native.darb_bin_sort_workspace(n, W, H, capacity) + 4 * capacity + 52 * n
                + (3 + 1 + 1) * 4 * W * H + 8 * ((W + 15) // 16) * ((H + 15) // 16))

    def _capacity(self, key) -> int:
        if key not in self.cap_hint:
            # sizing renders of a few poses of this key (blocking readback of K)
            import torch

            from . import pipeline

            scene_id, W, H = key
            sp = self.scenes[scene_id]
            K = 0
            fr = None
            for cam in self._probe_cameras(W, H, self.n_probe):
                fr = pipeline.render(sp, cam, self.kernel, self.opts, frame=fr, k_capacity=1 << 16)
                K = max(K, int(fr.K))
            # the last raster pass may still run: finish it before its buffers go back
            # to the allocator, where a slot on another stream could pick them up
            torch.cuda.current_stream().synchronize()
            del fr
            self.cap_hint[key] = K
        return int(self.cap_hint[key] * self.k_margin) + 4096

    @staticmethod
    def _probe_cameras(W: int, H: int, n: int) -> list:
        from . import scenes

        rng = np.random.Generator(np.random.PCG64(W * 7919 + H))
        return [scenes.orbit_camera(rng, W, H) for _ in range(n)]

    def _need(self, key) -> int:
        scene_id, W, H = key
        n = int(self.scenes[scene_id]["means"].shape[1])
        return self.slot_bytes(n, W, H, self._capacity(key))

    def _make_slot(self, key, _hint):
        return RenderSlot(self, key, self._capacity(key))

    def serve(self, requests, keep_images: bool = False):
        return self.sched.run(requests, keep_images=keep_images)


def sequential_baseline(server: RenderServer, requests, keep_images: bool = False):
    """One request at a time: the server's own slots and graphs (no new captures
    once warm), a single request in flight."""
    sched = server.sched
    saved = sched.max_inflight
    sched.max_inflight = 1
    try:
        return sched.run(requests, keep_images=keep_images)
    finally:
        sched.max_inflight = saved


def make_requests(seed: int, n: int, rate_hz: float, n_scenes: int) -> list:
    from . import scenes

    return [Request(i, r["arrival"], r["scene"], r["camera"])
            for i, r in enumerate(scenes.serving_requests(seed, n, rate_hz, n_scenes))]
