"""Continuous-batching render server (forward only) over libdarb.

Scenes stay resident in HBM.  Requests of one (scene, W, H) key are batched:
a *render slot* holds the buffers of up to B views of its key, a device array
of B cameras, a stream, and one captured HIP graph per batch size b = 1..B of
the multi-view forward -- one preprocess launch over the b views (cameras read
from the device array) -> a bin/sort per view (no host readback) -> one raster
launch over the tiles of all b views.  A replay renders every request of the
batch; an image in a batch has the bits of the same request rendered alone
(every launch is atomic-free and per view).

Admission is by memory: the oldest waiting request starts when an idle slot of
its key exists, or when a new slot fits in the memory budget (idle slots of
other keys are freed, least recently used first, to make room), and takes up
to B-1 more waiting requests of its key into the same replay; otherwise it
waits, first in first out.  Requests that arrive while others run are admitted
as slots and memory free up, and the graphs of several slots run concurrently
on separate streams.  The instance count K is decided on the device before any
instance is written, so a too-small capacity only sets a flag; the server
checks it at completion, grows the slot, re-captures its graphs and renders
that batch again.

The scheduling core (:class:`Scheduler`) takes a slot factory, so the policy can
be exercised without a GPU.
"""
from __future__ import annotations

import gc
import math
import time
import weakref
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
    """FIFO admission by memory over slots made by ``factory``, with batching.

    ``factory(key, capacity_hint)`` returns a slot with attributes ``key``,
    ``nbytes``, ``max_batch`` (requests per launch, optional: 1) and methods
    ``launch(requests)`` (a list of 1..max_batch requests of the slot's key),
    ``poll() -> bool`` (finished), ``finish() -> (ok, K)`` (ok False when a
    capacity overflowed; then K is the largest count needed),
    ``rerun(requests, K)`` (blocking re-render with room for K),
    ``image_copy(i)`` (image of the i-th request of the batch) and ``free()``.
    ``need(key)`` estimates a new slot's bytes.
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
        self.peak_batch = 0
        self.batch_limit = None  # cap on requests per launch (None: each slot's max_batch)

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
        # no cyclic garbage collection while requests are timed (a full collection
        # over the process's tensors stalls the loop for milliseconds); it runs
        # once the run is over
        enabled = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests, keep_images, poll_sleep)
        finally:
            if enabled:
                gc.enable()

    def _run(self, requests, keep_images: bool, poll_sleep: float):
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue = deque()
        results = []
        # statistics of this run only
        retries0, evictions0 = self.retries, self.evictions
        self.peak_slots, self.peak_bytes = self.n_slots, self.mem_used
        self.peak_batch = 0
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
            while i < min(len(queue), self.lookahead) and sum(len(b) for _, b, _ in self.busy) < self.max_inflight:
                r = queue[i]
                s = None if r.key in blocked else self.acquire(r)
                if s is None:
                    blocked.add(r.key)
                    i += 1
                    continue
                del queue[i]
                batch = [r]
                # continuous batching: waiting requests of the same key join the launch
                j = i
                limit = getattr(s, "max_batch", 1)
                if self.batch_limit is not None:
                    limit = min(limit, self.batch_limit)
                while len(batch) < limit and j < min(len(queue), self.lookahead):
                    if queue[j].key == r.key:
                        batch.append(queue[j])
                        del queue[j]
                    else:
                        j += 1
                s.launch(batch)
                self.busy.append((s, batch, self.clock() - t0))
                peak_inflight = max(peak_inflight, sum(len(b) for _, b, _ in self.busy))
                self.peak_batch = max(self.peak_batch, len(batch))
                progressed = True
            still = []
            for s, batch, start in self.busy:
                if s.poll():
                    ok, K = s.finish()
                    retried = False
                    if not ok:
                        self.retries += 1
                        retried = True
                        old = s.nbytes
                        s.rerun(batch, K)
                        self.mem_used += s.nbytes - old
                        self.peak_bytes = max(self.peak_bytes, self.mem_used)
                    end = self.clock() - t0
                    for q, req in enumerate(batch):
                        results.append(Result(req.rid, req.key, req.arrival, start, end, req.pixels, retried,
                                              s.image_copy(q) if keep_images else None,
                                              s.counts(q) if hasattr(s, "counts") else None))
                    self.release(s)
                    progressed = True
                else:
                    still.append((s, batch, start))
            self.busy = still
            if not progressed:
                if not self.busy and not queue and pending:
                    self.sleep(max(0.0, min(pending[0].arrival - (self.clock() - t0), 1e-3)))
                else:
                    self.sleep(poll_sleep)
        wall = max(r.end for r in results) - min(r.arrival for r in results) if results else 0.0
        st = summarize(results, max(wall, 1e-9), self.retries - retries0, self.peak_slots, self.peak_bytes,
                       self.evictions - evictions0, peak_inflight)
        st.extra["peak_batch"] = self.peak_batch
        return results, st


# ---------------------------------------------------------------------------
# GPU slots
# ---------------------------------------------------------------------------

def _round16(n: int) -> int:
    return (n + 15) // 16 * 16


class RenderSlot:
    """Buffers of up to ``max_batch`` views of one (scene, W, H) key, a device
    array of their cameras, a stream, and a captured graph per batch size."""

    def __init__(self, server, key, capacity: int):
        import torch

        from . import native, pipeline

        self.torch, self.native, self.pipeline = torch, native, pipeline
        # the server owns its slots: a weak reference keeps the pair out of a
        # reference cycle, so a dropped server frees its graphs, streams and
        # buffers at once instead of whenever the cyclic collector runs
        self.server = weakref.proxy(server)
        self.key = key
        scene_id, W, H = key
        self.splats = server.scenes[scene_id]
        self.n = int(self.splats["means"].shape[1])
        self.W, self.H = W, H
        self.max_batch = server.max_batch
        B = self.max_batch
        self.stream = torch.cuda.Stream()
        cb = native.CAMERA_NBYTES  # a multiple of 16: the array keeps every camera aligned
        self.cams_dev = torch.zeros(B * cb, dtype=torch.uint8, device="cuda")
        self.cams_host = torch.zeros(B * cb, dtype=torch.uint8, pin_memory=True)
        self.ovf_dev = torch.zeros((B, 4), dtype=torch.int32, device="cuda")
        self.k_dev = torch.zeros((B, 2), dtype=torch.int64, device="cuda")
        self.ovf_host = torch.zeros((B, 4), dtype=torch.int32, pin_memory=True)
        self.k_host = torch.zeros((B, 2), dtype=torch.int64, pin_memory=True)
        # a valid camera of this size for the host-side checks (the device cameras are used)
        self.template = server.probe_camera(W, H)
        self.done = torch.cuda.Event()
        self.batch = 0
        self._alloc(capacity)

    def _alloc(self, capacity: int):
        pipeline = self.pipeline
        self.graphs = None
        self.frames = None
        # the batch's bin/sorts run one after another on the slot's stream: one workspace
        first = pipeline.alloc_frame(self.n, self.W, self.H, capacity, "cuda", dcolor=False)
        self.frames = [first] + [pipeline.alloc_frame(self.n, self.W, self.H, capacity, "cuda", dcolor=False,
                                                      ws=first.ws) for _ in range(self.max_batch - 1)]
        for v, fr in enumerate(self.frames):  # per-view flags and counts in the slot's own arrays
            fr.overflow = self.ovf_dev[v]
            fr.k_dev = self.k_dev[v]
        self.views = [dict(cam=self.template, proj=fr.proj, k_capacity=fr.capacity, vals=fr.vals, ranges=fr.ranges,
                           overflow_dev=fr.overflow, image=fr.image, final_T=fr.final_T, last=fr.last)
                      for fr in self.frames]
        self.nbytes = self.server.slot_bytes(self.n, self.W, self.H, capacity, self.max_batch)
        self._capture()

    def _enqueue(self, b: int):
        native, srv = self.native, self.server
        native.darb_preprocess_multi_cam_dev(self.views[:b], self.cams_dev, srv.kernel, self.n, self.splats)
        for fr in self.frames[:b]:
            native.darb_bin_sort(fr.proj, self.n, self.W, self.H, fr.capacity, fr.ws, None, fr.vals, fr.ranges,
                                 fr.k_dev, fr.overflow)
        native.darb_raster_fwd_multi(self.views[:b], self.n, srv.kernel, srv.opts)

    def _capture(self):
        torch = self.torch
        self._write_cameras([self.template] * self.max_batch)
        self.cams_dev.copy_(self.cams_host)
        graphs = {}
        for b in range(1, self.max_batch + 1):
            with torch.cuda.stream(self.stream):
                self._enqueue(b)  # warm-up outside the graph
            self.stream.synchronize()
            g = torch.cuda.CUDAGraph()
            # no cyclic collection inside the capture: a finalizer that destroys a
            # graph, event or stream, or frees device memory, is rejected while a
            # stream captures (torch.cuda.graph collects once before it begins)
            enabled = gc.isenabled()
            gc.disable()
            try:
                with torch.cuda.graph(g, stream=self.stream):
                    self._enqueue(b)
            finally:
                if enabled:
                    gc.enable()
            graphs[b] = g
        self.graphs = graphs

    def _write_cameras(self, cams: list):
        cb = self.native.CAMERA_NBYTES
        host = self.cams_host.numpy()
        for v, cam in enumerate(cams):
            host[v * cb:(v + 1) * cb] = np.frombuffer(self.native.camera_bytes(cam), dtype=np.uint8)

    def launch(self, reqs: list):
        torch = self.torch
        b = len(reqs)
        self.batch = b
        self._write_cameras([r.camera for r in reqs])
        with torch.cuda.stream(self.stream):
            self.cams_dev.copy_(self.cams_host, non_blocking=True)
            self.graphs[b].replay()
            self.ovf_host.copy_(self.ovf_dev, non_blocking=True)
            self.k_host.copy_(self.k_dev, non_blocking=True)
            self.done.record(self.stream)

    def poll(self) -> bool:
        return self.done.query()

    def finish(self):
        b = self.batch
        ok = all(int(self.ovf_host[v, 0]) == 0 for v in range(b))
        return ok, max(int(self.k_host[v, 0]) for v in range(b))

    def counts(self, i: int = 0):
        """(K, N_v) of the i-th render of the last completed batch."""
        return int(self.k_host[i, 0]), int(self.k_host[i, 1])

    def rerun(self, reqs: list, K: int):
        """Capacity overflow: grow, re-capture, render the batch again (blocking)."""
        self.server.cap_hint[self.key] = max(self.server.cap_hint.get(self.key, 0), K)
        self._alloc(int(K * self.server.k_margin) + 4096)
        self.launch(reqs)
        self.done.synchronize()

    def image_copy(self, i: int = 0):
        # copied on the slot's stream, so the slot's next replay cannot overwrite
        # the image before the copy has read it; returned ready to use
        with self.torch.cuda.stream(self.stream):
            img = self.frames[i].image.clone()
        self.stream.synchronize()
        return img

    def free(self):
        self.graphs = None
        self.frames = None
        self.views = None


class RenderServer:
    """Scenes resident on the GPU + a :class:`Scheduler` of :class:`RenderSlot`s."""

    def __init__(self, scenes: list, kernel, opts: dict | None = None, mem_budget: int = 24 << 30,
                 max_slots: int = 8, k_margin: float = 2.0, n_probe: int = 16, max_inflight: int | None = None,
                 max_batch: int = 4):
        from . import pipeline

        if not 1 <= max_batch <= 16:
            raise ValueError("max_batch must be in [1, 16] (views per multi-view launch)")
        self.scenes = scenes
        self.kernel = kernel
        self.max_batch = int(max_batch)
        self.opts = opts or pipeline.DEFAULT_OPTS
        self.k_margin = k_margin
        self.n_probe = n_probe
        self.cap_hint = {}
        me = weakref.ref(self)  # the scheduler calls back without holding the server (no reference cycle)
        self.sched = Scheduler(lambda key, hint: me()._make_slot(key, hint), lambda key: me()._need(key), mem_budget,
                               max_slots, max_inflight=max_inflight)

    @staticmethod
    def slot_bytes(n: int, W: int, H: int, capacity: int, views: int = 1) -> int:
        """Device bytes of a slot of ``views`` renders sharing one bin/sort workspace."""
        from . import native

        return (native.darb_bin_sort_workspace(n, W, H, capacity) + views * (
            4 * capacity + 52 * n + (3 + 1 + 1) * 4 * W * H + 8 * ((W + 15) // 16) * ((H + 15) // 16)))

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

    def probe_camera(self, W: int, H: int) -> dict:
        return self._probe_cameras(W, H, 1)[0]

    def _need(self, key) -> int:
        scene_id, W, H = key
        n = int(self.scenes[scene_id]["means"].shape[1])
        return self.slot_bytes(n, W, H, self._capacity(key), self.max_batch)

    def _make_slot(self, key, _hint):
        return RenderSlot(self, key, self._capacity(key))

    def serve(self, requests, keep_images: bool = False):
        return self.sched.run(requests, keep_images=keep_images)


def sequential_baseline(server: RenderServer, requests, keep_images: bool = False):
    """One request at a time: the server's own slots and graphs (the batch-of-one
    graph, no new captures once warm), a single request in flight."""
    sched = server.sched
    saved = sched.max_inflight, sched.batch_limit
    sched.max_inflight, sched.batch_limit = 1, 1
    try:
        return sched.run(requests, keep_images=keep_images)
    finally:
        sched.max_inflight, sched.batch_limit = saved


def make_requests(seed: int, n: int, rate_hz: float, n_scenes: int) -> list:
    from . import scenes

    return [Request(i, r["arrival"], r["scene"], r["camera"])
            for i, r in enumerate(scenes.serving_requests(seed, n, rate_hz, n_scenes))]
