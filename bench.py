"""Benchmark: forward + backward of the DARBF rasterizer on one MI355X.

Workload: the scene-scale view -- 3M clustered splats (SH degree 3), one
1297x840 view, half-cosine DARBF (psi = 1.36, xi = 18/pi).  One step is the
whole hot path over that view with inputs resident in HBM:
preprocess -> bin/sort -> raster forward -> raster backward -> preprocess
backward.  The upstream gradient dL/dimage (mean-L1 to a random target) is
formed once before timing.  Prints one JSON line (metric: Mpix/s).

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--kernel half_cos]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# An estimate of VALU lane-operations per (pixel, splat) pair -- E (5
# FMA), the support and alpha tests, one transcendental, the 3 colour FMAs and
# the T update in the forward; the backward adds the T recovery division, the 9
# partial sums and the reduction.  Used only when no committed counter summary
# (VALU instructions per launch) matches the raster sources.
LANE_OPS_PER_PAIR_FWD = 25
LANE_OPS_PER_PAIR_BWD = 60
PEAK_HBM_GBS = 8000.0            # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3         # MI355X FP32 vector, packed FMA (2 flops x 2 lanes per lane-op)
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # the same without packed FP32 (how every kernel here is built)
PEAK_LANE_OPS = 39.3e12          # 256 CU x 64 lanes x 2.4 GHz: VALU lane-operations per second


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measure_ceilings(reps: int = 5):
    """Measured ceilings of this GPU (best of ``reps`` after a warm-up, HIP
    events): a 1 GiB copy (2 GiB moved) and a 1 GiB fill -- the library's probes
    and torch's elementwise kernels, the faster of the two -- and FMA chains in
    FP32 (non-packed, as every kernel is built) and FP64 (the library's probe)."""
    import torch

    from paper_2501_12369_amd import native

    def best(fn):
        fn()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b) * 1e-3)
        return min(ts)
    n = 1 << 28  # floats: 1 GiB
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    t_copy = best(lambda: native.darb_probe_copy(src, dst))
    t_fill = best(lambda: native.darb_probe_fill(dst))
    # torch's own elementwise kernels as a second opinion: the ceiling is the faster
    t_neg = best(lambda: torch.neg(src, out=dst))
    t_zero = best(lambda: dst.zero_())
    del src, dst
    lanes, iters = 1 << 21, 1024
    out32 = torch.empty(lanes, device="cuda")
    out64 = torch.empty(lanes, dtype=torch.float64, device="cuda")
    chains = native.darb_probe_fma(out32, iters)
    t32 = best(lambda: native.darb_probe_fma(out32, iters))
    t64 = best(lambda: native.darb_probe_fma(out64, iters))
    flops = 2.0 * chains * iters * lanes
    props = torch.cuda.get_device_properties(0)
    copy = dict(probe=round(8.0 * n / t_copy / 1e9, 1), torch_neg=round(8.0 * n / t_neg / 1e9, 1))
    fill = dict(probe=round(4.0 * n / t_fill / 1e9, 1), torch_zero=round(4.0 * n / t_zero / 1e9, 1))
    return dict(copy_gbs=max(copy.values()), fill_gbs=max(fill.values()), copy_detail=copy, fill_detail=fill,
                fma32_tflops=round(flops / t32 / 1e12, 2), fma64_tflops=round(flops / t64 / 1e12, 2),
                device=getattr(props, "name", ""), compute_units=int(props.multi_processor_count),
                arch=getattr(props, "gcnArchName", ""))


def algorithmic_bytes(n, n_vis, K, P, pairs, split=False):
    """Algorithmic bytes per stage by per-unit counts of what the method must
    move (one read of each needed input, one write of each output; the sort as
    one read + write pass of K keys and values):
      a1 preprocess        12 N + 224 N_v + 48 N_v + 4 N
      a2 duplicate         20 N_v + 12 K
      a3 sort              24 K
      a4 raster forward    40 K_trav + 20 P
      a5 raster backward   76 K_trav + 32 P
      a6 preprocess bwd    308 N_v + 236 N
    With the preprocess in two launches (split=True) a1 is divided between them
    by what each moves of it: the geometry part reads the mean and cull data of
    every splat (16 N) and scale, quaternion and opacity (32 B) of each visible
    one, and writes the geometric 36 B of its record (xy, conic and opacity,
    depth, radius, tile box); the colour part reads the 48 SH coefficients
    (192 B) and writes the colour (12 B) of each visible splat:
      geometry 16 N + 68 N_v,  colour 204 N_v  (together a1's 16 N + 272 N_v).
    K_trav, the instances a tile list traverses, is taken as the pairs up to each
    pixel's last blend divided by the 256 pixels of a tile."""
    k_trav = pairs / 256.0
    d = dict(preprocess=16 * n + 272 * n_vis, bin_sort=20 * n_vis + 36 * K, raster_fwd=40 * k_trav + 20 * P,
             raster_bwd=76 * k_trav + 32 * P, preprocess_bwd=308 * n_vis + 236 * n)
    if split:
        d.update(preprocess=16 * n + 68 * n_vis, colour=204 * n_vis)
    return d


def stage_bytes(n, n_vis, split=False):
    """The kernels' own algorithmic HBM bytes per launch of the single-kernel
    stages (one read of each input it needs, one write of each output), per
    splat / per visible splat:
      preprocess      12 B mean + 4 B cull data of every splat; 224 B of parameters
                      (scale, quaternion, opacity, 48 SH) read and 48 B of projected
                      record written per visible splat; the 36 B colour checkpoint
                      (d colour / d direction) and the 8 B tile box written for
                      every splat:                                60 N + 272 N_v
      split in two launches (split=True), the stage is the geometry part: mean,
      scale, quaternion and opacity read (44 B), xy, depth, radius, tile box and
      conic_o written (40 B), for every splat:                    84 N
      and the colour part beside the binning reads the radius (4 B) of every splat
      and the mean and 48 SH (204 B) of each visible one, and writes rgb, clamp
      bits and the colour checkpoint (49 B) of every splat:       53 N + 204 N_v
      preprocess_bwd  the radius (4 B) of every splat; per visible splat 113 B read
                      (mean 12, scale 12, quaternion 16, 2D gradients 36, colour
                      checkpoint 36 + clamp bits 1); the full gradient written for
                      every splat (236 B):                        113 N_v + 240 N
    """
    if split:
        return dict(preprocess=84 * n, colour=53 * n + 204 * n_vis, preprocess_bwd=113 * n_vis + 240 * n)
    return dict(preprocess=60 * n + 272 * n_vis, preprocess_bwd=113 * n_vis + 240 * n)


# kernel of each single-kernel stage, and the sources it is built from
STAGE_KERNEL = {"preprocess": ("k_preprocess<3>", ("preprocess.hip", "common.h")),
                "colour": ("k_preprocess_colour<3>", ("preprocess.hip", "common.h")),
                "preprocess_bwd": ("k_preprocess_bwd<3, true>", ("preprocess.hip", "common.h"))}


def sources_digest(files) -> str:
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2501_12369_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


# raster kernels' VALU work: the committed counter summary (profiles/valu.json)
# holds SQ_INSTS_VALU per dispatch of the scene step's full-size call
RASTER_KERNEL = {"raster_fwd": ("k_raster_fwd<1, OneView, false>", ("raster.hip", "common.h")),
                 "raster_bwd": ("k_raster_bwd_split<1, OneView>", ("raster.hip", "common.h"))}


def measured_valu_insts(stage: str):
    """Wave-level VALU instructions of the stage's kernel per launch, from the
    committed rocprofv3 counter summary, or None when its sources changed since."""
    path = os.path.join(ROOT, "profiles", "valu.json")
    if not os.path.exists(path):
        return None
    name, files = RASTER_KERNEL[stage]
    with open(path) as fh:
        rec = json.load(fh).get(name)
    if not rec or rec.get("sources_sha256") != sources_digest(files):
        return None
    return int(rec["valu_insts"])


def measured_traffic(stage: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (profiles/traffic.json), or None when the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    name, files = STAGE_KERNEL.get(stage) or RASTER_KERNEL[stage]
    with open(path) as fh:
        rec = json.load(fh).get(name)
    if not rec or rec.get("sources_sha256") != sources_digest(files):
        return None
    return int(rec["fetch_bytes"] + rec["write_bytes"])


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_oracle_run(sc, kernel_name, rows_every: int, threads: int, log_fn=log):
    """The FP64 oracle (as is) on a bounded sample of the scene step on ``threads``
    host threads: preprocess and its backward over all splats, composite
    forward+backward over every ``rows_every``-th image row; the per-pixel time
    is scaled to the full view.  Returns (Mpix/s, sample text, seconds)."""
    import oracle
    from paper_2501_12369_amd import scenes

    oracle.set_num_threads(threads)
    sp, camd = sc["splats"], sc["camera"]
    W, H = camd["width"], camd["height"]
    f32 = lambda v: float(np.float32(v))
    presets = {"half_cos": (oracle.HALF_COS, 18.0 / np.pi, 1.36), "gauss": (oracle.GAUSS, 2.0, 1.0)}
    kind, xi, psi = presets[kernel_name]
    k = oracle.KernelSpec(kind, f32(xi), f32(psi), 9.0)
    cam = oracle.camera_from_scene(camd)
    opts = oracle.make_opts(f32(1 / 255), f32(0.99), f32(1e-4))
    rows = np.arange(0, H, rows_every)
    ys, xs = np.meshgrid(rows, np.arange(W), indexing="ij")
    pix = np.stack([xs.ravel(), ys.ravel()], 1).astype(np.int32)
    G = scenes.upstream_grad(99, W, H).transpose(1, 2, 0).reshape(-1, 3)
    Gs = G[pix[:, 1] * W + pix[:, 0]].astype(np.float64)
    t0 = time.perf_counter()
    proj = oracle.preprocess(cam, k, sp["means"], sp["scales"], sp["quats"], sp["sh"], sp["sh_degree"])
    t1 = time.perf_counter()
    oracle.composite(proj, sp["opacity"], k, opts, W, H, pix=pix)
    t2 = time.perf_counter()
    g2d = oracle.composite_bwd(proj, sp["opacity"], k, opts, W, H, Gs, pix=pix)
    t3 = time.perf_counter()
    oracle.preprocess_bwd(cam, k, sp["means"], sp["scales"], sp["quats"], sp["sh"], sp["sh_degree"], g2d)
    t4 = time.perf_counter()
    frac = len(pix) / (W * H)
    total = (t1 - t0) + (t4 - t3) + (t3 - t1) / frac
    log_fn(f"cpu oracle on {threads} threads: preprocess {t1-t0:.2f}s composite {t2-t1:.2f}s composite_bwd "
           f"{t3-t2:.2f}s preprocess_bwd {t4-t3:.2f}s on {len(pix)} px; full-view estimate {total:.1f}s")
    sample = (f"FP64 oracle: preprocess + preprocess backward over all {sp['means'].shape[1]} splats, composite "
              f"forward + backward over every {rows_every}th row ({len(pix)} of {W*H} pixels); per-pixel time "
              f"scaled to the full view; measured {t4 - t0:.1f}s")
    return W * H / total / 1e6, sample, t4 - t0


def cpu_baseline(sc, kernel_name, rows_every: int, log_fn=log):
    """The oracle on all host threads (the reported baseline) and on one thread
    (a sparser row sample), with the host CPU named."""
    import oracle

    all_threads = oracle.num_threads()
    v, sample, _ = cpu_oracle_run(sc, kernel_name, rows_every, all_threads, log_fn)
    v1, sample1, _ = cpu_oracle_run(sc, kernel_name, rows_every * 8, 1, log_fn)
    oracle.set_num_threads(all_threads)
    model = cpu_model()
    log_fn(f"cpu: {model}; oracle {v:.5f} Mpix/s on {all_threads} threads, {v1:.5f} Mpix/s on 1 thread")
    return dict(value=round(v, 6), unit="Mpix/s", cores=all_threads, kind="oracle", sample=sample, cpu_model=model,
                one_core=dict(value=round(v1, 6), unit="Mpix/s", cores=1, sample=sample1))


def serving_bench(kernel_name: str, seconds: float, rate_hz: float, mem_budget_gb: float, max_slots: int,
                  max_batch: int = 4, sweep=(100.0, 200.0, 400.0, 800.0, 1600.0, 2400.0, 3200.0),
                  sweep_seconds: float = 2.0,
                  slo_p99_ms: float = 10.0):
    """Forward-only serving of Poisson requests over four resident scenes, with
    requests of one (scene, resolution) batched into multi-view graph replays;
    a sweep of arrival rates (p50/p99, Mpix/s and the forward's HBM fraction at
    each), the highest rate whose p99 meets ``slo_p99_ms``, and the same
    requests one at a time through the same slots."""
    import torch

    from paper_2501_12369_amd import pipeline, scenes, serving

    t0 = time.time()
    sc = [pipeline.splats_to_device(scenes.scene_splats(41 + i, n))
          for i, n in enumerate(scenes.SERVING_SCENE_SIZES)]
    log(f"serving scenes generated in {time.time() - t0:.1f}s")
    kern = pipeline.KERNELS[kernel_name]
    srv = serving.RenderServer(sc, kern, mem_budget=int(mem_budget_gb * (1 << 30)), max_slots=max_slots,
                               max_batch=max_batch)
    # warm-up: every (scene, resolution) key sized and captured before the measured
    # sessions, with two slots per key (two requests of a key at once, one per
    # launch), so that the first overlaps of a key do not allocate and capture a
    # slot inside a timed session
    warm = []
    rng = np.random.Generator(np.random.PCG64(1234))
    for s in range(len(sc)):
        for (w, h) in scenes.SERVING_RESOLUTIONS:
            for _ in range(2):
                warm.append(serving.Request(len(warm), 0.0, s, scenes.orbit_camera(rng, w, h)))
    srv.sched.batch_limit = 1
    srv.serve(warm)
    srv.sched.batch_limit = None
    torch.cuda.synchronize()
    sizes = list(scenes.SERVING_SCENE_SIZES)

    def fwd_bytes(results):
        """Algorithmic forward bytes (preprocess 16 N + 272 N_v, duplicate 20 N_v + 12 K,
        sort 24 K, image 20 P; the traversed-record reads of the raster are left out:
        a lower bound)."""
        tot = 0
        for r in results:
            K, nv = r.work
            tot += 16 * sizes[r.key[0]] + 292 * nv + 36 * K + 20 * r.pixels
        return tot

    def point(res, st):
        hbm = fwd_bytes(res) / st.wall_s / 1e9
        return dict(p50_ms=round(st.p50_ms, 3), p99_ms=round(st.p99_ms, 3), mean_ms=round(st.mean_ms, 3),
                    mpix_per_s=round(st.mpix_per_s, 2), req_per_s=round(st.req_per_s, 2), requests=st.n,
                    fwd_gbs=round(hbm, 1), hbm_frac=round(hbm / PEAK_HBM_GBS, 4), peak_batch=st.extra["peak_batch"],
                    peak_inflight=st.peak_inflight, retries=st.retries)

    n_req = max(1, int(seconds * rate_hz))
    reqs = serving.make_requests(77, n_req, rate_hz, len(sc))
    res, st = srv.serve(reqs)
    main_pt = point(res, st)
    log(f"serving: {st.n} requests at {rate_hz}/s: p50 {st.p50_ms:.2f} ms p99 {st.p99_ms:.2f} ms, "
        f"{st.mpix_per_s:.1f} Mpix/s, {main_pt['fwd_gbs']:.0f} GB/s of forward bytes, peak batch "
        f"{main_pt['peak_batch']}, peak slots {st.peak_slots}, peak in flight {st.peak_inflight}, retries {st.retries}")
    sweep_pts = []
    for i, rate in enumerate(sweep):
        rq = serving.make_requests(500 + i, max(16, int(sweep_seconds * rate)), rate, len(sc))
        pt = dict(rate_hz=rate, **point(*srv.serve(rq)))
        sweep_pts.append(pt)
        log(f"  sweep {rate:7.0f} req/s: p50 {pt['p50_ms']:.2f} p99 {pt['p99_ms']:.2f} ms, {pt['mpix_per_s']:.0f} "
            f"Mpix/s, {pt['fwd_gbs']:.0f} GB/s ({pt['hbm_frac']:.3f} of HBM), peak batch {pt['peak_batch']}")
    meets = [p for p in sweep_pts if p["p99_ms"] <= slo_p99_ms]
    best = max(meets, key=lambda p: p["rate_hz"]) if meets else None
    # saturation: a burst of the same mix arriving at once (a first, untimed burst
    # creates the slots that many requests of one key in flight need)
    srv.serve(serving.make_requests(79, max(64, n_req // 2), 1e9, len(sc)))
    torch.cuda.synchronize()
    burst = serving.make_requests(78, max(64, n_req // 2), 1e9, len(sc))
    sat = point(*srv.serve(burst))
    log(f"saturation: {sat['requests']} requests at once: {sat['mpix_per_s']:.1f} Mpix/s, {sat['req_per_s']:.1f} "
        f"req/s, {sat['fwd_gbs']:.0f} GB/s of forward bytes ({sat['hbm_frac']:.3f} of HBM peak)")
    seq_res, seq = serving.sequential_baseline(srv, reqs)
    log(f"one-at-a-time: p50 {seq.p50_ms:.2f} ms p99 {seq.p99_ms:.2f} ms, {seq.mpix_per_s:.1f} Mpix/s")
    bseq = point(*serving.sequential_baseline(srv, burst))
    log(f"one-at-a-time saturation: {bseq['mpix_per_s']:.1f} Mpix/s, {bseq['req_per_s']:.1f} req/s")
    return dict(workload=f"4 resident scenes {sizes} splats, Poisson {rate_hz} req/s for {seconds}s, resolutions "
                         f"{[f'{w}x{h}' for w, h in scenes.SERVING_RESOLUTIONS]}, forward only, {kernel_name}, "
                         f"batches of up to {max_batch} requests per graph replay",
                **main_pt, peak_slots=st.peak_slots, peak_gb=round(st.peak_bytes / 2**30, 2),
                rate_sweep=sweep_pts, slo_p99_ms=slo_p99_ms,
                max_rate_meeting_slo=best["rate_hz"] if best else None,
                at_max_rate=best, saturation=sat,
                one_at_a_time=dict(p50_ms=round(seq.p50_ms, 3), p99_ms=round(seq.p99_ms, 3),
                                   mpix_per_s=round(seq.mpix_per_s, 2), saturation_mpix_per_s=bseq["mpix_per_s"],
                                   saturation_req_per_s=bseq["req_per_s"]))


def variants_bench(spd, cam, steps: int, warmup: int):
    """The scene step with the Gaussian kernel (plain path), and the half-cosine
    step through the torch.autograd.Function (loss sum(G * image))."""
    import torch

    from paper_2501_12369_amd import native, pipeline
    from paper_2501_12369_amd.autograd import Rasterizer

    n = int(spd["means"].shape[1])
    W, H = cam["width"], cam["height"]
    out = {}
    kern = pipeline.KERNELS["gauss"]
    fr = pipeline.render(spd, cam, kern, k_capacity=1 << 20)
    frame = pipeline.alloc_frame(n, W, H, int(fr.K * 1.02) + 4096, "cuda")
    del fr
    G = torch.randn((3, H, W), device="cuda", generator=torch.Generator("cuda").manual_seed(9)) * 1e-6
    pipeline.render(spd, cam, kern, frame=frame, read_k=True)
    grads = pipeline.alloc_grads(n, 3)

    side = torch.cuda.Stream()

    def plain():
        pipeline.forward_overlapped(spd, cam, kern, frame, side, zero_g2d=grads[0])
        native.darb_raster_bwd(frame.proj, n, frame.vals, frame.ranges, frame.overflow, W, H, kern,
                               pipeline.DEFAULT_OPTS, G, frame.final_T, frame.last, grads[0], g2d_zeroed=True)
        native.darb_preprocess_bwd(cam, kern, n, spd, grads[0], grads[1], proj=frame.proj)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    t_g = timed(plain)
    assert int(frame.overflow[0].item()) == 0
    out["gauss_plain_ms"] = round(t_g * 1e3, 4)
    out["gauss_instances"] = int(frame.K)
    del frame, grads
    R = Rasterizer("half_cos")
    params = [spd[k].clone().requires_grad_(True) for k in ("means", "scales", "quats", "opacity", "sh")]

    def autograd_step():
        for p in params:
            p.grad = None
        img = R(*params, cam, sh_degree=3)
        (img * G).sum().backward()

    t_a = timed(autograd_step)
    out["half_cos_autograd_ms"] = round(t_a * 1e3, 4)
    log(f"variants: gauss plain {t_g*1e3:.3f} ms/step (K={out['gauss_instances']}), "
        f"half_cos autograd {t_a*1e3:.3f} ms/step")
    return out


def small_configs_bench(steps: int, warmup: int, cpu: bool):
    """The tiny (64 splats, 64x64; Gaussian and half-cosine) and object-scale
    (100k splats, 800x800, SH degree 3, half-cosine) workloads: the GPU step
    (preprocess, bin/sort, raster forward and backward, preprocess backward,
    one stream) beside the FP64 oracle on all host threads and on one thread
    (median of three runs each; the object's composite on a row sample, scaled
    to the full view)."""
    import torch

    import oracle
    from paper_2501_12369_amd import native, pipeline, scenes

    rows = []
    for name, sc, kname, every_all, every_one in (("tiny", scenes.tiny(seed=1), "gauss", 1, 1),
                                                  ("tiny", scenes.tiny(seed=1), "half_cos", 1, 1),
                                                  ("object", scenes.object_scale(seed=2), "half_cos", 4, 32)):
        cam, kern = sc["camera"], pipeline.KERNELS[kname]
        W, H = cam["width"], cam["height"]
        spd = pipeline.splats_to_device(sc["splats"])
        n = int(spd["means"].shape[1])
        fr = pipeline.render(spd, cam, kern, k_capacity=max(64 * n, 1 << 16))
        frame = pipeline.alloc_frame(n, W, H, int(fr.K * 1.1) + 4096, "cuda")
        del fr
        K = int(pipeline.render(spd, cam, kern, frame=frame, read_k=True).K)
        G = torch.randn((3, H, W), device="cuda", generator=torch.Generator("cuda").manual_seed(3)) * 1e-4
        grads = pipeline.alloc_grads(n, int(spd["sh_degree"]))

        def step():
            pipeline.render(spd, cam, kern, frame=frame, read_k=False, zero_g2d=grads[0])
            pipeline.render_backward(frame, G, spd, cam, kern, grads=grads, g2d_zeroed=True)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        gpu_s = (time.perf_counter() - t) / steps
        assert int(frame.overflow[0].item()) == 0
        row = dict(config=name, kernel=kname, n_splats=n, width=W, height=H, instances=K,
                   gpu_ms=round(gpu_s * 1e3, 4), gpu_mpix_per_s=round(W * H / gpu_s / 1e6, 2))
        if cpu:
            nt = oracle.num_threads()
            full = [cpu_oracle_run(sc, kname, every_all, nt, log_fn=lambda *a: None) for _ in range(3)]
            one = [cpu_oracle_run(sc, kname, every_one, 1, log_fn=lambda *a: None) for _ in range(3)]
            oracle.set_num_threads(nt)
            v_all = float(np.median([r[0] for r in full]))
            v_one = float(np.median([r[0] for r in one]))
            row.update(cpu_all_mpix_per_s=round(v_all, 5), cpu_threads=nt, cpu_1core_mpix_per_s=round(v_one, 5),
                       cpu_rows_every=(every_all, every_one),
                       gpu_over_cpu_all=round(W * H / gpu_s / 1e6 / v_all, 1))
        rows.append(row)
        log(f"{name} {kname}: GPU {gpu_s*1e3:.3f} ms/step ({row['gpu_mpix_per_s']} Mpix/s, K={row['instances']})"
            + (f"; oracle {row['cpu_all_mpix_per_s']} Mpix/s on {row['cpu_threads']} threads, "
               f"{row['cpu_1core_mpix_per_s']} on 1" if cpu else ""))
        del frame, grads, spd
    return rows


def multiview_bench(kernel_name: str, n: int, n_views: int, steps: int, warmup: int, bin_streams: int = 4):
    """Batched multi-view training step: n clustered splats, n_views views at uneven
    resolutions, mean-L1 loss to random targets.  The multi-view step (one
    preprocess launch, the views' bin/sorts on ``bin_streams`` concurrent
    streams, one fused forward+loss+backward launch
    over all views' tiles, one summed preprocess backward) against the same step
    as single-view calls made view after view."""
    import torch

    from paper_2501_12369_amd import native, pipeline, scenes

    t0 = time.time()
    spd = pipeline.splats_to_device(scenes.scene_splats(5, n))
    cams = scenes.multiview_cameras(5, n_views)
    log(f"multiview scene generated in {time.time() - t0:.1f}s; views "
        + " ".join(f"{c['width']}x{c['height']}" for c in cams))
    kern = pipeline.KERNELS[kernel_name]
    gen = torch.Generator("cuda").manual_seed(11)
    targets = [torch.rand((3, c["height"], c["width"]), device="cuda", generator=gen) for c in cams]
    caps = []
    for c in cams:
        fr = pipeline.render(spd, c, kern, k_capacity=1 << 20)
        caps.append(int(fr.K * 1.05) + 4096)
    del fr
    mf = pipeline.alloc_multiview(n, cams, caps)
    _, g3d = pipeline.alloc_grads(n, int(spd["sh_degree"]))
    pix = sum(c["width"] * c["height"] for c in cams)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        assert not pipeline.multiview_overflowed(mf), "instance capacity overflow during timing"
        return dt

    fused = timed(lambda: pipeline.multiview_step(spd, mf, targets, kern, g3d, fused=True, bin_streams=bin_streams))
    split = timed(lambda: pipeline.multiview_step(spd, mf, targets, kern, g3d, fused=False, bin_streams=bin_streams))
    seq = timed(lambda: pipeline.sequential_step(spd, mf, targets, kern, g3d))
    K = sum(fr.K for fr in mf.frames)
    log(f"multiview {n_views} views, {pix/1e6:.2f} Mpix, K={K}: fused {fused*1e3:.3f} ms, "
        f"multi (separate launches) {split*1e3:.3f} ms, sequential single-view {seq*1e3:.3f} ms")
    sizes = [f"{c['width']}x{c['height']}" for c in cams]
    return dict(workload=f"{n} clustered splats (SH degree 3), {n_views} views at uneven resolutions "
                         f"{sizes}, {kernel_name} DARBF, mean-L1 loss, fwd+bwd training step",
                pixels=pix, instances=int(K),
                bin_streams=bin_streams,
                fused_ms=round(fused * 1e3, 4), multi_ms=round(split * 1e3, 4), sequential_ms=round(seq * 1e3, 4),
                fused_mpix_per_s=round(pix / fused / 1e6, 2), sequential_mpix_per_s=round(pix / seq / 1e6, 2),
                speedup_vs_sequential=round(seq / fused, 3))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--kernel", default="half_cos", choices=["half_cos", "gauss"])
    ap.add_argument("--n", type=int, default=3_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the preprocess as one kernel instead of its colour part beside the binning")
    ap.add_argument("--cpu-rows-every", type=int, default=16)
    ap.add_argument("--small-configs", type=int, default=1, help="0 skips the tiny and object-scale legs")
    ap.add_argument("--serve-seconds", type=float, default=5.0, help="0 disables the serving leg")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-mem-gb", type=float, default=96.0)
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--serve-batch", type=int, default=4, help="requests per multi-view graph replay")
    ap.add_argument("--multiview-views", type=int, default=8, help="0 disables the multi-view leg")
    ap.add_argument("--multiview-n", type=int, default=2_000_000)
    ap.add_argument("--multiview-bin-streams", type=int, default=4,
                    help="concurrent streams for the views' bin/sorts in the multi-view step")
    ap.add_argument("--variants", type=int, default=1, help="0 skips the Gaussian and autograd steps")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run a plain elementwise copy of this size (counter calibration for profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: it has no multi-GPU path (requested --gpus {args.gpus}); "
              f"run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2501_12369_amd import native, pipeline, scenes

    if not torch.cuda.is_available():
        print("no GPU visible: bench.py needs an MI355X", file=sys.stderr)
        sys.exit(3)
    native.lib()  # fails loudly when the HIP library is missing

    t0 = time.time()
    sc = scenes.scene(seed=3, n=args.n)
    log(f"scene generated in {time.time()-t0:.1f}s")
    cam = sc["camera"]
    W, H = cam["width"], cam["height"]
    P = W * H
    kern = pipeline.KERNELS[args.kernel]
    spd = pipeline.splats_to_device(sc["splats"])
    n = args.n

    # sizing pass: K read back once, then every timed step runs without host syncs
    fr = pipeline.render(spd, cam, kern, k_capacity=1)
    K = fr.K
    frame = pipeline.alloc_frame(n, W, H, int(K * 1.02) + 4096, "cuda")
    pipeline.render(spd, cam, kern, frame=frame, read_k=True)
    del fr
    n_vis = int((frame.proj["radius"] > 0).sum())
    target = torch.rand((3, H, W), device="cuda", generator=torch.Generator("cuda").manual_seed(7))
    G = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
    native.darb_image_loss(frame.image, target, W, H, native.LOSS_L1, dL_dimage=G)  # mean-L1 gradient
    grads = pipeline.alloc_grads(n, 3)
    log(f"N={n} visible={n_vis} K={K} tiles={pipeline.n_tiles(W, H)}")

    stages = ["preprocess", "bin_sort", "raster_fwd", "raster_bwd", "preprocess_bwd"]

    # The colour part of the preprocess (SH colour and its checkpoint, most of the
    # stage's bytes) is not an input of the binning: it runs on a second stream
    # (default priority) beside the latency-bound bin/sort kernels and is joined
    # before the raster forward.  Stage "preprocess" is then the geometry part and
    # "bin_sort" ends at the join; "colour" is timed on the side stream.
    overlap = not args.no_overlap
    side = torch.cuda.Stream()
    main = torch.cuda.current_stream()
    if overlap:
        STAGE_KERNEL["preprocess"] = ("k_preprocess_geom", ("preprocess.hip", "common.h"))

    # event points of a step: name -> the stream it is recorded on
    side_points = ("col_start", "col_end")
    # a stage's (first, last) point; "colour" is the side stream's kernel
    spans = {"preprocess": ("start", "pre_end"), "bin_sort": ("pre_end", "bin_end"),
             "bin_sort_own": ("pre_end", "bin_own_end"), "raster_fwd": ("bin_end", "fwd_end"),
             "raster_bwd": ("fwd_end", "bwd_end"), "preprocess_bwd": ("bwd_end", "pbwd_end"),
             "colour": side_points}

    def step(ev=None):
        def mark(name):
            if ev is not None and name in ev:
                ev[name].record(side if name in side_points else main)

        mark("start")
        native.darb_preprocess(cam, kern, n, spd, frame.proj, parts=native.PRE_GEOMETRY if overlap else 3)
        mark("pre_end")
        if overlap:
            side.wait_stream(main)
            mark("col_start")
            native.darb_preprocess(cam, kern, n, spd, frame.proj, parts=native.PRE_COLOUR, stream=side)
            mark("col_end")
        native.darb_bin_sort(frame.proj, n, W, H, frame.capacity, frame.ws, None, frame.vals, frame.ranges,
                             frame.k_dev, frame.overflow)
        mark("bin_own_end")  # the binning's own end, before the join
        if overlap:
            main.wait_stream(side)
        mark("bin_end")
        native.darb_raster_fwd(frame.proj, n, frame.vals, frame.ranges, frame.overflow, W, H, kern,
                               pipeline.DEFAULT_OPTS, frame.image, frame.final_T, frame.last, zero_g2d=grads[0])
        mark("fwd_end")
        native.darb_raster_bwd(frame.proj, n, frame.vals, frame.ranges, frame.overflow, W, H, kern,
                               pipeline.DEFAULT_OPTS, G, frame.final_T, frame.last, grads[0], g2d_zeroed=True)
        mark("bwd_end")
        native.darb_preprocess_bwd(cam, kern, n, spd, grads[0], grads[1], proj=frame.proj)
        mark("pbwd_end")

    def new_events(points):
        return [{p: torch.cuda.Event(enable_timing=True) for p in points} for _ in range(args.steps)]

    def span_ms(evs, stage):
        a, b = spans[stage]
        return float(np.mean([e[a].elapsed_time(e[b]) for e in evs]))

    for _ in range(args.warmup):
        step()
    # Stage breakdown: K steps with events at every stage boundary (each event
    # recorded between two kernels costs the stream a few microseconds, ~37 us per
    # step in all, so these steps are not the timed ones).
    all_points = [p for pair in spans.values() for p in pair]
    evs = new_events(set(all_points) if overlap else set(all_points) - set(side_points))
    torch.cuda.synchronize()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    per_stage = {s: span_ms(evs, s) for s in stages}
    colour_ms = span_ms(evs, "colour") if overlap else None
    bin_own_ms = span_ms(evs, "bin_sort_own")
    # the dominant kernel: the longest single kernel of the step, the colour part
    # on the side stream included (the bin/sort stage is ~20 launches, none of
    # them longer than these)
    single = ["preprocess", "raster_fwd", "raster_bwd", "preprocess_bwd"] + (["colour"] if overlap else [])
    stage_time = dict(per_stage, colour=colour_ms)
    dom_stage = max(single, key=lambda st: stage_time[st])
    # The timed steps: events only around the dominant kernel, on its stream.
    evd = new_events(spans[dom_stage])
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(evd[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    assert int(frame.overflow[0].item()) == 0, "instance capacity overflow during timing"
    dom_ms = span_ms(evd, dom_stage)
    ms_per_step = wall * 1e3 / args.steps
    mpix = P * args.steps / wall / 1e6
    log("per-stage ms (steps with stage events): " + ", ".join(f"{k}={v:.3f}" for k, v in per_stage.items()) +
        f"; timed step {ms_per_step:.3f} ms (events around {dom_stage} only: {dom_ms:.3f} ms)")
    log(f"bin/sort kernels on the main stream: {bin_own_ms:.3f} ms (stage to the join {per_stage['bin_sort']:.3f})")
    if overlap:
        log(f"colour part on the side stream (beside bin_sort): {colour_ms:.3f} ms, "
            f"{stage_bytes(n, n_vis, True)['colour'] / (colour_ms * 1e-3) / 1e9:.1f} GB/s")

    # pairs up to each pixel's last blended splat (the backward walks exactly these;
    # the forward at least these), from the checkpoint
    last = frame.last.to(torch.int64) & 0xFFFFFFFF
    ranges = frame.ranges.to(torch.int64)
    gx = (W + 15) // 16
    yy, xx = torch.meshgrid(torch.arange(H, device="cuda"), torch.arange(W, device="cuda"), indexing="ij")
    tile = (yy // 16) * gx + (xx // 16)
    start = ranges[tile, 0]
    has = last != 0xFFFFFFFF
    pairs = int(torch.where(has, last - start + 1, torch.zeros_like(last)).sum())
    own = stage_bytes(n, n_vis, overlap)
    svy = algorithmic_bytes(n, n_vis, K, P, pairs, overlap)
    ceilings = measure_ceilings()
    log("measured ceilings: " + ", ".join(f"{k}={v}" for k, v in ceilings.items()))

    def hbm(stage, t_ms, kernel, own_bytes=None):
        b = svy.get(stage, own_bytes)
        r = dict(bound="hbm", kernel=kernel, us=round(t_ms * 1e3, 2), algorithmic_bytes=int(b),
                 achieved=round(b / (t_ms * 1e-3) / 1e9, 2), peak=PEAK_HBM_GBS, unit="GB/s")
        r["frac"] = round(r["achieved"] / PEAK_HBM_GBS, 4)
        r["frac_of_measured"] = round(r["achieved"] / ceilings["copy_gbs"], 4)
        if own_bytes is not None and stage in svy:
            r["own_bytes"] = int(own_bytes)
            r["own_frac"] = round(own_bytes / (t_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
        return r

    def valu(stage, t_ms, kernel, ops_per_pair):
        # counted VALU lane-operations (VALU instructions x 64 lanes) when the
        # committed counter summary matches the sources, else the
        # per-pair estimate
        insts = measured_valu_insts(stage)
        if insts is not None:
            ops, rule = insts * 64, "counted: SQ_INSTS_VALU x 64 (profiles/valu.json)"
        else:
            ops, rule = pairs * ops_per_pair, f"estimated: {ops_per_pair} lane-ops per pair"
        rate = ops / (t_ms * 1e-3)
        return dict(bound="alu", kernel=kernel, us=round(t_ms * 1e3, 2), pairs=pairs, lane_ops=int(ops),
                    lane_ops_rule=rule, lane_ops_per_pair=round(ops / max(pairs, 1), 2),
                    achieved=round(2 * rate / 1e12, 2), unit="TFLOP/s (FMA-equivalent: 2 x lane-ops)",
                    peak=PEAK_FP32_NONPACKED_TFLOPS, frac=round(rate / PEAK_LANE_OPS, 4),
                    frac_of_packed=round(2 * rate / 1e12 / PEAK_FP32_TFLOPS, 4),
                    frac_of_measured=round(2 * rate / 1e12 / ceilings["fma32_tflops"], 4))

    pre_kernel = "k_preprocess_geom" if overlap else "k_preprocess<3>"
    stage_roofs = {
        "preprocess": hbm("preprocess", per_stage["preprocess"], pre_kernel, own["preprocess"]),
        "bin_sort": hbm("bin_sort", per_stage["bin_sort"], "20 launches (keys .. level-2 scatter), to the join"),
        "bin_sort_own": hbm("bin_sort", bin_own_ms, "20 launches (keys .. level-2 scatter), own time"),
        "raster_fwd": valu("raster_fwd", per_stage["raster_fwd"], "k_raster_fwd<1, OneView, false>",
                           LANE_OPS_PER_PAIR_FWD),
        "raster_bwd": valu("raster_bwd", per_stage["raster_bwd"], "k_raster_bwd_split<1, OneView>",
                           LANE_OPS_PER_PAIR_BWD),
        "preprocess_bwd": hbm("preprocess_bwd", per_stage["preprocess_bwd"], "k_preprocess_bwd<3, true>",
                              own["preprocess_bwd"]),
    }
    if overlap:
        stage_roofs["colour_side_stream"] = hbm("colour", colour_ms, "k_preprocess_colour<3>", own["colour"])
    # the dominant kernel's figures from the timed steps' own events
    if dom_stage == "colour":
        r = hbm("colour", dom_ms, "k_preprocess_colour<3>", own["colour"])
    elif dom_stage in ("raster_fwd", "raster_bwd"):
        r = valu(dom_stage, dom_ms, stage_roofs[dom_stage]["kernel"],
                 LANE_OPS_PER_PAIR_FWD if dom_stage == "raster_fwd" else LANE_OPS_PER_PAIR_BWD)
    else:
        r = hbm(dom_stage, dom_ms, stage_roofs[dom_stage]["kernel"], own[dom_stage])
    traffic = measured_traffic(dom_stage)
    if r["bound"] == "hbm":
        roofline = dict(bound="hbm", achieved=r["achieved"], peak=PEAK_HBM_GBS, unit="GB/s", frac=r["frac"],
                        traffic=traffic, kernel=r["kernel"], kernel_us=r["us"],
                        algorithmic_bytes=r["algorithmic_bytes"], bytes_rule="per-unit algorithmic counts",
                        own_bytes=r.get("own_bytes"), own_frac=r.get("own_frac"),
                        measured_peak=ceilings["copy_gbs"], frac_of_measured=r["frac_of_measured"])
    else:
        roofline = dict(bound="alu", achieved=r["achieved"], peak=PEAK_FP32_NONPACKED_TFLOPS,
                        unit="TFLOP/s", frac=r["frac"], traffic=traffic, kernel=r["kernel"], kernel_us=r["us"],
                        pairs=pairs, frac_of_packed=r["frac_of_packed"], measured_peak=ceilings["fma32_tflops"],
                        frac_of_measured=r["frac_of_measured"])
    step_bytes = sum(svy.values())
    step_roof = dict(algorithmic_bytes=int(step_bytes), achieved=round(step_bytes / (ms_per_step * 1e-3) / 1e9, 2),
                     frac=round(step_bytes / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS, 4))
    ranked = sorted(stage_roofs, key=lambda st: -stage_roofs[st]["us"])
    log("stages by time: " + "; ".join(f"{st} {stage_roofs[st]['us']} us {stage_roofs[st]['achieved']} "
                                      f"{stage_roofs[st]['unit'].split(' ')[0]} (frac {stage_roofs[st]['frac']})"
                                      for st in ranked))
    log(f"dominant kernel {roofline['kernel']}: {roofline['kernel_us']} us, {roofline['achieved']} {roofline['unit']} "
        f"({roofline['frac']:.3f} of peak, {roofline['frac_of_measured']:.3f} of the measured ceiling), "
        f"traffic {traffic}; whole step {step_roof['achieved']} GB/s ({step_roof['frac']:.3f})")

    if args.calibrate_copy_mib > 0:
        # a plain elementwise copy of known size: what the HBM counters read for it
        # calibrates the per-kernel FETCH_SIZE / WRITE_SIZE of a counter run
        xc = torch.ones(args.calibrate_copy_mib << 18, device="cuda")
        yc = torch.empty_like(xc)
        for _ in range(3):
            torch.neg(xc, out=yc)
        torch.cuda.synchronize()
        del xc, yc

    variants = variants_bench(spd, cam, args.steps, args.warmup) if args.variants else None
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(sc, args.kernel, args.cpu_rows_every)
        # the same view with the Gaussian profile (the oracle on all threads)
        import oracle

        other = "gauss" if args.kernel == "half_cos" else "half_cos"
        v, sample, _ = cpu_oracle_run(sc, other, args.cpu_rows_every, oracle.num_threads())
        cpu["other_kernel"] = dict(kernel=other, value=round(v, 6), unit="Mpix/s", cores=oracle.num_threads(),
                                   sample=sample)
    small = small_configs_bench(max(10, args.steps), 3, not args.no_cpu_baseline) if args.small_configs else None
    del frame, grads, spd
    torch.cuda.empty_cache()
    multiview_stats = None
    if args.multiview_views > 0:
        multiview_stats = multiview_bench(args.kernel, args.multiview_n, args.multiview_views, max(3, args.steps // 2),
                                          2, bin_streams=args.multiview_bin_streams)
        torch.cuda.empty_cache()
    serving_stats = None
    if args.serve_seconds > 0:
        serving_stats = serving_bench(args.kernel, args.serve_seconds, args.serve_rate, args.serve_mem_gb,
                                      args.serve_slots, args.serve_batch)

    out = {
        "metric": "fwd+bwd Mpix/s at 3M splats 1297x840; serving p50/p99 render latency",
        "value": round(mpix, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"scene: {n} clustered splats (SH degree 3), one {W}x{H} view, {args.kernel} DARBF, "
                               f"preprocess+bin/sort+raster fwd+raster bwd+preprocess bwd",
                   "n_splats": n, "width": W, "height": H, "kernel": args.kernel, "visible": n_vis, "instances": K,
                   "splats_per_s": round(n * args.steps / wall, 1),
                   "stage_ms": {k: round(v, 4) for k, v in per_stage.items()},
                   "timing": "timed steps carry events around the dominant kernel only; stage_ms from as many "
                             "further steps with events at every stage boundary",
                   "colour_side_stream_ms": round(colour_ms, 4) if overlap else None,
                   "bin_sort_own_ms": round(bin_own_ms, 4), "variants": variants},
        "roofline": roofline,
        "measured_ceilings": ceilings,
        "stage_rooflines": stage_roofs,
        "step_roofline": step_roof,
        "cpu_baseline": cpu,
        "small_configs": small,
        "multiview": multiview_stats,
        "serving": serving_stats,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
