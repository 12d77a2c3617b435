"""Benchmark: Mrays/s on the 1920x1080 four-primitive teaser scene on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-batch] [--no-served] [--no-c3] [--no-next] [--served-seconds S]
                    [--only c3|c4|c5] [--compact N]

One step = one full frame of the teaser workload: 1920x1080, 1 sample per
pixel, two pac-men + quaternion Julia + power-8 Mandelbulb, 256 march steps,
eps 1e-4, primary + shadow rays + one mirror bounce (with its shadow ray),
rendered by ``pr_render`` on one stream with inputs resident in HBM.

Printed JSON line (rank 0): the metric value is total rays launched per
second (primary, shadow, bounce and bounce-shadow, counted by the
instrumented build on the same frame); ``roofline`` reports the algorithmic
FP32 work of the tracing kernel -- estimator evaluations and fractal
iterations counted per launch times a fixed per-evaluation flop table
(below) -- over its average duration measured with HIP events on the launch
stream; ``cpu_baseline`` times the FP64 oracle on a bounded pixel sample.
Sub-objects time C3 (1024 instances, 4 spp) and the batched form (64 requests
in one persistent launch vs 64 plain launches), each with its own roofline;
the served form (a 2 s warm-up, then a 30 s open-loop Poisson trace at
200 req/s and at 100 req/s, server vs FIFO plain launches, and what the GPU
sustains on that request mix as back-to-back batches); and the next-step
workloads: the sample scene with its triangle plane, the cut Julia set, the
Mandelbulb animation, and the teaser with its pac-men as a user hit group.
``--only c3|c4|c5`` times just that workload (for profiling).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector peak (256 CU x 2.4 GHz x 256 flop/clk)
METRIC = "Mrays/s (primary+shadow) 1080p 4-primitive scene; p50/p99 latency served"

# ---------------------------------------------------------------------------
# Algorithmic flop table: flops of the minimal formula per estimator
# evaluation (add/sub/mul/min/max = 1, FMA = 2, sqrt/rsqrt/div/log = 1,
# abs free), split into a per-evaluation base and a per-executed-iteration
# part for the fractals.  Every sphere-tracing step adds STEP_FLOPS for the
# march point o' + t d' (6), the world scaling sigma * DE (1) and t += v (1).
DE_BASE = {0: 7, 1: 19, 2: 10, 3: 50, 4: 18, 5: 12, 6: 10}
DE_ITER = {0: 0, 1: 0, 2: 0, 3: 0, 4: 0, 5: 19, 6: 52}
STEP_FLOPS = 8
NODE_FLOPS = 50        # visited interior node: two child slab tests + ordering
CLIP_FLOPS = 60        # candidate: local transform (33) + local slab clip (27)
RAYGEN_FLOPS = 60      # camera basis + jitter-free direction + normalisation
SHADE_FLOPS = 70       # normal mapping, light vector, Lambert, secondary-ray setup


def algorithmic_flops(counts: np.ndarray) -> float:
    c = counts.astype(np.float64)
    f = 0.0
    for t in range(7):
        f += c[t] * (DE_BASE[t] + STEP_FLOPS) + c[7 + t] * DE_ITER[t]
        f += c[14 + t] * DE_BASE[t] + c[21 + t] * DE_ITER[t]
    normals = c[14:21].sum() / 6.0
    f += c[32] * NODE_FLOPS + c[33] * CLIP_FLOPS + c[28] * RAYGEN_FLOPS + normals * SHADE_FLOPS
    return f


def ray_breakdown(counts):
    return dict(primary=int(counts[28]), shadow=int(counts[29]), bounce=int(counts[30]),
                bounce_shadow=int(counts[31]))


def cpu_baseline():
    """The FP64 oracle over the full 1080p teaser frame on the host cores.

    P worker processes, P = the cores this process may run on, at most 16
    (one GPU's share of the host cores).  The frame is split into 4P equal pixel chunks; the one-core rate is
    one more chunk of the same size traced in this process (the same fixed
    set-up cost per chunk as in the pool)."""
    import multiprocessing as mp
    import workloads as W
    affinity = len(os.sched_getaffinity(0))
    cores = max(1, min(16, affinity))
    pix = np.arange(1920 * 1080, dtype=np.int64)
    chunks = np.array_split(pix, cores * 4)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_chunk, chunks)
    wall = time.perf_counter() - t0
    rays = sum(sum(r["rays"].values()) for r in res)
    # one core: a chunk of the pool's size from a different part of the frame
    one = W.pixel_sample(1920, 1080, chunks[0].size, seed=103)
    t0 = time.perf_counter()
    r1 = _oracle_chunk(one)
    one_core = sum(r1["rays"].values()) / (time.perf_counter() - t0) / 1e6
    return {"value": rays / wall / 1e6, "unit": "Mrays/s", "cores": cores, "kind": "oracle",
            "sample": f"the full 1920x1080 teaser frame ({rays} rays: primary, shadow, bounce, "
                      f"bounce-shadow), FP64 NumPy oracle in {cores} processes over {len(chunks)} "
                      f"chunks of {chunks[0].size} pixels, {wall:.1f} s wall",
            "one_core_value": round(one_core, 4),
            "one_core_sample": f"{one.size} seeded pixels of the same frame in one process",
            "affinity_cores": affinity, "cpu_model": _cpu_model()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_chunk(pix):
    import workloads as W
    from oracle import tracer as T
    wl = W.c2()
    req = wl.requests[0]
    out = T.render(wl.scenes[0], req.camera, req.opts, pixels=pix)
    return {"rays": out["counts"]["rays"]}


# the kernel and the host code that sets its launch (grid, burst budget, tile
# order, request records)
KERNEL_SOURCES = ["paper_2012_10357_amd/csrc/trace.hip", "paper_2012_10357_amd/csrc/de.h",
                  "paper_2012_10357_amd/csrc/internal.h", "paper_2012_10357_amd/csrc/render.cpp"]
TRAFFIC_PROFILE = "profiles/trace_kernel_teaser_1080p_pmc.md"
C3_PROFILE = "profiles/trace_kernel_c3_1080p_4spp_pmc.md"
C4_PROFILE = "profiles/trace_kernel_c4_batch_64req_pmc.md"
C5_PROFILE = "profiles/trace_kernel_c5_served_mix_pmc.md"


def kernel_source_hash() -> str:
    """sha256 (16 hex digits) over the kernel sources with comments and
    whitespace removed: the counters depend on the code, not on its comments."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, f), encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def committed_counters(profile=None):
    """Machine-readable figures of a committed counter profile (HBM bytes
    per launch, VALU issue utilisation, active-lane fraction), if it was taken
    on the current kernel source (else an empty dict).  Default: the teaser's."""
    path = os.path.join(ROOT, profile or TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return {}
    fields = {}
    for line in open(path):
        k, sep, v = line.partition(":")
        if sep and k.strip() in ("kernel_source_sha256", "traffic_bytes_per_launch",
                                 "valu_issue_utilisation", "active_lane_fraction"):
            fields[k.strip()] = v.strip()
    if fields.pop("kernel_source_sha256", None) != kernel_source_hash():
        return {}
    out = {}
    for k, v in fields.items():
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


def committed_traffic():
    """HBM bytes per launch from the committed counter profile, if it was taken
    on the current kernel source (else None)."""
    return committed_counters().get("traffic_bytes_per_launch")


def bench_batched(P, W, torch, dev, reps=5, compare=True):
    """64 requests over the teaser scene: one persistent launch (graph-captured,
    autotuned) vs one plain pr_render launch per request, same stream.
    compare=False times the batched launch alone, with the tuned-or-default
    launch settings and no autotuning (for profiling)."""
    wl = W.c4()
    sc = P.Scene(wl.scenes[0])
    outs = [torch.empty((r.opts.height, r.opts.width, 3), dtype=torch.float32, device=dev)
            for r in wl.requests]
    rays, flops = 0, 0.0
    for r, o in zip(wl.requests, outs):
        c = P.render_counts(sc, r.camera, r.opts, o)
        rays += int(c[28:32].sum())
        flops += algorithmic_flops(c)
    reqs = P.make_requests([(sc, r.camera, r.opts, o, None, None, i)
                            for i, (r, o) in enumerate(zip(wl.requests, outs))])
    best = P.autotune(reqs) if compare else P.BatchOpts(0, 0, 0, 0, 0)
    stream = torch.cuda.Stream(device=dev)

    def run(fn):
        with torch.cuda.stream(stream):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def plain():
        for r, o in zip(wl.requests, outs):
            P.render(sc, r.camera, r.opts, o, stream=stream)

    def batched():
        P.render_batch(reqs, tile=(best.tile_w, best.tile_h), step_budget=best.step_budget,
                       use_graph=True, stream=stream, compact=best.compact_pct)

    t_plain = run(plain) if compare else float("nan")
    t_batch = run(batched)
    # kernel time of the batched launch alone (HIP events on its stream)
    with torch.cuda.stream(stream):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            batched()
        b.record(stream)
    torch.cuda.synchronize()
    k_ms = a.elapsed_time(b) / reps
    sc.close()
    return {"requests": len(wl.requests), "rays_per_batch": rays,
            "roofline": roofline_of(flops, k_ms, "trace_kernel (one persistent launch, graph replay)",
                                    profile=C4_PROFILE),
            "batched_mrays_s": round(rays / t_batch / 1e6, 2), "batched_ms": round(t_batch * 1e3, 3),
            "plain_mrays_s": round(rays / t_plain / 1e6, 2), "plain_ms": round(t_plain * 1e3, 3),
            "speedup": round(t_plain / t_batch, 3),
            "tuned": {"tile": [best.tile_w, best.tile_h], "step_budget": best.step_budget,
                      "regrouping": ("off" if best.compact_pct == P.PR_COMPACT_NEVER
                                     else f"{best.compact_pct} %")}}


def _frame_rate(P, torch, dev, sc, cam, opts, reps=5):
    """Rays, algorithmic flops and mean kernel time of one frame."""
    rgb = torch.empty((opts.height, opts.width, 3), dtype=torch.float32, device=dev)
    counts = P.render_counts(sc, cam, opts, rgb)
    rays = int(sum(ray_breakdown(counts).values()))
    flops = algorithmic_flops(counts)
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        P.render(sc, cam, opts, rgb, stream=stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            P.render(sc, cam, opts, rgb, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return {"ms": round(ms, 3), "mrays_s": round(rays / ms / 1e3, 1),
            "tflops": round(float(flops) / ms / 1e9, 3), "rays": rays}


def bench_next(P, W, torch, dev):
    """The next-step features at 1080p: the sample scene with its triangle
    plane, the Julia set cut by each plane, and the twelve-frame step-budget
    animation of the Mandelbulb rendered as one batched launch."""
    out = {}
    wl = W.f2_sample()
    sc = P.Scene(wl.scenes[0])
    out["sample_scene_plane_1080p"] = _frame_rate(P, torch, dev, sc, wl.requests[0].camera, wl.requests[0].opts)
    sc.close()
    wl = W.f1_julia_cut(1920, 1080)
    for k, r in enumerate(wl.requests):
        sc = P.Scene(wl.scenes[r.scene_index])
        out[f"julia_cut{k}_1080p"] = _frame_rate(P, torch, dev, sc, r.camera, r.opts)
        sc.close()
    wl = W.f1_mandelbulb_anim(1024, 1024)
    sc = P.Scene(wl.scenes[0])
    outs = [torch.empty((r.opts.height, r.opts.width, 3), dtype=torch.float32, device=dev) for r in wl.requests]
    rays = 0
    for r, o in zip(wl.requests, outs):
        rays += int(sum(ray_breakdown(P.render_counts(sc, r.camera, r.opts, o)).values()))
    reqs = P.make_requests([(sc, r.camera, r.opts, o, None, None, i) for i, (r, o) in enumerate(zip(wl.requests, outs))])
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        P.render_batch(reqs, use_graph=True, stream=stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(3):
            P.render_batch(reqs, use_graph=True, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / 3
    out["mandelbulb_animation_12x1024sq_batched"] = {"ms": round(ms, 3), "frames_s": round(12e3 / ms, 1),
                                                     "mrays_s": round(rays / ms / 1e3, 1), "rays": rays}
    sc.close()
    return out


# A programmable hit group over the teaser frame: the two pac-men as a user
# type whose estimator and closest-hit function are HIP C++ source compiled
# into the trace kernel at run time (parameters R, cos a, sin a of the wedge
# half-angle a), shaded by a restated Lambert term.
F3_PACMAN_BODY = """
  const R ca = (R)p[1], sa = (R)p[2];
  const R len = sqrt(x * x + y * y + z * z);
  const R qy = fabs(y);
  const R qn = ca * qy - sa * x, qu = ca * x + sa * qy;
  const R w = (qn > (R)0 && qu < (R)0) ? sqrt(x * x + qy * qy) : qn;
  return fmax(len - (R)p[0], -w);
"""
F3_LAMBERT_BODY = """
  const float lam = fmaxf(0.f, nx * lx + ny * ly + nz * lz);
  for (int c = 0; c < 3; ++c) rgb[c] = albedo[c] * (ambient + lit * lam * light_rgb[c]);
"""


def f3_scene(W, gtype):
    """The teaser scene with its pac-man geometry given as the user type."""
    import dataclasses
    s = W.c2_scene()
    sel = s.geom_type == W.PACMAN
    prm = s.geom_params.copy()
    half = prm[sel, 1].astype(np.float64)
    prm[sel, 1] = np.cos(half)
    prm[sel, 2] = np.sin(half)
    return dataclasses.replace(s, geom_type=np.where(sel, np.uint32(gtype), s.geom_type).astype(np.uint32),
                               geom_params=prm)


def bench_f3(P, W, torch, dev):
    """The teaser frame with its pac-men as a user hit group, beside the same
    frame with the built-in pac-man, timed alike (kernel time per frame)."""
    base = P.Scene(W.c2_scene())
    builtin = _frame_rate(P, torch, dev, base, W.c2_camera(), W.c2_opts())
    base.close()
    t0 = time.monotonic()
    gtype = P.register_estimator("bench_user_pacman", F3_PACMAN_BODY)
    P.register_closest_hit(gtype, F3_LAMBERT_BODY)
    sc = P.Scene(f3_scene(W, gtype))
    rgb = torch.empty((1080, 1920, 3), dtype=torch.float32, device=dev)
    P.render(sc, W.c2_camera(), W.c2_opts(), rgb)      # builds the kernel with the user code
    torch.cuda.synchronize()
    build_s = time.monotonic() - t0
    user = _frame_rate(P, torch, dev, sc, W.c2_camera(), W.c2_opts())
    sc.close()
    return {"ms": user["ms"], "mrays_s": user["mrays_s"], "rays": user["rays"],
            "builtin_ms": builtin["ms"], "builtin_rays": builtin["rays"], "first_build_s": round(build_s, 1)}


def bench_served(P, W, torch, dev, seconds, rate_hz=200.0, warmup_s=2.0):
    """Open-loop Poisson trace over 8 resident scenes (256..4096 instances,
    sides 256..2048, 1..4 spp): requests arrive for warmup_s + seconds; those
    arriving in the first warmup_s are served but not measured.  The
    continuous-batching server against FIFO per-request pr_render launches on
    the same arrival trace.  Latency = completion (the device flag seen by the
    host for the server; the stream synchronised for FIFO) minus the scheduled
    arrival; throughput = rays of the measured requests over the window from
    the first measured arrival to the last measured completion."""
    import threading
    scenes = [P.Scene(s) for s in W.c5_scenes()]
    n_req = max(20, int(rate_hz * (seconds + warmup_s)))
    reqs = W.c5_requests(n_req, rate_hz=rate_hz)
    measured = np.array([r.arrival_s >= warmup_s for r in reqs])
    prim = np.array([r.opts.width * r.opts.height * r.opts.spp for r in reqs], np.float64)

    # --- server
    srv = P.Server(16 << 30, max_inflight=4, max_batch=64, use_graph=False)
    for sc_ in scenes:
        srv.add_scene(sc_)
    tickets = [None] * n_req
    t_base = time.monotonic() + 0.2
    sub_err = []

    def submitter():
        try:
            for i, r in enumerate(reqs):
                dt = t_base + r.arrival_s - time.monotonic()
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = srv.submit(scenes[r.scene_index], r.camera, r.opts, tag=i)
        except Exception as e:   # surfaced below
            sub_err.append(e)

    th = threading.Thread(target=submitter)
    th.start()
    lat = np.zeros(n_req)
    done = np.zeros(n_req)
    shadow = np.zeros(n_req)
    for i in range(n_req):
        while tickets[i] is None and th.is_alive():
            time.sleep(0.0005)
        if tickets[i] is None:
            break
        res = srv.wait(tickets[i], 600000)
        lat[i] = res.t_done - (t_base + reqs[i].arrival_s)
        done[i] = res.t_done - t_base
        shadow[i] = res.rays_shadow
        srv.release(tickets[i])
    th.join()
    if sub_err:
        raise sub_err[0]
    stats = srv.stats()
    srv.close()
    t0 = min(r.arrival_s for r, m in zip(reqs, measured) if m)
    span = float(done[measured].max()) - t0
    served = {"p50_ms": round(float(np.percentile(lat[measured], 50)) * 1e3, 2),
              "p99_ms": round(float(np.percentile(lat[measured], 99)) * 1e3, 2),
              "primary_mrays_s": round(prim[measured].sum() / span / 1e6, 2),
              "primary_shadow_mrays_s": round((prim[measured].sum() + shadow[measured].sum()) / span / 1e6, 2),
              "launches": int(stats.launches)}

    # --- FIFO baseline: one pr_render per request in arrival order, synchronised
    stream = torch.cuda.Stream(device=dev)
    lat_f = np.zeros(n_req)
    done_f = np.zeros(n_req)
    buf = {}
    t_base = time.monotonic() + 0.2
    with torch.cuda.stream(stream):
        for i, r in enumerate(reqs):
            dt = t_base + r.arrival_s - time.monotonic()
            if dt > 0:
                time.sleep(dt)
            key = (r.opts.height, r.opts.width)
            if key not in buf:
                buf[key] = torch.empty((r.opts.height, r.opts.width, 3), dtype=torch.float32, device=dev)
            P.render(scenes[r.scene_index], r.camera, r.opts, buf[key], stream=stream)
            stream.synchronize()
            done_f[i] = time.monotonic() - t_base
            lat_f[i] = done_f[i] - r.arrival_s
    for sc_ in scenes:
        sc_.close()
    span_f = float(done_f[measured].max()) - t0
    fifo = {"p50_ms": round(float(np.percentile(lat_f[measured], 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat_f[measured], 99)) * 1e3, 2),
            "primary_mrays_s": round(prim[measured].sum() / span_f / 1e6, 2)}
    return {"requests": n_req, "measured": int(measured.sum()), "rate_hz": rate_hz, "warmup_s": warmup_s,
            "trace_s": round(reqs[-1].arrival_s, 2), "offered_primary_mrays_s":
                round(prim[measured].sum() / (reqs[-1].arrival_s - t0) / 1e6, 1),
            "server": served, "fifo_plain": fifo}


def bench_served_ceiling(P, W, torch, dev, n_req=480, batch=120, counts=True, plain=True):
    """What the GPU sustains on the served request mix: the first n_req
    requests of the 200 req/s trace rendered back to back as batches of
    ``batch`` requests on one stream (no arrivals, no admission), against
    one plain pr_render per request.  With ``counts`` the roofline of a batch
    launch: algorithmic flops from the instrumented build run on every
    request (the per-ray work does not depend on the batch), over the batch
    launches' mean duration from HIP events on the launch stream."""
    scenes = [P.Scene(s) for s in W.c5_scenes()]
    reqs = W.c5_requests(n_req, rate_hz=200.0)
    prim = float(sum(r.opts.width * r.opts.height * r.opts.spp for r in reqs))
    outs = [torch.empty((r.opts.height, r.opts.width, 3), dtype=torch.float32, device=dev) for r in reqs]
    flops = 0.0
    rays = None
    if counts:
        for r, o in zip(reqs, outs):
            c = P.render_counts(scenes[r.scene_index], r.camera, r.opts, o)
            flops += algorithmic_flops(c)
            rays = c[28:32].astype(np.float64) if rays is None else rays + c[28:32]
    items = [(scenes[r.scene_index], r.camera, r.opts, o, None, None, i)
             for i, (r, o) in enumerate(zip(reqs, outs))]
    batches = [P.make_requests(items[i:i + batch]) for i in range(0, n_req, batch)]
    stream = torch.cuda.Stream(device=dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in batches]
    with torch.cuda.stream(stream):
        P.render_batch(batches[0], stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (a, b), bt in zip(ev, batches):
            a.record(stream)
            P.render_batch(bt, stream=stream)
            b.record(stream)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        t_plain = None
        if plain:
            t0 = time.perf_counter()
            for r, o in zip(reqs, outs):
                P.render(scenes[r.scene_index], r.camera, r.opts, o, stream=stream)
            torch.cuda.synchronize()
            t_plain = time.perf_counter() - t0
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    for sc_ in scenes:
        sc_.close()
    out = {"requests": n_req, "batch": batch, "primary_rays": int(prim),
           "batched_primary_mrays_s": round(prim / t_batch / 1e6, 1)}
    if t_plain is not None:
        out["plain_primary_mrays_s"] = round(prim / t_plain / 1e6, 1)
    if counts:
        out["rays"] = dict(primary=int(rays[0]), shadow=int(rays[1]), bounce=int(rays[2]),
                           bounce_shadow=int(rays[3]))
        out["roofline"] = roofline_of(flops / len(batches), launch_ms,
                                      f"trace_kernel (one launch of {batch} served requests)",
                                      profile=C5_PROFILE)
    return out


def roofline_of(flops, kernel_ms, name, profile=None, **extra):
    """FP32 roofline of one launch; HBM traffic, VALU issue utilisation and
    active-lane fraction from the workload's committed counter profile when
    it was taken on the current kernel source (else null)."""
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    c = committed_counters(profile) if profile else {}
    out = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
           "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": c.get("traffic_bytes_per_launch"),
           "kernel": name, "kernel_ms": round(kernel_ms, 4), "flops_per_launch": float(flops),
           "valu_issue_frac": c.get("valu_issue_utilisation"), "active_lane_frac": c.get("active_lane_fraction")}
    out.update(extra)
    return out


def bench_c3(P, W, torch, dev, reps=5, compact=0):
    """C3: 1080p, 4 jittered samples, 1024 instances of five types, SAH BVH,
    shadows: rays and algorithmic flops from the instrumented build, kernel
    time from HIP events around reps launches on the launch stream."""
    wl = W.c3()
    sc = P.Scene(wl.scenes[0])
    r = wl.requests[0]
    rgb = torch.empty((r.opts.height, r.opts.width, 3), dtype=torch.float32, device=dev)
    counts = P.render_counts(sc, r.camera, r.opts, rgb, compact=compact)
    rays = ray_breakdown(counts)
    flops = algorithmic_flops(counts)
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        P.render(sc, r.camera, r.opts, rgb, stream=stream, compact=compact)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            P.render(sc, r.camera, r.opts, rgb, stream=stream, compact=compact)
        b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    sc.close()
    return {"workload": "C3: 1920x1080, 4 spp jittered, 1024 instances (sphere, torus, box-frame, "
                        "Mandelbulb, Julia), shadows", "ms": round(ms, 3),
            "mrays_s": round(sum(rays.values()) / ms / 1e3, 1), "rays": rays,
            "roofline": roofline_of(flops, ms, "trace_kernel", profile=C3_PROFILE)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-next", action="store_true", help="skip the cut / mesh / animation lines")
    ap.add_argument("--no-c3", action="store_true", help="skip the C3 (1024-instance, 4 spp) line")
    ap.add_argument("--served-seconds", type=float, default=30.0,
                    help="measured length of each open-loop served trace")
    ap.add_argument("--served-warmup", type=float, default=2.0,
                    help="arrivals before this (seconds) are served but not measured")
    ap.add_argument("--only", choices=["c3", "c4", "c5"], default=None,
                    help="time only this workload (for profiling): C3, the 64-request batch, or "
                         "the served request mix as batches")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--budget", type=int, default=0)
    ap.add_argument("--compact", type=int, default=0,
                    help="regrouping threshold (0 = tuned default, 1..100, 1000 = never)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run one plain device copy of 256 MiB (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1 "
                                   "(rays are independent: multi-GPU sharding is a design note only)"}))
        sys.exit(2)

    import torch
    import paper_2012_10357_amd as P
    import workloads as W

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4}))
        return
    if args.only == "c3":
        print(json.dumps({"c3": bench_c3(P, W, torch, dev, reps=args.steps, compact=args.compact)}), flush=True)
        return
    if args.only == "c5":
        print(json.dumps({"served_ceiling": bench_served_ceiling(P, W, torch, dev, counts=False, plain=False)}),
              flush=True)
        return
    if args.only == "c4":
        print(json.dumps({"batched": bench_batched(P, W, torch, dev, reps=args.steps, compare=False)}),
              flush=True)
        return
    wl = W.c2()
    scene_desc, req = wl.scenes[0], wl.requests[0]
    Wd, H = req.opts.width, req.opts.height
    sc = P.Scene(scene_desc)
    rgb = torch.empty((H, Wd, 3), dtype=torch.float32, device=dev)
    tile = (args.tile, 64 // args.tile) if args.tile else (0, 0)

    # work counts of this frame (instrumented build, untimed)
    counts = P.render_counts(sc, req.camera, req.opts, rgb, tile=tile, step_budget=args.budget,
                             compact=args.compact)
    rays = ray_breakdown(counts)
    rays_per_frame = sum(rays.values())
    flops_per_frame = algorithmic_flops(counts)

    stream = torch.cuda.Stream(device=dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            P.render(sc, req.camera, req.opts, rgb, stream=stream, tile=tile, step_budget=args.budget,
                     compact=args.compact)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            ev[i][0].record(stream)
            P.render(sc, req.camera, req.opts, rgb, stream=stream, tile=tile, step_budget=args.budget,
                     compact=args.compact)
            ev[i][1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    per_launch_ms = np.array([a.elapsed_time(b) for a, b in ev])
    ms_per_step = wall * 1e3 / args.steps
    value = rays_per_frame * args.steps / wall / 1e6
    kern_ms = float(np.mean(per_launch_ms))
    achieved = flops_per_frame / (kern_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mrays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded teaser-like scene; no dataset)",
        "config": {"workload": "teaser 1920x1080 1spp: 2 pac-men + quaternion Julia + "
                               "power-8 Mandelbulb, 256 steps, eps 1e-4, shadows + 1 mirror bounce",
                   "rays_per_frame": rays, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": None, "kernel": "trace_kernel", "kernel_ms": round(kern_ms, 4),
                     "flops_per_launch": flops_per_frame},
    }
    cus, wg_per_cu = P.launch_shape()
    out["roofline"]["grid"] = {"compute_units": cus, "workgroups_per_cu": wg_per_cu}
    print(f"# frame: {rays_per_frame} rays, {flops_per_frame / 1e9:.2f} GFLOP, "
          f"kernel {kern_ms:.3f} ms (min {per_launch_ms.min():.3f}), "
          f"{cus} CUs x {wg_per_cu} workgroups", file=sys.stderr, flush=True)
    # HBM traffic and issue figures from the committed counter profile of this
    # kernel source (null when the source has changed since it was taken)
    counters = committed_counters()
    out["roofline"]["traffic"] = counters.get("traffic_bytes_per_launch")
    out["roofline"]["valu_issue_frac"] = counters.get("valu_issue_utilisation")
    out["roofline"]["active_lane_frac"] = counters.get("active_lane_fraction")
    sc.close()
    if not args.no_c3:
        out["c3"] = bench_c3(P, W, torch, dev, compact=args.compact)
        print(f"# c3: {out['c3']}", file=sys.stderr, flush=True)
    if not args.no_batch:
        out["batched"] = bench_batched(P, W, torch, dev)
        print(f"# batched: {out['batched']}", file=sys.stderr, flush=True)
    if not args.no_served:
        out["served"] = bench_served(P, W, torch, dev, args.served_seconds, warmup_s=args.served_warmup)
        print(f"# served: {out['served']}", file=sys.stderr, flush=True)
        # the same requests at half the rate, below the GPU's capacity: the
        # latency of batching and execution rather than of a growing queue
        out["served_100hz"] = bench_served(P, W, torch, dev, args.served_seconds, rate_hz=100.0,
                                           warmup_s=args.served_warmup)
        print(f"# served at 100 req/s: {out['served_100hz']}", file=sys.stderr, flush=True)
        out["served_ceiling"] = bench_served_ceiling(P, W, torch, dev)
        print(f"# served mix, back-to-back batches: {out['served_ceiling']}", file=sys.stderr, flush=True)
    if not args.no_next:
        out["next"] = bench_next(P, W, torch, dev)
        print(f"# next: {out['next']}", file=sys.stderr, flush=True)
        # last on the GPU: registering a user type builds a second kernel
        out["next"]["teaser_user_pacmen_1080p"] = bench_f3(P, W, torch, dev)
        print(f"# user hit group: {out['next']['teaser_user_pacmen_1080p']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
