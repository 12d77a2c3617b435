"""GPU tests of the batched and served forms and of scheduling invariance.

Results must not depend on how work is scheduled: tile shape, step budget,
BVH build options, batch composition, hipGraph replay or the server's mix
all give bitwise-identical pixels."""
import time

import numpy as np
import pytest

import workloads as W
from oracle import tracer as T
from tests import parity
from tests.gpu_util import require_gpu, gpu_render, alloc, flat, d2h

pytestmark = pytest.mark.gpu


def _eq(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y, equal_nan=True)


def test_tile_and_budget_invariance():
    P = require_gpu()
    wl = W.c2(320, 180)
    sc = P.Scene(wl.scenes[0])
    req = wl.requests[0]
    ref = gpu_render(P, sc, req.camera, req.opts)
    for tile in ((16, 4), (32, 2), (64, 1)):
        for budget in (1, 5, 64):
            _eq(ref, gpu_render(P, sc, req.camera, req.opts, tile=tile, step_budget=budget))


@pytest.mark.parametrize("case", ["teaser 320x180", "teaser 61x37", "teaser 1x97", "teaser 130x1",
                                  "close-up", "fractal behind", "tile 64x1"])
def test_first_region_order_is_invisible(case):
    """Handing out the fractals' screen rectangle first (the default) and
    plain row-major order give the same bits, with every pixel written."""
    P = require_gpu()
    desc = W.c2_scene()
    sc = P.Scene(desc)
    tile = (0, 0)
    if case.startswith("teaser"):
        w, h = (int(v) for v in case.split()[1].split("x"))
        cam, opts = W.c2_camera(), W.c2_opts(w, h)
    elif case == "close-up":          # the Mandelbulb's box overfills the frame
        cam, opts = W.camera((0.9, 0.6, -2.4), (0.9, 0.1, -0.9)), W.c2_opts(200, 120)
    elif case == "fractal behind":    # box corners behind the eye: row-major order
        cam, opts = W.camera((0.9, 0.1, -1.2), (0.9, 0.1, -5.0)), W.c2_opts(96, 64)
    else:
        cam, opts, tile = W.c2_camera(), W.c2_opts(257, 75), (64, 1)
    a = gpu_render(P, sc, cam, opts, tile=tile)
    rgb, t, inst = alloc(opts.width, opts.height)
    P.render(sc, cam, opts, rgb, t, inst, tile=tile, natural_order=True)
    import torch
    torch.cuda.synchronize()
    b = (rgb.cpu().numpy(), t.cpu().numpy(), inst.cpu().numpy())
    assert np.isfinite(a[0]).all() and (a[2] >= -1).all()
    _eq(a, b)


def test_bvh_option_invariance():
    P = require_gpu()
    desc = W.random_instances_scene(np.random.default_rng(3), 300, W.C3_KINDS)
    cam = W.camera((0, 0, -45))
    opts = W.RenderOpts(256, 144, spp=2, jitter=1, seed=5, max_steps=256, tmax=200.0)
    ref = gpu_render(P, P.Scene(desc), cam, opts)
    for bo in (P.BvhOpts(8, 1, 1.0, 4.0, 0), P.BvhOpts(64, 4, 1.0, 1.0, 0), P.BvhOpts(16, 8, 2.0, 1.0, 0)):
        _eq(ref, gpu_render(P, P.Scene(desc, bvh=bo), cam, opts))


def _c4_small(n=24):
    """Small batched requests over the teaser scene; every other one with the
    mirror bounce (and so with shadow rays handed between lanes)."""
    wl = W.c4(n_requests=n, lo=64, hi=320)
    for i, r in enumerate(wl.requests):
        r.opts.bounces = i % 2
    return wl


def test_batch_equals_alone_and_graph_replays():
    P = require_gpu()
    import torch
    wl = _c4_small()
    sc = P.Scene(wl.scenes[0])
    outs, alone = [], []
    for r in wl.requests:
        alone.append(gpu_render(P, sc, r.camera, r.opts))
        outs.append(alloc(r.opts.width, r.opts.height))
    reqs = P.make_requests([(sc, r.camera, r.opts, *o, i) for i, (r, o) in enumerate(zip(wl.requests, outs))])
    P.render_batch(reqs)
    torch.cuda.synchronize()
    for o, a in zip(outs, alone):
        _eq([x.cpu().numpy() for x in o], a)
    # graph capture + replays, with eager work and synchronisation in between
    stream = torch.cuda.Stream()
    for rep in range(3):
        for o in outs:
            for x in o:
                x.fill_(-3)
        with torch.cuda.stream(stream):
            P.render_batch(reqs, use_graph=True, stream=stream)
        torch.cuda.synchronize()
        for o, a in zip(outs, alone):
            _eq([x.cpu().numpy() for x in o], a)
        gpu_render(P, sc, wl.requests[0].camera, wl.requests[0].opts)   # eager work between replays


def test_batch_mixed_scenes_and_parity():
    P = require_gpu()
    import torch
    s1 = W.c2_scene()
    s2 = W.random_instances_scene(np.random.default_rng(4), 200, W.C5_KINDS)
    sc1, sc2 = P.Scene(s1), P.Scene(s2)
    items = [(sc1, s1, W.c2_camera(), W.RenderOpts(97, 61, max_steps=256, bounces=1)),
             (sc2, s2, W.camera((0, 5, -50)), W.RenderOpts(80, 80, spp=3, jitter=1, seed=11, max_steps=256, tmax=200.0)),
             (sc1, s1, W.camera((3, 2, -4)), W.RenderOpts(64, 48, max_steps=256))]
    outs = [alloc(o.width, o.height) for _, _, _, o in items]
    reqs = P.make_requests([(sc, cam, o, *out, i) for i, ((sc, _, cam, o), out) in enumerate(zip(items, outs))])
    P.render_batch(reqs)
    torch.cuda.synchronize()
    for (sc, desc, cam, o), out in zip(items, outs):
        g = [x.cpu().numpy() for x in out]
        _eq(g, gpu_render(P, sc, cam, o))
        rep = parity.compare(*flat(*g), T.render(desc, cam, o), f"batch {o.width}x{o.height}")
        print(parity.fmt(rep))
        assert rep["pass"]


def test_autotune_returns_valid_choice():
    P = require_gpu()
    wl = W.c4(n_requests=4, lo=64, hi=128)
    sc = P.Scene(wl.scenes[0])
    outs = [alloc(r.opts.width, r.opts.height) for r in wl.requests]
    reqs = P.make_requests([(sc, r.camera, r.opts, *o, i) for i, (r, o) in enumerate(zip(wl.requests, outs))])
    best = P.autotune(reqs)
    assert best.tile_w * best.tile_h == 64 and best.step_budget >= 1


def test_server_mix_equals_alone():
    P = require_gpu()
    scenes = [W.c2_scene(), W.random_instances_scene(np.random.default_rng(5), 300, W.C5_KINDS)]
    dev = [P.Scene(s) for s in scenes]
    srv = P.Server(256 << 20, max_inflight=3, max_batch=16)
    for d in dev:
        srv.add_scene(d)
    reqs = W.c5_requests(24, lo=64, hi=256, n_scenes=2, seed=77)
    tickets = []
    for i, r in enumerate(reqs):
        if r.scene_index == 0:
            r.camera = W.camera((1.0 * (i % 3), 1.5, -6.0))
            r.opts.bounces = 1
        tickets.append(srv.submit(dev[r.scene_index], r.camera, r.opts, tag=i))
    import torch
    for tk, r in zip(tickets, reqs):
        res = srv.wait(tk, 60000)
        H, Wd = res.height, res.width
        got = (d2h(res.rgb, (H, Wd, 3), np.float32), d2h(res.t, (H, Wd), np.float32),
               d2h(res.inst, (H, Wd), np.int32))
        _eq(got, gpu_render(P, dev[r.scene_index], r.camera, r.opts))
        assert res.t_submit <= res.t_admit <= res.t_launch <= res.t_done
        # the ray counts the device reported for this request in the mix
        c = P.render_counts(dev[r.scene_index], r.camera, r.opts,
                            torch.empty((H, Wd, 3), dtype=torch.float32, device="cuda"))
        assert res.rays_primary == int(c[28])
        assert (res.rays_shadow, res.rays_bounce) == (int(c[29] + c[31]), int(c[30]))
        srv.release(tk)
    st = srv.stats()
    assert st.completed == 24 and st.pool_bytes_in_use == 0
    srv.close()


def test_launch_shape_keeps_three_workgroups_per_cu():
    """The kernel's registers and LDS must leave room for three 256-thread
    workgroups per compute unit (12 waves): the grid is sized from this, and
    one workgroup fewer costs about a third of the throughput of dense scenes."""
    P = require_gpu()
    cus, wg = P.launch_shape()
    assert cus >= 1
    assert wg == 3, (cus, wg)


def test_counts_match_oracle_work():
    """The instrumented kernel's work counts against the oracle's canonical
    front-to-back counts on the same frame (BVH order and float32 step
    sequences differ slightly, so this is a tolerance check)."""
    P = require_gpu()
    import torch
    wl = W.c2(160, 90)
    scene, req = wl.scenes[0], wl.requests[0]
    sc = P.Scene(scene)
    rgb = torch.empty((90, 160, 3), device="cuda")
    c = P.render_counts(sc, req.camera, req.opts, rgb).astype(np.float64)
    orc = T.render(scene, req.camera, req.opts)["counts"]
    print("gpu evals", c[:7], "oracle", orc["evals"])
    print("gpu rays", c[28:32], "oracle", orc["rays"])
    assert list(c[28:32]) == [orc["rays"][k] for k in ("primary", "shadow", "bounce", "bounce_shadow")]
    ev_g, ev_o = c[:7].sum(), float(sum(orc["evals"]))
    assert abs(ev_g - ev_o) / ev_o < 0.1
    it_g, it_o = c[7:14].sum(), float(sum(orc["iters"]))
    assert abs(it_g - it_o) / it_o < 0.1
    assert np.array_equal(c[14:21], np.array(orc["normal_evals"], np.float64))


def _regroup_cases():
    import dataclasses
    c2 = W.c2(320, 180)
    c3 = W.c3()
    f2 = W.f2_sample()
    f1 = W.f1_julia_cut(160, 90)
    dense = W.random_instances_scene(np.random.default_rng(8), 600, W.C5_KINDS)
    return {
        "teaser + bounce": (c2.scenes[0], c2.requests[0].camera, c2.requests[0].opts),
        "c3 dense 2 spp": (c3.scenes[0], c3.requests[0].camera,
                           dataclasses.replace(c3.requests[0].opts, width=256, height=144, spp=2)),
        "c5 kinds 3 spp": (dense, W.camera((0.0, 5.0, -50.0)),
                           W.RenderOpts(192, 108, spp=3, jitter=1, seed=4, max_steps=256, tmax=200.0)),
        "sample scene with plane": (f2.scenes[0], f2.requests[0].camera,
                                    dataclasses.replace(f2.requests[0].opts, width=160, height=90)),
        "oblique julia cut": (f1.scenes[f1.requests[1].scene_index], f1.requests[1].camera, f1.requests[1].opts),
    }


@pytest.mark.parametrize("case", list(_regroup_cases().keys()))
def test_regrouping_invariance(case):
    """Pooling a workgroup's sphere-trace queries by primitive type (any
    threshold, tile, budget; single render, batch with graph replay, the
    allocation-free path) gives the bits of waves marching their own lanes,
    and the instrumented build counts the same work."""
    P = require_gpu()
    import torch
    desc, cam, opts = _regroup_cases()[case]
    sc = P.Scene(desc)

    def run(**kw):
        rgb, t, inst = alloc(opts.width, opts.height)
        P.render(sc, cam, opts, rgb, t, inst, **kw)
        torch.cuda.synchronize()
        return rgb.cpu().numpy(), t.cpu().numpy(), inst.cpu().numpy()

    ref = run(compact=P.PR_COMPACT_NEVER)
    assert (ref[2] >= 0).any()
    for cp in (1, 50, 100):
        _eq(ref, run(compact=cp))
    _eq(ref, run(compact=100, tile=(16, 4), step_budget=5))
    _eq(ref, run(compact=30, tile=(64, 1), step_budget=64))
    out = alloc(opts.width, opts.height)
    reqs = P.make_requests([(sc, cam, opts, *out, 0)])
    for _ in range(2):
        P.render_batch(reqs, use_graph=True, compact=100, stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
        _eq(ref, [x.cpu().numpy() for x in out])
    na = alloc(opts.width, opts.height)
    P.render_noalloc(sc, cam, opts, *na, compact=100)
    torch.cuda.synchronize()
    _eq(ref, [x.cpu().numpy() for x in na])
    rgb = torch.empty((opts.height, opts.width, 3), device="cuda")
    c_plain = P.render_counts(sc, cam, opts, rgb, compact=P.PR_COMPACT_NEVER)
    c_pool = P.render_counts(sc, cam, opts, rgb, compact=100)
    assert np.array_equal(c_plain, c_pool), (c_plain, c_pool)
    sc.close()


def test_server_requests_complete_on_their_own():
    """Requests launched together complete when their own pixels are done
    (device flag), smallest first: small requests batched with a large one
    are done, correct and releasable before the large one finishes."""
    P = require_gpu()
    desc = W.random_instances_scene(np.random.default_rng(6), 1500, W.C5_KINDS)
    sc = P.Scene(desc)
    srv = P.Server(2 << 30, max_inflight=1, max_batch=16)
    srv.add_scene(sc)
    cam = W.camera((0.0, 8.0, -55.0))
    big = W.RenderOpts(2048, 2048, spp=4, jitter=1, seed=1, max_steps=256, tmax=200.0)
    small = [W.RenderOpts(64 + 16 * i, 48, spp=1 + i % 3, jitter=1, seed=10 + i, max_steps=256, tmax=200.0)
             for i in range(6)]
    # a first request keeps the single slot busy while the rest queue up, so
    # the large request and the small ones are launched together (the rest
    # are submitted once the first one's launch has started)
    first = srv.submit(sc, cam, W.RenderOpts(2048, 2048, spp=2, jitter=1, seed=2, max_steps=256, tmax=200.0))
    t0 = time.monotonic()
    while srv.stats().launches < 1:
        assert time.monotonic() - t0 < 30.0, "the first request was never launched"
        time.sleep(0.0002)
    t_big = srv.submit(sc, cam, big)
    t_small = [srv.submit(sc, cam, o, tag=i) for i, o in enumerate(small)]
    srv.wait(first, 120000)
    srv.release(first)
    done_small = []
    for tk, o in zip(t_small, small):
        res = srv.wait(tk, 120000)
        got = (d2h(res.rgb, (o.height, o.width, 3), np.float32), d2h(res.t, (o.height, o.width), np.float32),
               d2h(res.inst, (o.height, o.width), np.int32))
        done_small.append((res.t_launch, res.t_done))
        srv.release(tk)       # while the large request may still be rendering
        _eq(got, gpu_render(P, sc, cam, o))
    rb = srv.wait(t_big, 120000)
    srv.release(t_big)
    st = srv.stats()
    srv.close()
    assert st.launches == 2, st.launches
    assert all(tl == rb.t_launch for tl, _ in done_small)
    assert max(td for _, td in done_small) < rb.t_done
    print("small done after launch (ms):", [round((td - tl) * 1e3, 2) for tl, td in done_small],
          "large:", round((rb.t_done - rb.t_launch) * 1e3, 2), flush=True)
