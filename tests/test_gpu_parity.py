"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Inputs are the seeded workloads; the oracle runs on the same float32 arrays.
Full frames where the oracle finishes in seconds (several tiles and ragged
edges), and seeded pixel samples of the full-size frames rendered in the
launch configuration the benchmark times.
"""
import numpy as np
import pytest

import workloads as W
from oracle import tracer as T
from tests import parity
from tests import oracle_pool as OP
from tests.gpu_util import require_gpu, gpu_render, flat

pytestmark = pytest.mark.gpu


def _check(rep):
    print(parity.fmt(rep), flush=True)
    assert rep["pass"], parity.fmt(rep)


def test_c1_full_frame():
    P = require_gpu()
    wl = W.c1()
    scene, req = wl.scenes[0], wl.requests[0]
    sc = P.Scene(scene)
    g = gpu_render(P, sc, req.camera, req.opts)
    orc = T.render(scene, req.camera, req.opts)
    rep = parity.compare(*flat(*g), orc, "c1 64x64")
    _check(rep)
    assert rep["mask_all"] >= 0.999


@pytest.mark.parametrize("size", [(200, 113), (61, 37)])
def test_c2_small_full_frame(size):
    P = require_gpu()
    wl = W.c2(*size)
    scene, req = wl.scenes[0], wl.requests[0]
    sc = P.Scene(scene)
    g = gpu_render(P, sc, req.camera, req.opts)
    orc = T.render(scene, req.camera, req.opts)
    _check(parity.compare(*flat(*g), orc, f"c2 {size}"))


def test_c2_1080p_full_frame():
    """The benchmark's frame -- the 1920x1080 teaser in the launch
    configuration the benchmark times -- against the oracle on every pixel
    (the oracle runs in worker processes)."""
    P = require_gpu()
    wl = W.c2()
    scene, req = wl.scenes[0], wl.requests[0]
    sc = P.Scene(scene)
    g = gpu_render(P, sc, req.camera, req.opts)
    assert np.isfinite(g[0]).all()
    orc = OP.render(scene, req.camera, req.opts)
    rep = parity.compare(*flat(*g), orc, "c2 1080p full frame")
    _check(rep)
    # the frame passes the gate with E1-E3 alone, and its mask and distance
    # lines even with no exclusion
    assert rep["pass_strict"], parity.fmt(rep)
    assert rep["mask_all"] >= 0.999 and rep["t_frac_all"] >= 0.999


def test_c3_1080p_4spp_sampled():
    """C3 (1024 instances of five types, 4 jittered samples, shadows) at 1080p
    against the oracle on a seeded uniform sample of 65,536 pixels."""
    P = require_gpu()
    wl = W.c3()
    scene, req = wl.scenes[0], wl.requests[0]
    sc = P.Scene(scene)
    g = gpu_render(P, sc, req.camera, req.opts)
    assert np.isfinite(g[0]).all()
    pix = W.pixel_sample(1920, 1080, 65536, seed=9)
    assert pix.size == 65536
    orc = OP.render(scene, req.camera, req.opts, pixels=pix)
    rep = parity.compare(*flat(*g, pixels=pix), orc, "c3 1080p 4spp 65536 px")
    _check(rep)
    assert rep["pass_strict"], parity.fmt(rep)


def test_max_instances_sampled():
    """A scene at the item limit (16384 instances of two kinds, shadows),
    480x270 on the GPU against the oracle on a seeded sample of 65,536 pixels."""
    P = require_gpu()
    rng = np.random.default_rng(7)
    scene = W.random_instances_scene(rng, 16384, ["sphere", "torus"])
    cam = W.camera((0.0, 0.0, -45.0))
    opts = W.RenderOpts(480, 270, max_steps=256, shadows=1, bounces=0)
    g = gpu_render(P, P.Scene(scene), cam, opts)
    assert np.isfinite(g[0]).all()
    pix = W.pixel_sample(480, 270, 65536, seed=13)
    orc = OP.render(scene, cam, opts, pixels=pix)
    rep = parity.compare(*flat(*g, pixels=pix), orc, "16384 instances 480x270 65536 px")
    _check(rep)
    assert rep["pass_strict"], parity.fmt(rep)
    assert rep["hit_frac"] > 0.2


@pytest.mark.parametrize("wh", [(16384, 3), (5, 16384)])
def test_max_image_side_sampled(wh):
    """Images at the largest side the boundary accepts (16384), with ragged
    tiles the other way, against the oracle on a seeded pixel sample."""
    P = require_gpu()
    w, h = wh
    wl = W.c2(w, h)
    scene, req = wl.scenes[0], wl.requests[0]
    g = gpu_render(P, P.Scene(scene), req.camera, req.opts)
    assert np.isfinite(g[0]).all()
    # plus the middle of the frame, where the scene's objects are (a few
    # columns wide at 16384 x 3)
    cx, cy = w // 2, h // 2
    mid = [y * w + x for y in range(max(0, cy - 24), min(h, cy + 25)) for x in range(max(0, cx - 24), min(w, cx + 25))]
    pix = np.union1d(W.pixel_sample(w, h, 1200, seed=17), np.array(mid, np.int64))
    orc = T.render(scene, req.camera, req.opts, pixels=pix)
    rep = parity.compare(*flat(*g, pixels=pix), orc, f"max side {wh} sampled")
    _check(rep)
    assert rep["hit_frac"] > 0


@pytest.mark.parametrize("wh", [(1, 1), (1, 97), (130, 1), (65, 3)])
def test_degenerate_and_ragged_sizes(wh):
    P = require_gpu()
    wl = W.c2(*wh)
    scene, req = wl.scenes[0], wl.requests[0]
    # point the camera at the Mandelbulb so tiny images still hit something
    cam = W.camera((0.9, 0.3, -3.0), (0.9, 0.1, -0.9))
    sc = P.Scene(scene)
    g = gpu_render(P, sc, cam, req.opts)
    orc = T.render(scene, cam, req.opts)
    rep = parity.compare(*flat(*g), orc, f"ragged {wh}")
    print(parity.fmt(rep))
    keep = (orc["excl"] & parity.GATE_RULES) == 0
    assert np.array_equal((flat(*g)[2] >= 0)[keep], (orc["inst"] >= 0)[keep])


def test_spp_jitter_matches_oracle():
    P = require_gpu()
    scene = W.c1_scene()
    cam = W.camera((0, 1, -4))
    opts = W.RenderOpts(48, 40, spp=5, jitter=1, seed=(1 << 40) + 12345, max_steps=128, eps=1e-4,
                        tmax=100.0, shadows=1)
    sc = P.Scene(scene)
    g = gpu_render(P, sc, cam, opts)
    orc = T.render(scene, cam, opts)
    _check(parity.compare(*flat(*g), orc, "c1 5spp jitter"))


@pytest.mark.parametrize("spp,wh", [(16, (24, 20)), (64, (16, 12))])
def test_many_samples_match_oracle(spp, wh):
    """Up to the maximum of 64 samples per pixel: a 64-job chunk is then one
    pixel's samples (summed in the wave when they finish together), and a
    16-sample pixel spans a quarter chunk."""
    P = require_gpu()
    scene = W.c1_scene()
    cam = W.camera((0, 1, -4))
    opts = W.RenderOpts(wh[0], wh[1], spp=spp, jitter=1, seed=977 + spp, max_steps=128, eps=1e-4,
                        tmax=100.0, shadows=1)
    sc = P.Scene(scene)
    g = gpu_render(P, sc, cam, opts)
    orc = T.render(scene, cam, opts)
    _check(parity.compare(*flat(*g), orc, f"c1 {spp}spp jitter"))


def test_all_types_scene_with_bounce():
    """Every primitive type, non-trivial rotations and scales, shadows and a bounce."""
    P = require_gpu()
    rng = np.random.default_rng(31)
    b = W._SceneBuilder()
    geoms = [W.geom_sphere(1.0), W.geom_box((0.1, 0, 0), (0.6, 0.4, 0.5)), W.geom_torus(1.0, 0.3),
             W.geom_boxframe(1.0, 0.05), W.geom_pacman(0.8, 60.0),
             W.geom_julia(rng.uniform(-0.8, 0.8, 4), 12, 4.0), W.geom_mandelbulb(8, 10, 2.0)]
    for i, gg in enumerate(geoms):
        gi = b.geometry(gg)
        mi = b.material(rng.uniform(0.2, 0.9, 3), 0.4)
        pos = (-4.5 + 1.5 * i, 0.3 * (i % 2), 0.5 * (i % 3))
        b.instance(gi, mi, W.xform(W.random_rotation(rng), 0.6 + 0.1 * i, pos))
    gnd = b.geometry(W.geom_box((0, -1.6, 0), (8, 0.1, 8)))
    b.instance(gnd, b.material((0.7, 0.7, 0.7), 0.2), W.xform(np.eye(3), 1.0, (0, 0, 0)))
    scene = b.build(light_pos=(3, 6, -4))
    cam = W.camera((0, 2.0, -8.0), (0, 0, 0.3), vfov_deg=55)
    opts = W.RenderOpts(160, 72, spp=1, max_steps=256, eps=1e-4, tmax=100.0, shadows=1, bounces=1)
    sc = P.Scene(scene)
    g = gpu_render(P, sc, cam, opts)
    orc = T.render(scene, cam, opts)
    _check(parity.compare(*flat(*g), orc, "all types + bounce"))


def test_stacked_instances_four_wide_tree():
    """150 identical spheres stacked in one place among 150 scattered spheres
    and tori: a BVH too large for LDS, so the launch traverses the four-wide
    tree, whose nodes hold children with equal entry distances.  Against the
    oracle; a pixel that hits the stack reports its lowest instance id (equal
    distances, lowest id wins); and bit for bit the image of the regrouping
    variant, which walks the two-wide tree in another order."""
    import torch
    P = require_gpu()
    rng = np.random.default_rng(77)
    b = W._SceneBuilder()
    gs, gt = b.geometry(W.geom_sphere(1.0)), b.geometry(W.geom_torus(1.0, 0.3))
    m0, m1 = b.material((0.9, 0.3, 0.2)), b.material((0.3, 0.7, 0.9))
    for _ in range(150):
        b.instance(gs, m0, W.xform(np.eye(3), 3.0, (0.0, 0.0, 0.0)))
    for i in range(150):
        b.instance(gs if i % 2 else gt, m1,
                   W.xform(W.random_rotation(rng), rng.uniform(0.3, 0.8), rng.uniform(-8.0, 8.0, 3)))
    scene = b.build(light_pos=(10, 12, -10))
    cam = W.camera((0, 2, -18), (0, 0, 0), vfov_deg=60)
    opts = W.RenderOpts(96, 72, spp=1, max_steps=256, eps=1e-4, tmax=100.0, shadows=1)
    sc = P.Scene(scene)
    g = gpu_render(P, sc, cam, opts)
    inst = g[2].reshape(-1)
    stack = (inst >= 0) & (inst < 150)
    assert stack.sum() > 200 and (inst[stack] == 0).all(), np.unique(inst[stack])
    rgb, t, ins = (torch.empty_like(torch.from_numpy(x)).cuda() for x in g)
    P.render(sc, cam, opts, rgb, t, ins, compact=100)
    torch.cuda.synchronize()
    for a, v in zip(g, (rgb, t, ins)):
        assert np.array_equal(a, v.cpu().numpy(), equal_nan=True)
    orc = T.render(scene, cam, opts)
    _check(parity.compare(*flat(*g), orc, "stacked instances, four-wide tree"))
    sc.close()


@pytest.mark.parametrize("eye_z", [3.0, -3.0])
def test_mandelbulb_down_its_polar_axis(eye_z):
    """A Mandelbulb seen along its polar axis, odd image size: the central
    rays run on or within rounding of the axis, where the azimuth of the map
    is undefined and the orbit follows the real recurrence z <- |z|^8 + c."""
    P = require_gpu()
    b = W._SceneBuilder()
    gi = b.geometry(W.geom_mandelbulb(8, 10, 2.0))
    b.instance(gi, b.material((0.8, 0.6, 0.4), 0.3), W.xform(np.eye(3), 1.0, (0, 0, 0)))
    scene = b.build(light_pos=(2, 5, 4 * np.sign(eye_z)))
    cam = W.camera((0, 0, eye_z), (0, 0, 0), vfov_deg=30)
    opts = W.RenderOpts(33, 33, spp=1, max_steps=256, eps=1e-4, tmax=100.0, shadows=1, bounces=1)
    sc = P.Scene(scene)
    g = gpu_render(P, sc, cam, opts)
    assert g[2][16, 16] >= 0                      # the axis ray hits
    orc = T.render(scene, cam, opts)
    _check(parity.compare(*flat(*g), orc, f"mandelbulb polar axis, eye z {eye_z}"))


def test_c1_against_golden_fixture():
    """The GPU against the stored oracle values of tests/golden (no oracle
    run at test time)."""
    import os
    P = require_gpu()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_16x12_oracle.txt")
    rows = [ln.split() for ln in open(path) if not ln.startswith("#")]
    orc = dict(inst=np.array([int(r[1]) for r in rows]), excl=np.array([int(r[2]) for r in rows]),
               t=np.array([float(r[3]) for r in rows]),
               rgb=np.array([[float(v) for v in r[4:7]] for r in rows]))
    wl = W.c1(16, 12)
    g = gpu_render(P, P.Scene(wl.scenes[0]), wl.requests[0].camera, wl.requests[0].opts)
    rep = parity.compare(*flat(*g), orc, "c1 16x12 vs golden")
    _check(rep)
    assert rep["mask_all"] == 1.0
