"""GPU parity of the next-step features: primitives cut by a plane (Fig. 5)
and the step-budget animation of the Mandelbulb (Fig. 6), through the C ABI
against the FP64 oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import tracer as T
from tests import parity
from tests.gpu_util import require_gpu, gpu_render, alloc, flat

pytestmark = pytest.mark.gpu


def _check(rep):
    print(parity.fmt(rep), flush=True)
    assert rep["pass"], parity.fmt(rep)


@pytest.mark.parametrize("k", [0, 1])
def test_julia_cut_full_frame(k):
    P = require_gpu()
    wl = W.f1_julia_cut(160, 90)
    req = wl.requests[k]
    scene = wl.scenes[req.scene_index]
    g = gpu_render(P, P.Scene(scene), req.camera, req.opts)
    orc = T.render(scene, req.camera, req.opts)
    _check(parity.compare(*flat(*g), orc, f"julia cut {k} 160x90"))


def test_cut_sphere_and_ground_full_frame():
    """The C1 scene with its sphere cut by an oblique plane, shadows on."""
    P = require_gpu()
    wl = W.c1(72, 56)
    scene, req = wl.scenes[0], wl.requests[0]
    scene.geom_cut = np.array([[1.0, 2.0, -2.0, 0.9], [0.0, 0.0, 0.0, 0.0]], np.float32)
    g = gpu_render(P, P.Scene(scene), req.camera, req.opts)
    orc = T.render(scene, req.camera, req.opts)
    rep = parity.compare(*flat(*g), orc, "c1 cut sphere 72x56")
    _check(rep)
    assert rep["mask_all"] >= 0.999


def test_far_cut_plane_changes_nothing_bitwise():
    """A plane beyond every primitive: max(DE, n.p - d) = DE exactly, so the
    frame is bit-identical to the uncut one."""
    P = require_gpu()
    wl = W.c2(200, 113)
    req = wl.requests[0]
    ref = gpu_render(P, P.Scene(wl.scenes[0]), req.camera, req.opts)
    far = W.c2_scene()
    far.geom_cut = np.tile(np.array([0.0, 1.0, 0.0, 50.0], np.float32), (len(far.geom_type), 1))
    got = gpu_render(P, P.Scene(far), req.camera, req.opts)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b, equal_nan=True)


def test_mandelbulb_animation_batch():
    """All frames of the step-budget animation in one batched launch; each
    frame against the oracle, and the hit set grows with the budget."""
    P = require_gpu()
    import torch
    wl = W.f1_mandelbulb_anim(96, 96)
    scene = wl.scenes[0]
    sc = P.Scene(scene)
    outs = [alloc(r.opts.width, r.opts.height) for r in wl.requests]
    reqs = P.make_requests([(sc, r.camera, r.opts, *o, i) for i, (r, o) in enumerate(zip(wl.requests, outs))])
    P.render_batch(reqs)
    torch.cuda.synchronize()
    masks = []
    for r, o in zip(wl.requests, outs):
        g = tuple(x.cpu().numpy() for x in o)
        orc = T.render(scene, r.camera, r.opts)
        _check(parity.compare(*flat(*g), orc, f"anim steps {r.opts.max_steps}"))
        masks.append(g[2].reshape(-1) >= 0)
    for a, b in zip(masks[:-1], masks[1:]):
        assert np.all(b[a])
    assert masks[0].sum() < masks[-1].sum()
