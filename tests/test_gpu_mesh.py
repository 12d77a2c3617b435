"""GPU parity of triangle meshes beside procedural instances (the paper's
sample scene puts a triangle plane under its procedural objects, Fig. 4):
closed-form triangle hits in the same traversal, against the FP64 oracle."""
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


def _sphere_on_quads():
    """A unit sphere over a ground quad, plus a tilted quad placed twice."""
    b = W._SceneBuilder()
    m_s = b.material((0.9, 0.2, 0.2), 0.4)
    m_g = b.material((0.8, 0.8, 0.8))
    m_w = b.material((0.2, 0.5, 0.9), 0.2)
    b.instance(b.geometry(W.geom_sphere(1.0)), m_s, W.xform(np.eye(3), 1.0, (0, 0, 0)))
    b.mesh(W.QUAD_VERTICES, W.QUAD_INDICES,
           [(m_g, W.xform(np.eye(3), 10.0, (0.0, -1.0, 0.0))),
            (m_w, W.xform(W._rot_x(1.2), 1.5, (2.2, 0.2, 1.0))),
            (m_w, W.xform(W._rot_y(0.7) @ W._rot_x(1.4), 1.2, (-2.4, 0.0, 1.5)))])
    return b.build(light_pos=(2, 4, -3))


def test_sphere_on_quads_full_frame():
    P = require_gpu()
    scene = _sphere_on_quads()
    cam = W.camera((0.0, 1.0, -5.0))
    opts = W.RenderOpts(96, 72, max_steps=256, shadows=1, bounces=1)
    g = gpu_render(P, P.Scene(scene), cam, opts)
    orc = T.render(scene, cam, opts)
    rep = parity.compare(*flat(*g), orc, "sphere on quads 96x72")
    _check(rep)
    assert rep["inst"] >= 0.999


@pytest.mark.parametrize("size", [(200, 113), (61, 37)])
def test_sample_scene_full_frame(size):
    P = require_gpu()
    wl = W.f2_sample(*size)
    scene, req = wl.scenes[0], wl.requests[0]
    g = gpu_render(P, P.Scene(scene), req.camera, req.opts)
    orc = T.render(scene, req.camera, req.opts)
    _check(parity.compare(*flat(*g), orc, f"sample scene {size}"))


def test_sample_scene_1080p_sampled():
    P = require_gpu()
    wl = W.f2_sample()
    scene, req = wl.scenes[0], wl.requests[0]
    g = gpu_render(P, P.Scene(scene), req.camera, req.opts)
    assert np.isfinite(g[0]).all()
    pix = W.pixel_sample(1920, 1080, 4000, seed=21)
    orc = T.render(scene, req.camera, req.opts, pixels=pix)
    _check(parity.compare(*flat(*g, pixels=pix), orc, "sample scene 1080p sampled"))


def test_mesh_scene_scheduling_invariance():
    """Tile shape, step budget, BVH options and batching leave the bits alone."""
    P = require_gpu()
    import torch
    scene = _sphere_on_quads()
    cam = W.camera((0.5, 1.5, -5.0))
    opts = W.RenderOpts(130, 70, spp=2, jitter=1, seed=3, max_steps=256, shadows=1, bounces=1)
    sc = P.Scene(scene)
    ref = gpu_render(P, sc, cam, opts)
    others = [gpu_render(P, sc, cam, opts, tile=(32, 2), step_budget=3),
              gpu_render(P, P.Scene(scene, bvh=P.BvhOpts(8, 4, 1.0, 1.0, 0)), cam, opts)]
    out = alloc(opts.width, opts.height)
    small = W.RenderOpts(40, 30, max_steps=256)
    out2 = alloc(40, 30)
    reqs = P.make_requests([(sc, cam, opts, *out, 0), (sc, W.camera((3, 2, -4)), small, *out2, 1)])
    P.render_batch(reqs)
    torch.cuda.synchronize()
    others.append(tuple(x.cpu().numpy() for x in out))
    for o in others:
        for a, b in zip(ref, o):
            assert np.array_equal(a, b, equal_nan=True)
