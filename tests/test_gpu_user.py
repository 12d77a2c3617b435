"""GPU parity of programmable primitives: estimators and closest-hit
functions registered as HIP C++ source, compiled into the trace kernel at run
time, next to built-in primitives and a triangle plane, against the FP64
oracle running NumPy twins of the same functions."""
import numpy as np
import pytest

import bench
import workloads as W
from oracle import de as D
from oracle import tracer as T
from tests import parity
from tests import user_estimators as U
from tests.gpu_util import require_gpu, gpu_render, alloc, flat

pytestmark = pytest.mark.gpu

_types = {}


def _register(P):
    # everything is registered before the first render, so the module builds
    # one code object
    if not _types:
        _types["cyl"] = P.register_estimator("gpu_test_cylinder", U.CYLINDER_BODY)
        _types["oct"] = P.register_estimator("gpu_test_octahedron", U.OCTAHEDRON_BODY)
        # the same cylinder, shaded by user closest-hit functions
        _types["cyl_ch"] = P.register_estimator("gpu_test_cylinder_striped", U.CYLINDER_BODY)
        _types["cyl_lam"] = P.register_estimator("gpu_test_cylinder_lambert", U.CYLINDER_BODY)
        P.register_closest_hit(_types["cyl_ch"], U.STRIPED_CH_BODY)
        P.register_closest_hit(_types["cyl_lam"], U.LAMBERT_CH_BODY)
        # the benchmark's user hit group: the teaser's pac-man and Lambert shading restated
        _types["cyl_signed"] = P.register_estimator("gpu_test_cylinder_signed", U.CYLINDER_BODY)
        P.register_closest_hit(_types["cyl_signed"], U.SIGNED_CH_BODY)
        _types["pac"] = P.register_estimator("gpu_test_user_pacman", bench.F3_PACMAN_BODY)
        P.register_closest_hit(_types["pac"], bench.F3_LAMBERT_BODY)
        D.register_estimator(_types["pac"],
                             lambda p, k: D.de_pacman(p, k[:, 0], np.arctan2(k[:, 2], k[:, 1])))
        D.register_closest_hit(_types["pac"], U.lambert_ch_np)
        for k in ("cyl", "cyl_ch", "cyl_lam", "cyl_signed"):
            D.register_estimator(_types[k], U.cylinder_np)
        D.register_closest_hit(_types["cyl_signed"], U.signed_ch_np)
        D.register_estimator(_types["oct"], U.octahedron_np)
        D.register_closest_hit(_types["cyl_ch"], U.striped_ch_np)
        D.register_closest_hit(_types["cyl_lam"], U.lambert_ch_np)
    return _types


def _scene(types, cyl="cyl"):
    b = W._SceneBuilder()
    m_c = b.material((0.2, 0.7, 0.4), 0.3)
    m_o = b.material((0.9, 0.6, 0.2), 0.0)
    m_s = b.material((0.6, 0.6, 0.9), 0.2)
    m_g = b.material((0.75, 0.75, 0.75))
    aabb, prm = U.cylinder_geom(0.5, 0.9)
    g_c = b.geometry((types[cyl], aabb, prm))
    aabb, prm = U.octahedron_geom(0.8)
    g_o = b.geometry((types["oct"], aabb, prm))
    b.instance(g_c, m_c, W.xform(W._rot_x(0.4), 1.0, (-1.4, 0.0, 0.3)))
    b.instance(g_c, m_c, W.xform(W._rot_y(0.6) @ W._rot_x(1.2), 0.7, (1.6, -0.3, -0.4)))
    b.instance(g_o, m_o, W.xform(W._rot_y(0.5), 1.1, (0.1, 0.1, 0.6)))
    b.instance(b.geometry(W.geom_sphere(0.6)), m_s, W.xform(np.eye(3), 1.0, (0.2, -0.4, -1.2)))
    b.mesh(W.QUAD_VERTICES, W.QUAD_INDICES, [(m_g, W.xform(np.eye(3), 8.0, (0.0, -1.0, 0.0)))])
    return b.build(light_pos=(2, 4, -3))


def test_user_estimators_full_frame():
    P = require_gpu()
    types = _register(P)
    scene = _scene(types)
    cam = W.camera((0.0, 1.2, -5.0))
    opts = W.RenderOpts(128, 96, max_steps=256, shadows=1, bounces=1)
    g = gpu_render(P, P.Scene(scene), cam, opts)
    orc = T.render(scene, cam, opts)
    rep = parity.compare(*flat(*g), orc, "user estimators 128x96")
    print(parity.fmt(rep), flush=True)
    assert rep["pass"], parity.fmt(rep)
    # every instance (both user types, the sphere, the plane) shows up
    assert set(np.unique(g[2])) >= {0, 1, 2, 3, 4}


@pytest.mark.parametrize("cyl", ["cyl", "cyl_ch"])
def test_user_estimators_batch_counts_and_schedule(cyl):
    """Batched with a built-in-only request, graph-captured, other tile and
    budget: bitwise equal to single renders; the instrumented build runs too
    (user estimators alone, and with a user closest-hit function)."""
    P = require_gpu()
    import torch
    types = _register(P)
    scene = _scene(types, cyl)
    sc = P.Scene(scene)
    teaser = P.Scene(W.c2_scene())
    cam = W.camera((1.0, 2.0, -4.5), (0.0, -0.2, 0.0))
    opts = W.RenderOpts(97, 61, spp=2, jitter=1, seed=9, max_steps=256, shadows=1, bounces=1)
    ref = gpu_render(P, sc, cam, opts)
    _eq = lambda a, b: all(np.array_equal(x, y, equal_nan=True) for x, y in zip(a, b))
    assert _eq(ref, gpu_render(P, sc, cam, opts, tile=(16, 4), step_budget=5))
    t_opts = W.c2_opts(80, 45)
    out1, out2 = alloc(opts.width, opts.height), alloc(80, 45)
    reqs = P.make_requests([(sc, cam, opts, *out1, 0), (teaser, W.c2_camera(), t_opts, *out2, 1)])
    for _ in range(3):
        P.render_batch(reqs, use_graph=True)
        torch.cuda.synchronize()
        assert _eq(ref, tuple(x.cpu().numpy() for x in out1))
    rgb = torch.empty((opts.height, opts.width, 3), device="cuda")
    c = P.render_counts(sc, cam, opts, rgb)
    assert int(c[28]) == opts.width * opts.height * opts.spp


def test_graph_cache_tells_kernels_apart():
    """A launch context that replayed a captured graph of the built-in kernel
    must not replay it for a batch that needs the user-estimator kernel, even
    with the same table size, grid, budget and stream."""
    P = require_gpu()
    import torch
    types = _register(P)
    user_sc = P.Scene(_scene(types))
    teaser = P.Scene(W.c2_scene())
    cam = W.camera((0.0, 1.2, -5.0))
    opts = W.RenderOpts(256, 192, max_steps=256, shadows=1, bounces=1)
    stream = torch.cuda.Stream()
    a = alloc(256, 192)
    ra = P.make_requests([(teaser, W.c2_camera(), opts, *a, 0)])
    b = alloc(256, 192)
    rb = P.make_requests([(user_sc, cam, opts, *b, 1)])
    for _ in range(2):
        P.render_batch(ra, tile=(8, 8), step_budget=16, use_graph=True, stream=stream)
        torch.cuda.synchronize()
        P.render_batch(rb, tile=(8, 8), step_budget=16, use_graph=True, stream=stream)
        torch.cuda.synchronize()
        want = gpu_render(P, user_sc, cam, opts)
        got = tuple(x.cpu().numpy() for x in b)
        for x, y in zip(want, got):
            assert np.array_equal(x, y, equal_nan=True)


def test_user_closest_hit_full_frame():
    """Cylinders shaded by a registered closest-hit function (stripes in world
    y, Lambert, a Blinn-Phong highlight, a parameter term), reflective, with
    shadows cast on and by them, beside built-in primitives and a triangle
    plane: parity with the oracle running the function's NumPy twin."""
    P = require_gpu()
    types = _register(P)
    scene = _scene(types, "cyl_ch")
    cam = W.camera((0.0, 1.2, -5.0))
    opts = W.RenderOpts(128, 96, max_steps=256, shadows=1, bounces=1)
    g = gpu_render(P, P.Scene(scene), cam, opts)
    orc = T.render(scene, cam, opts)
    rep = parity.compare(*flat(*g), orc, "user closest-hit 128x96")
    print(parity.fmt(rep), flush=True)
    assert rep["pass"], parity.fmt(rep)
    # the function's colours differ from the built-in Lambert ones on the cylinders
    plain = gpu_render(P, P.Scene(_scene(types)), cam, opts)
    cyl = (g[2] == 0) | (g[2] == 1)
    assert cyl.sum() > 300
    assert np.max(np.abs(g[0][cyl] - plain[0][cyl])) > 0.05


def test_closest_hit_restating_lambert_matches_builtin():
    """A closest-hit function that restates the built-in Lambert term renders
    the built-in image (to float32 rounding: the light direction is
    normalised before the dot product), though its hits trace their own
    shadow ray instead of handing it to another lane."""
    P = require_gpu()
    types = _register(P)
    cam = W.camera((0.0, 1.2, -5.0))
    opts = W.RenderOpts(128, 96, max_steps=256, shadows=1, bounces=1)
    a = gpu_render(P, P.Scene(_scene(types)), cam, opts)
    b = gpu_render(P, P.Scene(_scene(types, "cyl_lam")), cam, opts)
    assert np.array_equal(a[2], b[2])
    assert np.max(np.abs(a[0] - b[0])) < 1e-5


def test_user_pacmen_teaser_against_oracle_and_builtin():
    """The benchmark's user-hit-group frame -- the teaser with its pac-men as a
    user type restating the built-in estimator and Lambert shading -- against
    the oracle (running the built-in pac-man as the twin), and against the
    built-in frame: the same pixels hit the same instances."""
    P = require_gpu()
    types = _register(P)
    scene = bench.f3_scene(W, types["pac"])
    cam, opts = W.c2_camera(), W.c2_opts(200, 113)
    g = gpu_render(P, P.Scene(scene), cam, opts)
    orc = T.render(scene, cam, opts)
    rep = parity.compare(*flat(*g), orc, "teaser with user pac-men 200x113")
    print(parity.fmt(rep), flush=True)
    assert rep["pass"], parity.fmt(rep)
    gb = gpu_render(P, P.Scene(W.c2_scene()), cam, opts)
    assert np.mean(g[2] == gb[2]) >= 0.999
    assert set(np.unique(g[2])) >= {0, 1, 2, 3}


def _signed_scene(types):
    """Cylinders shaded by the signed closest-hit function, a sphere of
    negative albedo in two channels and a plane, nothing reflective."""
    b = W._SceneBuilder()
    m_c = b.material((0.2, 0.7, 0.4), 0.0)
    m_s = b.material((-0.6, 0.6, -0.9), 0.0)
    m_g = b.material((0.75, -0.5, 0.75), 0.0)
    aabb, prm = U.cylinder_geom(0.5, 0.9)
    g_c = b.geometry((types["cyl_signed"], aabb, prm))
    b.instance(g_c, m_c, W.xform(W._rot_x(0.4), 1.0, (-1.4, 0.0, 0.3)))
    b.instance(g_c, m_c, W.xform(W._rot_y(0.6) @ W._rot_x(1.2), 0.7, (1.6, -0.3, -0.4)))
    b.instance(b.geometry(W.geom_sphere(0.6)), m_s, W.xform(np.eye(3), 1.0, (0.2, -0.4, -1.2)))
    b.mesh(W.QUAD_VERTICES, W.QUAD_INDICES, [(m_g, W.xform(np.eye(3), 8.0, (0.0, -1.0, 0.0)))])
    return b.build(light_pos=(2, 4, -3), background=(-0.25, 0.0, 0.5))


@pytest.mark.parametrize("spp", [1, 4])
def test_signed_and_clamped_colours_against_oracle(spp):
    """Signed colours (negative albedo and background, a user closest-hit
    returning a signed normal component), a channel beyond the colour bound
    (clamped to 2^24) and NaN channels, averaged over 4 jittered samples by the
    fixed-point accumulators: parity with the oracle, the same NaN pixels, and
    the clamped channel exactly 2^24 where every sample hits a cylinder."""
    P = require_gpu()
    types = _register(P)
    scene = _signed_scene(types)
    cam = W.camera((0.0, 1.2, -5.0))
    opts = W.RenderOpts(128, 96, spp=spp, jitter=1, seed=77, max_steps=256, shadows=1, bounces=0)
    g = gpu_render(P, P.Scene(scene), cam, opts)
    orc = T.render(scene, cam, opts)
    g_rgb = g[0].reshape(-1, 3).astype(np.float64)
    keep = orc["excl"] == 0
    nan_g, nan_o = np.isnan(g_rgb), np.isnan(orc["rgb"])
    assert nan_o[:, 1].sum() > 100 and not nan_o[:, [0, 2]].any()
    assert np.mean((nan_g == nan_o).all(axis=1)[keep]) >= 0.999
    assert (g_rgb < 0).any() and (orc["rgb"] < 0).any()
    both = ~(nan_g | nan_o)
    g_rgb = np.where(both, g_rgb, 0.0)
    o_rgb = np.where(both, orc["rgb"], 0.0)
    # the clamped channel: exactly 2^24 where every sample hits a cylinder;
    # a mean of mixed samples (up to 2^24) is compared at float32 resolution
    full = o_rgb[:, 2] == 2.0 ** 24
    assert full.sum() > 300
    assert np.all(g_rgb[full & keep, 2] == 2.0 ** 24)
    agree = keep & ((g[2].reshape(-1) >= 0) == (orc["inst"] >= 0))
    err2 = np.abs(g_rgb[:, 2] - o_rgb[:, 2])
    assert np.mean((err2 <= 1e-3 + np.abs(o_rgb[:, 2]) * 2.0 ** -23)[agree]) >= 0.999
    g_rgb[:, 2] = 0.0
    o_rgb[:, 2] = 0.0
    rep = parity.compare(g_rgb, g[1], g[2], dict(orc, rgb=o_rgb), f"signed colours spp={spp}")
    print(parity.fmt(rep), flush=True)
    assert rep["pass"], parity.fmt(rep)
