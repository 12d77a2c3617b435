"""Seeded generators: determinism, parameter ranges, AABBs that contain the surface."""
import math

import numpy as np

import workloads as W
from oracle import de as D


def _bytes(scene):
    return b"".join(np.ascontiguousarray(getattr(scene, k)).tobytes()
                    for k in ("geom_type", "geom_aabb", "geom_params", "inst_geom", "inst_mat",
                              "inst_xform", "mat_albedo", "mat_refl"))


def test_same_seed_same_bytes():
    assert _bytes(W.c2_scene()) == _bytes(W.c2_scene())
    assert _bytes(W.c3_scene()) == _bytes(W.c3_scene())
    r1 = W.c5_requests(50)
    r2 = W.c5_requests(50)
    assert [(r.scene_index, r.opts.width, r.opts.spp, r.arrival_s) for r in r1] == \
           [(r.scene_index, r.opts.width, r.opts.spp, r.arrival_s) for r in r2]


def test_c3_ranges():
    s = W.c3_scene()
    assert s.n_inst == 1024
    xf = s.inst_xform.reshape(-1, 3, 4).astype(np.float64)
    assert np.all(np.abs(xf[:, :, 3]) <= 20)
    sv = np.linalg.svd(xf[:, :, :3], compute_uv=False)
    assert np.all((sv >= 0.5 - 1e-5) & (sv <= 2 + 1e-5))
    assert np.allclose(sv[:, 0], sv[:, 2], rtol=1e-5)          # rotation x uniform scale
    types = s.geom_type[s.inst_geom]
    assert set(np.unique(types)) == {W.SPHERE, W.TORUS, W.BOXFRAME, W.MANDELBULB, W.JULIA}
    jul = s.geom_params[s.inst_geom][types == W.JULIA]
    assert np.all(np.abs(jul[:, :4]) <= 0.8)
    assert np.all((s.mat_albedo >= 0.2) & (s.mat_albedo <= 0.9))


def test_c4_c5_distributions():
    c4 = W.c4()
    sides = np.array([r.opts.width for r in c4.requests])
    assert len(sides) == 64 and sides.min() >= 128 and sides.max() <= 1024
    reqs = W.c5_requests(2000)
    gaps = np.diff([0.0] + [r.arrival_s for r in reqs])
    assert abs(gaps.mean() - 1 / 200) < 0.0005
    sides = np.array([r.opts.width for r in reqs])
    assert sides.min() >= 256 and sides.max() <= 2048
    # log-uniform: the median side is near the geometric mean of the range
    assert abs(math.log(np.median(sides)) - 0.5 * (math.log(256) + math.log(2048))) < 0.1
    assert set(r.opts.spp for r in reqs) == {1, 2, 3, 4}
    for r in reqs[:50]:
        assert 45 <= np.linalg.norm(r.camera.eye) <= 60 + 1e-4


def test_fractal_aabb_faces_clear_of_the_surface():
    """Every Julia/Mandelbulb AABB face point has an estimator well above eps."""
    rng = np.random.default_rng(0)
    scenes = [W.c2_scene(), W.c3_scene()]
    for s in scenes:
        for g in range(s.geom_type.shape[0]):
            gt = int(s.geom_type[g])
            if gt not in (W.JULIA, W.MANDELBULB):
                continue
            lo, hi = s.geom_aabb[g, :3].astype(np.float64), s.geom_aabb[g, 3:].astype(np.float64)
            pts = rng.uniform(lo, hi, (200, 3))
            ax = rng.integers(0, 3, 200)
            side = rng.integers(0, 2, 200)
            pts[np.arange(200), ax] = np.where(side == 0, lo[ax], hi[ax])
            v, _ = D.de_eval(gt, pts, s.geom_params[g])
            assert v.min() > 2e-4, (gt, v.min())
