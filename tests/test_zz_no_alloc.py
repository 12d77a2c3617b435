"""pr_render_noalloc through the C ABI against pr_render: the same frames,
bit for bit, on consecutive calls that reuse the fixed scratch (a
multi-sample frame, then a smaller one, then a single-sample one)."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import require_gpu, alloc

pytestmark = pytest.mark.gpu


def _both(P, sc, cam, opts, tile=(0, 0)):
    import torch
    a = alloc(opts.width, opts.height)
    P.render(sc, cam, opts, *a, tile=tile)
    b = alloc(opts.width, opts.height)
    P.render_noalloc(sc, cam, opts, *b, tile=tile)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in a], [x.cpu().numpy() for x in b]


def _same(a, b):
    return all(np.array_equal(x, y, equal_nan=True) for x, y in zip(a, b))


def test_noalloc_matches_render_on_consecutive_calls():
    P = require_gpu()
    sc = P.Scene(W.c2_scene())
    cam = W.c2_camera()
    import dataclasses
    base = W.c2_opts(320, 180)
    cases = [dataclasses.replace(base, spp=4, jitter=1, seed=5),
             dataclasses.replace(W.c2_opts(150, 83), spp=2, jitter=1, seed=6),
             W.c2_opts(97, 61)]
    for opts in cases:
        a, b = _both(P, sc, cam, opts)
        print(f"noalloc {opts.width}x{opts.height} spp={opts.spp}: hits {int((a[2] >= 0).sum())}", flush=True)
        assert np.isfinite(a[0]).all() and (a[2] >= 0).any()
        assert _same(a, b), f"{opts.width}x{opts.height} spp={opts.spp}"
    # a C3-like dense scene at 4 samples, and a tile shape other than the default
    c3 = W.c3()
    sc3 = P.Scene(c3.scenes[0])
    o3 = dataclasses.replace(c3.requests[0].opts, width=256, height=144)
    a, b = _both(P, sc3, c3.requests[0].camera, o3, tile=(16, 4))
    assert _same(a, b)
    sc.close()
    sc3.close()
