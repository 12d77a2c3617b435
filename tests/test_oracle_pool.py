"""The worker-process oracle returns exactly what the oracle returns in one
process (test infrastructure used by the full-size GPU parity tests)."""
import numpy as np

import workloads as W
from oracle import tracer as T
from tests import oracle_pool as OP


def test_pool_equals_single_process():
    wl = W.c2(40, 24)
    scene, req = wl.scenes[0], wl.requests[0]
    pix = W.pixel_sample(40, 24, 700, seed=3)
    a = T.render(scene, req.camera, req.opts, pixels=pix)
    b = OP.render(scene, req.camera, req.opts, pixels=pix, chunk=97, procs=3)
    for k in ("rgb", "t", "inst", "excl"):
        assert np.array_equal(a[k], b[k]), k
    assert a["counts"]["rays"] == b["counts"]["rays"]
    c, d = OP.render_many([(scene, req.camera, req.opts, pix[:50]), (scene, req.camera, req.opts, pix[50:])],
                          chunk=64, procs=2)
    assert np.array_equal(np.concatenate([c["rgb"], d["rgb"]]), a["rgb"])
