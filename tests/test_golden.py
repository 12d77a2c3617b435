"""Golden fixtures (tests/golden/, written by tests/golden/make_golden.py
from the oracle and the seeded generators only): the oracle and the input
generators must keep reproducing them.  The paper prints no numeric worked
example, so these are regression anchors, not paper values; the oracle's
correctness is pinned in test_oracle_pins.py."""
import os

import numpy as np

import workloads as W
from tests.golden import make_golden as G

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    return [ln.split() for ln in open(os.path.join(HERE, name)) if not ln.startswith("#")]


def test_c1_oracle_render_matches_golden():
    out = G.c1_render()
    rows = _rows("c1_16x12_oracle.txt")
    assert len(rows) == out["t"].size
    for r in rows:
        i = int(r[0])
        assert int(r[1]) == out["inst"][i] and int(r[2]) == out["excl"][i]
        want = np.array([float(v) for v in r[3:7]])
        got = np.array([out["t"][i], *out["rgb"][i]])
        assert np.allclose(got, want, rtol=1e-12, atol=1e-15) or (np.isinf(want[0]) and np.isinf(got[0]))


def test_teaser_scene_generator_matches_golden():
    s = W.c2_scene()
    rows = _rows("teaser_scene.txt")
    geoms = [r for r in rows if r[0] == "geom"]
    insts = [r for r in rows if r[0] == "inst"]
    mats = [r for r in rows if r[0] == "mat"]
    assert [int(r[1]) for r in geoms] == s.geom_type.tolist()
    assert np.array_equal(np.array([[float(v) for v in r[2:]] for r in geoms], np.float32), s.geom_params)
    assert np.array_equal(np.array([[float(v) for v in r[3:]] for r in insts], np.float32), s.inst_xform)
    assert np.array_equal(np.array([[float(v) for v in r[1:4]] for r in mats], np.float32), s.mat_albedo)
