"""Writes the golden fixtures of this directory.  It calls only the oracle
and the seeded input generators (never the HIP path):

    python -m tests.golden.make_golden

The paper prints no numeric worked example (its device code is in another
chapter), so the fixtures here are regression anchors: the C1 scene (unit
sphere over a ground box) rendered by the FP64 oracle at 16 x 12, and the
seeded teaser scene's parameters."""
import os

import numpy as np

import workloads as W
from oracle import tracer as T

HERE = os.path.dirname(os.path.abspath(__file__))


def c1_render():
    wl = W.c1(16, 12)
    return T.render(wl.scenes[0], wl.requests[0].camera, wl.requests[0].opts)


def write_c1(path):
    out = c1_render()
    with open(path, "w") as f:
        f.write("# C1 (unit sphere over a ground box) 16x12, 1 spp, 128 steps, eps 1e-4, shadows;\n")
        f.write("# FP64 oracle, written by tests/golden/make_golden.py\n")
        f.write("# pixel inst excl t r g b\n")
        for i in range(out["t"].size):
            r, g, b = out["rgb"][i]
            vals = " ".join(repr(float(v)) for v in (out["t"][i], r, g, b))
            f.write(f"{i} {int(out['inst'][i])} {int(out['excl'][i])} {vals}\n")


def write_teaser(path):
    s = W.c2_scene()
    with open(path, "w") as f:
        f.write("# seeded teaser scene (config seed 1035702): geometry types, parameters, instance\n")
        f.write("# transforms, materials; written by tests/golden/make_golden.py\n")
        for g in range(len(s.geom_type)):
            f.write("geom %d %s\n" % (int(s.geom_type[g]), " ".join(repr(float(v)) for v in s.geom_params[g])))
        for i in range(s.n_inst):
            f.write("inst %d %d %s\n" % (int(s.inst_geom[i]), int(s.inst_mat[i]),
                                        " ".join(repr(float(v)) for v in s.inst_xform[i])))
        for m in range(len(s.mat_refl)):
            f.write("mat %s %r\n" % (" ".join(repr(float(v)) for v in s.mat_albedo[m]), float(s.mat_refl[m])))


if __name__ == "__main__":
    write_c1(os.path.join(HERE, "c1_16x12_oracle.txt"))
    write_teaser(os.path.join(HERE, "teaser_scene.txt"))
    print("written")
