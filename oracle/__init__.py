"""FP64 CPU oracle for procedural-primitive ray tracing — TEST INFRASTRUCTURE.

This package is the correctness authority for the HIP path.  It is a plain,
slow, vectorised NumPy implementation in float64 of what the method computes:
camera rays, brute-force intersection against every instance (no BVH), sphere
tracing of each primitive's distance estimator inside its AABB, closest hit,
central-difference normals, Lambert shading with one shadow ray per hit and an
optional mirror bounce.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP path and never
imports ``paper_2012_10357_amd``; the two sides share only the seeded input
generators in ``workloads``, which contain none of the method's arithmetic.

Paper context (Proceduray, da Silva, Novello, Lopes, Velho): the ray-tracing
pipeline of Sec. 2.2.3 (ray generation shader launching one ray per pixel;
intersection shaders computing hits inside a BLAS AABB; closest-hit, miss and
shadow rays of Listings "Ray creation" and "Hit group creation"), intersection
in each instance's local space (Sec. 4.1, "Instance buffer creation"), and
the sphere-traced fractals and CSG pac-men of the sample scene (Sec. 4,
Figs. 4-6).  The paper gives no device code, so every formula is the textbook
definition named in each function's docstring.

Beyond the sample scene's primitives it follows the same definitions for
primitives cut by a plane (CSG with a half-space, Fig. 5), triangle meshes
placed by instance transforms (the plane of Fig. 4; closed-form hits), and
estimators and closest-hit functions a test registers as NumPy functions
(``de.register_estimator``, ``de.register_closest_hit``: the twins of the
user hit groups compiled into the kernel).

Parity status per function is stated in the module headers and checked in
``tests/test_oracle_pins.py``: the fractal estimators are pinned by the planes
in which they reduce to complex recurrences (the Julia set on its real axis
and the plane of c; the Mandelbulb on its polar axis and its slices through
it) and, at generic points, by their symmetries and a second, algebraically
independent form of their maps.
"""
from .de import de_eval, TYPE_NAMES  # noqa: F401
from .tracer import prepare, render, camera_rays, lowbias32  # noqa: F401
