"""Two user estimators for the programmable-primitive tests: HIP C++ bodies
for the library and NumPy twins for the oracle (test infrastructure)."""
import numpy as np

# capped cylinder about the local y axis: radius p[0], half height p[1] (exact SDF)
CYLINDER_BODY = """
  R a = sqrt(x * x + z * z) - (R)p[0];
  R h = fabs(y) - (R)p[1];
  R ao = fmax(a, (R)0), ho = fmax(h, (R)0);
  return fmin(fmax(a, h), (R)0) + sqrt(ao * ao + ho * ho);
"""


def cylinder_np(p, prm):
    a = np.sqrt(p[:, 0] ** 2 + p[:, 2] ** 2) - prm[:, 0]
    h = np.abs(p[:, 1]) - prm[:, 1]
    return np.minimum(np.maximum(a, h), 0.0) + np.sqrt(np.maximum(a, 0.0) ** 2 + np.maximum(h, 0.0) ** 2)


# octahedron |x| + |y| + |z| <= p[0]: the plane distance of its faces, a lower bound
OCTAHEDRON_BODY = """
  return (fabs(x) + fabs(y) + fabs(z) - (R)p[0]) * (R)0.57735026918962576;
"""


def octahedron_np(p, prm):
    return (np.abs(p).sum(axis=1) - prm[:, 0]) * 0.57735026918962576


def cylinder_geom(r, hh):
    prm = np.zeros(8, np.float32); prm[0] = r; prm[1] = hh
    m = 0.01
    return [-r - m, -hh - m, -r - m, r + m, hh + m, r + m], prm


def octahedron_geom(s):
    prm = np.zeros(8, np.float32); prm[0] = s
    m = 0.01
    return [-s - m] * 3 + [s + m] * 3, prm
