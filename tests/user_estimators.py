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


# Closest-hit functions (the shading half of a user hit group), HIP C++ bodies
# and NumPy twins.  The arguments: hit point p, unit normal n, unit direction
# toward the ray origin v, unit direction toward the light l, lit (0/1),
# albedo, ambient, light rgb, params k; out: rgb.

# the built-in Lambert term, restated
LAMBERT_CH_BODY = """
  const float lam = fmaxf(0.f, nx * lx + ny * ly + nz * lz);
  for (int c = 0; c < 3; ++c) rgb[c] = albedo[c] * (ambient + lit * lam * light_rgb[c]);
"""


def lambert_ch_np(p, n, v, l, lit, albedo, ambient, light_rgb, k):
    lam = np.maximum(0.0, np.sum(n * l, axis=1))
    return albedo * (ambient + (lit * lam)[:, None] * light_rgb[None, :])


# stripes across world y on the albedo, Lambert, a Blinn-Phong highlight
# (exponent 16) and a term from the geometry's first parameter
STRIPED_CH_BODY = """
  const float stripe = 0.6f + 0.4f * cosf(6.f * py);
  const float lam = fmaxf(0.f, nx * lx + ny * ly + nz * lz);
  const float hx = lx + vx, hy = ly + vy, hz = lz + vz;
  const float hl = sqrtf(hx * hx + hy * hy + hz * hz);
  const float sp = hl > 0.f ? fmaxf(0.f, (nx * hx + ny * hy + nz * hz) / hl) : 0.f;
  const float s2 = sp * sp, s4 = s2 * s2, s8 = s4 * s4, s16 = s8 * s8;
  for (int c = 0; c < 3; ++c)
    rgb[c] = stripe * albedo[c] * (ambient + lit * lam * light_rgb[c]) + lit * 0.5f * s16 * light_rgb[c] +
             0.1f * k[0];
"""


def striped_ch_np(p, n, v, l, lit, albedo, ambient, light_rgb, k):
    stripe = 0.6 + 0.4 * np.cos(6.0 * p[:, 1])
    lam = np.maximum(0.0, np.sum(n * l, axis=1))
    h = l + v
    hl = np.linalg.norm(h, axis=1)
    sp = np.where(hl > 0.0, np.maximum(0.0, np.sum(n * h, axis=1) / np.where(hl > 0.0, hl, 1.0)), 0.0)
    return (stripe[:, None] * albedo * (ambient + (lit * lam)[:, None] * light_rgb[None, :])
            + (lit * 0.5 * sp ** 16)[:, None] * light_rgb[None, :] + 0.1 * k[:, 0:1])


# Signed, out-of-range and NaN colours: a signed normal component, a
# negated Lambert term that is NaN above world height 0.2, and a channel far
# beyond the library's colour bound (clamped to 2^24 on both sides).
SIGNED_CH_BODY = """
  const float lam = fmaxf(0.f, nx * lx + ny * ly + nz * lz);
  rgb[0] = nx - 0.25f * ny;
  rgb[1] = py > 0.2f ? __builtin_nanf("") : -albedo[1] * (ambient + lit * lam * light_rgb[1]);
  rgb[2] = 1e30f;
"""


def signed_ch_np(p, n, v, l, lit, albedo, ambient, light_rgb, k):
    lam = np.maximum(0.0, np.sum(n * l, axis=1))
    out = np.empty((p.shape[0], 3))
    out[:, 0] = n[:, 0] - 0.25 * n[:, 1]
    out[:, 1] = np.where(p[:, 1] > 0.2, np.nan, -albedo[:, 1] * (ambient + lit * lam * light_rgb[1]))
    out[:, 2] = 1e30
    return out
