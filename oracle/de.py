"""Distance estimators in float64 (test infrastructure; see package header).

Every function takes local-space points ``p`` of shape (m, 3) and parameter
arrays broadcastable to (m,) and returns the estimator value (m,).  Fractal
estimators also return the number of map iterations executed per point, so
that the oracle can count the work of a render.

Definitions (textbook mathematics; the paper names the primitives -- sphere,
CSG pac-man, quaternion Julia set, Mandelbulb (Sec. 4, Figs. 1, 4-6) -- but
defers their device code to a separate chapter):

* sphere:     |p| - r                                   exact SDF
* box:        |max(q,0)| + min(max_i q_i, 0), q = |p-c| - h      exact SDF
* torus:      |(sqrt(px^2+pz^2) - R, py)| - r (axis local y)     exact SDF
* box-frame:  min over the 12 edge bars (half-thickness e, flush with the
              cube [-b,b]^3) of the bar box SDFs; by mirror symmetry the min
              over 12 equals the min over the 3 bars at the (+,+,+) corner
              evaluated at |p|.                         exact outside
* pac-man:    max(|p| - R, -W(p)), W = signed distance to the dihedral wedge
              {|atan2(py, px)| <= alpha} extruded along z.     CSG bound
* Julia:      quaternion z <- z^2 + c from z0 = (px, py, pz, 0), scalar
              derivative m <- 2|z| m, bailout on |z| > R_b (a radius),
              DE = |z| ln|z| / (2 m).                   estimator
* Mandelbulb: spherical power map (theta from +z, phi = atan2(y, x)),
              dr <- P r^(P-1) dr + 1, bailout r > R_b (a radius), then a
              fresh r = |z| and DE = ln(r) r / (2 dr).   estimator

Parity: sphere, box, torus, box-frame and pac-man are pinned by closed-form
ray intersections and the distance lower-bound invariant; the Julia estimator
is pinned at c = 0 (exactly |p| ln|p| / 2), at real c (complex Julia), and at
generic quaternion c by the complex planes span{1, u} that its orbits keep
(real axis; the plane of (c1, c2) when c3 = 0), by its invariance under
rotations of the imaginary part and by the 2x2 complex matrix representation
of the quaternions; the Mandelbulb on its polar axis (real recurrence
|x|^P + c), on the slice y = 0 and its rotated copies at azimuth 2 pi k / 7
(a folded complex multibrot, the same recurrence written with complex
powers), by its (P-1)-fold rotational and mirror symmetries and by the
agreement of its trigonometric and algebraic power maps.  At a generic
azimuth off those half-planes the Mandelbulb has no closed-form reduction:
there the symmetries and the algebraic map are its pins.
"""
from __future__ import annotations

import numpy as np

TYPE_NAMES = ["sphere", "box", "torus", "boxframe", "pacman", "julia", "mandelbulb"]
SPHERE, BOX, TORUS, BOXFRAME, PACMAN, JULIA, MANDELBULB = range(7)

TINY = 1e-300


def _norm(p):
    return np.sqrt(np.sum(p * p, axis=-1))


def de_sphere(p, r):
    return _norm(p) - r


def de_box(p, c, h):
    """Exact box SDF; c, h are (3,) or (m, 3)."""
    q = np.abs(p - c) - h
    outside = _norm(np.maximum(q, 0.0))
    inside = np.minimum(np.max(q, axis=-1), 0.0)
    return outside + inside


def de_torus(p, R, r):
    a = np.sqrt(p[:, 0] ** 2 + p[:, 2] ** 2) - R
    return np.sqrt(a * a + p[:, 1] ** 2) - r


def de_boxframe(p, b, e):
    """Union of the 12 edge bars of the cube [-b, b]^3, each of half-thickness e."""
    b = np.broadcast_to(np.asarray(b, np.float64), p.shape[:1])
    e = np.broadcast_to(np.asarray(e, np.float64), p.shape[:1])
    a = np.abs(p)
    k = b - e
    z = np.zeros_like(b)
    bars = [
        (np.stack([z, k, k], -1), np.stack([b, e, e], -1)),   # along x at (+y,+z)
        (np.stack([k, z, k], -1), np.stack([e, b, e], -1)),   # along y at (+x,+z)
        (np.stack([k, k, z], -1), np.stack([e, e, b], -1)),   # along z at (+x,+y)
    ]
    return np.min(np.stack([de_box(a, c, h) for c, h in bars], -1), axis=-1)


def wedge_sdf(p, alpha):
    """Signed distance (positive outside) to {|atan2(py, px)| <= alpha}, any z."""
    qx = p[:, 0]
    qy = np.abs(p[:, 1])
    ca, sa = np.cos(alpha), np.sin(alpha)
    qn = -sa * qx + ca * qy           # q . n, n = (-sin a, cos a)
    qu = ca * qx + sa * qy            # q . u, u = (cos a, sin a)
    apex = np.sqrt(qx * qx + qy * qy)
    return np.where((qn > 0.0) & (qu < 0.0), apex, qn)


def de_pacman(p, R, alpha):
    return np.maximum(_norm(p) - R, -wedge_sdf(p, alpha))


def de_julia(p, c, n_iter, bailout):
    """Quaternion Julia estimator; c is (4,) or (m, 4).  Returns (DE, iterations)."""
    m_pts = p.shape[0]
    c = np.broadcast_to(np.asarray(c, np.float64), (m_pts, 4))
    n_iter = np.broadcast_to(np.asarray(n_iter), (m_pts,)).astype(np.int64)
    bailout = np.broadcast_to(np.asarray(bailout, np.float64), (m_pts,))
    z = np.zeros((m_pts, 4))
    z[:, :3] = p
    md = np.ones(m_pts)
    iters = np.zeros(m_pts, np.int64)
    live = np.ones(m_pts, bool)
    for n in range(int(n_iter.max(initial=0))):
        zn = _norm(z)
        live &= (n < n_iter) & ~(zn > bailout)
        if not live.any():
            break
        md = np.where(live, 2.0 * zn * md, md)
        x, y, w2, w3 = z[:, 0], z[:, 1], z[:, 2], z[:, 3]
        sq = np.stack([x * x - y * y - w2 * w2 - w3 * w3, 2 * x * y, 2 * x * w2, 2 * x * w3], -1)
        z = np.where(live[:, None], sq + c, z)
        iters += live
    zn = _norm(z)
    with np.errstate(divide="ignore", invalid="ignore"):
        de = 0.5 * zn * np.log(zn) / md
    return np.where(zn < TINY, 0.0, de), iters


def _bulb_map_trig(z, r, power):
    """r^P (sin P th cos P ph, sin P th sin P ph, cos P th) with th from +z."""
    with np.errstate(divide="ignore", invalid="ignore"):
        th = np.where(r > 0, np.arccos(np.clip(z[:, 2] / np.where(r > 0, r, 1.0), -1.0, 1.0)), 0.0)
    ph = np.arctan2(z[:, 1], z[:, 0])
    rp = r ** power
    return np.stack([rp * np.sin(power * th) * np.cos(power * ph),
                     rp * np.sin(power * th) * np.sin(power * ph),
                     rp * np.cos(power * th)], -1)


def _bulb_map_algebraic8(z):
    """The power-8 map without trigonometry.

    With rho = sqrt(x^2 + y^2): (z + i rho)^8 = r^8 (cos 8th + i sin 8th) and
    (x + i y)^8 / rho^8 = cos 8ph + i sin 8ph, so the map is
    (Im A * Re B, Im A * Im B, Re A) with A = (z + i rho)^8, B = ((x+iy)/rho)^8,
    and B = 1 on the polar axis (phi = atan2(0, 0) = 0).
    """
    x, y, zz = z[:, 0], z[:, 1], z[:, 2]
    rho = np.sqrt(x * x + y * y)
    a = (zz + 1j * rho) ** 8
    with np.errstate(divide="ignore", invalid="ignore"):
        b = np.where(rho > 0, ((x + 1j * y) / np.where(rho > 0, rho, 1.0)) ** 8, 1.0 + 0j)
    return np.stack([a.imag * b.real, a.imag * b.imag, a.real], -1)


def de_mandelbulb(p, power, n_iter, bailout, algebraic=False):
    """Mandelbulb estimator.  Returns (DE, iterations)."""
    m_pts = p.shape[0]
    power = np.broadcast_to(np.asarray(power, np.float64), (m_pts,))
    n_iter = np.broadcast_to(np.asarray(n_iter), (m_pts,)).astype(np.int64)
    bailout = np.broadcast_to(np.asarray(bailout, np.float64), (m_pts,))
    z = p.astype(np.float64).copy()
    dr = np.ones(m_pts)
    iters = np.zeros(m_pts, np.int64)
    live = np.ones(m_pts, bool)
    for n in range(int(n_iter.max(initial=0))):
        r = _norm(z)
        live &= (n < n_iter) & ~(r > bailout)
        if not live.any():
            break
        dr = np.where(live, power * r ** (power - 1.0) * dr + 1.0, dr)
        if algebraic:
            if not np.all(power == 8.0):
                raise ValueError("algebraic form is for power 8 only")
            zp = _bulb_map_algebraic8(z)
        else:
            zp = _bulb_map_trig(z, r, power[:, None][:, 0])
        z = np.where(live[:, None], zp + p, z)
        iters += live
    r = _norm(z)
    with np.errstate(divide="ignore", invalid="ignore"):
        de = 0.5 * np.log(r) * r / dr
    return np.where(r < TINY, 0.0, de), iters


# User estimators (the programmable primitives of the library): type id ->
# function (points (m, 3), params (m, 8)) -> distance bounds (m,), float64.
USER = {}


def register_estimator(gtype: int, fn) -> None:
    USER[int(gtype)] = fn


# User closest-hit functions (the shading half of a hit group, Sec. 2.2.3):
# type id -> function (hit points, unit normals, unit directions toward the
# ray origins, unit directions toward the light, lit (0/1), albedo (m, 3),
# ambient, light rgb (3,), params (m, 8)) -> colours (m, 3), float64.
CLOSEST_HIT = {}


def register_closest_hit(gtype: int, fn) -> None:
    CLOSEST_HIT[int(gtype)] = fn


def de_eval(gtype: int, p: np.ndarray, prm: np.ndarray):
    """Evaluate the estimator of one primitive type at points p (m, 3).

    ``prm`` holds the 8 parameters, either (8,) or per point (m, 8), in the
    layout of the scene records.  Returns (DE, fractal iterations).
    """
    prm = np.asarray(prm, np.float64)
    if prm.ndim == 1:
        prm = np.broadcast_to(prm, (p.shape[0], 8))
    zero = np.zeros(p.shape[0], np.int64)
    if gtype in USER:
        return np.asarray(USER[gtype](p, prm), np.float64), zero
    if gtype == SPHERE:
        return de_sphere(p, prm[:, 0]), zero
    if gtype == BOX:
        return de_box(p, prm[:, 0:3], prm[:, 3:6]), zero
    if gtype == TORUS:
        return de_torus(p, prm[:, 0], prm[:, 1]), zero
    if gtype == BOXFRAME:
        return de_boxframe(p, prm[:, 0], prm[:, 1]), zero
    if gtype == PACMAN:
        return de_pacman(p, prm[:, 0], prm[:, 1]), zero
    if gtype == JULIA:
        return de_julia(p, prm[:, 0:4], prm[:, 4].astype(np.int64), prm[:, 5])
    if gtype == MANDELBULB:
        return de_mandelbulb(p, prm[:, 0], prm[:, 1].astype(np.int64), prm[:, 2])
    raise ValueError(f"unknown primitive type {gtype}")
