"""Closed-form ray intersections used to pin the oracle (test-side only).

None of these reuse the oracle's code: they solve the intersection problem
directly (quadratics, quartics, slab entries, plane crossings) instead of
marching an estimator.
"""
from __future__ import annotations

import math

import numpy as np


def ray_sphere(o, d, c, r):
    """First root t >= 0 of |o + t d - c| = r (d unit), and closest-approach distance."""
    oc = o - c
    b = np.sum(oc * d, axis=-1)
    cc = np.sum(oc * oc, axis=-1) - r * r
    disc = b * b - cc
    closest = np.sqrt(np.maximum(np.sum(oc * oc, axis=-1) - b * b, 0.0))
    sq = np.sqrt(np.maximum(disc, 0.0))
    t = -b - sq
    t = np.where(t < 0, -b + sq, t)
    hit = (disc >= 0) & (t >= 0)
    return np.where(hit, t, np.inf), closest


def ray_aabb(o, d, lo, hi):
    """Slab entry/exit of an axis-aligned box (d components non-zero)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        a = (lo - o) / d
        b = (hi - o) / d
    tn = np.max(np.minimum(a, b), axis=-1)
    tf = np.min(np.maximum(a, b), axis=-1)
    return tn, tf


def ray_torus_roots(o, d, R, r):
    """Smallest positive real root of the torus quartic (axis y) per ray."""
    out = np.full(o.shape[0], np.inf)
    for i in range(o.shape[0]):
        ox, oy, oz = o[i]
        dx, dy, dz = d[i]
        # (|p|^2 + R^2 - r^2)^2 = 4 R^2 (px^2 + pz^2), p = o + t d
        a = dx * dx + dy * dy + dz * dz
        b = 2 * (ox * dx + oy * dy + oz * dz)
        c = ox * ox + oy * oy + oz * oz + R * R - r * r
        # (a t^2 + b t + c)^2 - 4R^2 ((dx^2+dz^2) t^2 + 2 (ox dx + oz dz) t + ox^2 + oz^2)
        e2 = dx * dx + dz * dz
        e1 = 2 * (ox * dx + oz * dz)
        e0 = ox * ox + oz * oz
        coef = [a * a, 2 * a * b, b * b + 2 * a * c - 4 * R * R * e2,
                2 * b * c - 4 * R * R * e1, c * c - 4 * R * R * e0]
        roots = np.roots(coef)
        real = roots[np.abs(roots.imag) < 1e-7].real
        real = real[real > 0]
        if real.size:
            out[i] = real.min()
    return out


def torus_sdf(p, R, r):
    """Distance to the torus: distance to its core circle minus r."""
    q = np.sqrt(p[:, 0] ** 2 + p[:, 2] ** 2) - R
    return np.sqrt(q * q + p[:, 1] ** 2) - r


def boxframe_bars(b, e):
    """The 12 edge bars of the frame of [-b,b]^3 as (lo, hi) boxes."""
    k = b - e
    bars = []
    for s1 in (-1, 1):
        for s2 in (-1, 1):
            for axis in range(3):
                c = [0.0, 0.0, 0.0]
                h = [e, e, e]
                h[axis] = b
                others = [i for i in range(3) if i != axis]
                c[others[0]] = s1 * k
                c[others[1]] = s2 * k
                bars.append((np.array(c) - np.array(h), np.array(c) + np.array(h)))
    return bars


def ray_boxframe(o, d, b, e):
    """First entry into any of the 12 bars (min over bar slab entries)."""
    best = np.full(o.shape[0], np.inf)
    for lo, hi in boxframe_bars(b, e):
        tn, tf = ray_aabb(o, d, lo, hi)
        ok = (tn <= tf) & (tf >= 0)
        best = np.where(ok, np.minimum(best, np.maximum(tn, 0.0)), best)
    return best


def ray_pacman(o, d, R, alpha):
    """First point inside the sphere |p| <= R and outside the wedge |atan2(y,x)| <= alpha."""
    out = np.full(o.shape[0], np.inf)
    for i in range(o.shape[0]):
        oi, di = o[i], d[i]
        b = float(oi @ di)
        cc = float(oi @ oi) - R * R
        disc = b * b - cc
        if disc < 0:
            continue
        t_in, t_out = -b - math.sqrt(disc), -b + math.sqrt(disc)
        cands = [t_in]
        for sgn in (1.0, -1.0):
            # half-plane through the z axis at angle sgn*alpha: normal (-sin, cos) rotated
            nx, ny = -math.sin(sgn * alpha), math.cos(sgn * alpha)
            den = nx * di[0] + ny * di[1]
            if den != 0.0:
                cands.append(-(nx * oi[0] + ny * oi[1]) / den)
        for t in sorted(cands):
            if t < t_in - 1e-12 or t > t_out + 1e-12 or t < 0:
                continue
            p = oi + t * di
            ang = math.atan2(p[1], p[0])
            inside_wedge = abs(ang) < alpha - 1e-12
            if not inside_wedge:
                out[i] = t
                break
    return out


def complex_julia_de(w, c0, n_iter, bailout):
    """Complex-plane Julia estimator |w| ln|w| / (2 |dw|) with the same stopping rule."""
    m = 1.0
    for _ in range(n_iter):
        if abs(w) > bailout:
            break
        m = 2.0 * abs(w) * m
        w = w * w + c0
    a = abs(w)
    return 0.5 * a * math.log(a) / m


def real_bulb_axis_de(x, c, n_iter, bailout, power=8):
    """The Mandelbulb on its polar axis: x <- |x|^P + c, dr <- P |x|^(P-1) dr + 1."""
    dr = 1.0
    z = x
    for _ in range(n_iter):
        r = abs(z)
        if r > bailout:
            break
        dr = power * r ** (power - 1) * dr + 1.0
        z = r ** power + c
    r = abs(z)
    return 0.5 * math.log(r) * r / dr


def folded_multibrot_slice_de(x, z, n_iter, bailout, power=8):
    """The Mandelbulb on its slice y = 0, as a complex recurrence.

    A point (x, 0, z) has azimuth 0 or pi, so P times its azimuth is a
    multiple of 2 pi and the power map keeps it in the slice; with
    w = z + i x its polar angle (from +z) is |arg w|, so the slice map is
    w <- (Re w + i |Im w|)^P + c with c = z + i x, a folded multibrot.  The
    derivative and estimator rules are the Mandelbulb's (r = |w|)."""
    c = complex(z, x)
    w = c
    dr = 1.0
    for _ in range(n_iter):
        r = abs(w)
        if r > bailout:
            break
        dr = power * r ** (power - 1) * dr + 1.0
        w = complex(w.real, abs(w.imag)) ** power + c
    r = abs(w)
    return 0.5 * math.log(r) * r / dr


def quaternion_matrix_julia_de(p, c, n_iter, bailout):
    """Quaternion Julia estimator computed in the 2x2 complex matrix
    representation of the quaternions: a + b i + c j + d k is the matrix
    [[a + b i, c + d i], [-c + d i, a - b i]], quaternion products are
    matrix products and |q|^2 = det(Q).  The orbit Z <- Z Z + C starts at
    the slice point (p_x, p_y, p_z, 0); the derivative m <- 2 |Z| m and the
    escape and estimator rules are those of the quaternion definition."""
    def mat(a, b, cc, d):
        return np.array([[complex(a, b), complex(cc, d)], [complex(-cc, d), complex(a, -b)]])

    Z = mat(p[0], p[1], p[2], 0.0)
    C = mat(*c)
    m = 1.0
    for _ in range(n_iter):
        r = math.sqrt(max(np.linalg.det(Z).real, 0.0))
        if r > bailout:
            break
        m = 2.0 * r * m
        Z = Z @ Z + C
    r = math.sqrt(max(np.linalg.det(Z).real, 0.0))
    return 0.5 * r * math.log(r) / m
