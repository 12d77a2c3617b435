"""Scalar pure-Python twin of the vectorised oracle (test infrastructure).

It renders tiny images one ray at a time with the ``math`` module, and is
deliberately formulated differently from ``tracer.py`` so that a masking or
vectorisation slip in either shows up as a disagreement:

* instances are visited in index order with the running best distance
  pruning each march (closest hit) or stopping at the first hit (shadow),
  instead of marching every candidate and taking the minimum afterwards;
* the box-frame is the minimum over all 12 explicit edge bars (no folding);
* the wedge distance of the pac-man is computed from the two boundary
  half-lines explicitly;
* quaternion products are written out component by component;
* triangles are intersected with the Moeller-Trumbore formulation instead
  of the plane equation and signed areas.

Same definitions otherwise (pinhole camera, local-space slab clip, sphere
tracing v = sigma DE, eps stop, central-difference normal, Lambert with a
shadow ray, optional single mirror bounce).  No diagnostics.
"""
from __future__ import annotations

import math

from .tracer import sample_offsets

INF = float("inf")


def _sub(a, b): return (a[0] - b[0], a[1] - b[1], a[2] - b[2])
def _add(a, b): return (a[0] + b[0], a[1] + b[1], a[2] + b[2])
def _mul(a, s): return (a[0] * s, a[1] * s, a[2] * s)
def _dot(a, b): return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]
def _len(a): return math.sqrt(_dot(a, a))
def _nrm(a):
    n = _len(a)
    return (a[0] / n, a[1] / n, a[2] / n)
def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _box(p, c, h):
    q = [abs(p[i] - c[i]) - h[i] for i in range(3)]
    out = math.sqrt(sum(max(x, 0.0) ** 2 for x in q))
    return out + min(max(q), 0.0)


def _de(gt, p, prm):
    from .de import USER
    if gt in USER:
        import numpy as np
        return float(USER[gt](np.array([p], np.float64), np.array([prm], np.float64))[0]), 0
    return _de_builtin(gt, p, prm)


def _de_builtin(gt, p, prm):
    """Returns (DE, iterations)."""
    if gt == 0:
        return _len(p) - prm[0], 0
    if gt == 1:
        return _box(p, prm[0:3], prm[3:6]), 0
    if gt == 2:
        a = math.hypot(p[0], p[2]) - prm[0]
        return math.hypot(a, p[1]) - prm[1], 0
    if gt == 3:
        b, e = prm[0], prm[1]
        k = b - e
        best = INF
        for s1 in (-1.0, 1.0):
            for s2 in (-1.0, 1.0):
                best = min(best,
                           _box(p, (0.0, s1 * k, s2 * k), (b, e, e)),
                           _box(p, (s1 * k, 0.0, s2 * k), (e, b, e)),
                           _box(p, (s1 * k, s2 * k, 0.0), (e, e, b)))
        return best, 0
    if gt == 4:
        R, al = prm[0], prm[1]
        # distance to the wedge {|angle| <= al} in the xy-plane: outside the
        # wedge it is the distance to the nearer boundary half-line, inside it
        # is minus the distance to the nearer half-line.
        x, y = p[0], p[1]
        ang = math.atan2(y, x)
        dists = []
        for sgn in (1.0, -1.0):
            ux, uy = math.cos(al), sgn * math.sin(al)
            s = max(0.0, x * ux + y * uy)
            dists.append(math.hypot(x - s * ux, y - s * uy))
        dw = min(dists)
        w = -dw if abs(ang) <= al else dw
        return max(_len(p) - R, -w), 0
    if gt == 5:
        c = prm[0:4]
        n_it, rb = int(prm[4]), prm[5]
        z = [p[0], p[1], p[2], 0.0]
        m = 1.0
        it = 0
        for _ in range(n_it):
            zn = math.sqrt(sum(v * v for v in z))
            if zn > rb:
                break
            m = 2.0 * zn * m
            a, b1, c1, d1 = z
            z = [a * a - b1 * b1 - c1 * c1 - d1 * d1 + c[0], a * b1 + b1 * a + c[1],
                 a * c1 + c1 * a + c[2], a * d1 + d1 * a + c[3]]
            it += 1
        zn = math.sqrt(sum(v * v for v in z))
        if zn < 1e-300:
            return 0.0, it
        return 0.5 * zn * math.log(zn) / m, it
    if gt == 6:
        pw, n_it, rb = prm[0], int(prm[1]), prm[2]
        z = tuple(p)
        dr = 1.0
        it = 0
        for _ in range(n_it):
            r = _len(z)
            if r > rb:
                break
            th = math.acos(max(-1.0, min(1.0, z[2] / r))) if r > 0 else 0.0
            ph = math.atan2(z[1], z[0])
            dr = pw * r ** (pw - 1.0) * dr + 1.0
            rp = r ** pw
            z = (rp * math.sin(pw * th) * math.cos(pw * ph) + p[0],
                 rp * math.sin(pw * th) * math.sin(pw * ph) + p[1],
                 rp * math.cos(pw * th) + p[2])
            it += 1
        r = _len(z)
        if r < 1e-300:
            return 0.0, it
        return 0.5 * math.log(r) * r / dr, it
    raise ValueError(gt)


class ScalarScene:
    def __init__(self, scene):
        import numpy as np
        self.inst = []
        for k in range(scene.n_inst):
            xf = [float(v) for v in scene.inst_xform[k]]
            A = [[xf[0], xf[1], xf[2]], [xf[4], xf[5], xf[6]], [xf[8], xf[9], xf[10]]]
            b = (xf[3], xf[7], xf[11])
            An = np.array(A)
            Ainv = [list(map(float, row)) for row in np.linalg.inv(An)]
            sigma = float(np.linalg.svd(An, compute_uv=False)[-1])
            g = int(scene.inst_geom[k])
            m = int(scene.inst_mat[k])
            aabb = [float(v) for v in scene.geom_aabb[g]]
            raw = getattr(scene, "geom_cut", None)
            cut = [0.0, 0.0, 0.0, 0.0] if raw is None else [float(v) for v in raw[g]]
            nn = math.sqrt(cut[0] * cut[0] + cut[1] * cut[1] + cut[2] * cut[2])
            cut = [v / nn for v in cut] if nn > 0 else None
            self.inst.append(dict(cut=cut,
                Ainv=Ainv, b=b, sigma=sigma, lo=aabb[0:3], hi=aabb[3:6],
                gt=int(scene.geom_type[g]), prm=[float(v) for v in scene.geom_params[g]],
                albedo=[float(v) for v in scene.mat_albedo[m]], refl=float(scene.mat_refl[m])))
        # mesh triangles in world space (float64 placement), ids after the instances
        self.tri = []
        n_proc = len(self.inst)
        for mesh in (getattr(scene, "meshes", None) or []):
            verts = [tuple(float(c) for c in v) for v in mesh["vertices"]]
            for mat, xf in zip(mesh["inst_mat"], mesh["inst_xform"]):
                x = [float(c) for c in xf]
                def place(p):
                    return tuple(x[4 * r] * p[0] + x[4 * r + 1] * p[1] + x[4 * r + 2] * p[2] + x[4 * r + 3]
                                 for r in range(3))
                for f in mesh["indices"]:
                    a, b_, c = (place(verts[int(i)]) for i in f)
                    e1, e2 = _sub(b_, a), _sub(c, a)
                    self.tri.append(dict(v0=a, e1=e1, e2=e2, n=_nrm(_cross(e1, e2)),
                                         albedo=[float(v) for v in scene.mat_albedo[int(mat)]],
                                         refl=float(scene.mat_refl[int(mat)]),
                                         id=n_proc + len(self.tri)))
        self.light = tuple(float(v) for v in scene.light_pos)
        self.light_rgb = tuple(float(v) for v in scene.light_rgb)
        self.ambient = float(scene.ambient)
        self.bg = tuple(float(v) for v in scene.background)


def _mv(M, v):
    return tuple(M[i][0] * v[0] + M[i][1] * v[1] + M[i][2] * v[2] for i in range(3))


def _mtv(M, v):
    return tuple(M[0][i] * v[0] + M[1][i] * v[1] + M[2][i] * v[2] for i in range(3))


def _clip(ol, dl, lo, hi, tmin, tmax):
    t0, t1 = tmin, tmax
    for i in range(3):
        if dl[i] == 0.0:
            if ol[i] < lo[i] or ol[i] > hi[i]:
                return None
            continue
        a = (lo[i] - ol[i]) / dl[i]
        b = (hi[i] - ol[i]) / dl[i]
        t0 = max(t0, min(a, b))
        t1 = min(t1, max(a, b))
    return (t0, t1) if t0 <= t1 else None


def _cut_de(ins, p):
    """Estimator of the instance, intersected with its kept half-space
    n.p <= d when it has a cutting plane (Fig. 5)."""
    v, _ = _de(ins["gt"], p, ins["prm"])
    c = ins["cut"]
    if c is not None and v == v:
        g = c[0] * p[0] + c[1] * p[1] + c[2] * p[2] - c[3]
        if g > v:
            v = g
    return v


def _march(ins, ol, dl, t0, t1, n_max, eps):
    t = t0
    for _ in range(n_max):
        v = _cut_de(ins, _add(ol, _mul(dl, t)))
        v *= ins["sigma"]
        if v != v:
            return None
        if v < eps:
            return t
        t += v
        if t > t1:
            return None
    return None


def _tri_hit(tr, o, d, tmin, tmax):
    """Moeller-Trumbore: distance of the ray's hit on the triangle (both
    sides, closed edges) inside [tmin, tmax], or None."""
    p = _cross(d, tr["e2"])
    det = _dot(tr["e1"], p)
    if det == 0.0:
        return None
    s = _sub(o, tr["v0"])
    u = _dot(s, p) / det
    if u < 0.0 or u > 1.0:
        return None
    q = _cross(s, tr["e1"])
    v = _dot(d, q) / det
    if v < 0.0 or u + v > 1.0:
        return None
    t = _dot(tr["e2"], q) / det
    return t if tmin <= t <= tmax else None


def trace_closest(sc, o, d, tmin, tmax, opts):
    best_t, best_k = INF, -1
    for k, ins in enumerate(sc.inst):
        ol = _mv(ins["Ainv"], _sub(o, ins["b"]))
        dl = _mv(ins["Ainv"], d)
        lim = min(tmax, best_t)
        iv = _clip(ol, dl, ins["lo"], ins["hi"], tmin, lim)
        if iv is None:
            continue
        th = _march(ins, ol, dl, iv[0], iv[1], opts.max_steps, opts.eps)
        if th is not None and (th < best_t or (th == best_t and k < best_k)):
            best_t, best_k = th, k
    for tr in sc.tri:
        th = _tri_hit(tr, o, d, tmin, min(tmax, best_t))
        if th is not None and (th < best_t or (th == best_t and tr["id"] < best_k)):
            best_t, best_k = th, tr["id"]
    return best_t, best_k


def trace_any(sc, o, d, tmax, opts):
    for ins in sc.inst:
        ol = _mv(ins["Ainv"], _sub(o, ins["b"]))
        dl = _mv(ins["Ainv"], d)
        iv = _clip(ol, dl, ins["lo"], ins["hi"], 0.0, tmax)
        if iv is None:
            continue
        if _march(ins, ol, dl, iv[0], iv[1], opts.max_steps, opts.eps) is not None:
            return True
    return any(_tri_hit(tr, o, d, 0.0, tmax) is not None for tr in sc.tri)


def _normal(ins, o, d, t, h_fd):
    ol = _mv(ins["Ainv"], _sub(o, ins["b"]))
    dl = _mv(ins["Ainv"], d)
    p = _add(ol, _mul(dl, t))
    h = h_fd / ins["sigma"]
    g = []
    for ax in range(3):
        e = [0.0, 0.0, 0.0]; e[ax] = h
        g.append(_cut_de(ins, _add(p, e)) - _cut_de(ins, _sub(p, e)))
    nw = _mtv(ins["Ainv"], g)
    ln = _len(nw)
    return _mul(d, -1.0) if not ln > 0 else _mul(nw, 1.0 / ln)


def _item(sc, k):
    return sc.inst[k] if k < len(sc.inst) else sc.tri[k - len(sc.inst)]


def _shade(sc, o, d, t, k, opts):
    ins = _item(sc, k)
    if k < len(sc.inst):
        n = _normal(ins, o, d, t, opts.fd_h)
    else:
        n = ins["n"] if _dot(ins["n"], d) <= 0.0 else _mul(ins["n"], -1.0)
    p = _add(o, _mul(d, t))
    V = 1.0
    if opts.shadows:
        ps = _add(p, _mul(n, opts.shadow_offset))
        ls = _sub(sc.light, ps)
        dist = _len(ls)
        if trace_any(sc, ps, _mul(ls, 1.0 / dist), dist, opts):
            V = 0.0
    ell = _nrm(_sub(sc.light, p))
    lam = max(0.0, _dot(n, ell))
    c = tuple(ins["albedo"][i] * (sc.ambient + V * lam * sc.light_rgb[i]) for i in range(3))
    return c, n, p


def render(scene, cam, opts):
    """Whole image; returns (rgb list of H*W tuples, t list, inst list)."""
    import numpy as np
    sc = ScalarScene(scene)
    W, H = opts.width, opts.height
    eye = tuple(float(v) for v in cam.eye)
    f = _nrm(_sub(tuple(float(v) for v in cam.target), eye))
    r = _nrm(_cross(tuple(float(v) for v in cam.up), f))
    u = _cross(f, r)
    sh = math.tan(math.radians(float(cam.vfov_deg)) / 2.0)
    rgb, tt, ii = [], [], []
    pix_all = np.arange(W * H)
    offs = [sample_offsets(opts, pix_all, s) for s in range(opts.spp)]
    for pix in range(W * H):
        x, y = pix % W, pix // W
        acc = [0.0, 0.0, 0.0]
        for s in range(opts.spp):
            jx, jy = float(offs[s][0][pix]), float(offs[s][1][pix])
            sx = (2.0 * (x + jx) / W - 1.0) * sh * (W / H)
            sy = (1.0 - 2.0 * (y + jy) / H) * sh
            d = _nrm(_add(_add(f, _mul(r, sx)), _mul(u, sy)))
            t, k = trace_closest(sc, eye, d, opts.tmin, opts.tmax, opts)
            if k < 0:
                c = sc.bg
            else:
                c, n, p = _shade(sc, eye, d, t, k, opts)
                rho = _item(sc, k)["refl"]
                if opts.bounces >= 1 and rho > 0:
                    dn = _dot(d, n)
                    rd = _sub(d, _mul(n, 2.0 * dn))
                    ob = _add(p, _mul(n, opts.shadow_offset))
                    t2, k2 = trace_closest(sc, ob, rd, 0.0, opts.tmax, opts)
                    cref = sc.bg if k2 < 0 else _shade(sc, ob, rd, t2, k2, opts)[0]
                    c = tuple((1.0 - rho) * c[i] + rho * cref[i] for i in range(3))
            for i in range(3):
                acc[i] += c[i]
            if s == 0:
                tt.append(t); ii.append(k)
        rgb.append(tuple(a / opts.spp for a in acc))
    return rgb, tt, ii
