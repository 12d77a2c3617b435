"""FP64 brute-force sphere tracer (test infrastructure; see package header).

The render follows the per-ray pipeline of the paper's Sec. 2.2.3 and
Sec. 4.1 in this order:

1. ray generation: a pinhole camera ray from the eye through each pixel
   (the ray-generation shader's role);
2. candidate search: every instance's local AABB is slab-tested in the
   instance's local space (Sec. 4.1: the transforms live in an instance
   buffer so intersection works in local space).  Brute force over all
   instances -- no BVH -- so that the GPU's BVH is checked too;
3. intersection: sphere tracing of the primitive's estimator inside the
   clipped interval [t0, t1] (the intersection-shader role);
4. closest hit: the lexicographic minimum of (t, instance index) over all
   candidates.  Each candidate's march is a fixed sequence, so marching it
   fully and taking the minimum afterwards gives the same answer as pruning
   with the running best in any visiting order;
5. closest-hit shading: central-difference normal, Lambert term with one
   shadow ray (the shadow hit groups are intersection-only, Listing "Hit
   group creation", so a shadow ray is occluded when *any* instance reports
   a hit) and an optional mirror bounce shaded the same way;
6. miss: the background colour (the radiance miss shader).

Triangle meshes (Sec. 4.1, listing "Triangle geometry creation"; the plane
of the sample scene, Fig. 4) are placed by their instance transforms in
float64 and intersected in closed form -- the plane equation and signed-area
barycentric coordinates, both sides of a triangle -- against every ray;
their hits join the same lexicographic closest-hit rule, with ids following
the procedural instances.

Readings of points the paper leaves open are listed in the project's design
notes; the ones that fix arithmetic are restated where they are used below.

Besides colour, distance and instance index the oracle reports, per pixel,
whether any traced ray passed within 1e-3 of a surface without stopping
(E1), ran out of march steps (E2), stopped with a value in [0.98 eps, eps)
(E3), or hit where the normal itself is ill-conditioned -- it turns by more
than 1e-3 when the hit point moves by 1e-7 t, about the float32 error of a
hit point, along any of four fixed directions; for a bounce hit also by the
displacement its direction inherits from the primary normal (E4) -- the
places where float32 and float64 may legitimately differ -- and per-type
counts of estimator evaluations and fractal iterations in canonical
front-to-back order (for work accounting).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import de as D
from .de import de_eval, JULIA, MANDELBULB

HIT, MISS_EXIT, MISS_BUDGET, MISS_NAN = 0, 1, 2, 3
E1_GRAZE, E2_BUDGET, E3_MARGINAL, E4_NORMAL, E5_TRIANGLE = 1, 2, 4, 8, 16
# E5: a triangle decision float32 may take differently -- the ray passes
# within 1e-5 (barycentric) of a triangle's edge, meets its plane at a
# grazing angle (|n.d| < 1e-3), or hits a triangle and a procedural surface
# at distances within 1e-5 relative of each other.
TRI_EDGE = 1e-5
TRI_GRAZE = 1e-3
TRI_TIE = 1e-5
GRAZE_V = 1e-3
# E4: displacement of the hit point (relative to t) at which the normal's
# conditioning is probed -- about four float32 ulps of the hit distance --
# and the normal change that flags it (half the radiance tolerance).
E4_REL_SHIFT = 1e-7
E4_MAX_DN = 1e-3
_E4_DIRS = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], np.float64) / np.sqrt(3.0)

M32 = 0xFFFFFFFF
# magnitude bound of a user closest-hit colour (outputs beyond it are clamped)
USER_COLOUR_BOUND = 2.0 ** 24


def lowbias32(x):
    """Wellons' 'lowbias32' 32-bit integer hash (public domain, 2018).

    Three xor-shifts and two odd multiplies modulo 2^32; works on Python ints
    or uint32/uint64 numpy arrays.
    """
    if isinstance(x, np.ndarray):
        x = x.astype(np.uint64) & M32
        x ^= x >> np.uint64(16)
        x = (x * np.uint64(0x7FEB352D)) & np.uint64(M32)
        x ^= x >> np.uint64(15)
        x = (x * np.uint64(0x846CA68B)) & np.uint64(M32)
        x ^= x >> np.uint64(16)
        return x
    x &= M32
    x ^= x >> 16
    x = (x * 0x7FEB352D) & M32
    x ^= x >> 15
    x = (x * 0x846CA68B) & M32
    x ^= x >> 16
    return x


@dataclass
class Prepared:
    A: np.ndarray        # (N, 3, 3)
    b: np.ndarray        # (N, 3)
    Ainv: np.ndarray     # (N, 3, 3)
    sigma: np.ndarray    # (N,)
    lo: np.ndarray       # (N, 3)
    hi: np.ndarray       # (N, 3)
    gtype: np.ndarray    # (N,)
    prm: np.ndarray      # (N, 8)
    cut: np.ndarray      # (N, 4): unit normal n and offset d of the kept half-space n.p <= d; zeros = none
    albedo: np.ndarray   # (N + T, 3): procedural instances, then triangles
    refl: np.ndarray     # (N + T,)
    tri: np.ndarray      # (T, 3, 3) world-space triangle vertices
    tri_n: np.ndarray    # (T, 3) unit face normals
    n_proc: int          # N: triangle j reports id N + j
    light: np.ndarray
    light_rgb: np.ndarray
    ambient: float
    background: np.ndarray


def unit_cuts(scene) -> np.ndarray:
    """Cutting planes per geometry (Fig. 5: the Julia set cut by planes) as
    (n / |n|, d / |n|), so that n.p - d is the signed distance to the plane;
    a zero normal (or no ``geom_cut`` at all) means no cut."""
    G = len(scene.geom_type)
    raw = getattr(scene, "geom_cut", None)
    c = np.zeros((G, 4)) if raw is None else np.asarray(raw, np.float64).reshape(G, 4).copy()
    nn = np.linalg.norm(c[:, :3], axis=1)
    on = nn > 0
    c[on] /= nn[on, None]
    return c


def apply_cut(v, pts, cut):
    """CSG intersection of a primitive with its kept half-space: the
    estimator becomes max(DE, n.p - d) where a cut is set (a NaN estimate
    stays NaN).  ``cut`` is (m, 4) or (4,) per point."""
    cut = np.broadcast_to(np.asarray(cut, np.float64), (pts.shape[0], 4))
    on = np.any(cut[:, :3] != 0.0, axis=1)
    if not on.any():
        return v
    g = np.einsum("mi,mi->m", pts, cut[:, :3]) - cut[:, 3]
    return np.where(on, np.maximum(v, g), v)


def mesh_triangles(scene):
    """World-space triangles of the scene's meshes, instance-major (every
    placement of a mesh, then its triangles in index order), and their
    material indices.  Vertices are placed in float64: v_w = A v + b."""
    tris, mats = [], []
    for mesh in (getattr(scene, "meshes", None) or []):
        v = np.asarray(mesh["vertices"], np.float64).reshape(-1, 3)
        f = np.asarray(mesh["indices"], np.int64).reshape(-1, 3)
        xf = np.asarray(mesh["inst_xform"], np.float64).reshape(-1, 3, 4)
        for mat, x in zip(np.asarray(mesh["inst_mat"], np.int64).reshape(-1), xf):
            w = v @ x[:, :3].T + x[:, 3]
            tris.append(w[f])
            mats.append(np.full(f.shape[0], mat, np.int64))
    if not tris:
        return np.zeros((0, 3, 3)), np.zeros(0, np.int64)
    return np.concatenate(tris), np.concatenate(mats)


def triangle_hits(prep, o, d, tmin, tmax):
    """Every ray against every triangle: the ray meets the triangle's plane
    at t = n.(v0 - o) / n.d and hits when the signed-area barycentric
    coordinates of that point are all >= 0 and t lies in [tmin, tmax].

    Returns the hit distance t (m, T) (+inf where no hit), the plane
    distance (m, T) whether or not the point is inside, the smallest
    barycentric coordinate of the plane point (m, T) and |n.d| (m, T)."""
    m, T = o.shape[0], prep.tri.shape[0]
    if T == 0:
        z = np.zeros((m, 0))
        return z + np.inf, z + np.inf, z, z
    n = prep.tri_n
    v0, v1, v2 = prep.tri[:, 0], prep.tri[:, 1], prep.tri[:, 2]
    nd = d @ n.T
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (np.sum(v0 * n, axis=1)[None, :] - o @ n.T) / nd
    p = o[:, None, :] + t[..., None] * d[:, None, :]
    area = np.sum(np.cross(v1 - v0, v2 - v0) * n, axis=1)          # twice the area
    lam = [np.sum(np.cross(b[None] - p, c[None] - p) * n[None], axis=2) / area[None]
           for b, c in ((v1, v2), (v2, v0), (v0, v1))]
    bmin = np.minimum(np.minimum(lam[0], lam[1]), lam[2])
    tmin = np.broadcast_to(np.asarray(tmin, np.float64), (m,))[:, None]
    tmax = np.broadcast_to(np.asarray(tmax, np.float64), (m,))[:, None]
    ok = (nd != 0.0) & (bmin >= 0.0) & (t >= tmin) & (t <= tmax)
    bmin = np.where(np.isfinite(bmin), bmin, np.inf)
    t_plane = np.where(np.isfinite(t), t, np.inf)
    return np.where(ok, t, np.inf), t_plane, bmin, np.abs(nd)


def prepare(scene) -> Prepared:
    """Per-instance local frames from the float32 scene, upcast to float64.

    The instance transform is a 3x4 local-to-world affine [A | b]; the local
    ray is o' = A^-1 (o - b), d' = A^-1 d (not renormalised, so t is shared
    between frames), and sigma = the smallest singular value of A scales a
    local distance into a world-space lower bound.
    """
    xf = np.asarray(scene.inst_xform, np.float64).reshape(-1, 3, 4)
    A = xf[:, :, :3]
    b = xf[:, :, 3]
    Ainv = np.linalg.inv(A)
    sigma = np.linalg.svd(A, compute_uv=False)[:, -1]
    g = np.asarray(scene.inst_geom, np.int64)
    aabb = np.asarray(scene.geom_aabb, np.float64)[g]
    mat = np.asarray(scene.inst_mat, np.int64)
    tri, tri_mat = mesh_triangles(scene)
    e1, e2 = tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0]
    nrm = np.cross(e1, e2)
    tri_n = nrm / np.maximum(np.linalg.norm(nrm, axis=1), 1e-300)[:, None]
    alb = np.asarray(scene.mat_albedo, np.float64)
    rfl = np.asarray(scene.mat_refl, np.float64)
    return Prepared(
        A=A, b=b, Ainv=Ainv, sigma=sigma, lo=aabb[:, 0:3], hi=aabb[:, 3:6],
        gtype=np.asarray(scene.geom_type, np.int64)[g],
        prm=np.asarray(scene.geom_params, np.float64)[g],
        cut=unit_cuts(scene)[g],
        albedo=np.concatenate([alb[mat], alb[tri_mat]]),
        refl=np.concatenate([rfl[mat], rfl[tri_mat]]),
        tri=tri, tri_n=tri_n, n_proc=int(g.shape[0]),
        light=np.asarray(scene.light_pos, np.float64),
        light_rgb=np.asarray(scene.light_rgb, np.float64),
        ambient=float(scene.ambient),
        background=np.asarray(scene.background, np.float64),
    )


def _normalize(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def sample_offsets(opts, pix, s):
    """Sub-pixel offsets (jx, jy) of sample s for flat pixel indices pix.

    Pixel centres when spp = 1 and jitter is off; otherwise
    k = H(H(H(seed_lo ^ H(seed_hi)) ^ (y W + x)) ^ s) and
    jx = (H(k ^ 0xA511E9B3) >> 8) 2^-24, jy = (H(k ^ 0x63D83595) >> 8) 2^-24.
    """
    pix = np.asarray(pix, np.int64)
    if opts.spp == 1 and not opts.jitter:
        h = np.full(pix.shape, 0.5)
        return h, h.copy()
    seed = int(opts.seed) & 0xFFFFFFFFFFFFFFFF
    s_lo, s_hi = seed & M32, seed >> 32
    k0 = lowbias32(s_lo ^ lowbias32(s_hi))
    lin = (pix.astype(np.uint64) & np.uint64(M32))
    k = lowbias32(lowbias32(np.uint64(k0) ^ lin) ^ np.uint64(s))
    jx = (lowbias32(k ^ np.uint64(0xA511E9B3)) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
    jy = (lowbias32(k ^ np.uint64(0x63D83595)) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
    return jx, jy


def camera_rays(cam, opts, pix, s=0):
    """Pinhole camera, vertical field of view, left-handed (D3D) frame.

    f = normalize(target - eye), r = normalize(up x f), u = f x r;
    s_x = (2 (x + jx) / W - 1) tan(fov/2) W/H, s_y = (1 - 2 (y + jy) / H) tan(fov/2);
    d = normalize(f + s_x r + s_y u); row 0 is the top of the image.
    """
    eye = np.asarray(cam.eye, np.float64)
    f = _normalize(np.asarray(cam.target, np.float64) - eye)
    r = _normalize(np.cross(np.asarray(cam.up, np.float64), f))
    u = np.cross(f, r)
    W, H = opts.width, opts.height
    sh = math.tan(math.radians(float(cam.vfov_deg)) / 2.0)
    pix = np.asarray(pix, np.int64)
    x = (pix % W).astype(np.float64)
    y = (pix // W).astype(np.float64)
    jx, jy = sample_offsets(opts, pix, s)
    sx = (2.0 * (x + jx) / W - 1.0) * sh * (W / H)
    sy = (1.0 - 2.0 * (y + jy) / H) * sh
    d = _normalize(f[None, :] + sx[:, None] * r[None, :] + sy[:, None] * u[None, :])
    o = np.broadcast_to(eye, d.shape).copy()
    return o, d


def slab(o_l, d_l, lo, hi, tmin, tmax):
    """Closed-interval slab test in local space.

    Per axis with d_i != 0 the entry/exit are the ordered (lo_i - o_i)/d_i and
    (hi_i - o_i)/d_i; with d_i == 0 the axis is unconstrained when
    lo_i <= o_i <= hi_i and empty otherwise.  t0 = max(entries, tmin),
    t1 = min(exits, tmax); the instance is a candidate iff t0 <= t1.
    """
    t0 = np.asarray(tmin, np.float64) + np.zeros(o_l.shape[:-1])
    t1 = np.asarray(tmax, np.float64) + np.zeros(o_l.shape[:-1])
    empty = np.zeros(o_l.shape[:-1], bool)
    for i in range(3):
        oi, di = o_l[..., i], d_l[..., i]
        zero = di == 0.0
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (lo[..., i] - oi) / np.where(zero, 1.0, di)
            tb = (hi[..., i] - oi) / np.where(zero, 1.0, di)
        tl = np.where(zero, -np.inf, np.minimum(ta, tb))
        th = np.where(zero, np.inf, np.maximum(ta, tb))
        empty |= zero & ((oi < lo[..., i]) | (oi > hi[..., i]))
        t0 = np.maximum(t0, tl)
        t1 = np.minimum(t1, th)
    return t0, t1, (t0 <= t1) & ~empty


def march(gtype, o_l, d_l, t0, t1, prm, sigma, n_max, eps, cut=None):
    """Sphere tracing of one primitive type over many (ray, instance) pairs.

    For each pair: t = t0; repeat at most n_max times: v = sigma DE(o' + t d')
    (DE cut by the pair's plane when ``cut`` is given, see apply_cut);
    if v < eps: hit at t; t += v; if t > t1: miss.  Running out of steps is a
    miss; a NaN value ends the march as a miss.  Returns the full histories
    (t_i, v_i, iterations_i) for the diagnostics and the work count.
    """
    P = t0.shape[0]
    T = np.full((P, n_max), np.inf)
    V = np.full((P, n_max), np.inf)
    IT = np.zeros((P, n_max), np.int32)
    n = np.zeros(P, np.int64)
    out = np.full(P, MISS_BUDGET, np.int64)
    thit = np.full(P, np.inf)
    t = t0.astype(np.float64).copy()
    idx = np.arange(P)
    for i in range(n_max):
        if idx.size == 0:
            break
        pts = o_l[idx] + t[idx, None] * d_l[idx]
        v, it = de_eval(gtype, pts, prm[idx])
        if cut is not None:
            v = apply_cut(v, pts, cut[idx])
        v = sigma[idx] * v
        T[idx, i] = t[idx]
        V[idx, i] = v
        IT[idx, i] = it
        n[idx] = i + 1
        nan = np.isnan(v)
        hit = v < eps
        out[idx[hit]] = HIT
        thit[idx[hit]] = t[idx[hit]]
        out[idx[nan]] = MISS_NAN
        keep = ~hit & ~nan
        idx = idx[keep]
        t[idx] = t[idx] + v[keep]
        gone = t[idx] > t1[idx]
        out[idx[gone]] = MISS_EXIT
        idx = idx[~gone]
    return dict(T=T, V=V, IT=IT, n=n, out=out, thit=thit)


def _pair_flags(T, V, n, out, t_lim, eps, departure):
    """E1/E2/E3 flags of marches restricted to steps with t_i <= t_lim.

    E1: a local minimum v_i < 1e-3 among those steps (v_{i-1} >= v_i <= v_{i+1};
    the last considered step of a march that did not hit needs only
    v_{i-1} >= v_i) other than the terminal hit step, outside the initial
    non-decreasing run of a secondary ray leaving its own surface.
    E2: all n_max steps considered and the march ran out of steps.
    E3: terminal hit value in [0.98 eps, eps) (evaluated by the caller).
    """
    P, N = V.shape
    steps = np.arange(N)[None, :]
    rel_mask = (T <= t_lim[:, None]) & (steps < n[:, None])
    rel = rel_mask.sum(1)
    terminal = (out == HIT) & (rel == n)
    Vp = np.concatenate([np.full((P, 1), np.inf), V[:, :-1]], 1)
    Vn = np.concatenate([V[:, 1:], np.full((P, 1), np.inf)], 1)
    last = steps == (rel - 1)[:, None]
    with np.errstate(invalid="ignore"):
        prev_ok = Vp >= V
        next_ok = np.where(last, True, V <= Vn)
        small = V < GRAZE_V
        # departure run: indices before the first decrease
        dec = (Vn < V) & (steps < (n - 1)[:, None])
    first_dec = np.where(dec.any(1), dec.argmax(1), N)
    dep_len = np.where(departure, first_dec + 1, 0)
    in_dep = steps < dep_len[:, None]
    term_step = terminal[:, None] & (steps == (n - 1)[:, None])
    graze = rel_mask & prev_ok & next_ok & small & ~term_step & ~in_dep
    e1 = graze.any(1)
    e2 = (out == MISS_BUDGET) & (rel == n) & (n == N)
    vt = V[np.arange(P), np.maximum(n - 1, 0)]
    e3 = (out == HIT) & (vt >= 0.98 * eps) & (vt < eps)
    return e1, e2, e3, rel_mask


class _Counts:
    def __init__(self):
        self.evals = np.zeros(7, np.int64)
        self.iters = np.zeros(7, np.int64)
        self.normal_evals = np.zeros(7, np.int64)
        self.normal_iters = np.zeros(7, np.int64)
        self.rays = {"primary": 0, "shadow": 0, "bounce": 0, "bounce_shadow": 0}

    def as_dict(self):
        return dict(evals=self.evals.tolist(), iters=self.iters.tolist(),
                    normal_evals=self.normal_evals.tolist(),
                    normal_iters=self.normal_iters.tolist(), rays=dict(self.rays))


def _candidates(prep, o, d, tmin, tmax, block=256):
    """All (ray, instance) pairs whose local AABB interval is non-empty."""
    m = o.shape[0]
    N = prep.gtype.shape[0]
    R, K, T0, T1, OL, DL = [], [], [], [], [], []
    for k0 in range(0, N, block):
        ks = slice(k0, min(N, k0 + block))
        Ainv = prep.Ainv[ks]                                   # (B,3,3)
        ol = np.einsum("kij,mkj->mki", Ainv, o[:, None, :] - prep.b[ks][None])
        dl = np.einsum("kij,mj->mki", Ainv, d)
        t0, t1, cand = slab(ol, dl, prep.lo[ks][None], prep.hi[ks][None],
                            tmin[:, None], tmax[:, None])
        r_i, k_i = np.nonzero(cand)
        R.append(r_i); K.append(k_i + k0)
        T0.append(t0[r_i, k_i]); T1.append(t1[r_i, k_i])
        OL.append(ol[r_i, k_i]); DL.append(dl[r_i, k_i])
    cat = np.concatenate
    return cat(R), cat(K), cat(T0), cat(T1), cat(OL).reshape(-1, 3), cat(DL).reshape(-1, 3)


def trace(prep, o, d, tmin, tmax, opts, mode, source=None, counts=None):
    """Trace rays against all instances.

    mode 'closest': returns t (inf on miss), instance (-1 on miss), the winning
    pair's local point data and per-ray exclusion bits.  mode 'any': returns
    occlusion and exclusion bits.  ``source`` (per ray, -1 for none) names the
    instance a secondary ray leaves, for the departure-run rule.
    """
    m = o.shape[0]
    tmin = np.broadcast_to(np.asarray(tmin, np.float64), (m,)).copy()
    tmax = np.broadcast_to(np.asarray(tmax, np.float64), (m,)).copy()
    R, K, T0, T1, OL, DL = _candidates(prep, o, d, tmin, tmax)
    P = R.shape[0]
    n_max, eps = int(opts.max_steps), float(opts.eps)
    res = dict(out=np.full(P, MISS_BUDGET), thit=np.full(P, np.inf), n=np.zeros(P, np.int64))
    hist = {}
    for gt in np.unique(prep.gtype[K]) if P else []:
        sel = np.nonzero(prep.gtype[K] == gt)[0]
        h = march(int(gt), OL[sel], DL[sel], T0[sel], T1[sel], prep.prm[K[sel]],
                  prep.sigma[K[sel]], n_max, eps, cut=prep.cut[K[sel]])
        res["out"][sel] = h["out"]; res["thit"][sel] = h["thit"]; res["n"][sel] = h["n"]
        hist[int(gt)] = (sel, h)

    excl = np.zeros(m, np.int64)
    src = np.full(m, -1, np.int64) if source is None else np.asarray(source, np.int64)
    departure_pair = (src[R] == K) if P else np.zeros(0, bool)

    if mode == "closest":
        t_best = np.full(m, np.inf)
        inst = np.full(m, -1, np.int64)
        win = np.full(m, -1, np.int64)
        hit_pairs = np.nonzero(res["out"] == HIT)[0]
        if hit_pairs.size:
            order = np.lexsort((K[hit_pairs], res["thit"][hit_pairs], R[hit_pairs]))
            hp = hit_pairs[order]
            first = np.ones(hp.size, bool)
            first[1:] = R[hp][1:] != R[hp][:-1]
            hp = hp[first]
            t_best[R[hp]] = res["thit"][hp]
            inst[R[hp]] = K[hp]
            win[R[hp]] = hp
        # triangles: the nearest triangle hit wins over a procedural hit only
        # when strictly nearer (its id, n_proc + j, is larger)
        tt, tpl, bmin, cosd = triangle_hits(prep, o, d, tmin, tmax)
        if tt.shape[1]:
            j = np.argmin(tt, axis=1)
            rows = np.arange(m)
            t_tri = tt[rows, j]
            better = np.isfinite(t_tri) & (t_tri < t_best)
            both = np.isfinite(t_tri) & np.isfinite(t_best)
            gap = np.abs(np.where(both, t_tri, 0.0) - np.where(both, t_best, 0.0))
            tie = both & (gap <= TRI_TIE * np.maximum(1.0, np.where(both, np.minimum(t_tri, t_best), 0.0)))
            t_best = np.where(better, t_tri, t_best)
            inst = np.where(better, prep.n_proc + j, inst)
            win = np.where(better, -1, win)
            t_lim = np.where(np.isfinite(t_best), t_best, tmax)
            edge = (np.abs(bmin) < TRI_EDGE) & (tpl >= tmin[:, None]) & (tpl <= t_lim[:, None] * (1 + TRI_TIE))
            graze = better & (cosd[rows, j] < TRI_GRAZE)
            excl |= np.where(edge.any(axis=1) | graze | tie, E5_TRIANGLE, 0)
        t_lim_ray = np.where(np.isfinite(t_best), t_best, tmax)
        for gt, (sel, h) in hist.items():
            e1, e2, e3, rel_mask = _pair_flags(h["T"], h["V"], h["n"], h["out"],
                                               t_lim_ray[R[sel]], eps, departure_pair[sel])
            is_win = win[R[sel]] == sel
            bits = e1 * E1_GRAZE | e2 * E2_BUDGET | (e3 & is_win) * E3_MARGINAL
            np.bitwise_or.at(excl, R[sel], bits.astype(np.int64))
        if counts is not None:
            _count_canonical(prep, R, K, T0, res, hist, m, "closest", counts)
        return dict(t=t_best, inst=inst, win=win, pairs=(R, K, OL, DL), excl=excl)

    # any-hit (shadow rays): occluded if any instance reports a hit
    occluded = np.zeros(m, bool)
    robust = np.zeros(m, bool)
    flagged = np.zeros(m, bool)
    for gt, (sel, h) in hist.items():
        e1, e2, e3, _ = _pair_flags(h["T"], h["V"], h["n"], h["out"], T1[sel], eps,
                                    departure_pair[sel])
        hit = h["out"] == HIT
        np.logical_or.at(occluded, R[sel], hit)
        np.logical_or.at(robust, R[sel], hit & ~e3)
        np.logical_or.at(flagged, R[sel], e1 | e2 | e3)
        bits = e1 * E1_GRAZE | e2 * E2_BUDGET | e3 * E3_MARGINAL
        np.bitwise_or.at(excl, R[sel], bits.astype(np.int64))
    tt, tpl, bmin, cosd = triangle_hits(prep, o, d, tmin, tmax)
    if tt.shape[1]:
        th = np.isfinite(tt)
        occluded |= th.any(axis=1)
        robust |= (th & (np.abs(bmin) >= TRI_EDGE) & (cosd >= TRI_GRAZE)).any(axis=1)
        edge = (np.abs(bmin) < TRI_EDGE) & (tpl >= tmin[:, None]) & (tpl <= tmax[:, None])
        e5 = edge.any(axis=1) | (th & (cosd < TRI_GRAZE)).any(axis=1)
        excl |= np.where(e5, E5_TRIANGLE, 0)
    excl = np.where(robust, 0, excl)
    if counts is not None:
        _count_canonical(prep, R, K, T0, res, hist, m, "any", counts)
    return dict(occluded=occluded, excl=excl)


def _count_canonical(prep, R, K, T0, res, hist, m, mode, counts):
    """Estimator evaluations in front-to-back order of AABB entry.

    Pairs of a ray are visited by ascending (t0, instance); a closest-hit ray
    skips pairs entering beyond its running best and stops each march once t
    passes it; an any-hit ray stops after its first hit.
    """
    P = R.shape[0]
    if P == 0:
        return
    order = np.lexsort((K, T0, R))
    Rs = R[order]
    rank = np.zeros(P, np.int64)
    if P > 1:
        starts = np.r_[0, np.nonzero(Rs[1:] != Rs[:-1])[0] + 1]
        run = np.zeros(P, np.int64)
        run[starts] = starts
        run = np.maximum.accumulate(run)
        rank = np.arange(P) - run
    pair_of = np.empty(P, np.int64)
    pair_of[:] = order
    where = {}
    for gt, (sel, h) in hist.items():
        for j, pidx in enumerate(sel):
            where[pidx] = (gt, j)
    best = np.full(m, np.inf)
    done = np.zeros(m, bool)
    for r in range(int(rank.max()) + 1):
        pp = pair_of[rank == r]
        for pidx in pp:
            ray = R[pidx]
            if done[ray] or T0[pidx] > best[ray]:
                continue
            gt, j = where[pidx]
            h = hist[gt][1]
            nn = h["n"][j]
            Tj = h["T"][j, :nn]
            use = Tj <= best[ray]
            if gt < counts.evals.size:   # user estimators are not counted
                counts.evals[gt] += int(use.sum())
                counts.iters[gt] += int(h["IT"][j, :nn][use].sum())
            if h["out"][j] == HIT:
                if mode == "any":
                    done[ray] = True
                elif h["thit"][j] < best[ray]:
                    best[ray] = h["thit"][j]


def normals(prep, inst, ol, dl, t, d_world, h_fd, counts=None):
    """Central-difference normal at the hit, mapped to world space.

    p_l = o' + t d', h_l = h_fd / sigma, g_i = DE(p_l + h_l e_i) - DE(p_l - h_l e_i),
    n = normalize(A^-T g); n = -d when g = 0.
    """
    p_l = ol + t[:, None] * dl
    h_l = h_fd / prep.sigma[inst]
    g = np.zeros_like(p_l)
    for gt in np.unique(prep.gtype[inst]):
        sel = np.nonzero(prep.gtype[inst] == gt)[0]
        prm = prep.prm[inst[sel]]
        for ax in range(3):
            e = np.zeros(3); e[ax] = 1.0
            dp = h_l[sel, None] * e[None, :]
            vp, itp = de_eval(int(gt), p_l[sel] + dp, prm)
            vm, itm = de_eval(int(gt), p_l[sel] - dp, prm)
            vp = apply_cut(vp, p_l[sel] + dp, prep.cut[inst[sel]])
            vm = apply_cut(vm, p_l[sel] - dp, prep.cut[inst[sel]])
            g[sel, ax] = vp - vm
            if counts is not None:
                if gt < counts.normal_evals.size:
                    counts.normal_evals[gt] += 2 * sel.size
                    counts.normal_iters[gt] += int(itp.sum() + itm.sum())
    nw = np.einsum("kji,kj->ki", prep.Ainv[inst], g)       # A^-T g
    ln = np.linalg.norm(nw, axis=1)
    zero = ~(ln > 0)
    nw = np.where(zero[:, None], -d_world, nw / np.where(zero, 1.0, ln)[:, None])
    return nw


def normal_sensitivity(prep, inst, ol, dl, t, d_world, h_fd, shift):
    """Largest change of the normal when the hit point moves by ``shift``
    (world units, per hit) along any of four fixed directions."""
    n0 = normals(prep, inst, ol, dl, t, d_world, h_fd)
    worst = np.zeros(t.shape[0])
    for v in _E4_DIRS:
        dv = (prep.Ainv[inst] @ v) * shift[:, None]          # world shift mapped to local space
        n1 = normals(prep, inst, ol + dv, dl, t, d_world, h_fd)
        worst = np.maximum(worst, np.linalg.norm(n1 - n0, axis=1))
    return worst


def _shade_hits(prep, opts, o, d, tr, counts, kind_shadow, extra_shift=None):
    """Lambert shading (with shadow ray) of the rays of ``tr`` that hit.

    Returns colour (m,3), exclusion bits (m,), normals, hit points and the
    normal sensitivity (for E4) of the hits.  ``extra_shift`` (per ray) is
    an additional expected displacement of the hit point, e.g. a bounce ray
    whose direction inherits the float32 error of the primary normal.
    """
    m = o.shape[0]
    hit = tr["inst"] >= 0
    col = np.broadcast_to(prep.background, (m, 3)).copy()
    excl = tr["excl"].copy()
    hidx = np.nonzero(hit)[0]
    nrm = np.zeros((m, 3))
    pw = np.zeros((m, 3))
    sens = np.zeros(m)
    if hidx.size == 0:
        return col, excl, nrm, pw, hit, sens
    R, K, OL, DL = tr["pairs"]
    inst = tr["inst"][hidx]
    t = tr["t"][hidx]
    n = np.zeros((hidx.size, 3))
    dn = np.zeros(hidx.size)
    proc = inst < prep.n_proc
    if proc.any():
        wp = tr["win"][hidx[proc]]
        ip, tp = inst[proc], t[proc]
        n[proc] = normals(prep, ip, OL[wp], DL[wp], tp, d[hidx[proc]], float(opts.fd_h), counts)
        shift = E4_REL_SHIFT * np.maximum(tp, 1.0)
        if extra_shift is not None:
            shift = np.maximum(shift, extra_shift[hidx[proc]])
        dn[proc] = normal_sensitivity(prep, ip, OL[wp], DL[wp], tp, d[hidx[proc]], float(opts.fd_h), shift)
    if (~proc).any():
        # triangles are double-sided: the face normal turned toward the ray
        fn = prep.tri_n[inst[~proc] - prep.n_proc]
        side = np.where(np.sum(fn * d[hidx[~proc]], axis=1) > 0.0, -1.0, 1.0)
        n[~proc] = fn * side[:, None]
    excl[hidx] |= np.where(dn > E4_MAX_DN, E4_NORMAL, 0)
    sens[hidx] = dn
    p = o[hidx] + t[:, None] * d[hidx]
    V = np.ones(hidx.size)
    if opts.shadows:
        ps = p + float(opts.shadow_offset) * n
        ls = prep.light[None, :] - ps
        dist = np.linalg.norm(ls, axis=1)
        sd = ls / dist[:, None]
        sh = trace(prep, ps, sd, 0.0, dist, opts, "any", source=inst, counts=counts)
        counts.rays[kind_shadow] += hidx.size
        V = np.where(sh["occluded"], 0.0, 1.0)
        excl[hidx] |= sh["excl"]
    ell = _normalize(prep.light[None, :] - p)
    lam = np.maximum(0.0, np.sum(n * ell, axis=1))
    c = prep.albedo[inst] * (prep.ambient + (V * lam)[:, None] * prep.light_rgb[None, :])
    # hits on a user type with a closest-hit function take their colour from
    # it, clamped to the library's colour bound of 2^24 in magnitude (a NaN
    # stays NaN): the boundary states this clamp for user shading outputs
    if D.CLOSEST_HIT and proc.any():
        gt = np.full(hidx.size, -1, np.int64)
        gt[proc] = prep.gtype[inst[proc]]
        for ty, fn in D.CLOSEST_HIT.items():
            sel = gt == ty
            if sel.any():
                cu = np.asarray(fn(p[sel], n[sel], -d[hidx[sel]], ell[sel], V[sel], prep.albedo[inst[sel]],
                                   float(prep.ambient), prep.light_rgb, prep.prm[inst[sel]]), np.float64)
                c[sel] = np.clip(cu, -USER_COLOUR_BOUND, USER_COLOUR_BOUND)
    col[hidx] = c
    nrm[hidx] = n
    pw[hidx] = p
    return col, excl, nrm, pw, hit, sens


def _f32_opts(opts):
    """The render options as the float32 values a device receives, upcast."""
    from copy import copy
    o = copy(opts)
    for k in ("eps", "tmin", "tmax", "shadow_offset", "fd_h"):
        setattr(o, k, float(np.float32(getattr(opts, k))))
    return o


def render(scene, cam, opts, pixels=None, prep=None, chunk=4096):
    """Render flat pixel indices ``pixels`` (default: the whole image).

    Returns dict(rgb (m,3), t (m,), inst (m,), excl (m,) bit flags, counts).
    Colour is the mean over samples summed in sample order; t and inst come
    from the primary ray of sample 0 (t = +inf and inst = -1 on a miss).
    """
    if prep is None:
        prep = prepare(scene)
    opts = _f32_opts(opts)
    W, H = opts.width, opts.height
    if pixels is None:
        pixels = np.arange(W * H, dtype=np.int64)
    pixels = np.asarray(pixels, np.int64)
    counts = _Counts()
    out_rgb = np.zeros((pixels.size, 3))
    out_t = np.full(pixels.size, np.inf)
    out_inst = np.full(pixels.size, -1, np.int64)
    out_excl = np.zeros(pixels.size, np.int64)
    for c0 in range(0, pixels.size, chunk):
        pix = pixels[c0:c0 + chunk]
        acc = np.zeros((pix.size, 3))
        for s in range(int(opts.spp)):
            o, d = camera_rays(cam, opts, pix, s)
            counts.rays["primary"] += pix.size
            tr = trace(prep, o, d, float(opts.tmin), float(opts.tmax), opts, "closest",
                       counts=counts)
            col, excl, n, p, hit, sens = _shade_hits(prep, opts, o, d, tr, counts, "shadow")
            if opts.bounces >= 1:
                rho = np.where(hit, prep.refl[np.maximum(tr["inst"], 0)], 0.0)
                bidx = np.nonzero(hit & (rho > 0))[0]
                if bidx.size:
                    dd = d[bidx]
                    nn = n[bidx]
                    rdir = dd - 2.0 * np.sum(dd * nn, axis=1)[:, None] * nn
                    ob = p[bidx] + float(opts.shadow_offset) * nn
                    counts.rays["bounce"] += bidx.size
                    trb = trace(prep, ob, rdir, 0.0, float(opts.tmax), opts, "closest",
                                source=tr["inst"][bidx], counts=counts)
                    # the mirror direction inherits twice the primary normal's
                    # float32 uncertainty, displacing the bounce hit by 2 dn t_b
                    tb = np.where(np.isfinite(trb["t"]), trb["t"], 0.0)
                    cref, exb, _, _, _, _ = _shade_hits(prep, opts, ob, rdir, trb, counts,
                                                        "bounce_shadow",
                                                        extra_shift=2.0 * sens[bidx] * tb)
                    rb = rho[bidx][:, None]
                    col[bidx] = (1.0 - rb) * col[bidx] + rb * cref
                    excl[bidx] |= exb
            acc += col
            out_excl[c0:c0 + pix.size] |= excl
            if s == 0:
                out_t[c0:c0 + pix.size] = tr["t"]
                out_inst[c0:c0 + pix.size] = tr["inst"]
        out_rgb[c0:c0 + pix.size] = acc / float(opts.spp)
    return dict(rgb=out_rgb, t=out_t, inst=out_inst, excl=out_excl, counts=counts.as_dict(),
                pixels=pixels)
