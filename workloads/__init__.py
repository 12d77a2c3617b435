"""Seeded synthetic inputs for procedural-primitive ray tracing.

This module only *builds input data*: geometry records (primitive type, local
AABB, parameters), instance transforms, materials, scene constants, cameras,
render options and request traces.  It holds none of the rendering method's
arithmetic (no distance estimators, no ray generation, no marching, no
shading), so that both the FP64 CPU oracle and the HIP path can consume the
very same FP32 arrays without sharing any of the method's code.

The paper (Proceduray, Sec. 4.1, listings "Procedural geometry creation" and
"Instance buffer creation") describes a scene as procedural geometries given
by an AABB, each with a vector of instance transforms, plus per-instance
material and primitive-type records; the numeric values of its sample scene
are elided there, so the seeded scenes below stand in for it.

Parameter layout per primitive type (``params[0..7]``, unused entries zero):

=============  ==========================================================
SPHERE         r
BOX            cx, cy, cz, hx, hy, hz          (centre, half extents)
TORUS          R, r                             (axis = local y)
BOXFRAME       b, e                             (cube half-size, bar half-thickness)
PACMAN         R, alpha                         (sphere radius, wedge half-angle, rad)
JULIA          c0, c1, c2, c3, n_iter, bailout  (quaternion c, component 0 real)
MANDELBULB     power, n_iter, bailout           (polar axis = local z)
=============  ==========================================================
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

SPHERE, BOX, TORUS, BOXFRAME, PACMAN, JULIA, MANDELBULB = range(7)
TYPE_NAMES = ["sphere", "box", "torus", "boxframe", "pacman", "julia", "mandelbulb"]

MASTER_SEED = 10357


def config_seed(k: int) -> int:
    """Seed of workload configuration ``k`` (1-based)."""
    return MASTER_SEED * 100 + k


@dataclass
class Scene:
    geom_type: np.ndarray      # (G,) uint32
    geom_aabb: np.ndarray      # (G, 6) float32: lo xyz, hi xyz (local space)
    geom_params: np.ndarray    # (G, 8) float32
    inst_geom: np.ndarray      # (N,) uint32
    inst_mat: np.ndarray       # (N,) uint32
    inst_xform: np.ndarray     # (N, 12) float32, row-major 3x4 local->world [A | b]
    mat_albedo: np.ndarray     # (M, 3) float32
    mat_refl: np.ndarray       # (M,) float32
    light_pos: np.ndarray      # (3,) float32
    light_rgb: np.ndarray      # (3,) float32
    ambient: float
    background: np.ndarray     # (3,) float32
    geom_cut: Optional[np.ndarray] = None   # (G, 4) float32: kept half-space n.p <= d; n = 0: none
    # triangle meshes: dicts of vertices (V, 3) f32, indices (F, 3) u32 and one
    # placement per entry of inst_mat (K,) u32 / inst_xform (K, 12) f32
    meshes: Optional[list] = None

    @property
    def n_inst(self) -> int:
        return int(self.inst_geom.shape[0])


@dataclass
class Camera:
    eye: np.ndarray            # (3,) float32
    target: np.ndarray         # (3,) float32
    up: np.ndarray             # (3,) float32
    vfov_deg: float


@dataclass
class RenderOpts:
    width: int
    height: int
    spp: int = 1
    jitter: int = 0
    seed: int = 0
    max_steps: int = 256
    eps: float = 1e-4
    tmin: float = 0.0
    tmax: float = 100.0
    shadows: int = 1
    bounces: int = 0
    shadow_offset: float = 1e-3
    fd_h: float = 1e-3


@dataclass
class Request:
    scene_index: int
    camera: Camera
    opts: RenderOpts
    arrival_s: float = 0.0


@dataclass
class Workload:
    name: str
    scenes: List[Scene]
    requests: List[Request]
    notes: str = ""


# --------------------------------------------------------------------------
# small builders (input construction only)
# --------------------------------------------------------------------------

def _f32(x):
    return np.asarray(x, dtype=np.float32)


def _rot_x(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=np.float64)


def _rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], dtype=np.float64)


def _quat_to_matrix(q):
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ], dtype=np.float64)


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Rotation from a normalised 4-D Gaussian quaternion (uniform on SO(3))."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    return _quat_to_matrix(q)


def xform(rot: np.ndarray, scale: float, pos) -> np.ndarray:
    m = np.zeros((3, 4), dtype=np.float64)
    m[:, :3] = rot * scale
    m[:, 3] = pos
    return m.reshape(12).astype(np.float32)


def julia_escape_halfwidth(c) -> float:
    """Half-width of a cube containing the filled quaternion Julia set of c.

    Any |z| > (1 + sqrt(1 + 4|c|)) / 2 grows under z -> z^2 + c; a 0.05 margin
    keeps the estimator well above eps on the box faces.
    """
    cn = float(np.linalg.norm(np.asarray(c, dtype=np.float64)))
    return (1.0 + math.sqrt(1.0 + 4.0 * cn)) / 2.0 + 0.05


def geom_sphere(r=1.0):
    p = np.zeros(8, np.float32); p[0] = r
    return SPHERE, [-r, -r, -r, r, r, r], p


def geom_box(c, h):
    p = np.zeros(8, np.float32); p[0:3] = c; p[3:6] = h
    lo = np.asarray(c, np.float64) - np.asarray(h, np.float64)
    hi = np.asarray(c, np.float64) + np.asarray(h, np.float64)
    return BOX, list(lo) + list(hi), p


def geom_torus(R=1.0, r=0.3):
    p = np.zeros(8, np.float32); p[0] = R; p[1] = r
    a = R + r
    return TORUS, [-a, -r, -a, a, r, a], p


def geom_boxframe(b=1.0, e=0.05):
    p = np.zeros(8, np.float32); p[0] = b; p[1] = e
    return BOXFRAME, [-b, -b, -b, b, b, b], p


def geom_pacman(R=0.8, mouth_deg=60.0):
    p = np.zeros(8, np.float32); p[0] = R; p[1] = math.radians(mouth_deg) / 2.0
    return PACMAN, [-R, -R, -R, R, R, R], p


def geom_julia(c, n_iter=12, bailout=4.0):
    p = np.zeros(8, np.float32); p[0:4] = c; p[4] = n_iter; p[5] = bailout
    # the half-width is computed from the float32 value of c that is stored
    h = julia_escape_halfwidth(p[0:4].astype(np.float64))
    return JULIA, [-h, -h, -h, h, h, h], p


def geom_mandelbulb(power=8, n_iter=10, bailout=2.0, half=1.2):
    p = np.zeros(8, np.float32); p[0] = power; p[1] = n_iter; p[2] = bailout
    return MANDELBULB, [-half, -half, -half, half, half, half], p


class _SceneBuilder:
    def __init__(self):
        self.gt, self.ga, self.gp, self.gc = [], [], [], []
        self.meshes = []
        self.ig, self.im, self.ix = [], [], []
        self.alb, self.refl = [], []

    def material(self, albedo, refl=0.0) -> int:
        self.alb.append(albedo); self.refl.append(refl)
        return len(self.alb) - 1

    def geometry(self, g, cut=(0.0, 0.0, 0.0, 0.0)) -> int:
        t, aabb, p = g
        self.gt.append(t); self.ga.append(aabb); self.gp.append(p); self.gc.append(cut)
        return len(self.gt) - 1

    def instance(self, geom: int, mat: int, xf: np.ndarray):
        self.ig.append(geom); self.im.append(mat); self.ix.append(xf)

    def mesh(self, vertices, indices, placements):
        """placements: sequence of (material, 3x4 row-major local-to-world)."""
        self.meshes.append(dict(
            vertices=_f32(vertices).reshape(-1, 3),
            indices=np.asarray(indices, np.uint32).reshape(-1, 3),
            inst_mat=np.asarray([m for m, _ in placements], np.uint32),
            inst_xform=_f32([x for _, x in placements]).reshape(-1, 12)))

    def build(self, light_pos, light_rgb=(1, 1, 1), ambient=0.1, background=(0, 0, 0)) -> Scene:
        return Scene(
            geom_type=np.asarray(self.gt, np.uint32),
            geom_aabb=_f32(self.ga).reshape(-1, 6),
            geom_params=_f32(self.gp).reshape(-1, 8),
            inst_geom=np.asarray(self.ig, np.uint32),
            inst_mat=np.asarray(self.im, np.uint32),
            inst_xform=_f32(self.ix).reshape(-1, 12),
            mat_albedo=_f32(self.alb).reshape(-1, 3),
            mat_refl=_f32(self.refl).reshape(-1),
            light_pos=_f32(light_pos), light_rgb=_f32(light_rgb),
            ambient=float(np.float32(ambient)), background=_f32(background),
            geom_cut=_f32(self.gc).reshape(-1, 4),
            meshes=self.meshes or None,
        )


def camera(eye, target=(0, 0, 0), up=(0, 1, 0), vfov_deg=60.0) -> Camera:
    return Camera(_f32(eye), _f32(target), _f32(up), float(np.float32(vfov_deg)))


def log_uniform_side(rng, lo, hi) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


# --------------------------------------------------------------------------
# the five workload configurations
# --------------------------------------------------------------------------

def c1_scene() -> Scene:
    """Unit sphere in [-1,1]^3 plus a ground box y in [-1.1,-1], x,z in [-10,10]."""
    b = _SceneBuilder()
    m_sph = b.material((0.9, 0.2, 0.2))
    m_gnd = b.material((0.8, 0.8, 0.8))
    g_sph = b.geometry(geom_sphere(1.0))
    g_gnd = b.geometry(geom_box((0.0, -1.05, 0.0), (10.0, 0.05, 10.0)))
    ident = np.eye(3)
    b.instance(g_sph, m_sph, xform(ident, 1.0, (0, 0, 0)))
    b.instance(g_gnd, m_gnd, xform(ident, 1.0, (0, 0, 0)))
    return b.build(light_pos=(2, 4, -3))


def c1(width=64, height=64) -> Workload:
    opts = RenderOpts(width, height, spp=1, jitter=0, max_steps=128, eps=1e-4,
                      tmax=100.0, shadows=1, bounces=0)
    req = Request(0, camera((0, 1, -4)), opts)
    return Workload("c1_sphere_ground_64x64", [c1_scene()], [req])


def c2_scene(seed: Optional[int] = None) -> Scene:
    """Teaser-like scene: two pac-men, a quaternion Julia set and a Mandelbulb."""
    rng = np.random.default_rng(config_seed(2) if seed is None else seed)
    b = _SceneBuilder()
    m_pac = b.material((1.0, 0.85, 0.1), 0.3)
    m_jul = b.material((0.3, 0.6, 1.0), 0.3)
    m_man = b.material((0.9, 0.4, 0.3), 0.3)
    g_pac = b.geometry(geom_pacman(0.8, 60.0))
    c = rng.uniform(-0.8, 0.8, 4)
    g_jul = b.geometry(geom_julia(c, 12, 4.0))
    g_man = b.geometry(geom_mandelbulb(8, 10, 2.0))
    yaw0, yaw1 = rng.uniform(0.0, 2.0 * math.pi, 2)
    b.instance(g_pac, m_pac, xform(_rot_y(yaw0), 1.0, (-2.2, 0.0, 0.5)))
    b.instance(g_pac, m_pac, xform(_rot_y(yaw1), 1.0, (2.2, 0.0, 0.5)))
    b.instance(g_jul, m_jul, xform(np.eye(3), 0.6, (-0.8, 0.1, -0.6)))
    b.instance(g_man, m_man, xform(_rot_x(-math.pi / 2), 0.9, (0.9, 0.1, -0.9)))
    return b.build(light_pos=(2, 4, -3))


def c2_opts(width=1920, height=1080) -> RenderOpts:
    return RenderOpts(width, height, spp=1, jitter=0, max_steps=256, eps=1e-4,
                      tmax=100.0, shadows=1, bounces=1)


def c2_camera() -> Camera:
    return camera((0, 1.2, -5.5))


def c2(width=1920, height=1080) -> Workload:
    return Workload("c2_teaser_1080p", [c2_scene()],
                    [Request(0, c2_camera(), c2_opts(width, height))])


def random_instances_scene(rng, n_inst: int, kinds: List[str]) -> Scene:
    """Instances at U[-20,20]^3, scale U[0.5,2], uniform random rotation.

    ``kinds`` lists the primitive kinds drawn uniformly per instance; every
    instance gets its own geometry record (Julia c is drawn per instance).
    """
    b = _SceneBuilder()
    for _ in range(n_inst):
        pos = rng.uniform(-20.0, 20.0, 3)
        scale = rng.uniform(0.5, 2.0)
        rot = random_rotation(rng)
        kind = kinds[int(rng.integers(0, len(kinds)))]
        if kind == "sphere":
            g = geom_sphere(1.0)
        elif kind == "torus":
            g = geom_torus(1.0, 0.3)
        elif kind == "boxframe":
            g = geom_boxframe(1.0, 0.05)
        elif kind == "mandelbulb":
            g = geom_mandelbulb(8, 10, 2.0)
        elif kind == "julia":
            g = geom_julia(rng.uniform(-0.8, 0.8, 4), 12, 4.0)
        elif kind == "pacman":
            g = geom_pacman(0.8, 60.0)
        else:
            raise ValueError(kind)
        gi = b.geometry(g)
        if kinds == C5_KINDS:
            mi = b.material(C2_ALBEDO[kind], 0.0)
        else:
            mi = b.material(rng.uniform(0.2, 0.9, 3), 0.0)
        b.instance(gi, mi, xform(rot, scale, pos))
    return b.build(light_pos=(40, 60, -50))


C3_KINDS = ["sphere", "torus", "boxframe", "mandelbulb", "julia"]
C5_KINDS = ["pacman", "julia", "mandelbulb"]
C2_ALBEDO = {"pacman": (1.0, 0.85, 0.1), "julia": (0.3, 0.6, 1.0), "mandelbulb": (0.9, 0.4, 0.3)}


def c3_scene() -> Scene:
    rng = np.random.default_rng(config_seed(3))
    return random_instances_scene(rng, 1024, C3_KINDS)


def c3_opts(width=1920, height=1080) -> RenderOpts:
    return RenderOpts(width, height, spp=4, jitter=1, seed=config_seed(3), max_steps=256,
                      eps=1e-4, tmax=200.0, shadows=1, bounces=0)


def c3(width=1920, height=1080) -> Workload:
    return Workload("c3_1024inst_1080p_4spp", [c3_scene()],
                    [Request(0, camera((0, 0, -60)), c3_opts(width, height))])


def c4(n_requests=64, lo=128, hi=1024) -> Workload:
    """Batched: seeded cameras over the teaser scene, log-uniform square sides."""
    rng = np.random.default_rng(config_seed(4))
    reqs = []
    for j in range(n_requests):
        a = rng.uniform(-math.pi, math.pi)
        e = math.radians(rng.uniform(5.0, 45.0))
        R = rng.uniform(4.0, 8.0)
        eye = (R * math.cos(e) * math.sin(a), R * math.sin(e), -R * math.cos(e) * math.cos(a))
        s = log_uniform_side(rng, lo, hi)
        opts = RenderOpts(s, s, spp=1, jitter=0, seed=config_seed(4) + j, max_steps=256,
                          eps=1e-4, tmax=100.0, shadows=1, bounces=0)
        reqs.append(Request(0, camera(eye), opts))
    return Workload("c4_batched_64req", [c2_scene()], reqs)


def c5_scenes(n_scenes=8, lo=256, hi=4096) -> List[Scene]:
    rng = np.random.default_rng(config_seed(5))
    scenes = []
    for _ in range(n_scenes):
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        scenes.append(random_instances_scene(rng, n, C5_KINDS))
    return scenes


def c5_requests(n_requests: int, rate_hz=200.0, lo=256, hi=2048, n_scenes=8,
                seed: Optional[int] = None) -> List[Request]:
    """Poisson arrivals (exponential gaps), seeded cameras, sides and spp."""
    base = config_seed(5) * 1000 if seed is None else seed
    rng = np.random.default_rng(base)
    reqs, t = [], 0.0
    for j in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        v = rng.standard_normal(3); v /= np.linalg.norm(v)
        R = rng.uniform(45.0, 60.0)
        s = log_uniform_side(rng, lo, hi)
        spp = int(rng.integers(1, 5))
        opts = RenderOpts(s, s, spp=spp, jitter=1 if spp > 1 else 0, seed=base + j,
                          max_steps=256, eps=1e-4, tmax=200.0, shadows=1, bounces=0)
        up = (0, 1, 0) if abs(v[1]) < 0.99 else (1, 0, 0)
        reqs.append(Request(int(rng.integers(0, n_scenes)), camera(R * v, up=up), opts, t))
    return reqs


def c5(n_requests=6000, n_scenes=8) -> Workload:
    return Workload("c5_served_200rps", c5_scenes(n_scenes), c5_requests(n_requests, n_scenes=n_scenes))


# --------------------------------------------------------------------------
# next-step workloads: the cut Julia set and the animated Mandelbulb
# --------------------------------------------------------------------------

# Two cutting planes in the Julia set's local frame (Fig. 5 shows the set cut
# by two different planes): the front half facing the camera removed, and an
# oblique cut.  Stored unnormalised on purpose; the library normalises.
F1_JULIA_CUTS = [(0.0, 0.0, -1.0, 0.0), (1.0, 1.0, -1.0, 0.15)]


def f1_julia_cut_scene(cut) -> Scene:
    """The teaser's Julia set alone, enlarged, cut by one plane."""
    rng = np.random.default_rng(config_seed(2))
    c = rng.uniform(-0.8, 0.8, 4)          # the same c as the teaser's Julia set
    b = _SceneBuilder()
    m = b.material(C2_ALBEDO["julia"], 0.0)
    g = b.geometry(geom_julia(c, 12, 4.0), cut=cut)
    b.instance(g, m, xform(np.eye(3), 1.5, (0.0, 0.0, 0.0)))
    return b.build(light_pos=(2, 4, -3))


def f1_julia_cut(width=320, height=180) -> Workload:
    """One request per cutting plane, camera in front of the cut face."""
    scenes = [f1_julia_cut_scene(c) for c in F1_JULIA_CUTS]
    opts = RenderOpts(width, height, spp=1, jitter=0, max_steps=256, eps=1e-4, tmax=100.0,
                      shadows=1, bounces=0)
    reqs = [Request(i, camera((0.0, 0.8, -4.0)), opts) for i in range(len(scenes))]
    return Workload("f1_julia_cut", scenes, reqs)


# Ray-marching step budgets of the animation frames (Fig. 6: the Mandelbulb
# is animated by varying the number of ray-marching iterations over time).
F1_ANIM_STEPS = [6, 8, 11, 16, 23, 32, 45, 64, 91, 128, 181, 256]


def f1_mandelbulb_anim_scene() -> Scene:
    b = _SceneBuilder()
    m = b.material(C2_ALBEDO["mandelbulb"], 0.0)
    g = b.geometry(geom_mandelbulb(8, 10, 2.0))
    b.instance(g, m, xform(_rot_x(-math.pi / 2), 1.5, (0.0, 0.0, 0.0)))
    return b.build(light_pos=(2, 4, -3))


def f1_mandelbulb_anim(width=256, height=256, steps=None) -> Workload:
    """One request per animation frame; frame k marches at most steps[k]."""
    steps = F1_ANIM_STEPS if steps is None else steps
    reqs = [Request(0, camera((0.0, 1.0, -4.5)),
                    RenderOpts(width, height, spp=1, jitter=0, max_steps=int(n), eps=1e-4,
                               tmax=100.0, shadows=1, bounces=0))
            for n in steps]
    return Workload("f1_mandelbulb_animation", [f1_mandelbulb_anim_scene()], reqs)


# The paper's sample scene (Fig. 4): a triangle plane mesh under the two
# pac-men, the Julia set and the Mandelbulb of the teaser.
QUAD_VERTICES = [(-1.0, 0.0, -1.0), (1.0, 0.0, -1.0), (1.0, 0.0, 1.0), (-1.0, 0.0, 1.0)]
QUAD_INDICES = [(0, 1, 2), (0, 2, 3)]


def f2_sample_scene() -> Scene:
    """The teaser scene plus a 16 x 16 grey plane of two triangles at y = -1.1."""
    rng = np.random.default_rng(config_seed(2))
    b = _SceneBuilder()
    m_pac = b.material((1.0, 0.85, 0.1), 0.3)
    m_jul = b.material((0.3, 0.6, 1.0), 0.3)
    m_man = b.material((0.9, 0.4, 0.3), 0.3)
    m_pln = b.material((0.75, 0.75, 0.75), 0.0)
    g_pac = b.geometry(geom_pacman(0.8, 60.0))
    c = rng.uniform(-0.8, 0.8, 4)
    g_jul = b.geometry(geom_julia(c, 12, 4.0))
    g_man = b.geometry(geom_mandelbulb(8, 10, 2.0))
    yaw0, yaw1 = rng.uniform(0.0, 2.0 * math.pi, 2)
    b.instance(g_pac, m_pac, xform(_rot_y(yaw0), 1.0, (-2.2, 0.0, 0.5)))
    b.instance(g_pac, m_pac, xform(_rot_y(yaw1), 1.0, (2.2, 0.0, 0.5)))
    b.instance(g_jul, m_jul, xform(np.eye(3), 0.6, (-0.8, 0.1, -0.6)))
    b.instance(g_man, m_man, xform(_rot_x(-math.pi / 2), 0.9, (0.9, 0.1, -0.9)))
    b.mesh(QUAD_VERTICES, QUAD_INDICES, [(m_pln, xform(np.eye(3), 8.0, (0.0, -1.1, 0.0)))])
    return b.build(light_pos=(2, 4, -3))


def f2_sample(width=1920, height=1080) -> Workload:
    return Workload("f2_sample_scene_plane", [f2_sample_scene()],
                    [Request(0, c2_camera(), c2_opts(width, height))])


def pixel_sample(width: int, height: int, n: int, seed: int) -> np.ndarray:
    """Seeded uniform subset of flat pixel indices (y * width + x), sorted."""
    rng = np.random.default_rng(seed)
    n = min(n, width * height)
    return np.sort(rng.choice(width * height, size=n, replace=False)).astype(np.int64)
