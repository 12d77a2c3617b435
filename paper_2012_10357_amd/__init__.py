"""Python binding of libprocray (argument marshalling only).

Every step of the rendering path runs in the HIP kernels behind the C ABI in
``include/procray.h``; this module converts Python/NumPy scene descriptions
into the ABI's POD structs, passes torch tensor device pointers and HIP
stream handles through, and raises ``ProcrayError`` on any non-OK status.
There is no CPU fallback: if the built library is missing, importing the
binding works but every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprocray.so")

PR_OK, PR_ERR_INVALID_ARG, PR_ERR_OUT_OF_MEMORY, PR_ERR_DEVICE, PR_ERR_NOT_BUILT, \
    PR_ERR_BUSY, PR_ERR_UNSUPPORTED, PR_ERR_TIMEOUT = range(8)
STATUS_NAMES = ["PR_OK", "PR_ERR_INVALID_ARG", "PR_ERR_OUT_OF_MEMORY", "PR_ERR_DEVICE",
                "PR_ERR_NOT_BUILT", "PR_ERR_BUSY", "PR_ERR_UNSUPPORTED", "PR_ERR_TIMEOUT"]
PR_NUM_COUNTS = 34
PR_BVH_HOST_ONLY = 1

# every symbol the header declares
EXPORTS = [
    "pr_scene_create", "pr_scene_add_mesh", "pr_bvh_build", "pr_scene_bvh_export", "pr_scene_device_bytes",
    "pr_scene_destroy", "pr_render", "pr_render_counts", "pr_render_batch", "pr_autotune",
    "pr_server_create", "pr_server_create_simulated", "pr_server_add_scene", "pr_server_submit", "pr_server_wait",
    "pr_server_release", "pr_server_stats_get", "pr_server_destroy", "pr_last_error",
    "pr_abi_version", "pr_device_count", "pr_launch_shape", "pr_register_estimator", "pr_build_estimators",
    "pr_register_closest_hit", "pr_render_noalloc",
]


class ProcrayError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")


# ---------------------------------------------------------------- ABI structs
class Aabb(C.Structure):
    _fields_ = [("lo", C.c_float * 3), ("hi", C.c_float * 3)]


class Geometry(C.Structure):
    _fields_ = [("type", C.c_uint32), ("aabb", Aabb), ("params", C.c_float * 8), ("cut", C.c_float * 4)]


class Instance(C.Structure):
    _fields_ = [("geometry", C.c_uint32), ("material", C.c_uint32), ("xform", C.c_float * 12)]


class Material(C.Structure):
    _fields_ = [("albedo", C.c_float * 3), ("reflectivity", C.c_float)]


class SceneConsts(C.Structure):
    _fields_ = [("light_pos", C.c_float * 3), ("light_rgb", C.c_float * 3), ("ambient", C.c_float),
                ("background", C.c_float * 3)]


class CameraC(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float)]


class RenderOptsC(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("spp", C.c_uint32), ("jitter", C.c_uint32),
                ("max_steps", C.c_uint32), ("shadows", C.c_uint32), ("bounces", C.c_uint32),
                ("eps", C.c_float), ("tmin", C.c_float), ("tmax", C.c_float),
                ("shadow_offset", C.c_float), ("fd_h", C.c_float), ("tile_w", C.c_uint32),
                ("tile_h", C.c_uint32), ("step_budget", C.c_uint32), ("flags", C.c_uint32),
                ("compact_pct", C.c_uint32), ("reserved", C.c_uint32)]


class BvhOpts(C.Structure):
    _fields_ = [("sah_bins", C.c_uint32), ("max_leaf", C.c_uint32), ("c_node", C.c_float),
                ("c_leaf", C.c_float), ("flags", C.c_uint32)]


class BvhNode(C.Structure):
    _fields_ = [("lo", C.c_float * 3), ("first", C.c_uint32), ("hi", C.c_float * 3),
                ("count", C.c_uint32)]


class RequestC(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("cam", CameraC), ("opts", RenderOptsC),
                ("width", C.c_uint32), ("height", C.c_uint32), ("out_rgb", C.c_void_p),
                ("out_t", C.c_void_p), ("out_inst", C.c_void_p), ("user_tag", C.c_uint64)]


class BatchOpts(C.Structure):
    _fields_ = [("tile_w", C.c_uint32), ("tile_h", C.c_uint32), ("step_budget", C.c_uint32),
                ("use_graph", C.c_uint32), ("compact_pct", C.c_uint32)]


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("max_inflight", C.c_uint32),
                ("device", C.c_uint32), ("max_batch", C.c_uint32), ("use_graph", C.c_uint32)]


class RequestResult(C.Structure):
    _fields_ = [("status", C.c_int), ("rgb", C.c_void_p), ("t", C.c_void_p), ("inst", C.c_void_p),
                ("width", C.c_uint32), ("height", C.c_uint32), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_launch", C.c_double), ("t_done", C.c_double),
                ("rays_primary", C.c_uint64), ("rays_shadow", C.c_uint64), ("rays_bounce", C.c_uint64),
                ("user_tag", C.c_uint64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("admitted", C.c_uint64), ("completed", C.c_uint64),
                ("rejected", C.c_uint64), ("launches", C.c_uint64),
                ("pool_bytes_in_use", C.c_uint64), ("pool_bytes_peak", C.c_uint64)]


assert C.sizeof(Geometry) == 76 and C.sizeof(Instance) == 56 and C.sizeof(Material) == 16
assert C.sizeof(SceneConsts) == 40 and C.sizeof(CameraC) == 40 and C.sizeof(RenderOptsC) == 72
assert C.sizeof(BvhNode) == 32

# The C ABI revision these ctypes layouts and signatures describe.
PR_ABI_VERSION = 8

_lib = None


def lib():
    """Loads libprocray.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ProcrayError(PR_ERR_DEVICE, f"{LIB_PATH} is missing: run __graft_entry__.build() "
                                          "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    U32, U64 = C.c_uint32, C.c_uint64
    sig = {
        "pr_scene_create": [P, U32, P, U32, P, U32, P, C.POINTER(C.c_void_p)],
        "pr_bvh_build": [P, P],
        "pr_scene_add_mesh": [P, P, U32, P, U32, P, U32],
        "pr_scene_bvh_export": [P, P, U32, P, U32, C.POINTER(U32), C.POINTER(U32)],
        "pr_scene_device_bytes": [P, C.POINTER(U64)],
        "pr_scene_destroy": [P],
        "pr_render": [P, P, P, U32, U32, P, P, P, P],
        "pr_render_noalloc": [P, P, P, U32, U32, P, P, P, P],
        "pr_render_counts": [P, P, P, U32, U32, P, P],
        "pr_render_batch": [P, U32, P, P],
        "pr_autotune": [P, U32, P],
        "pr_server_create": [P, C.POINTER(C.c_void_p)],
        "pr_server_create_simulated": [P, U32, C.POINTER(C.c_void_p)],
        "pr_server_add_scene": [P, P, C.POINTER(U32)],
        "pr_server_submit": [P, P, C.POINTER(U64)],
        "pr_server_wait": [P, U64, U32, P],
        "pr_server_release": [P, U64],
        "pr_server_stats_get": [P, P],
        "pr_server_destroy": [P],
        "pr_launch_shape": [C.POINTER(U32), C.POINTER(U32)],
        "pr_register_estimator": [C.c_char_p, C.c_char_p, C.POINTER(U32)],
        "pr_build_estimators": [],
        "pr_register_closest_hit": [U32, C.c_char_p],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.pr_last_error.restype = C.c_char_p
    L.pr_last_error.argtypes = []
    L.pr_abi_version.restype = C.c_uint32
    L.pr_device_count.restype = C.c_uint32
    if L.pr_abi_version() != PR_ABI_VERSION:
        raise ProcrayError(PR_ERR_UNSUPPORTED, f"{LIB_PATH} has ABI version {L.pr_abi_version()}, "
                                               f"the binding expects {PR_ABI_VERSION}: rebuild")
    _lib = L
    return L


def _check(st: int):
    if st != PR_OK:
        raise ProcrayError(st, lib().pr_last_error().decode(errors="replace"))


def _arr(ctype, vals):
    a = ctype()
    for i, v in enumerate(vals):
        a[i] = v
    return a


def camera_c(cam) -> CameraC:
    return CameraC(_arr(C.c_float * 3, cam.eye), _arr(C.c_float * 3, cam.target),
                   _arr(C.c_float * 3, cam.up), float(cam.vfov_deg))


PR_RENDER_NATURAL_ORDER = 1
PR_COMPACT_NEVER = 1000


def opts_c(o, tile=(0, 0), step_budget=0, natural_order=False, compact=0) -> RenderOptsC:
    """compact: 0 = tuned choice, 1..100 = regrouping threshold, PR_COMPACT_NEVER = none."""
    return RenderOptsC(int(o.seed) & 0xFFFFFFFFFFFFFFFF, o.spp, o.jitter, o.max_steps, o.shadows,
                       o.bounces, o.eps, o.tmin, o.tmax, o.shadow_offset, o.fd_h, tile[0], tile[1],
                       step_budget, PR_RENDER_NATURAL_ORDER if natural_order else 0, compact, 0)


class Scene:
    """A scene on the device: pr_scene_create + pr_bvh_build."""

    def __init__(self, desc, bvh: Optional[BvhOpts] = None, build: bool = True):
        L = lib()
        G = len(desc.geom_type)
        geoms = (Geometry * G)()
        for g in range(G):
            geoms[g].type = int(desc.geom_type[g])
            geoms[g].aabb.lo = _arr(C.c_float * 3, desc.geom_aabb[g, :3])
            geoms[g].aabb.hi = _arr(C.c_float * 3, desc.geom_aabb[g, 3:])
            geoms[g].params = _arr(C.c_float * 8, desc.geom_params[g])
            cut = getattr(desc, "geom_cut", None)
            if cut is not None:
                geoms[g].cut = _arr(C.c_float * 4, cut[g])
        N = len(desc.inst_geom)
        insts = (Instance * N)()
        for i in range(N):
            insts[i].geometry = int(desc.inst_geom[i])
            insts[i].material = int(desc.inst_mat[i])
            insts[i].xform = _arr(C.c_float * 12, desc.inst_xform[i])
        M = len(desc.mat_refl)
        mats = (Material * M)()
        for m in range(M):
            mats[m].albedo = _arr(C.c_float * 3, desc.mat_albedo[m])
            mats[m].reflectivity = float(desc.mat_refl[m])
        consts = SceneConsts(_arr(C.c_float * 3, desc.light_pos), _arr(C.c_float * 3, desc.light_rgb),
                             float(desc.ambient), _arr(C.c_float * 3, desc.background))
        h = C.c_void_p()
        _check(L.pr_scene_create(geoms, G, insts, N, mats, M, C.byref(consts), C.byref(h)))
        self.handle = h
        self.n_inst = N
        for mesh in (getattr(desc, "meshes", None) or []):
            try:
                self.add_mesh(mesh["vertices"], mesh["indices"], mesh["inst_mat"], mesh["inst_xform"])
            except ProcrayError:
                self.close()
                raise
        if build:
            self.build(bvh)

    def add_mesh(self, vertices, indices, inst_mat, inst_xform):
        """pr_scene_add_mesh: vertices (V, 3), indices (F, 3), one placement per
        entry of inst_mat / inst_xform (K,), (K, 12); clears the build."""
        v = np.ascontiguousarray(vertices, np.float32).reshape(-1, 3)
        f = np.ascontiguousarray(indices, np.uint32).reshape(-1, 3)
        mats = np.asarray(inst_mat).reshape(-1)
        xf = np.asarray(inst_xform, np.float32).reshape(-1, 12)
        K = len(mats)
        insts = (Instance * K)()
        for i in range(K):
            insts[i].geometry = 0
            insts[i].material = int(mats[i])
            insts[i].xform = _arr(C.c_float * 12, xf[i])
        _check(lib().pr_scene_add_mesh(self.handle, v.ctypes.data_as(C.c_void_p), len(v),
                                       f.ctypes.data_as(C.c_void_p), len(f), insts, K))

    def build(self, bvh: Optional[BvhOpts] = None):
        _check(lib().pr_bvh_build(self.handle, C.byref(bvh) if bvh is not None else None))

    def bvh(self):
        L = lib()
        nn, no = C.c_uint32(), C.c_uint32()
        _check(L.pr_scene_bvh_export(self.handle, None, 0, None, 0, C.byref(nn), C.byref(no)))
        nodes = (BvhNode * nn.value)()
        order = (C.c_uint32 * no.value)()
        _check(L.pr_scene_bvh_export(self.handle, nodes, nn.value, order, no.value, None, None))
        lo = np.array([list(n.lo) for n in nodes], np.float32)
        hi = np.array([list(n.hi) for n in nodes], np.float32)
        first = np.array([n.first for n in nodes], np.int64)
        count = np.array([n.count for n in nodes], np.int64)
        return lo, hi, first, count, np.array(order[:], np.int64)

    def device_bytes(self) -> int:
        b = C.c_uint64()
        _check(lib().pr_scene_device_bytes(self.handle, C.byref(b)))
        return b.value

    def close(self):
        if self.handle:
            _check(lib().pr_scene_destroy(self.handle))
            self.handle = None


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        return None
    return C.c_void_p(int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream))


def render(scene: Scene, cam, opts, out_rgb, out_t=None, out_inst=None, stream=None,
           tile=(0, 0), step_budget=0, natural_order=False, compact=0):
    """pr_render into caller-owned torch CUDA tensors (H, W, 3) / (H, W) / (H, W)."""
    H, W = out_rgb.shape[0], out_rgb.shape[1]
    c, o = camera_c(cam), opts_c(opts, tile, step_budget, natural_order, compact)
    _check(lib().pr_render(scene.handle, C.byref(c), C.byref(o), W, H, _ptr(out_rgb), _ptr(out_t),
                           _ptr(out_inst), _stream_ptr(stream)))


def render_noalloc(scene: Scene, cam, opts, out_rgb, out_t=None, out_inst=None, stream=None,
                   tile=(0, 0), step_budget=0, natural_order=False, compact=0):
    """pr_render_noalloc: pr_render with no device allocation (fixed per-device
    scratch; overlapping calls on one device race)."""
    H, W = out_rgb.shape[0], out_rgb.shape[1]
    c, o = camera_c(cam), opts_c(opts, tile, step_budget, natural_order, compact)
    _check(lib().pr_render_noalloc(scene.handle, C.byref(c), C.byref(o), W, H, _ptr(out_rgb), _ptr(out_t),
                                   _ptr(out_inst), _stream_ptr(stream)))


def render_counts(scene: Scene, cam, opts, out_rgb, tile=(0, 0), step_budget=0, compact=0) -> np.ndarray:
    H, W = out_rgb.shape[0], out_rgb.shape[1]
    c, o = camera_c(cam), opts_c(opts, tile, step_budget, compact=compact)
    counts = (C.c_uint64 * PR_NUM_COUNTS)()
    _check(lib().pr_render_counts(scene.handle, C.byref(c), C.byref(o), W, H, _ptr(out_rgb), counts))
    return np.array(counts[:], np.uint64)


def make_requests(items) -> "C.Array":
    """items: sequence of (Scene, camera, opts, rgb, t, inst, tag)."""
    arr = (RequestC * len(items))()
    for i, (sc, cam, o, rgb, t, inst, tag) in enumerate(items):
        arr[i].scene = sc.handle
        arr[i].cam = camera_c(cam)
        arr[i].opts = opts_c(o)
        arr[i].width = rgb.shape[1]
        arr[i].height = rgb.shape[0]
        arr[i].out_rgb = None if rgb is None else rgb.data_ptr()
        arr[i].out_t = None if t is None else t.data_ptr()
        arr[i].out_inst = None if inst is None else inst.data_ptr()
        arr[i].user_tag = tag
    return arr


def render_batch(reqs, tile=(0, 0), step_budget=0, use_graph=False, stream=None, compact=0):
    bo = BatchOpts(tile[0], tile[1], step_budget, 1 if use_graph else 0, compact)
    _check(lib().pr_render_batch(reqs, len(reqs), C.byref(bo), _stream_ptr(stream)))


def autotune(reqs) -> BatchOpts:
    best = BatchOpts()
    _check(lib().pr_autotune(reqs, len(reqs), C.byref(best)))
    return best


class Server:
    """Continuous-batching server (pr_server_*).  ``simulated_us_per_mpix``
    selects the host-only simulated executor."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 2, device: int = 0,
                 max_batch: int = 256, use_graph: bool = False,
                 simulated_us_per_mpix: Optional[int] = None):
        L = lib()
        o = ServerOpts(hbm_budget_bytes, max_inflight, device, max_batch, 1 if use_graph else 0)
        h = C.c_void_p()
        if simulated_us_per_mpix is None:
            _check(L.pr_server_create(C.byref(o), C.byref(h)))
        else:
            _check(L.pr_server_create_simulated(C.byref(o), simulated_us_per_mpix, C.byref(h)))
        self.handle = h

    def add_scene(self, scene: Scene) -> int:
        slot = C.c_uint32()
        _check(lib().pr_server_add_scene(self.handle, scene.handle, C.byref(slot)))
        return slot.value

    def submit(self, scene: Scene, cam, opts, tag: int = 0) -> int:
        r = RequestC()
        r.scene = scene.handle
        r.cam = camera_c(cam)
        r.opts = opts_c(opts)
        r.width, r.height = opts.width, opts.height
        r.user_tag = tag
        t = C.c_uint64()
        _check(lib().pr_server_submit(self.handle, C.byref(r), C.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_ms: int = 60000) -> RequestResult:
        res = RequestResult()
        _check(lib().pr_server_wait(self.handle, ticket, timeout_ms, C.byref(res)))
        return res

    def release(self, ticket: int):
        _check(lib().pr_server_release(self.handle, ticket))

    def stats(self) -> ServerStats:
        s = ServerStats()
        _check(lib().pr_server_stats_get(self.handle, C.byref(s)))
        return s

    def close(self):
        if self.handle:
            _check(lib().pr_server_destroy(self.handle))
            self.handle = None


def device_count() -> int:
    return int(lib().pr_device_count())


def register_estimator(name: str, body: str) -> int:
    """pr_register_estimator: returns the new primitive type for pr_geometry."""
    t = C.c_uint32(0)
    _check(lib().pr_register_estimator(name.encode(), body.encode(), C.byref(t)))
    return int(t.value)


def register_closest_hit(gtype: int, body: str) -> None:
    """pr_register_closest_hit: the shading half of a user hit group."""
    _check(lib().pr_register_closest_hit(int(gtype), body.encode()))


def build_estimators():
    """pr_build_estimators: compile the registered estimators now."""
    _check(lib().pr_build_estimators())


def launch_shape():
    """(compute units, resident 256-thread workgroups per compute unit) of the
    persistent kernel on the current device."""
    cu, wg = C.c_uint32(0), C.c_uint32(0)
    _check(lib().pr_launch_shape(C.byref(cu), C.byref(wg)))
    return int(cu.value), int(wg.value)


def abi_version() -> int:
    return int(lib().pr_abi_version())
