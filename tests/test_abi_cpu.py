"""Host-side checks that need no GPU: the library loads and exports every
declared symbol, validation errors are reported before any device work, and
the BVH built on the host is well formed."""
import ctypes as C
import re
import os

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2012_10357_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_2012_10357_amd import build
        build.build()
    P.lib()
    return P


def test_exports_every_declared_symbol(P):
    hdr = open(os.path.join(ROOT, "include", "procray.h")).read()
    declared = set(re.findall(r"^(?:pr_status|const char\*|uint32_t)\s+(pr_\w+)\(", hdr, re.M))
    assert declared == set(P.EXPORTS)
    L = C.CDLL(P.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name
    assert P.abi_version() == P.PR_ABI_VERSION == 8
    assert P.device_count() >= 0


def _scene_arrays(desc):
    import paper_2012_10357_amd as P
    return desc


def test_invalid_scenes_rejected_before_device(P):
    good = W.c2_scene()
    P.Scene(good, build=False).close()
    bad = W.c2_scene(); bad.geom_type = bad.geom_type.copy(); bad.geom_type[0] = 9
    with pytest.raises(P.ProcrayError, match="INVALID_ARG"):
        P.Scene(bad, build=False)
    bad = W.c2_scene(); bad.inst_geom = bad.inst_geom.copy(); bad.inst_geom[1] = 17
    with pytest.raises(P.ProcrayError, match="INVALID_ARG"):
        P.Scene(bad, build=False)
    bad = W.c2_scene(); bad.inst_xform = bad.inst_xform.copy(); bad.inst_xform[0, :] = 0
    with pytest.raises(P.ProcrayError, match="det"):
        P.Scene(bad, build=False)
    bad = W.c2_scene(); bad.geom_aabb = bad.geom_aabb.copy(); bad.geom_aabb[0, 0] = 5
    with pytest.raises(P.ProcrayError, match="lo > hi"):
        P.Scene(bad, build=False)
    bad = W.c2_scene(); bad.geom_params = bad.geom_params.copy(); bad.geom_params[2, 0] = 7  # power 7
    with pytest.raises(P.ProcrayError, match="UNSUPPORTED"):
        P.Scene(bad, build=False)
    bad = W.c2_scene(); bad.mat_refl = np.array([0.3, 1.5, 0.3], np.float32)
    with pytest.raises(P.ProcrayError, match="rho"):
        P.Scene(bad, build=False)
    bad = W.c2_scene(); bad.geom_params = bad.geom_params.copy(); bad.geom_params[1, 4] = 0
    with pytest.raises(P.ProcrayError, match="n_iter"):
        P.Scene(bad, build=False)
    bad = W.c2_scene(); bad.geom_cut = bad.geom_cut.copy(); bad.geom_cut[1] = (0, 0, 1, np.nan)
    with pytest.raises(P.ProcrayError, match="non-finite cutting plane"):
        P.Scene(bad, build=False)
    bad = W.c2_scene(); bad.geom_cut = bad.geom_cut.copy(); bad.geom_cut[1] = (1e-20, 0, 0, 0)
    with pytest.raises(P.ProcrayError, match="normal too small"):
        P.Scene(bad, build=False)
    cut = W.c2_scene(); cut.geom_cut = cut.geom_cut.copy(); cut.geom_cut[1] = (0, 0, 3, 0.5)
    P.Scene(cut, build=False).close()


def test_colour_bound_validated(P):
    """Sample colours must stay within 2^24 in magnitude (multi-sample means
    are exact signed 32.32 fixed-point sums): background and
    |albedo| (|ambient| + |light_rgb|) beyond it are rejected; signed values
    within it are accepted."""
    ok = W.c2_scene(); ok.mat_albedo = np.array([[-0.5, 0.2, 3.0], [0.1, -2.0, 0.0], [1, 1, 1]], np.float32)
    ok.background = np.array([-1.0, 0.5, 2.0 ** 24], np.float32)
    P.Scene(ok, build=False).close()
    bad = W.c2_scene(); bad.background = np.array([0, 0, -2.0 ** 24 * 1.001], np.float32)
    with pytest.raises(P.ProcrayError, match="background"):
        P.Scene(bad, build=False)
    bad = W.c2_scene(); bad.mat_albedo = bad.mat_albedo.copy(); bad.mat_albedo[1, 2] = -1.6e7
    with pytest.raises(P.ProcrayError, match="albedo"):
        P.Scene(bad, build=False)   # 1.6e7 * (0.1 + 1) > 2^24
    bad = W.c2_scene(); bad.light_rgb = np.array([1, 1e20, 1], np.float32)
    with pytest.raises(P.ProcrayError, match="albedo"):
        P.Scene(bad, build=False)


def test_render_argument_errors_before_device(P):
    sc = P.Scene(W.c1_scene(), build=False)
    cam = W.camera((0, 1, -4))
    o = W.RenderOpts(64, 64, max_steps=128)
    fake = type("T", (), {"shape": (64, 64, 3), "data_ptr": lambda self: 0})()
    # not built yet
    with pytest.raises(P.ProcrayError, match="NOT_BUILT"):
        P.render(sc, cam, o, fake)
    sc.build(P.BvhOpts(32, 1, 1.0, 4.0, P.PR_BVH_HOST_ONLY))
    for bad_cam in (W.camera((0, 0, 0), (0, 0, 0)), W.camera((0, 5, 0), (0, 0, 0), up=(0, 1, 0)),
                    W.Camera(np.float32([0, 1, -4]), np.float32([0, 0, 0]), np.float32([0, 1, 0]), 180.0)):
        with pytest.raises(P.ProcrayError, match="INVALID_ARG"):
            P.render(sc, bad_cam, o, fake)
    for kw in (dict(spp=0), dict(spp=65), dict(max_steps=0), dict(eps=0.0), dict(tmin=5.0, tmax=1.0),
               dict(bounces=2)):
        oo = W.RenderOpts(64, 64, **{**dict(max_steps=128), **kw})
        with pytest.raises(P.ProcrayError):
            P.render(sc, cam, oo, fake)
    big = type("T", (), {"shape": (16385, 4, 3), "data_ptr": lambda self: 0})()
    with pytest.raises(P.ProcrayError, match="width and height"):
        P.render(sc, cam, o, big)
    with pytest.raises(P.ProcrayError, match="tile"):
        P.render(sc, cam, o, fake, tile=(8, 4))
    import ctypes as C
    oc = P.opts_c(o)
    oc.flags = 2
    st = P.lib().pr_render(sc.handle, C.byref(P.camera_c(cam)), C.byref(oc), 64, 64, None, None, None, None)
    assert st == P.PR_ERR_INVALID_ARG and b"flags" in P.lib().pr_last_error()
    for cp in (101, 999, 1001):
        with pytest.raises(P.ProcrayError, match="compact_pct"):
            P.render(sc, cam, o, fake, compact=cp)
    oc = P.opts_c(o)
    oc.reserved = 1
    st = P.lib().pr_render(sc.handle, C.byref(P.camera_c(cam)), C.byref(oc), 64, 64, None, None, None, None)
    assert st == P.PR_ERR_INVALID_ARG and b"reserved" in P.lib().pr_last_error()
    # host-only build: not uploaded, so rendering is refused before any device call
    with pytest.raises(P.ProcrayError, match="NOT_BUILT"):
        P.render(sc, cam, o, fake)
    # the allocation-free entry point: the same refusal, and requests whose
    # multi-sample accumulators would not fit its fixed scratch are rejected
    # before anything else (1920x1080 at 4 spp fits, 2048x2048 at 2 does not)
    with pytest.raises(P.ProcrayError, match="NOT_BUILT"):
        P.render_noalloc(sc, cam, W.RenderOpts(1920, 1080, spp=4, max_steps=128),
                         type("T", (), {"shape": (1080, 1920, 3), "data_ptr": lambda self: 0})())
    huge = type("T", (), {"shape": (2048, 2048, 3), "data_ptr": lambda self: 0})()
    with pytest.raises(P.ProcrayError, match="scratch"):
        P.render_noalloc(sc, cam, W.RenderOpts(2048, 2048, spp=2, max_steps=128), huge)
    with pytest.raises(P.ProcrayError, match="NOT_BUILT"):
        P.render_noalloc(sc, cam, W.RenderOpts(2048, 2048, spp=1, max_steps=128), huge)
    # batches: empty, more than 4096 requests, a tile that is not 64 pixels,
    # and a request whose scene is not on the device (named by its index)
    one = P.make_requests([(sc, cam, o, fake, None, None, 0)])
    L = P.lib()
    assert L.pr_render_batch(one, 0, None, None) == P.PR_ERR_INVALID_ARG
    assert L.pr_render_batch(one, 4097, None, None) == P.PR_ERR_INVALID_ARG
    assert L.pr_autotune(one, 0, C.byref(P.BatchOpts())) == P.PR_ERR_INVALID_ARG
    assert L.pr_render_batch(one, 1, C.byref(P.BatchOpts(8, 4, 0, 0)), None) == P.PR_ERR_INVALID_ARG
    with pytest.raises(P.ProcrayError, match="request 0"):
        P.render_batch(one)
    sc.close()


@pytest.mark.parametrize("max_leaf", [1, 4])
def test_bvh_well_formed_and_culls_like_brute_force(P, max_leaf):
    desc = W.c3_scene()
    sc = P.Scene(desc, build=False)
    sc.build(P.BvhOpts(32, max_leaf, 1.0, 4.0, P.PR_BVH_HOST_ONLY))
    lo, hi, first, count, order = sc.bvh()
    n = desc.n_inst
    assert sorted(order.tolist()) == list(range(n))
    leaves = np.nonzero(count > 0)[0]
    assert count[leaves].sum() == n and count.max() <= max_leaf
    covered = np.zeros(n, int)
    for l in leaves:
        covered[first[l]:first[l] + count[l]] += 1
    assert np.all(covered == 1)
    # world AABBs of instances from their 8 transformed corners
    xf = desc.inst_xform.reshape(-1, 3, 4).astype(np.float64)
    g = desc.geom_aabb[desc.inst_geom].astype(np.float64)
    corners = np.stack([np.stack([g[:, 0 + 3 * (c & 1)], g[:, 1 + 3 * ((c >> 1) & 1)],
                                  g[:, 2 + 3 * ((c >> 2) & 1)]], -1) for c in range(8)], 1)
    wc = np.einsum("kij,kcj->kci", xf[:, :, :3], corners) + xf[:, None, :, 3]
    wlo, whi = wc.min(1), wc.max(1)
    # parents contain children, leaves contain their instances
    def depth(i):
        return 0 if count[i] else 1 + max(depth(first[i]), depth(first[i] + 1))
    assert depth(0) <= 30
    for i in range(len(count)):
        if count[i] == 0:
            for c in (first[i], first[i] + 1):
                assert np.all(lo[i] <= lo[c]) and np.all(hi[i] >= hi[c])
        else:
            ids = order[first[i]:first[i] + count[i]]
            assert np.all(lo[i] <= wlo[ids]) and np.all(hi[i] >= whi[ids])
    # CPU traversal of the exported BVH == brute-force world-box test on random rays
    rng = np.random.default_rng(0)
    o = rng.uniform(-30, 30, (300, 3))
    d = rng.standard_normal((300, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)

    def box_hit(o1, d1, l, h):
        with np.errstate(divide="ignore", invalid="ignore"):
            a = (l - o1) / d1
            b = (h - o1) / d1
        return np.max(np.minimum(a, b)) <= max(np.min(np.maximum(a, b)), 0)

    for r in range(300):
        found = set()
        stack = [0]
        while stack:
            i = stack.pop()
            if not box_hit(o[r], d[r], lo[i], hi[i]):
                continue
            if count[i]:
                found |= set(order[first[i]:first[i] + count[i]].tolist())
            else:
                stack += [first[i], first[i] + 1]
        brute = {k for k in range(n) if box_hit(o[r], d[r], wlo[k], whi[k])}
        assert brute <= found
    sc.close()


def test_mesh_validation_and_bvh_items(P):
    """pr_scene_add_mesh validates before touching anything; every (placement,
    triangle) pair becomes one BVH leaf item after the procedural instances."""
    desc = W.f2_sample_scene()
    sc = P.Scene(desc, build=False)
    sc.build(P.BvhOpts(32, 1, 1.0, 4.0, P.PR_BVH_HOST_ONLY))
    order = sc.bvh()[4]
    assert sorted(order.tolist()) == list(range(desc.n_inst + 2))
    quad_v, quad_f = np.array(W.QUAD_VERTICES, np.float32), np.array(W.QUAD_INDICES, np.uint32)
    xf = [W.xform(np.eye(3), 1.0, (0, 0, 0))]
    with pytest.raises(P.ProcrayError, match="index"):
        sc.add_mesh(quad_v, np.array([[0, 1, 7]], np.uint32), [0], xf)
    bad_v = quad_v.copy(); bad_v[1, 1] = np.inf
    with pytest.raises(P.ProcrayError, match="non-finite"):
        sc.add_mesh(bad_v, quad_f, [0], xf)
    with pytest.raises(P.ProcrayError, match="degenerate"):
        sc.add_mesh(np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], np.float32), np.array([[0, 1, 2]], np.uint32),
                    [0], xf)
    with pytest.raises(P.ProcrayError, match="material"):
        sc.add_mesh(quad_v, quad_f, [99], xf)
    with pytest.raises(P.ProcrayError, match="det"):
        sc.add_mesh(quad_v, quad_f, [0], [np.zeros(12, np.float32)])
    with pytest.raises(P.ProcrayError, match="at most"):
        sc.add_mesh(quad_v, quad_f, [0] * 8200, xf * 8200)
    # the failed calls changed nothing: the build still holds 4 + 2 items;
    # a valid addition clears the build
    sc.add_mesh(quad_v, quad_f, [0, 1], xf * 2)
    with pytest.raises(P.ProcrayError, match="NOT_BUILT"):
        sc.bvh()
    sc.build(P.BvhOpts(32, 1, 1.0, 4.0, P.PR_BVH_HOST_ONLY))
    order = sc.bvh()[4]
    assert sorted(order.tolist()) == list(range(desc.n_inst + 2 + 4))
    sc.close()


def test_user_estimator_registration_and_build(P):
    """Registering validates the name and body and hands out types from
    PR_USER_TYPE_BASE; scenes accept registered types only; closest-hit
    functions attach to registered user types only; estimators and
    closest-hit functions compile with the library's flags without a device."""
    from tests import user_estimators as U
    t = P.register_estimator("cyl_cpu_test", U.CYLINDER_BODY)
    assert t >= 8
    with pytest.raises(P.ProcrayError, match="already registered"):
        P.register_estimator("cyl_cpu_test", U.CYLINDER_BODY)
    for bad in ("9abc", "", "a-b", "x" * 49):
        with pytest.raises(P.ProcrayError, match="name"):
            P.register_estimator(bad, U.CYLINDER_BODY)
    with pytest.raises(P.ProcrayError, match="body"):
        P.register_estimator("empty_body", "")
    b = W._SceneBuilder()
    m = b.material((0.5, 0.5, 0.5))
    aabb, prm = U.cylinder_geom(0.5, 1.0)
    b.instance(b.geometry((t, aabb, prm)), m, W.xform(np.eye(3), 1.0, (0, 0, 0)))
    desc = b.build(light_pos=(2, 4, -3))
    P.Scene(desc, build=False).close()
    desc.geom_type = np.array([t + 7], np.uint32)
    with pytest.raises(P.ProcrayError, match="unknown primitive type"):
        P.Scene(desc, build=False)
    # closest-hit functions attach to registered user types only
    for bad_type in (0, 7, t + 1, 1000):
        with pytest.raises(P.ProcrayError, match="not a registered user type"):
            P.register_closest_hit(bad_type, U.STRIPED_CH_BODY)
    with pytest.raises(P.ProcrayError, match="body"):
        P.register_closest_hit(t, "")
    P.register_closest_hit(t, U.LAMBERT_CH_BODY)
    P.register_closest_hit(t, U.STRIPED_CH_BODY)   # replaces the first
    P.build_estimators()


def test_user_estimator_compile_error_is_reported(tmp_path):
    """A body that does not compile fails pr_build_estimators with the
    compiler's message (in a child process, so the registry of this one stays
    valid)."""
    import subprocess, sys, os
    code = (
        "import paper_2012_10357_amd as P\n"
        "P.register_estimator('broken', 'return undeclared_thing + x;')\n"
        "try:\n"
        "    P.build_estimators()\n"
        "    print('NO ERROR')\n"
        "except P.ProcrayError as e:\n"
        "    print('ERROR', e)\n")
    env = dict(os.environ, PR_USER_CACHE=str(tmp_path))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300,
                       cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert "ERROR" in r.stdout and "INVALID_ARG" in r.stdout, r.stdout + r.stderr
    assert "undeclared_thing" in r.stdout


def test_binding_abi_version_matches_header(P):
    """The binding's struct layouts are written for the header's ABI revision."""
    import os, re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                            "procray.h")).read()
    v = int(re.search(r"#define PR_ABI_VERSION (\d+)", hdr).group(1))
    assert v == P.PR_ABI_VERSION == P.abi_version()


def _depth(first, count, i=0):
    return 1 if count[i] > 0 else 1 + max(_depth(first, count, first[i]), _depth(first, count, first[i] + 1))


def test_scene_size_limit_and_bvh_depth(P):
    """A scene holds at most 16384 items (16-bit traversal stack entries); at
    that size the BVH stays within the depth the LDS stack allows, also when
    every instance sits at the same place (no SAH split possible), and one
    instance more is rejected before any device work."""
    import sys
    sys.setrecursionlimit(10000)
    rng = np.random.default_rng(11)
    full = W.random_instances_scene(rng, 16384, ["sphere", "torus"])
    stacked = W.random_instances_scene(rng, 16384, ["sphere"])
    stacked.inst_xform = np.tile(np.float32([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]), (16384, 1))
    for desc in (full, stacked):
        sc = P.Scene(desc, build=False)
        sc.build(P.BvhOpts(32, 1, 1.0, 4.0, P.PR_BVH_HOST_ONLY))
        lo, hi, first, count, order = sc.bvh()
        assert sorted(order.tolist()) == list(range(16384))
        assert _depth(first, count) <= 30
        sc.close()
    over = W.random_instances_scene(rng, 16385, ["sphere"])
    with pytest.raises(P.ProcrayError, match="n_inst must be in 1..16384"):
        P.Scene(over, build=False)
