"""Serving logic on the host with the simulated executor (no device):
admission by footprint, the budget is never exceeded, FIFO without
starvation, oversize rejection, timeouts, latency accounting."""
import time

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def P():
    import os
    import paper_2012_10357_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_2012_10357_amd import build
        build.build()
    return P


@pytest.fixture(scope="module")
def scene(P):
    sc = P.Scene(W.c2_scene(), build=False)
    sc.build(P.BvhOpts(32, 1, 1.0, 4.0, P.PR_BVH_HOST_ONLY))
    yield sc


def _opts(side, spp=1):
    return W.RenderOpts(side, side, spp=spp, jitter=1 if spp > 1 else 0, max_steps=256)


def _fp(side, spp=1):
    """Pool bytes of one request: colour, depth and instance outputs, plus
    three 64-bit colour sums and a counter per pixel when spp > 1."""
    up = lambda b: (b + 255) // 256 * 256
    px = side * side
    b = up(px * 12) + 2 * up(px * 4)
    if spp > 1:
        b += up(px * 24) + up(px * 4)
    return b


def test_oversize_rejected_and_unregistered_scene(P, scene):
    srv = P.Server(_fp(256) * 2, max_inflight=2, simulated_us_per_mpix=100)
    srv.add_scene(scene)
    with pytest.raises(P.ProcrayError, match="OUT_OF_MEMORY"):
        srv.submit(scene, W.c2_camera(), _opts(1024))
    other = P.Scene(W.c1_scene(), build=False)
    other.build(P.BvhOpts(32, 1, 1.0, 4.0, P.PR_BVH_HOST_ONLY))
    with pytest.raises(P.ProcrayError, match="not registered"):
        srv.submit(other, W.c2_camera(), _opts(64))
    assert srv.stats().rejected == 1
    srv.close()


def test_footprint_counts_per_sample_scratch(P, scene):
    """A multi-sample request also reserves its per-sample colours and
    counters: it fits a budget of exactly that size and not one byte less."""
    need = _fp(256, spp=4)
    srv = P.Server(need, max_inflight=1, simulated_us_per_mpix=100)
    srv.add_scene(scene)
    tk = srv.submit(scene, W.c2_camera(), _opts(256, spp=4))
    srv.wait(tk, 10000)
    assert srv.stats().pool_bytes_peak == need
    srv.release(tk)
    srv.close()
    srv = P.Server(need - 1, max_inflight=1, simulated_us_per_mpix=100)
    srv.add_scene(scene)
    with pytest.raises(P.ProcrayError, match="OUT_OF_MEMORY"):
        srv.submit(scene, W.c2_camera(), _opts(256, spp=4))
    srv.close()


def test_budget_never_exceeded_fifo_and_all_complete(P, scene):
    budget = _fp(512) * 3 + 1000
    srv = P.Server(budget, max_inflight=2, max_batch=8, simulated_us_per_mpix=2000)
    srv.add_scene(scene)
    rng = np.random.default_rng(0)
    sides = [int(s) for s in rng.choice([64, 128, 256, 512], 60)]
    tickets = [srv.submit(scene, W.c2_camera(), _opts(s), tag=i) for i, s in enumerate(sides)]
    results = []
    for tk in tickets:
        r = srv.wait(tk, 20000)
        assert r.status == 0
        results.append((r.t_submit, r.t_admit, r.t_launch, r.t_done, r.user_tag))
        assert srv.stats().pool_bytes_peak <= budget
        srv.release(tk)
    st = srv.stats()
    assert st.completed == 60 and st.admitted == 60 and st.pool_bytes_in_use == 0
    assert st.pool_bytes_peak <= budget
    # FIFO admission: admit times are non-decreasing in submission order
    admits = [r[1] for r in results]
    assert all(a <= b for a, b in zip(admits, admits[1:]))
    for t_sub, t_adm, t_lau, t_done, _ in results:
        assert t_sub <= t_adm <= t_lau <= t_done
    # batching happened: fewer launches than requests
    assert st.launches < 60
    srv.close()


def test_large_request_not_starved(P, scene):
    """A request needing the whole budget is admitted once earlier ones are
    released, even while small requests keep arriving behind it."""
    budget = _fp(512)
    srv = P.Server(budget, max_inflight=2, simulated_us_per_mpix=500)
    srv.add_scene(scene)
    small = [srv.submit(scene, W.c2_camera(), _opts(128)) for _ in range(3)]
    big = srv.submit(scene, W.c2_camera(), _opts(512))
    later = [srv.submit(scene, W.c2_camera(), _opts(64)) for _ in range(5)]
    for tk in small:
        srv.wait(tk, 10000)
        srv.release(tk)
    rb = srv.wait(big, 10000)
    t_big_admit = rb.t_admit
    srv.release(big)          # the big request holds the whole budget until released
    # nothing submitted after the big request was admitted before it
    for tk in later:
        r = srv.wait(tk, 10000)
        assert r.t_admit >= t_big_admit
        srv.release(tk)
    srv.close()


def test_wait_timeout_and_release_busy(P, scene):
    srv = P.Server(_fp(512, spp=4), max_inflight=1, simulated_us_per_mpix=200000)
    srv.add_scene(scene)
    tk = srv.submit(scene, W.c2_camera(), _opts(512, spp=4))   # ~0.2 s simulated
    with pytest.raises(P.ProcrayError, match="TIMEOUT"):
        srv.wait(tk, 1)
    with pytest.raises(P.ProcrayError, match="BUSY"):
        srv.release(tk)
    r = srv.wait(tk, 10000)
    assert r.t_done - r.t_launch > 0.05
    srv.release(tk)
    srv.close()


def test_arrivals_overlap_inflight_launches(P, scene):
    """Continuous batching: requests arriving while a launch runs are launched
    on a second stream before the first finishes."""
    srv = P.Server(_fp(1024) * 4, max_inflight=2, simulated_us_per_mpix=100000)
    srv.add_scene(scene)
    a = srv.submit(scene, W.c2_camera(), _opts(1024))          # ~0.1 s
    time.sleep(0.01)
    b = srv.submit(scene, W.c2_camera(), _opts(64))
    rb = srv.wait(b, 10000)
    ra = srv.wait(a, 10000)
    assert rb.t_launch < ra.t_done and rb.t_done < ra.t_done
    srv.release(a)
    srv.release(b)
    srv.close()
