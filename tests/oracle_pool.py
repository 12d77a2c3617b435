"""The FP64 oracle over many pixels in worker processes (test infrastructure).

Workers are started with the "spawn" method, so they are fresh interpreters
that import only NumPy, the oracle and the workload generators -- never the
GPU runtime of the process that asks.  Pixels are split into chunks handed
out dynamically; results come back in pixel order, with the same fields as
``oracle.tracer.render`` (work counts summed).
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np


def workers() -> int:
    # the host cores this process may use, at most 16 (one GPU's share)
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _chunk(args):
    from oracle import tracer as T
    scene, cam, opts, pix = args
    o = T.render(scene, cam, opts, pixels=pix)
    return o["rgb"], o["t"], o["inst"], o["excl"], o["counts"]


def render(scene, cam, opts, pixels=None, chunk=2048, procs=None):
    """oracle.tracer.render(scene, cam, opts, pixels) computed in parallel."""
    if pixels is None:
        pixels = np.arange(opts.width * opts.height, dtype=np.int64)
    pixels = np.asarray(pixels, np.int64)
    return render_many([(scene, cam, opts, pixels)], chunk=chunk, procs=procs)[0]


def render_many(jobs, chunk=2048, procs=None):
    """Several (scene, cam, opts, pixels) renders through one worker pool."""
    tasks, owner = [], []
    for k, (scene, cam, opts, pixels) in enumerate(jobs):
        pixels = np.asarray(pixels, np.int64)
        for c0 in range(0, pixels.size, chunk):
            tasks.append((scene, cam, opts, pixels[c0:c0 + chunk]))
            owner.append(k)
    n = procs or workers()
    with mp.get_context("spawn").Pool(min(n, max(1, len(tasks)))) as pool:
        parts = pool.map(_chunk, tasks, chunksize=1)
    out = []
    for k, (_, _, _, pixels) in enumerate(jobs):
        mine = [p for p, o in zip(parts, owner) if o == k]
        rays = {}
        for p in mine:
            for key, v in p[4]["rays"].items():
                rays[key] = rays.get(key, 0) + v
        cat = (lambda i: np.concatenate([p[i] for p in mine])) if mine else (lambda i: np.zeros(0))
        out.append(dict(rgb=cat(0).reshape(-1, 3), t=cat(1), inst=cat(2).astype(np.int64),
                        excl=cat(3).astype(np.int64), counts={"rays": rays},
                        pixels=np.asarray(pixels, np.int64)))
    return out
