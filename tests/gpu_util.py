"""Helpers for GPU tests: device tensors and one-call renders through the C ABI."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible (HIP device required)")
    import paper_2012_10357_amd as P
    P.lib()   # raises if the HIP library is missing: no fallback
    return P


def alloc(W, H, dev="cuda"):
    rgb = torch.full((H, W, 3), float("nan"), dtype=torch.float32, device=dev)
    t = torch.full((H, W), float("nan"), dtype=torch.float32, device=dev)
    inst = torch.full((H, W), -7, dtype=torch.int32, device=dev)
    return rgb, t, inst


def gpu_render(P, scene, cam, opts, tile=(0, 0), step_budget=0, stream=None):
    rgb, t, inst = alloc(opts.width, opts.height)
    P.render(scene, cam, opts, rgb, t, inst, stream=stream, tile=tile, step_budget=step_budget)
    torch.cuda.synchronize()
    return rgb.cpu().numpy(), t.cpu().numpy(), inst.cpu().numpy()


def flat(rgb, t, inst, pixels=None):
    rgb = rgb.reshape(-1, 3)
    t = t.reshape(-1)
    inst = inst.reshape(-1)
    if pixels is not None:
        return rgb[pixels], t[pixels], inst[pixels]
    return rgb, t, inst


_hip = None


def d2h(ptr: int, shape, dtype):
    """Copies device memory at a raw pointer into a new NumPy array."""
    import ctypes as C
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    out = np.empty(shape, dtype)
    rc = _hip.hipMemcpy(out.ctypes.data, C.c_void_p(ptr), out.nbytes, 2)   # device -> host
    assert rc == 0, f"hipMemcpy failed: {rc}"
    return out
