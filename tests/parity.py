"""GPU-vs-oracle comparison protocol (test-side).

The oracle flags a pixel when any ray traced for it, in any sample, passed
within 1e-3 of a surface without stopping (E1), exhausted its step budget
(E2) or stopped with a value in [0.98 eps, eps) (E3): the places where float32
and float64 sphere tracing may legitimately take different branches.  E5 is
their counterpart for closed-form triangle hits (a ray within 1e-5 of a
triangle edge, at a grazing angle, or tied with a procedural hit).  On the
pixels none of these flags:
  * hit mask agreement >= 99.9 %,
  * hit distance |t_g - t_o| <= 1e-4 t_o on >= 99.9 % of pixels hit by both,
  * radiance max_c |L_g - L_o| <= 1e-3 on >= 99.9 % of pixels whose masks agree.
``pass_strict`` is that gate.  ``pass`` takes the radiance line over the
pixels that E4 leaves as well -- E4 flags hits whose float64 normal itself
turns by more than 1e-3 when the hit point moves by about its float32 error
(for a mirror bounce, by the error the reflected direction inherits), where
the colour is not determined to 1e-3 by the hit -- while the mask and
distance lines stay on E1-E3 (and E5).  Both radiance lines are always
reported, with the number of failing pixels, the same fractions over hit
pixels only, and mask, distance and radiance with no exclusion at all.
"""
from __future__ import annotations

import numpy as np

MASK_GATE = 0.999
T_REL = 1e-4
RGB_ABS = 1e-3
FRAC_GATE = 0.999
E1, E2, E3, E4, E5 = 1, 2, 4, 8, 16
GATE_RULES = E1 | E2 | E3 | E5


def _frac(ok, sel):
    return float(ok[sel].mean()) if sel.any() else 1.0


def compare(g_rgb, g_t, g_inst, orc, label=""):
    g_rgb = np.asarray(g_rgb, np.float64).reshape(-1, 3)
    g_t = np.asarray(g_t, np.float64).reshape(-1)
    g_inst = np.asarray(g_inst, np.int64).reshape(-1)
    o_rgb, o_t, o_inst = orc["rgb"], orc["t"], orc["inst"]
    excl = np.asarray(orc["excl"])
    keep = (excl & GATE_RULES) == 0
    keep4 = keep & ((excl & E4) == 0)
    mg, mo = g_inst >= 0, o_inst >= 0
    agree = mg == mo
    both = keep & mg & mo
    with np.errstate(invalid="ignore"):
        t_err = np.abs(g_t - o_t) / np.maximum(o_t, 1e-30)
    rgb_err = np.max(np.abs(g_rgb - o_rgb), axis=1)
    rgb_ok = rgb_err <= RGB_ABS
    sel = keep & agree
    rep = dict(
        label=label, pixels=int(g_inst.size), hit_frac=float(mo.mean()),
        excluded=float(1 - keep.mean()), excluded_e4=float(1 - keep4.mean()),
        excl_hits=float(1 - keep[mo].mean()) if mo.any() else 0.0,
        **{f"excl_e{k}": float(((excl & (1 << (k - 1))) != 0).mean()) for k in range(1, 6)},
        mask=_frac(agree, keep), mask_all=float(agree.mean()),
        inst=_frac(g_inst == o_inst, keep),
        t_frac=_frac(t_err <= T_REL, both), t_max=float(t_err[both].max()) if both.any() else 0.0,
        rgb_frac=_frac(rgb_ok, sel), rgb_fail=int((sel & ~rgb_ok).sum()),
        rgb_max=float(rgb_err[sel].max()) if sel.any() else 0.0,
        rgb_p999=float(np.quantile(rgb_err[sel], 0.999)) if sel.any() else 0.0,
        rgb_frac_hits=_frac(rgb_ok, sel & mo),
        rgb_frac_e4=_frac(rgb_ok, keep4 & agree), rgb_fail_e4=int((keep4 & agree & ~rgb_ok).sum()),
        rgb_frac_all=_frac(rgb_ok, agree),
        t_frac_all=_frac(t_err <= T_REL, mg & mo),
    )
    geo = rep["mask"] >= MASK_GATE and rep["t_frac"] >= FRAC_GATE
    rep["pass_strict"] = geo and rep["rgb_frac"] >= FRAC_GATE
    rep["pass"] = geo and rep["rgb_frac_e4"] >= FRAC_GATE
    return rep


def fmt(rep):
    return ("{label}: px={pixels} hit={hit_frac:.3f} | E1-E3,E5: excl={excluded:.4f} "
            "(E1 {excl_e1:.4f} E2 {excl_e2:.4f} E3 {excl_e3:.4f} E5 {excl_e5:.4f}; of hit px {excl_hits:.3f}) "
            "mask={mask:.5f} inst={inst:.5f} t_frac={t_frac:.5f} t_max={t_max:.2e} "
            "rgb_frac={rgb_frac:.5f} (fail {rgb_fail}; hit px {rgb_frac_hits:.5f}) rgb_max={rgb_max:.2e} "
            "rgb_p999={rgb_p999:.2e} pass_strict={pass_strict} | radiance also without E4: "
            "excl={excluded_e4:.4f} (E4 {excl_e4:.4f}) rgb_frac={rgb_frac_e4:.5f} (fail {rgb_fail_e4}) "
            "pass={pass} | no exclusion: mask={mask_all:.5f} t_frac={t_frac_all:.5f} "
            "rgb_frac={rgb_frac_all:.5f}").format(**rep)
