"""GPU-vs-oracle comparison protocol (test-side).

Pixels are excluded where the oracle saw any traced ray graze a surface
within 1e-3 without stopping (E1), exhaust its step budget (E2), stop with
a value in [0.98 eps, eps) (E3), hit where the normal is ill-conditioned
at the scale of float32 rounding of the hit point (E4), or meet a triangle
within 1e-5 of an edge, at a grazing angle, or tied with a procedural hit
(E5): there float32 and float64 may legitimately take different branches.  On the remaining pixels:
  * hit mask agreement >= 99.9 %,
  * hit distance |t_g - t_o| <= 1e-4 t_o on >= 99.9 % of pixels hit by both,
  * radiance max_c |L_g - L_o| <= 1e-3 on >= 99.9 % of pixels whose masks agree.
Agreement over *all* pixels (no exclusion) is reported next to it.
"""
from __future__ import annotations

import numpy as np

MASK_GATE = 0.999
T_REL = 1e-4
RGB_ABS = 1e-3
FRAC_GATE = 0.999


def compare(g_rgb, g_t, g_inst, orc, label=""):
    g_rgb = np.asarray(g_rgb, np.float64).reshape(-1, 3)
    g_t = np.asarray(g_t, np.float64).reshape(-1)
    g_inst = np.asarray(g_inst, np.int64).reshape(-1)
    o_rgb, o_t, o_inst = orc["rgb"], orc["t"], orc["inst"]
    keep = orc["excl"] == 0
    mg, mo = g_inst >= 0, o_inst >= 0
    agree = mg == mo
    n_keep = int(keep.sum())
    frac_mask = float(agree[keep].mean()) if n_keep else 1.0
    frac_mask_all = float(agree.mean())
    inst_agree = float((g_inst == o_inst)[keep].mean()) if n_keep else 1.0
    both = keep & mg & mo
    with np.errstate(invalid="ignore"):
        t_err = np.abs(g_t - o_t) / np.maximum(o_t, 1e-30)
    frac_t = float((t_err[both] <= T_REL).mean()) if both.any() else 1.0
    rgb_err = np.max(np.abs(g_rgb - o_rgb), axis=1)
    sel = keep & agree
    frac_rgb = float((rgb_err[sel] <= RGB_ABS).mean()) if sel.any() else 1.0
    rep = dict(
        label=label, pixels=int(g_inst.size), excluded=float(1 - keep.mean()),
        excl_e1=float(((orc["excl"] & 1) != 0).mean()), excl_e2=float(((orc["excl"] & 2) != 0).mean()),
        excl_e3=float(((orc["excl"] & 4) != 0).mean()),
        excl_e4=float(((orc["excl"] & 8) != 0).mean()),
        excl_e5=float(((orc["excl"] & 16) != 0).mean()),
        hit_frac=float(mo.mean()), mask=frac_mask, mask_all=frac_mask_all, inst=inst_agree,
        t_frac=frac_t, t_max=float(t_err[both].max()) if both.any() else 0.0,
        rgb_frac=frac_rgb, rgb_max=float(rgb_err[sel].max()) if sel.any() else 0.0,
        rgb_p999=float(np.quantile(rgb_err[sel], 0.999)) if sel.any() else 0.0,
        rgb_frac_all=float((rgb_err <= RGB_ABS).mean()),
    )
    rep["pass"] = frac_mask >= MASK_GATE and frac_t >= FRAC_GATE and frac_rgb >= FRAC_GATE
    return rep


def fmt(rep):
    return ("{label}: px={pixels} excl={excluded:.4f} (E1 {excl_e1:.4f} E2 {excl_e2:.4f} E3 {excl_e3:.4f} E4 {excl_e4:.4f} E5 {excl_e5:.4f}) "
            "hit={hit_frac:.3f} mask={mask:.5f} mask_all={mask_all:.5f} inst={inst:.5f} "
            "t_frac={t_frac:.5f} t_max={t_max:.2e} rgb_frac={rgb_frac:.5f} rgb_max={rgb_max:.2e} "
            "rgb_p999={rgb_p999:.2e} rgb_frac_all={rgb_frac_all:.5f} pass={pass}").format(**rep)
