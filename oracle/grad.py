"""Reference derivatives of the estimator with the hit selection held fixed.

Oracle code (test infrastructure only).

The march that selects each sample's hit pixel is piecewise constant in the
inputs and has no useful derivative (the paper differentiates its shading
with the screen-space tracing treated as a fixed selection).  With the hit
codes held fixed, every pixel's output is a smooth function of its own
G-buffer entries (normal, roughness, albedo, metallic: through the sampled
directions, the Fresnel and masking terms, the roughness mip level and the
environment lookups) and a linear function of the environment texels and
of the radiance at the hit pixels.

Derivatives of a scalar loss sum_p g_p . out_p are taken here by central
finite differences of the float64 forward (``shade_pixels`` with
``replay_hits``),
which needs no derivative formula at all; the environment derivatives use
the linearity exactly (one unit change of a texel).
"""

import numpy as np

from . import env as envmod
from .shade import shade_pixels


def _loss(out, g_out):
    return (np.asarray(out) * np.asarray(g_out)).sum(axis=-1)


def pixel_grads(cam, gbuf, env_rgb, params, pix, hits, g_out, eps=1e-6):
    """d(g_p . out_p) / d(normal_rough[p, 0..3], albedo_metal[p, 0..3]) for
    every pixel p of ``pix`` ([n][8], float64).  ``hits`` [n][S] are the
    fixed codes of those pixels, ``g_out`` [n][3] the loss weights.  A
    pixel's own inputs move only its own output when the hits are fixed, so
    all pixels are perturbed together."""
    pix = np.asarray(pix, np.int64).reshape(-1)
    mips = envmod.build_mips(np.asarray(env_rgb, np.float64))
    base = {k: np.array(v, np.float64) for k, v in gbuf.items()}
    out = np.zeros((pix.size, 8))
    for b, name in enumerate(("normal_rough", "albedo_metal")):
        for ch in range(4):
            vals = []
            for sgn in (1.0, -1.0):
                g = dict(base)
                arr = base[name].copy().reshape(-1, 4)
                arr[pix, ch] += sgn * eps
                g[name] = arr.reshape(base[name].shape)
                r = shade_pixels(cam, g, env_rgb, params, pix, mips=mips, replay_hits=hits,
                                 check_long_form=False)
                vals.append(_loss(r["out"], g_out))
            out[:, 4 * b + ch] = (vals[0] - vals[1]) / (2.0 * eps)
    return out


def env_grads(cam, gbuf, env_rgb, params, hits, g_out, texels):
    """d(sum_p g_p . out_p) / d env[y, x, c] for each (y, x, c) of ``texels``,
    over the whole frame (``hits`` [H][W][S], ``g_out`` [H][W][3]).  The
    output is linear in the texels (box-mean mips, trilinear and bilinear
    lookups), so one unit change gives the derivative exactly."""
    W, H = int(cam["width"]), int(cam["height"])
    pix = np.arange(W * H)
    hits = np.asarray(hits).reshape(W * H, -1)
    g_out = np.asarray(g_out, np.float64).reshape(W * H, 3)
    e0 = np.array(env_rgb, np.float64)

    def total(e):
        r = shade_pixels(cam, gbuf, e, params, pix, mips=envmod.build_mips(e), replay_hits=hits,
                         check_long_form=False)
        return float(_loss(r["out"], g_out).sum())

    base = total(e0)
    res = []
    for (y, x, c) in texels:
        e = e0.copy()
        e[y, x, c] += 1.0
        res.append(total(e) - base)
    return np.array(res)


def radiance_grads(cam, gbuf, env_rgb, params, hits, g_out):
    """d(sum_p g_p . out_p) / d radiance[q, c] for every pixel q ([H][W][3]):
    each sample that hits q contributes its weight.  Linear in the radiance,
    so one evaluation with a unit radiance per channel gives it exactly."""
    W, H = int(cam["width"]), int(cam["height"])
    hits = np.asarray(hits).reshape(W * H, -1)
    g_out = np.asarray(g_out, np.float64).reshape(W * H, 3)
    out = np.zeros((W * H, 3))
    # the radiance enters only through hit samples: shading with the
    # environment off (zero map) and radiance = e_q isolates q's weight
    pix = np.arange(W * H)
    zero_env = np.zeros_like(np.asarray(env_rgb, np.float64))
    g = {k: np.array(v, np.float64) for k, v in gbuf.items()}
    for q in np.unique(hits[hits >= 0]):
        for c in range(3):
            rad = np.zeros_like(g["radiance"]).reshape(-1, 4)
            rad[q, c] = 1.0
            gg = dict(g, radiance=rad.reshape(g["radiance"].shape))
            uses = np.nonzero((hits == q).any(axis=1))[0]
            r = shade_pixels(cam, gg, zero_env, params, pix[uses], replay_hits=hits[uses],
                             check_long_form=False, mips=envmod.build_mips(zero_env))
            out[q, c] = float(_loss(r["out"], g_out[uses]).sum())
    return out.reshape(H, W, 3)
