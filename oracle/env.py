"""Environment-map queries.

Oracle code (test infrastructure only).

The paper queries a learnable cubemap at a roughness-dependent mip level
lambda = log2(rho + 1) * lambda_max (Sec. 3.2, "Shading", the SampleEnvMap
equation).  Reading taken: an equirectangular map E_0 of He x We texels
(We = 2 He, powers of two), mip level k the plain 2x2 box mean of level k-1
down to 2 x 1, lambda_max = log2 He, bilinear filtering inside a level
(wrapping in longitude, clamped in latitude) and linear blending between the
two levels around lambda.

Direction d (unit) maps to u = 1/2 + atan2(d.x, -d.z) / (2 pi),
v = acos(d.y) / pi; level k has texel centres at ((x + 1/2) / We_k,
(y + 1/2) / He_k).
"""

import math

import numpy as np


def build_mips(env):
    """Levels 0..log2(He) as float64 arrays; level k = mean of 2x2 children."""
    lv = [np.asarray(env, np.float64)]
    while lv[-1].shape[0] > 1:
        e = lv[-1]
        h, w = e.shape[0] // 2, e.shape[1] // 2
        blocks = e.reshape(h, 2, w, 2, 3)
        lv.append(blocks.mean(axis=(1, 3)))
    return lv


def lambda_max(mips):
    return len(mips) - 1


def dir_to_uv(d):
    u = 0.5 + np.arctan2(d[..., 0], -d[..., 2]) / (2.0 * math.pi)
    v = np.arccos(np.clip(d[..., 1], -1.0, 1.0)) / math.pi
    return u, v


def bilinear(img, d):
    """Bilinear lookup of level ``img[h][w][3]`` in unit directions ``d[n][3]``."""
    h, w = img.shape[:2]
    u, v = dir_to_uv(d)
    x = u * w - 0.5
    y = v * h - 0.5
    x0 = np.floor(x)
    y0 = np.floor(y)
    fx = (x - x0)[..., None]
    fy = (y - y0)[..., None]
    ix0 = np.mod(x0.astype(np.int64), w)
    ix1 = np.mod(ix0 + 1, w)
    iy0 = np.clip(y0.astype(np.int64), 0, h - 1)
    iy1 = np.clip(y0.astype(np.int64) + 1, 0, h - 1)
    return ((1 - fx) * (1 - fy) * img[iy0, ix0] + fx * (1 - fy) * img[iy0, ix1]
            + (1 - fx) * fy * img[iy1, ix0] + fx * fy * img[iy1, ix1])


def trilinear(mips, d, lam):
    """E_lambda(d): blend of the two levels around ``lam`` (clamped to the top)."""
    top = lambda_max(mips)
    lam = np.clip(np.asarray(lam, np.float64), 0.0, top)
    k0 = np.floor(lam).astype(np.int64)
    k1 = np.minimum(k0 + 1, top)
    t = (lam - k0)[..., None]
    out = np.zeros(d.shape)
    for k in range(top + 1):
        sel0 = k0 == k
        if sel0.any():
            out[sel0] += (1 - t[sel0]) * bilinear(mips[k], d[sel0])
        sel1 = k1 == k
        if sel1.any():
            out[sel1] += t[sel1] * bilinear(mips[k], d[sel1])
    return out


def roughness_level(mips, rho):
    """lambda = log2(rho + 1) * lambda_max (Sec. 3.2, SampleEnvMap)."""
    return np.log2(np.asarray(rho, np.float64) + 1.0) * lambda_max(mips)
