"""The first shading pass that produces the radiance c1 the specular rays read.

Oracle code (test infrastructure only).

Sec. 3.2 ("Shading") computes, per pixel of the G-buffer, c1 = c_d + c_s
with the split-sum approximation (Karis 2013):

* c_d = (1 - m) a L_E(n, rho): the environment at the normal, at mip level
  lambda = log2(1 + rho) lambda_max (the same lookup as the direct term of
  the estimator);
* c_s = L_E(r, rho) F_s: the environment along the mirror direction
  r = 2 (v.n) n - v at the same level, times the BRDF integral F_s;
* F_s from a 2D table over (n.v, rho) holding the two integrals of the
  Schlick split (supplementary, split-sum details): A = int f_s/F (1 - Fc)
  cos, B = int f_s/F Fc cos with Fc = (1 - wo.h)^5, so F_s = F0 A + B with
  F0 = lerp(0.04, a, m) (reading taken: the split multiplies F0, the
  reflectance at normal incidence, where the text writes the albedo).  The
  table is the Monte-Carlo estimate of both integrals with visible-normal
  samples on a stratified K x K grid of (u1, u2) cell centres (a fixed rule,
  so two implementations produce the same table).

Sec. 3.2 also takes the shading normal from the depth buffer by finite
differences (the "depth normal"): the world positions of neighbouring pixel
centres give two tangents whose cross product is the normal.

Readings taken: central differences where both neighbours of a pixel are
surface pixels inside the image, one-sided differences where only one is,
and the direction toward the camera where neither is; normals face the
camera; background pixels get a zero normal and zero radiance; back-facing
pixels (n.v <= 0) get no specular term; table texels sit at cell centres
((i + 1/2)/N) and are read bilinearly with clamping at the edges.
"""

import math

import numpy as np

from . import brdf, camera, env


def _tangents(cam, depth):
    """World points of the pixel centres and the two tangents of each pixel."""
    c = camera.unpack(cam)
    W, H = c["W"], c["H"]
    D = np.asarray(depth, np.float64)
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    fin = np.isfinite(D)
    Dz = np.where(fin, D, 1.0)
    V = camera.pixel_view_point(c, ii.astype(np.float64), jj.astype(np.float64), Dz)
    P = c["pos"] + camera.view_to_world_dir(c, V.reshape(-1, 3)).reshape(H, W, 3)

    def tangent(axis):
        fwd = np.zeros_like(P)
        nxt = np.roll(P, -1, axis=axis)
        prv = np.roll(P, 1, axis=axis)
        fn = np.roll(fin, -1, axis=axis)
        fp = np.roll(fin, 1, axis=axis)
        idx = ii if axis == 1 else jj
        n_lim = W if axis == 1 else H
        fn = fn & (idx + 1 < n_lim)
        fp = fp & (idx - 1 >= 0)
        both = fn & fp
        fwd[both] = 0.5 * (nxt[both] - prv[both])
        only_n = fn & ~fp
        fwd[only_n] = nxt[only_n] - P[only_n]
        only_p = fp & ~fn
        fwd[only_p] = P[only_p] - prv[only_p]
        have = fn | fp
        return fwd, have

    dx, hx = tangent(1)
    dy, hy = tangent(0)
    return c, P, fin, dx, hx, dy, hy


def depth_normals(cam, depth):
    """World-space unit normals [H][W][3] from the depth buffer."""
    c, P, fin, dx, hx, dy, hy = _tangents(cam, depth)
    n = np.cross(dx, dy)
    to_cam = c["pos"] - P
    ok = hx & hy & (np.linalg.norm(n, axis=-1) > 0)
    n = np.where(ok[..., None], n, to_cam)
    n = n / np.linalg.norm(n, axis=-1, keepdims=True)
    flip = (n * to_cam).sum(-1) < 0
    n[flip] = -n[flip]
    n[~fin] = 0.0
    return n


def depth_normal_condition(cam, depth):
    """|t_x| |t_y| / |t_x x t_y| per pixel: how much a relative error in the
    two tangents turns the normal (one over the sine of their angle).  Inf
    where the cross product vanishes; 1 where the normal falls back to the
    direction toward the camera.  The conditioning of the pixel, not part of
    the method."""
    _, _, fin, dx, hx, dy, hy = _tangents(cam, depth)
    cr = np.linalg.norm(np.cross(dx, dy), axis=-1)
    num = np.linalg.norm(dx, axis=-1) * np.linalg.norm(dy, axis=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        k = np.where(cr > 0, num / np.where(cr > 0, cr, 1.0), np.inf)
    k = np.where(hx & hy, k, 1.0)
    return np.where(fin, k, 0.0)


def brdf_lut(n=128, k=64):
    """[n][n][2] table: rows rho_j = (j + 1/2)/n, columns mu_i = (i + 1/2)/n,
    entries (A, B) of the Schlick split, each the mean over the k x k
    stratified visible-normal samples u = ((a + 1/2)/k, (b + 1/2)/k)."""
    mu = (np.arange(n) + 0.5) / n
    rho = (np.arange(n) + 0.5) / n
    ua = (np.arange(k) + 0.5) / k
    u1, u2 = np.meshgrid(ua, ua, indexing="ij")
    u1, u2 = u1.reshape(-1), u2.reshape(-1)
    out = np.zeros((n, n, 2))
    for j, r in enumerate(rho):
        for i, m in enumerate(mu):
            wo = np.array([math.sqrt(1.0 - m * m), 0.0, m])
            h = brdf.sample_vndf(np.broadcast_to(wo, (u1.size, 3)), np.full(u1.size, r), u1, u2)
            cos_oh = h @ wo
            l = 2.0 * cos_oh[:, None] * h - wo
            cnl = l[:, 2]
            ok = cnl > 0
            g1 = np.zeros(u1.size)
            g1[ok] = brdf.smith_g1(cnl[ok], np.full(ok.sum(), r))
            fc = (1.0 - cos_oh) ** 5
            out[j, i, 0] = np.mean((1.0 - fc) * g1)
            out[j, i, 1] = np.mean(fc * g1)
    return out


def lut_lookup(lut, mu, rho):
    """Bilinear read at (n.v, rho), texel centres at (i + 1/2)/n, clamped."""
    n = lut.shape[0]
    x = np.clip(np.asarray(mu, np.float64) * n - 0.5, 0.0, n - 1.0)
    y = np.clip(np.asarray(rho, np.float64) * n - 0.5, 0.0, n - 1.0)
    x0 = np.minimum(np.floor(x).astype(np.int64), n - 2) if n > 1 else np.zeros_like(x, np.int64)
    y0 = np.minimum(np.floor(y).astype(np.int64), n - 2) if n > 1 else np.zeros_like(y, np.int64)
    fx = (x - x0)[..., None]
    fy = (y - y0)[..., None]
    x1 = np.minimum(x0 + 1, n - 1)
    y1 = np.minimum(y0 + 1, n - 1)
    return ((1 - fx) * (1 - fy) * lut[y0, x0] + fx * (1 - fy) * lut[y0, x1]
            + (1 - fx) * fy * lut[y1, x0] + fx * fy * lut[y1, x1])


def first_pass_bound(cam, gbuf, env_rgb, lut, eps=1e-6, pix=None):
    """How far each c1 can move, to first order, when a component of the
    stored normal is off by a relative eps (its rounding; zero components stay
    zero) or the mirror direction is turned by eps radians (the rounding of
    the directions derived from the normal and the view ray): the
    conditioning of the pixel, not part of the method."""
    mips = env.build_mips(np.asarray(env_rgb, np.float64))
    base = first_pass(cam, gbuf, env_rgb, lut, pix=pix, mips=mips)
    worst = np.zeros_like(base)
    for k in range(3):
        for sgn in (1.0, -1.0):
            g = dict(gbuf)
            nr = np.array(gbuf["normal_rough"], np.float64)
            nr[..., k] *= 1.0 + sgn * eps
            g["normal_rough"] = nr
            worst = np.maximum(worst, np.abs(first_pass(cam, g, env_rgb, lut, pix=pix,
                                                        mips=mips) - base))
    for k in range(2):
        for sgn in (1.0, -1.0):
            worst = np.maximum(worst, np.abs(first_pass(cam, gbuf, env_rgb, lut, pix=pix, mips=mips,
                                                        _turn_r=(k, sgn * eps)) - base))
    return worst


def first_pass(cam, gbuf, env_rgb, lut, pix=None, mips=None, _turn_r=None):
    """c1 [H][W][4] = (c_d + c_s, 0) per pixel (float64); with ``pix`` (flat
    pixel indices) only those pixels, as [n][4].  (``_turn_r`` = (k, angle)
    turns each mirror direction toward its k-th tangent, for the bound.)"""
    c = camera.unpack(cam)
    W, H = c["W"], c["H"]
    D = np.asarray(gbuf["depth"], np.float64).reshape(-1)
    nr = np.asarray(gbuf["normal_rough"], np.float64).reshape(-1, 4)
    am = np.asarray(gbuf["albedo_metal"], np.float64).reshape(-1, 4)
    if mips is None:
        mips = env.build_mips(np.asarray(env_rgb, np.float64))
    sel = np.arange(W * H) if pix is None else np.asarray(pix, np.int64).reshape(-1)
    out = np.zeros((W * H, 4))
    shape = (H, W, 4) if pix is None else (sel.size, 4)
    fg = sel[np.isfinite(D[sel])]
    if fg.size == 0:
        return out[sel].reshape(shape)
    i, j = fg % W, fg // W
    V0 = camera.pixel_view_point(c, i.astype(np.float64), j.astype(np.float64), D[fg])
    wo = -camera.view_to_world_dir(c, V0)
    wo /= np.linalg.norm(wo, axis=-1, keepdims=True)
    n = brdf.normalize(nr[fg, :3])
    rho = np.clip(nr[fg, 3], 0.0, 1.0)
    a = am[fg, :3]
    m = np.clip(am[fg, 3], 0.0, 1.0)
    f0 = 0.04 * (1.0 - m)[:, None] + a * m[:, None]
    lam = env.roughness_level(mips, rho)
    cd = (1.0 - m)[:, None] * a * env.trilinear(mips, n, lam)
    cos_nv = brdf.dot(n, wo)
    r = 2.0 * cos_nv[:, None] * n - wo
    if _turn_r is not None:
        tan = brdf.onb(r)[_turn_r[0]]
        r = math.cos(_turn_r[1]) * r + math.sin(_turn_r[1]) * tan
    ab = lut_lookup(lut, np.clip(cos_nv, 0.0, 1.0), rho)
    fs = f0 * ab[:, 0:1] + ab[:, 1:2]
    cs = env.trilinear(mips, r, lam) * fs
    cs[cos_nv <= 0] = 0.0
    out[fg, :3] = cd + cs
    return out[sel].reshape(shape)
