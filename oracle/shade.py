"""The per-pixel shading estimator, end to end, in float64.

Oracle code (test infrastructure only).

For a pixel with finite depth (Sec. 3.2 and Sec. 3.3):

  1. un-project the pixel centre to p; wo = normalize(camera - p); n the
     normalised stored normal; rho and m clamped to [0, 1];
     F0 = lerp(0.04, a, m)  (Appendix B, Eq. fresnel);
  2. direct diffuse c_d = (1 - m) a E_lambda(n), lambda = log2(1 + rho) lambda_max
     (Sec. 3.2, the c_d expression and SampleEnvMap; as written there, with
     no 1/pi and no cosine);
  3. for s = 0..S-1: draw (u1, u2) from Philox keyed by (pixel, sample),
     sample h from the visible-normal density, reflect wo about h to get the
     ray direction l (a sample with n.l <= 0 contributes zero but still
     counts in S), march l in screen space, read the first-pass radiance c1
     at the hit pixel (reading taken for misses: the unfiltered environment
     E_0 in direction l), weight by F(wo.h) G1(n.l);
  4. c_s' = (1/S) sum of weight * radiance  (Sec. 3.3, the Monte-Carlo
     estimator); output c_d + c_s' in linear HDR (reading taken: tone
     mapping and gamma, which the paper leaves unspecified, are not part of
     the compared output).

Pixels with n.wo <= 0 get no specular term.  Background pixels (depth not
finite) output E_0 in the pixel's view direction.

Hit codes per sample: q >= 0 hit pixel, -1 left the screen or segment,
-2 direction below the surface (or back-facing pixel), -3 background pixel,
-4 iteration cap, -5 specular disabled by flag.
"""

import numpy as np

from . import brdf, camera, env, march, philox

NO_DIRECT = 1
NO_SPECULAR = 2
SAMPLER_NDF = 4     # draw h from D(h) (n.h) (Walter et al. 2007) instead of visible normals

HIT_INVALID = -2
HIT_BACKGROUND = -3
HIT_SKIPPED = -5


def shade_pixels(cam, gbuf, env_rgb, params, pix, pyramid=None, mips=None,
                 check_long_form=True, sensitivity=None, replay_hits=None, hiz_scan=False):
    """Shade the flat pixel indices ``pix``.

    ``gbuf``: dict with ``depth`` [H][W], ``normal_rough``, ``albedo_metal``,
    ``radiance`` [H][W][4] (any float dtype; widened to float64).
    Returns dict(out [n][3], hits [n][S], steps [n][S]).

    With ``replay_hits`` [n][S] (hit codes, as this function returns them) the march
    is not run: each valid sample reads the radiance its given code names.
    This is the estimator with the hit selection held fixed, the form whose
    derivatives the adjoint computes (the march itself is not
    differentiable).

    With ``hiz_scan`` the hierarchical march is replaced by its pyramid-free
    definition, ``march.brute_force_first_hit`` (no iteration cap; the
    iteration counts are then 0): the exact first crossing the traversal
    must find whenever it is not capped.

    With ``sensitivity=eps`` (radians) the result also holds ``bound`` [n][3]:
    how far each output can move when every direction the estimator looks up
    (the normal of the diffuse lookup, each sample's ray direction) is off by
    eps, to first order, with the hit pixels held fixed.  It is the
    conditioning of the pixel, not part of the method.
    """
    c = camera.unpack(cam)
    W = c["W"]
    S = int(params["spp"])
    flags = int(params.get("flags", 0))
    pix = np.asarray(pix, np.int64).reshape(-1)
    n = pix.shape[0]
    depth = np.asarray(gbuf["depth"], np.float64)
    nr = np.asarray(gbuf["normal_rough"], np.float64).reshape(-1, 4)[pix]
    am = np.asarray(gbuf["albedo_metal"], np.float64).reshape(-1, 4)[pix]
    rad = np.asarray(gbuf["radiance"], np.float64).reshape(-1, 4)
    if mips is None:
        mips = env.build_mips(env_rgb)
    if pyramid is None and int(params["march"]) == 1 and replay_hits is None and not hiz_scan:
        pyramid = (march.hiz_pyramid(depth), march.hiz_max_pyramid(depth))

    i = pix % W
    j = pix // W
    D = depth.reshape(-1)[pix]
    out = np.zeros((n, 3))
    hits = np.full((n, S), HIT_BACKGROUND, np.int64)
    steps = np.zeros((n, S), np.int64)

    bound = np.zeros((n, 3))
    res = dict(out=out, hits=hits, steps=steps)
    if sensitivity is not None:
        res["bound"] = bound

    bg = ~(D < np.inf)
    if bg.any():
        vd = camera.view_ray_dir(c, i[bg], j[bg])
        out[bg] = env.bilinear(mips[0], vd)
        if sensitivity is not None:
            bound[bg] = _spread(lambda d: env.bilinear(mips[0], d), vd, sensitivity)
    fg = np.nonzero(~bg)[0]
    if fg.size == 0:
        return res

    # 1. per-pixel setup
    V0 = camera.pixel_view_point(c, i[fg], j[fg], D[fg])
    wo = -camera.view_to_world_dir(c, V0)
    wo /= np.linalg.norm(wo, axis=-1, keepdims=True)
    nrm = brdf.normalize(nr[fg, :3])
    rho = np.clip(nr[fg, 3], 0.0, 1.0)
    alb = am[fg, :3]
    met = np.clip(am[fg, 3], 0.0, 1.0)
    f0 = 0.04 * (1.0 - met)[:, None] + alb * met[:, None]

    # 2. direct diffuse
    if not flags & NO_DIRECT:
        lam = env.roughness_level(mips, rho)
        kd = (1.0 - met)[:, None] * alb
        out[fg] += kd * env.trilinear(mips, nrm, lam)
        if sensitivity is not None:
            bound[fg] += kd * _spread_components(lambda d: env.trilinear(mips, d, lam), nrm,
                                                 sensitivity)

    if flags & NO_SPECULAR:
        hits[fg] = HIT_SKIPPED
        return res

    # 3. one ray per (pixel, sample)
    cos_no = brdf.dot(nrm, wo)
    front = cos_no > 0
    hits[fg] = HIT_INVALID
    pf = fg[front]                      # rows of the output that trace rays
    kf = np.nonzero(front)[0]           # rows of the per-pixel arrays above
    if pf.size == 0:
        return res
    rep = np.repeat(kf, S)
    sidx = np.tile(np.arange(S), kf.size)
    u1, u2 = philox.sample_uniforms(pix[np.repeat(pf, S)], sidx, params["frame"],
                                    params["seed"])
    n_r = nrm[rep]
    wo_r = wo[rep]
    a_r = rho[rep]
    t, b = brdf.onb(n_r)
    wo_local = np.stack([brdf.dot(wo_r, t), brdf.dot(wo_r, b), cos_no[rep]], axis=-1)
    ndf_sampling = bool(flags & SAMPLER_NDF)
    if ndf_sampling:
        hl = brdf.sample_ndf(a_r, u1, u2)
    else:
        hl = brdf.sample_vndf(wo_local, a_r, u1, u2)
    h = hl[:, 0:1] * t + hl[:, 1:2] * b + hl[:, 2:3] * n_r
    cos_oh = brdf.dot(wo_r, h)
    l = 2.0 * cos_oh[:, None] * h - wo_r
    cos_nl = brdf.dot(n_r, l)
    ok = cos_nl > 0
    if ndf_sampling:
        ok &= cos_oh > 0          # a half vector facing away from wo reflects nothing

    code = np.full(rep.shape[0], HIT_INVALID, np.int64)
    nit = np.zeros(rep.shape[0], np.int64)
    r_ok = np.nonzero(ok)[0]
    if replay_hits is not None:
        given = np.asarray(replay_hits, np.int64).reshape(n, S)[pf].reshape(-1)
        code[r_ok] = given[r_ok]
        # a replayed code only counts where the sample is valid here too
        ok &= (code >= 0) | (code == march.HIT_OFFSCREEN) | (code == march.HIT_CAP)
    else:
        org = np.stack([i[fg][rep[r_ok]], j[fg][rep[r_ok]]], axis=1)
        Dv = camera.world_to_view_dir(c, l[r_ok])
        V0r = V0[rep[r_ok]]
        if int(params["march"]) == 0:
            cc, it = march.march_linear(cam, depth, org, V0r, Dv, float(params["step_len"]),
                                        int(params["max_steps"]), float(params["max_dist"]),
                                        float(params["thickness"]))
        elif hiz_scan:
            cc = march.brute_force_first_hit(cam, depth, org, V0r, Dv, float(params["max_dist"]),
                                             float(params["thickness"]), bbox=True)
            it = np.zeros_like(cc)
        else:
            cc, it = march.march_hiz(cam, pyramid, org, V0r, Dv, int(params["max_steps"]),
                                     float(params["max_dist"]), float(params["thickness"]))
        code[r_ok] = cc
        nit[r_ok] = it

    # radiance along each valid ray: c1 at the hit pixel, else the environment
    L = np.zeros((rep.shape[0], 3))
    hit = code >= 0
    L[hit] = rad[code[hit], :3]
    miss = ok & ~hit
    L[miss] = env.bilinear(mips[0], l[miss])

    w = np.zeros((rep.shape[0], 3))
    if ndf_sampling:
        w[ok] = brdf.weight_ndf_short(f0[rep[ok]], cos_no[rep[ok]], cos_nl[ok], cos_oh[ok],
                                      hl[ok, 2], a_r[ok])
    else:
        w[ok] = brdf.weight_short(f0[rep[ok]], cos_oh[ok], cos_nl[ok], a_r[ok])
    if check_long_form:
        lf = ok & (a_r > 1e-3)
        if lf.any():
            long_form = brdf.weight_ndf_long if ndf_sampling else brdf.weight_long
            wl = long_form(f0[rep[lf]], cos_no[rep[lf]], cos_nl[lf], cos_oh[lf], hl[lf, 2], a_r[lf])
            assert np.allclose(wl, w[lf], rtol=1e-9, atol=1e-12), "weight forms disagree"
    contrib = (w * L).reshape(kf.size, S, 3)
    out[pf] += contrib.sum(axis=1) / S
    hits[pf] = code.reshape(kf.size, S)
    steps[pf] = nit.reshape(kf.size, S)

    if sensitivity is not None and ok.any():
        # each valid sample's contribution as a function of its direction,
        # with its hit pixel (or miss) held fixed
        f0o, woo, no, ao = f0[rep[ok]], wo_r[ok], n_r[ok], a_r[ok]
        cno = cos_no[rep[ok]]
        hit_o, code_o = hit[ok], code[ok]

        def contribution(d):
            hh = brdf.normalize(woo + d)
            cnl = brdf.dot(no, d)
            if ndf_sampling:
                ww = brdf.weight_ndf_short(f0o, cno, np.maximum(cnl, 0.0), brdf.dot(woo, hh),
                                           brdf.dot(no, hh), ao)
            else:
                ww = brdf.weight_short(f0o, brdf.dot(woo, hh), np.maximum(cnl, 0.0), ao)
            ww[cnl <= 0] = 0.0
            LL = np.empty_like(ww)
            LL[hit_o] = rad[code_o[hit_o], :3]
            LL[~hit_o] = env.bilinear(mips[0], d[~hit_o])
            return ww * LL

        sp = np.zeros((rep.shape[0], 3))
        sp[ok] = _spread(contribution, l[ok], sensitivity)
        bound[pf] += sp.reshape(kf.size, S, 3).sum(axis=1) / S
    return res


def _spread_components(fn, d, eps):
    """Largest change of fn when one component of the unit vector d is scaled
    by (1 +- eps) and d renormalised: the rounding of a stored, normalised
    input, which leaves zero components zero (so a normal exactly at a pole
    of the equirect map stays there)."""
    d = brdf.normalize(d)
    base = fn(d)
    worst = np.zeros_like(base)
    for k in range(3):
        for sgn in (1.0, -1.0):
            dd = d.copy()
            dd[:, k] *= 1.0 + sgn * eps
            worst = np.maximum(worst, np.abs(fn(brdf.normalize(dd)) - base))
    return worst


def _spread(fn, d, eps):
    """Largest change of fn over the four directions d rotated by eps radians
    towards two orthogonal tangents (fn maps [m][3] directions to [m][3])."""
    d = brdf.normalize(d)
    t, b = brdf.onb(d)
    base = fn(d)
    worst = np.zeros_like(base)
    for tan in (t, b):
        for sgn in (1.0, -1.0):
            dd = np.cos(eps) * d + sgn * np.sin(eps) * tan
            worst = np.maximum(worst, np.abs(fn(dd) - base))
    return worst


def shade_frame(cam, gbuf, env_rgb, params, chunk=1 << 14, sensitivity=None):
    """Shade every pixel; returns out [H][W][3], hits and steps [H][W][S]
    (and ``bound`` [H][W][3] with ``sensitivity``, see shade_pixels)."""
    W, H = int(cam["width"]), int(cam["height"])
    S = int(params["spp"])
    mips = env.build_mips(env_rgb)
    pyramid = ((march.hiz_pyramid(gbuf["depth"]), march.hiz_max_pyramid(gbuf["depth"]))
               if int(params["march"]) == 1 else None)
    out = np.zeros((H * W, 3))
    bound = np.zeros((H * W, 3))
    hits = np.zeros((H * W, S), np.int64)
    steps = np.zeros((H * W, S), np.int64)
    per = max(1, chunk // max(S, 1))
    for k in range(0, H * W, per):
        pix = np.arange(k, min(k + per, H * W))
        r = shade_pixels(cam, gbuf, env_rgb, params, pix, pyramid=pyramid, mips=mips,
                         sensitivity=sensitivity)
        out[pix], hits[pix], steps[pix] = r["out"], r["hits"], r["steps"]
        if sensitivity is not None:
            bound[pix] = r["bound"]
    res = dict(out=out.reshape(H, W, 3), hits=hits.reshape(H, W, S),
               steps=steps.reshape(H, W, S))
    if sensitivity is not None:
        res["bound"] = bound.reshape(H, W, 3)
    return res
