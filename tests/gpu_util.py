"""Helpers for the GPU tests: upload inputs, run the library, run the oracle,
compare the two."""

import numpy as np
import torch

import oracle
from scenes import quantise_gbuffer

BUFS = ("normal_rough", "albedo_metal", "radiance")


def f32_camera(cam):
    """Round every camera value to float32 (what the library sees)."""
    out = dict(cam)
    out["pos"] = np.asarray(cam["pos"], np.float32)
    out["rot"] = np.asarray(cam["rot"], np.float32).reshape(3, 3)
    for k in ("fx", "fy", "cx", "cy", "z_near"):
        out[k] = np.float32(cam[k])
    return out


def f32_gbuf(g):
    return {k: np.ascontiguousarray(np.asarray(v, np.float32)) for k, v in g.items()}


def gbuf_of(scene):
    return dict(depth=scene.depth, normal_rough=scene.normal_rough,
                albedo_metal=scene.albedo_metal, radiance=scene.radiance)


def untile(t, W, H):
    """Tile-major per-sample buffer [ceil(H/8) ceil(W/8)][S][64] -> [H][W][S]."""
    ty, tx = (H + 7) // 8, (W + 7) // 8
    S = t.shape[1]
    x = t.reshape(ty, tx, S, 8, 8).transpose(0, 3, 1, 4, 2).reshape(ty * 8, tx * 8, S)
    return x[:H, :W]


def run_gpu(ctx, cam, g, env, params, dtype="f32", want_hits=True, want_steps=True,
            env_mips=None, hiz=None, tiled=False):
    """Shade on cuda:0.  Returns numpy out/hits/steps and the G-buffer values
    the GPU actually read (quantised for f16/bf16).  With ``tiled`` the frame
    is traced and resolved with tile-major codes (the launch configuration the
    benchmark times) and the codes are returned in [H][W][S]."""
    dev = torch.device("cuda", 0)
    W, H, S = int(cam["width"]), int(cam["height"]), int(params["spp"])
    depth = torch.from_numpy(np.ascontiguousarray(g["depth"], np.float32)).to(dev)
    seen = dict(depth=np.asarray(g["depth"], np.float32))
    if dtype == "f32":
        bufs = {k: torch.from_numpy(np.ascontiguousarray(g[k], np.float32)).to(dev) for k in BUFS}
        for k in BUFS:
            seen[k] = np.asarray(g[k], np.float32)
    else:
        class _S:
            pass
        s = _S()
        for k in BUFS:
            setattr(s, k, np.asarray(g[k], np.float32))
        bits, vals = quantise_gbuffer(s, dtype)
        tdt = torch.float16 if dtype == "f16" else torch.bfloat16
        bufs = {k: torch.from_numpy(bits[k].view(np.int16)).to(dev).view(tdt) for k in BUFS}
        seen.update(vals)
    envt = torch.from_numpy(np.ascontiguousarray(env, np.float32)).to(dev)
    if tiled:
        from paper_2504_01358_amd import ssr
        pt = dict(params, flags=int(params.get("flags", 0)) | ssr.CODES_TILED)
        shape = ssr.codes_shape(W, H, S, ssr.CODES_TILED)
        hits = torch.full(shape, -99, dtype=torch.int32, device=dev)
        steps = torch.full(shape, -99, dtype=torch.int32, device=dev) if want_steps else None
        args = (cam, depth, bufs["normal_rough"], bufs["albedo_metal"], bufs["radiance"])
        ctx.trace(*args, pt, hiz=hiz, hits=hits, steps=steps)
        out = ctx.resolve(*args, envt, pt, hits, env_mips=env_mips)
        torch.cuda.synchronize()
        res = dict(out=out.cpu().numpy().astype(np.float64),
                   hits=untile(hits.cpu().numpy(), W, H).astype(np.int64))
        if want_steps:
            res["steps"] = untile(steps.cpu().numpy(), W, H).astype(np.int64)
        return res, seen
    hits = torch.full((H, W, S), -99, dtype=torch.int32, device=dev) if want_hits else None
    steps = torch.full((H, W, S), -99, dtype=torch.int32, device=dev) if want_steps else None
    out = ctx.shade(cam, depth, bufs["normal_rough"], bufs["albedo_metal"], bufs["radiance"],
                    envt, params, env_mips=env_mips, hiz=hiz, hits=hits, steps=steps)
    torch.cuda.synchronize()
    res = dict(out=out.cpu().numpy().astype(np.float64))
    if want_hits:
        res["hits"] = hits.cpu().numpy().astype(np.int64)
    if want_steps:
        res["steps"] = steps.cpu().numpy().astype(np.int64)
    return res, seen


# Direction error allowed for the float32 path when bounding its output: the
# sampled ray direction passes through about sixteen float32 operations
# between the stored inputs and the environment lookup, each rounding by at
# most 2^-24 relative, which bounds its error by ~1e-6 rad (component-wise
# for the stored normal of the diffuse lookup).
DIR_EPS = 1e-6


def oracle_frame(cam, g, env, params):
    return oracle.shade_frame(cam, g, env, params, sensitivity=DIR_EPS)


def rel_err(gpu, ref, floor=1e-6):
    return np.abs(gpu - ref) / np.maximum(np.abs(ref), floor)


# Codes of samples that never march: invalid direction or back-facing
# pixel, background pixel, specular switched off.
NO_MARCH = (-2, -3, -5)

# Share of agreeing pixels that must be within plain rel_tol relative error,
# counted over the well-conditioned ones (the oracle's own bound for a
# DIR_EPS direction error below rel_tol |ref|).  Every agreeing pixel, well
# conditioned or not, must be within rel_tol |ref| + bound.
MIN_PLAIN = 0.999


def compare(gpu_out, gpu_hits, ref_out, ref_hits, label="", ref_bound=None, rel_tol=1e-4):
    """Hit agreement and per-pixel error.  Hit agreement counts the samples
    that march on either side (codes other than -2, -3, -5 on the GPU or in
    the oracle); the non-marching samples are compared on their own.  The
    per-pixel error is taken on pixels whose samples all agree.  With
    ``ref_bound`` (the oracle's first-order output change for a DIR_EPS
    direction error) also the excess of each pixel's error over
    rel_tol * |ref| + bound (``excess_max`` <= 0 passes) and the plain share
    over well-conditioned pixels (bound <= rel_tol |ref| in every channel).
    Returns a dict of statistics (printed)."""
    nm_ref = np.isin(ref_hits, NO_MARCH)
    nm_gpu = np.isin(gpu_hits, NO_MARCH)
    marched = ~(nm_ref & nm_gpu)
    agree = gpu_hits == ref_hits
    frac = agree[marched].mean() if marched.any() else 1.0
    nm = nm_ref | nm_gpu
    nm_frac = agree[nm].mean() if nm.any() else 1.0
    pix_ok = agree.all(axis=-1)
    rel = rel_err(gpu_out, ref_out).max(axis=-1)
    r = rel[pix_ok]
    stats = dict(samples_marched=int(marched.sum()), hit_agreement=float(frac),
                 no_march_agreement=float(nm_frac),
                 pixels_compared=int(pix_ok.sum()), pixels=int(pix_ok.size),
                 rel_p50=float(np.quantile(r, 0.5)) if r.size else 0.0,
                 rel_p99=float(np.quantile(r, 0.99)) if r.size else 0.0,
                 rel_p999=float(np.quantile(r, 0.999)) if r.size else 0.0,
                 rel_max=float(r.max()) if r.size else 0.0,
                 frac_within_1e4=float((r <= rel_tol).mean()) if r.size else 1.0)
    if ref_bound is not None:
        err = np.abs(gpu_out - ref_out)
        allowed = rel_tol * np.abs(ref_out) + ref_bound
        ex = (err - allowed)[pix_ok]
        stats["excess_max"] = float(ex.max()) if ex.size else 0.0
        brel = (ref_bound / np.maximum(np.abs(ref_out), 1e-6)).max(axis=-1)
        well = (brel <= rel_tol) & pix_ok
        stats["bound_dominated"] = float(1.0 - well.sum() / max(1, pix_ok.sum()))
        rw = rel[well]
        stats["well_conditioned"] = int(well.sum())
        stats["frac_within_1e4_well"] = float((rw <= rel_tol).mean()) if rw.size else 1.0
        stats["rel_max_well"] = float(rw.max()) if rw.size else 0.0
    print(f"[{label}] " + " ".join(f"{k}={v:.6g}" if isinstance(v, float) else f"{k}={v}"
                                   for k, v in stats.items()), flush=True)
    return stats
