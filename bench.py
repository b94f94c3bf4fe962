"""Throughput of screen-space GGX shading on one MI355X.

One step = one frame of the whole hot path on the headline workload: build
the (min, max) inverse-depth pyramid of the frame's depth buffer, then shade every pixel
(direct diffuse + 16-sample Monte-Carlo specular with the hierarchical
march) of the 1920x1080 synthetic scene (ground plane, 40 spheres, 60 boxes,
512x256 lognormal(0, 2) environment; the paper's own data is not public).
Inputs are resident in HBM before timing; the env mip chain is built once
(the environment is an input that does not change between frames).

Prints one JSON line: Mrays/s (= W*H*spp / frame time), ms per frame, the
FP16 and BF16 G-buffer variants of the same frame, the roofline figure of the
shading kernel and the FP64 oracle timed on this host's cores.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="FP32 only")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="oracle sample: every k-th row (default 8)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--no-backward", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--no-first-pass", action="store_true", help="skip the first-pass timing")
    ap.add_argument("--serve-workspace-gib", type=float, default=6.0,
                    help="device memory for request workspaces in the serving run")
    ap.add_argument("--copy-reference", action="store_true",
                    help="also run one plain device copy of 256 MiB (the reference for "
                         "scaling hardware byte counters)")
    return ap.parse_args()


def upload(scene, dtype, dev):
    import torch

    from scenes import quantise_gbuffer
    t = dict(depth=torch.from_numpy(scene.depth).to(dev), env=torch.from_numpy(scene.env).to(dev))
    if dtype == "f32":
        for k in ("normal_rough", "albedo_metal", "radiance"):
            t[k] = torch.from_numpy(getattr(scene, k)).to(dev)
    else:
        bits, _ = quantise_gbuffer(scene, dtype)
        tdt = torch.float16 if dtype == "f16" else torch.bfloat16
        for k in ("normal_rough", "albedo_metal", "radiance"):
            t[k] = torch.from_numpy(bits[k].view(np.int16)).to(dev).view(tdt)
    return t


# Roofline of the path: HBM bandwidth on the method's algorithmic bytes, with
# the VALU rate beside it.  Per frame (P pixels, S samples each):
#
#   B = P (B_g + 12 + 16/3) + sum over samples of (4 n_iter + B_r)
#
#   B_g   G-buffer bytes per pixel: depth 4 + normal/roughness 16 +
#         albedo/metallic 16 + radiance 12 = 48 (FP32), 4 + 8 + 8 + 6 = 26
#         (FP16 / BF16; depth stays FP32)
#   12    the FP32 RGB output
#   16/3  the depth pyramid: 4 B of depth read + 4/3 B of pyramid written
#   4     one 4 B depth per march iteration (n_iter iterations of the sample)
#   B_r   the radiance read of a sample that reaches one: 12 at a hit (FP32;
#         6 FP16 / BF16) or of environment on a miss (-1, -4); 0 otherwise
#
# The trace kernel processes every pixel and sample of the frame, so its
# figure is B over its average launch time; the frame's is B over the frame
# time.  The trace's own share (depth 4 + normal 16 (8) per pixel, 4 B per
# iteration) is reported beside them.
#
# VALU: about 200 lane operations per sample (Philox, the visible-normal
# sample, the segment, the weight and the sum) plus 25 per march iteration.
# Peak: 157.3 TFLOP/s FP32 vector counts an FMA as two flops and a packed
# instruction as two lanes; single 32-bit lane operations issue at
# 256 CUs x 64 lanes x 2.4 GHz.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
ALU_OPS_PER_SAMPLE = 200
ALU_OPS_PER_ITER = 25

# A finer model of the implementation's own operation counts (an FMA, a
# compare, a select, a transcendental instruction each count one), kept as a
# separately named figure:
OPS_PER_HIZ_ITER = 54     # two cells (the cell and its parent), each: cell index 2,
                          # exit parameter per axis 3 (x2), nearer exit 1, ray
                          # inverse depth at the exit 1, texel address 2, front
                          # test 1, behind test 2 (= 15, x2 = 30); level-0 test 6;
                          # move / arm / level choice 8; advance 5; loop control 5
OPS_PER_LINEAR_STEP = 20  # point 3, projection 5, bounds 4, texel address 3, tests 5
OPS_PER_SAMPLE = 156      # Philox4x32-10 98 and the two 24-bit uniforms 6; the
                          # visible-normal sample (stretch, normalise, cap point,
                          # sin/cos, un-stretch, normalise) 30; to world 9;
                          # reflection and the two cosines 13
OPS_PER_SEGMENT = 35      # view direction 9, end point 8, projection 10, screen
                          # deltas and inverse depths 8
OPS_PER_PIXEL_SETUP = 48  # un-projection 3, view vector 17, normal 7, clamps 2,
                          # frame 10, local view vector 9


def work_model(scene, hits, steps, dtype):
    """Algorithmic bytes and operations of one frame from its hit codes and
    iteration counts (the model above)."""
    P = scene.width * scene.height
    S = hits.shape[-1]
    half = dtype != "f32"
    n_iter = int(steps.sum(dtype=np.int64))
    rays = (hits >= 0) | (hits == -1) | (hits == -4)  # samples that reach a radiance lookup
    n_hit = int((hits >= 0).sum())
    n_rays = int(rays.sum())
    n_env = n_rays - n_hit
    fg = int((hits[..., 0] != -3).sum())
    n_drawn = int((hits != -3).sum() - (hits == -5).sum())
    B_g = 26 if half else 48
    b_hit = 6 if half else 12
    frame_bytes = P * (B_g + 12) + (P * 16) // 3 + 4 * n_iter + b_hit * n_hit + 12 * n_env
    trace_bytes = P * (4 + (8 if half else 16)) + 4 * n_iter
    alu_ops = ALU_OPS_PER_SAMPLE * P * S + ALU_OPS_PER_ITER * n_iter
    hiz = scene.params["march"] == 1
    impl_ops = ((OPS_PER_HIZ_ITER if hiz else OPS_PER_LINEAR_STEP) * n_iter
                + OPS_PER_SAMPLE * n_drawn + OPS_PER_SEGMENT * n_rays + OPS_PER_PIXEL_SETUP * fg)
    return dict(frame_bytes=frame_bytes, trace_bytes=trace_bytes, alu_ops=alu_ops,
                impl_ops_trace=impl_ops, mean_iters=n_iter / max(1, n_rays),
                hit_frac=n_hit / max(1, n_rays), iterations=n_iter, rays=n_rays)


COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "trace_hiz_kernel_c2_1080p_16spp_counters.md")


KERNEL_SOURCES = ("device_math.h", "kernels.h", "pyramids.hip", "shade.hip", "shading.h")


def kernel_sources_digest():
    """SHA-256 over the sources the kernels are compiled from, in name order."""
    import hashlib
    d = os.path.join(ROOT, "paper_2504_01358_amd", "csrc")
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


# the "name = value" figures of the counter summary that the line reports
PROFILE_FIGURES = ("traffic_bytes_per_launch", "l2_hit_rate", "valu_busy", "valu_lane_utilisation")


def profile_figures():
    """The figures of the committed counter summary (HBM bytes per launch of
    the shading kernel, its L2 hit rate, VALU busy share and lane utilisation),
    or {} when the summary is absent or was taken from other sources."""
    try:
        with open(COUNTER_SUMMARY) as f:
            text = f.read()
    except OSError:
        return {}
    vals = {}
    for ln in text.splitlines():
        if "=" in ln and ln.strip().startswith(PROFILE_FIGURES + ("sources_sha256",)):
            k, v = ln.strip().strip("`").split("=", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.pop("sources_sha256", None) != kernel_sources_digest():
        return {}
    out = {}
    for k, v in vals.items():
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


def measured_traffic():
    """HBM bytes per launch of the shading kernel from the committed counter
    summary, or None when it is absent or was taken from other sources."""
    return profile_figures().get("traffic_bytes_per_launch")


def measured_counters():
    """L2 hit rate, VALU busy share and lane utilisation of the shading kernel
    from the committed counter summary (None under the same rule as the
    traffic)."""
    f = profile_figures()
    keys = ("l2_hit_rate", "valu_busy", "valu_lane_utilisation")
    if not all(k in f for k in keys):
        return None
    return dict({k: f[k] for k in keys},
                source=os.path.relpath(COUNTER_SUMMARY, ROOT))


def time_gpu(ctx, scene, dtype, steps, warmup, dev, mips):
    import torch

    from paper_2504_01358_amd import ssr
    t = upload(scene, dtype, dev)
    H, W, S = scene.height, scene.width, scene.params["spp"]
    out = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    hiz = torch.empty(ssr.hiz_floats(W, H), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    cam = ssr.make_camera(scene.camera)
    prm = ssr.make_params(scene.params)
    # the timed frames keep their codes tile-major, as ssr_shade does for its own
    # workspace (same values, far fewer partial-line writes)
    prm_t = ssr.make_params(dict(scene.params,
                                 flags=int(scene.params.get("flags", 0)) | ssr.CODES_TILED))
    codes = torch.empty(ssr.codes_shape(W, H, S, ssr.CODES_TILED), dtype=torch.int32, device=dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        ssr.hiz_build(t["depth"], scene.params["thickness"], out=hiz, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        ctx.trace(cam, t["depth"], t["normal_rough"], t["albedo_metal"], t["radiance"], prm_t,
                  hiz=hiz, hits=codes, stream=stream)
        if ev is not None:
            ev[2].record(stream)
        ctx.resolve(cam, t["depth"], t["normal_rough"], t["albedo_metal"], t["radiance"], t["env"],
                    prm_t, codes, env_mips=mips, out=out, stream=stream)
        if ev is not None:
            ev[3].record(stream)

    # untimed: the per-sample iteration counts and hit codes for the byte model
    hits = torch.empty((H, W, S), dtype=torch.int32, device=dev)
    nst = torch.empty((H, W, S), dtype=torch.int32, device=dev)
    ctx.shade(cam, t["depth"], t["normal_rough"], t["albedo_metal"], t["radiance"], t["env"], prm,
              env_mips=mips, out=out, hits=hits, steps=nst, stream=stream)
    torch.cuda.synchronize()
    hits_np, steps_np, out_np = hits.cpu().numpy(), nst.cpu().numpy(), out.cpu().numpy()
    del hits, nst

    for _ in range(warmup):
        step()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for k in range(steps):
        step(evs[k])
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    hiz_ms = [e[0].elapsed_time(e[1]) for e in evs]
    trace_ms = [e[1].elapsed_time(e[2]) for e in evs]
    resolve_ms = [e[2].elapsed_time(e[3]) for e in evs]
    frame_ms = [e[0].elapsed_time(e[3]) for e in evs]
    work = work_model(scene, hits_np, steps_np, dtype)
    return dict(ms_per_step=total_ms / steps, wall_ms_per_step=1e3 * wall / steps,
                frame_ms_p50=float(np.median(frame_ms)), frame_ms_p99=float(np.quantile(frame_ms, 0.99)),
                trace_ms=float(np.mean(trace_ms)), resolve_ms=float(np.mean(resolve_ms)),
                hiz_ms=float(np.mean(hiz_ms)), image=out_np, codes=hits_np,
                step_fn=step, **work)


def time_precision(runs, frames=100, warmup=10, block=10):
    """Frame times of the storage types side by side: blocks of `block`
    frames of each type in turn (so that clock and thermal drift fall on all
    of them alike) until each has `frames` timed frames, after `warmup`
    untimed frames each.  Per type: p50, p10 and p90 of the frame time and
    the p50 of the trace and resolve kernels, from HIP events on the stream
    the kernels run on."""
    import torch
    stream = torch.cuda.current_stream()
    for fn in runs.values():
        for _ in range(warmup):
            fn()
    times = {dt: [[], [], []] for dt in runs}
    while min(len(v[0]) for v in times.values()) < frames:
        for dt, fn in runs.items():
            evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(block)]
            for e in evs:
                fn(e)
            stream.synchronize()
            for e in evs:
                times[dt][0].append(e[0].elapsed_time(e[3]))
                times[dt][1].append(e[1].elapsed_time(e[2]))
                times[dt][2].append(e[2].elapsed_time(e[3]))
    out = {}
    for dt, (fr, tr, rs) in times.items():
        fr = np.array(fr)
        out[dt] = {"frames": int(fr.size), "frame_ms_p50": float(np.median(fr)),
                   "frame_ms_p10": float(np.quantile(fr, 0.1)),
                   "frame_ms_p90": float(np.quantile(fr, 0.9)),
                   "trace_ms_p50": float(np.median(tr)), "resolve_ms_p50": float(np.median(rs))}
    return out


def time_linear(ctx, scene, dev, mips, reps=20):
    """The same frame with the march of Algorithm 1 (the paper's linear
    march: 32 world-space steps of 0.125 up to a ray length of 4, the
    parameters of the small configuration) instead of the hierarchical one."""
    import torch

    from paper_2504_01358_amd import ssr
    t = upload(scene, "f32", dev)
    H, W, S = scene.height, scene.width, scene.params["spp"]
    prm = dict(scene.params, march=0, max_steps=32, step_len=0.125, max_dist=4.0)
    out = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    cam, p = ssr.make_camera(scene.camera), ssr.make_params(prm)

    def step():
        ctx.shade(cam, t["depth"], t["normal_rough"], t["albedo_metal"], t["radiance"], t["env"], p,
                  env_mips=mips, out=out, stream=stream)
    for _ in range(3):
        step()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"ms_per_step": ms, "value": H * W * S / (ms * 1e-3) / 1e6, "unit": "Mrays/s",
            "march": "linear (Algorithm 1): 32 steps of 0.125, ray length <= 4, thickness 0.05"}


def _oracle_rows(args):
    cfg, rows = args
    os.environ["OMP_NUM_THREADS"] = "1"
    import oracle
    import scenes
    sc = scenes.make_scene(cfg)
    g = dict(depth=sc.depth, normal_rough=sc.normal_rough, albedo_metal=sc.albedo_metal,
             radiance=sc.radiance)
    mips = oracle.env.build_mips(sc.env)
    pyr = ((oracle.march.hiz_pyramid(sc.depth), oracle.march.hiz_max_pyramid(sc.depth))
           if sc.params["march"] == 1 else None)
    t0 = time.perf_counter()
    n = 0
    outs, codes = [], []
    for r in rows:
        pix = np.arange(r * sc.width, (r + 1) * sc.width)
        res = oracle.shade_pixels(sc.camera, g, sc.env, sc.params, pix, pyramid=pyr, mips=mips)
        outs.append(res["out"])
        codes.append(res["hits"].astype(np.int32))
        n += pix.size
    return n, time.perf_counter() - t0, rows, outs, codes


# Worker processes of the CPU baseline: one per core the process may run on,
# at most 16 (the host share of one GPU on the machines this runs on).
CPU_WORKERS_MAX = 16


def cpu_baseline(cfg, scene, row_stride):
    """The FP64 oracle on every row_stride-th row of the frame, one worker
    process per available core (row-interleaved), wall-clock timed.  Returns
    the figure and the oracle's image and hit codes of those rows (for the
    error report of the GPU frames)."""
    import multiprocessing as mp
    affinity = len(os.sched_getaffinity(0))
    cores = min(affinity, CPU_WORKERS_MAX)
    rows = list(range(0, scene.height, row_stride))
    chunks = [rows[k::cores] for k in range(cores)]
    chunks = [c for c in chunks if c]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(len(chunks)) as pool:
        res = pool.map(_oracle_rows, [(cfg, c) for c in chunks])
    wall = time.perf_counter() - t0
    busy = max(r[1] for r in res)
    pixels = sum(r[0] for r in res)
    rays = pixels * scene.params["spp"]
    ref = {}
    for _, _, rr, outs, codes in res:
        for r, o, c in zip(rr, outs, codes):
            ref[r] = (o, c)
    order = sorted(ref)
    sample = dict(rows=np.array(order), out=np.stack([ref[r][0] for r in order]),
                  hits=np.stack([ref[r][1] for r in order]))
    fig = dict(value=rays / busy / 1e6, unit="Mrays/s", cores=len(chunks), kind="oracle",
               affinity_cores=affinity,
               sample=f"every {row_stride}th row of the frame ({len(rows)} rows, {pixels} pixels, "
                      f"{rays} rays), FP64 NumPy, {len(chunks)} worker processes (one per core "
                      f"of the {affinity} this process may use, at most {CPU_WORKERS_MAX}); "
                      f"{busy:.1f} s compute, {wall:.1f} s wall incl. start-up")
    return fig, sample


def error_report(gpu_image, gpu_codes, sample, tol):
    """The GPU frame against the FP64 oracle on the CPU baseline's rows:
    hit agreement over samples that march on either side, per-pixel relative
    error (p50, p99, max) over pixels whose samples all agree, the share of
    them within `tol`, and the image-level relative L1 over non-background
    pixels."""
    g = gpu_image[sample["rows"]].astype(np.float64).reshape(-1, 3)
    h = gpu_codes[sample["rows"]].reshape(g.shape[0], -1)
    o = sample["out"].reshape(-1, 3)
    oh = sample["hits"].reshape(g.shape[0], -1)
    nm = np.isin(h, (-2, -3, -5)) & np.isin(oh, (-2, -3, -5))
    agree = h == oh
    ok = agree.all(axis=1)
    rel = (np.abs(g - o) / np.maximum(np.abs(o), 1e-6)).max(axis=1)[ok]
    fg = oh[:, 0] != -3
    l1 = float(np.abs(g - o)[fg].sum() / max(np.abs(o)[fg].sum(), 1e-30))
    return {"pixels": int(g.shape[0]), "hit_agreement": float(agree[~nm].mean()),
            "pixels_all_agree": float(ok.mean()), "rel_p50": float(np.quantile(rel, 0.5)),
            "rel_p99": float(np.quantile(rel, 0.99)), "rel_max": float(rel.max()),
            f"frac_within_{tol:g}": float((rel <= tol).mean()), "image_rel_l1": l1}


def time_backward(ctx, dev, reps=20):
    """The differentiation workload (800x800, 8 spp, Hi-Z, FP32): one
    forward with hit codes, then the adjoint with every gradient output."""
    import torch

    import scenes
    sc = scenes.make_scene("c4")
    t = {k: torch.from_numpy(getattr(sc, k)).to(dev)
         for k in ("depth", "normal_rough", "albedo_metal", "radiance", "env")}
    H, W = sc.height, sc.width
    hits = torch.empty((H, W, sc.params["spp"]), dtype=torch.int32, device=dev)
    g_rgb = torch.randn((H, W, 3), dtype=torch.float32, device=dev)
    g_nr = torch.empty((H, W, 4), dtype=torch.float32, device=dev)
    g_am = torch.empty_like(g_nr)
    g_rad = torch.zeros_like(g_nr)
    g_env = torch.zeros_like(t["env"])
    stream = torch.cuda.current_stream(dev)
    args = (sc.camera, t["depth"], t["normal_rough"], t["albedo_metal"], t["radiance"], t["env"],
            sc.params)

    def fwd():
        ctx.shade(*args, hits=hits, stream=stream)

    def bwd():
        ctx.shade_backward(*args, hits, g_rgb, g_normal_rough=g_nr, g_albedo_metal=g_am,
                           g_env=g_env, g_radiance=g_rad, stream=stream)
    res = {}
    for name, fn in (("forward_ms", fwd), ("backward_ms", bwd)):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / reps
    res["backward_Mpixels_per_s"] = H * W / (res["backward_ms"] * 1e-3) / 1e6
    res["workload"] = ("c4: 800x800, 8 spp, Hi-Z, FP32; gradients for normal, roughness, albedo, "
                       "metallic, radiance and the 256x128 env (hit codes held fixed)")
    return res


def time_first_pass(ctx, scene, dev, reps=50):
    """The first shading pass on the benchmark frame: depth normals and c1
    (FP32 and FP16 G-buffers), average kernel time over `reps` launches.
    Algorithmic HBM bytes per pixel: depth normals read the depth (4 B; the
    neighbours come from cache) and write three channels; the first pass
    reads depth, normal_rough and albedo_metal and writes c1 (the 2 MB env
    mip chain stays in L2)."""
    import torch

    from paper_2504_01358_amd import ssr
    H, W = scene.height, scene.width
    stream = torch.cuda.current_stream(dev)
    cam = ssr.make_camera(scene.camera)
    res = {}
    for dt in ("f32", "f16"):
        t = upload(scene, dt, dev)
        mips = ssr.env_build_mips(t["env"], stream=stream)   # built once, as for the shading
        esz = 4 if dt == "f32" else 2
        nr = t["normal_rough"].clone()
        out = torch.empty_like(t["normal_rough"])
        ssr.depth_normals(cam, t["depth"], nr, stream=stream)          # first call: table
        ctx.first_pass(cam, t["depth"], t["normal_rough"], t["albedo_metal"], t["env"], env_mips=mips,
                       out=out, stream=stream)
        for name, fn, per_px in (
                ("depth_normals", lambda: ssr.depth_normals(cam, t["depth"], nr, stream=stream),
                 4 + 3 * esz),
                ("first_pass", lambda: ctx.first_pass(cam, t["depth"], t["normal_rough"],
                                                      t["albedo_metal"], t["env"], env_mips=mips,
                                                      out=out, stream=stream),
                 4 + 3 * 4 * esz)):
            for _ in range(3):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            gbs = per_px * W * H / (ms * 1e-3) / 1e9
            res[f"{name}_{dt}"] = {"kernel_ms": ms, "bytes_per_pixel": per_px, "hbm_gbs": gbs,
                                   "hbm_frac": gbs / HBM_PEAK_GBS}
        del t, nr, out
    res["workload"] = f"{W}x{H}, the shading benchmark's frame"
    return res


def _serving_scene_task(task):
    """One (scene, resolution) of the serving mix, FP16 G-buffer bits."""
    k, ri = task
    os.environ["OMP_NUM_THREADS"] = "1"
    import scenes
    w, h = scenes.SERVE["resolutions"][ri]
    sc = scenes.serving_scene(k, w, h)
    bits, _ = scenes.quantise_gbuffer(sc, scenes.SERVE["dtype"])
    return (k, ri, sc.camera, sc.depth, {b: bits[b] for b in ("normal_rough", "albedo_metal", "radiance")},
            sc.env, sc.params)


def serving_scenes():
    """All scenes of the serving mix at all resolutions, generated in parallel
    (largest first), before anything initialises the GPU."""
    import multiprocessing as mp

    import scenes
    tasks = [(k, ri) for ri in reversed(range(len(scenes.SERVE["resolutions"])))
             for k in range(scenes.SERVE["n_scenes"])]
    workers = min(len(os.sched_getaffinity(0)), 8)
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        out = list(pool.imap_unordered(_serving_scene_task, tasks))
    return out, time.perf_counter() - t0


def serve_run(data, workspace_bytes, dev, saturated=False, graphs=True):
    """The serving mix through an ssr_session: requests submitted at their
    arrival times (or, saturated, all at once, so that the delivered rate is
    the session's capacity), results collected as they finish."""
    import torch

    import scenes
    from paper_2504_01358_amd import ssr
    # the budget: the scenes (an upper bound of their session footprint) plus
    # the request workspace
    scene_bound = 0
    for k, ri, cam, depth, bits, env, params in data:
        px = cam["width"] * cam["height"]
        scene_bound += px * 28 + env.size * 4 + ssr.env_mips_floats(env.shape[1], env.shape[0]) * 4 + 8 * 256
    sess = ssr.Session(0, hbm_budget_bytes=int(scene_bound + workspace_bytes), max_slots=8,
                       max_bypass=8, graphs=graphs)
    ids, cams = {}, {}
    for k, ri, cam, depth, bits, env, params in data:
        t = {b: torch.from_numpy(bits[b].view(np.int16)).to(dev).view(torch.float16) for b in bits}
        ids[(k, ri)] = sess.add_scene(cam, torch.from_numpy(depth).to(dev), t["normal_rough"],
                                      t["albedo_metal"], t["radiance"], torch.from_numpy(env).to(dev))
        cams[(k, ri)] = cam
        base = params
    torch.cuda.synchronize()
    reqs = scenes.serving_requests()
    pending, done = {}, []

    def collect():
        for tk in list(pending):
            r = sess.poll(tk)
            if r is not None:
                r["rays"] = pending.pop(tk)
                done.append(r)

    t0 = time.perf_counter()
    for n, (ta, k, ri, spp) in enumerate(reqs):
        while not saturated and time.perf_counter() - t0 < ta:
            collect()
            time.sleep(0.0002)
        cam = cams[(k, ri)]
        prm = dict(base, spp=spp, seed=7000 + n, frame=n)
        tk, _ = sess.submit(ids[(k, ri)], prm)
        pending[tk] = cam["width"] * cam["height"] * spp
    for tk in list(pending):
        r = sess.wait(tk)
        r["rays"] = pending.pop(tk)
        done.append(r)
    st = sess.stats()
    sess.close()
    lat = np.array([r["t_done"] - r["t_submit"] for r in done]) * 1e3
    queue = np.array([r["t_admit"] - r["t_submit"] for r in done]) * 1e3
    span = max(r["t_done"] for r in done) - min(r["t_submit"] for r in done)
    rays = sum(r["rays"] for r in done)
    ev = sorted([(r["t_admit"], 1) for r in done] + [(r["t_done"], -1) for r in done])
    conc = peak = 0
    for _, d in ev:
        conc += d
        peak = max(peak, conc)
    return {"requests": len(done), "failed": int(sum(r["status"] != 0 for r in done)),
            "latency_ms_p50": float(np.median(lat)), "latency_ms_p99": float(np.quantile(lat, 0.99)),
            "latency_ms_mean": float(lat.mean()),
            "admission_wait_ms_p50": float(np.median(queue)),
            "admission_wait_ms_p99": float(np.quantile(queue, 0.99)),
            "value": rays / span / 1e6, "unit": "Mrays/s", "span_s": span,
            "offered_Mrays_per_s": (rays / reqs[-1][0] / 1e6) if not saturated else None,
            "peak_concurrent": peak, "scene_bytes": st["scene_bytes"],
            "workspace_bytes": st["arena_bytes"], "dtype": "f16",
            "frames": "graph replays" if graphs else "direct launches",
            "mix": "8 scenes (100-400 objects) x {640x360,1280x720,1920x1080,3840x2160}, spp "
                   "{4,16,64}, 512 requests, " + ("all submitted at once" if saturated else
                                                  "Poisson arrivals at 200/s")
                   + ", FP16 G-buffers, Hi-Z"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this path runs on one GPU; the multi-GPU layout is a design note only "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import scenes
    scene = scenes.make_scene(args.config)
    # the CPU leg runs first, before anything initialises the GPU, so its
    # worker processes start from a process with no device state
    cpu = sample = None
    if not args.no_cpu_baseline:
        cpu, sample = cpu_baseline(args.config, scene, args.cpu_rows or 8)
        print(f"bench: oracle {cpu['value']:.3f} Mrays/s on {cpu['cores']} cores "
              f"({cpu['affinity_cores']} available)", file=sys.stderr, flush=True)

    serve_data = None
    if not args.no_serve:
        serve_data, gen_s = serving_scenes()
        print(f"bench: serving scenes generated in {gen_s:.1f} s", file=sys.stderr, flush=True)

    import torch

    from paper_2504_01358_amd import ssr
    dev = torch.device("cuda", 0)
    ctx = ssr.Context(0)
    mips = ssr.env_build_mips(torch.from_numpy(scene.env).to(dev))
    print(f"bench: {args.config} {scene.width}x{scene.height} spp={scene.params['spp']}",
          file=sys.stderr, flush=True)
    res = {"f32": time_gpu(ctx, scene, "f32", args.steps, args.warmup, dev, mips)}
    print(f"bench: f32 {res['f32']['ms_per_step']:.3f} ms/frame", file=sys.stderr, flush=True)
    if not args.no_variants:
        for dt in ("f16", "bf16"):
            res[dt] = time_gpu(ctx, scene, dt, args.steps, args.warmup, dev, mips)
            print(f"bench: {dt} {res[dt]['ms_per_step']:.3f} ms/frame", file=sys.stderr, flush=True)
    if args.copy_reference:
        # 256 MiB read + 256 MiB written; 1 GiB written in between pushes the
        # source out of the 256 MB Infinity Cache so its reads reach HBM
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        flush = torch.empty(256 << 20, dtype=torch.float32, device=dev)
        flush.fill_(2.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst, flush
    rays = scene.width * scene.height * scene.params["spp"]
    r32 = res["f32"]
    trace_s, frame_s = r32["trace_ms"] * 1e-3, r32["ms_per_step"] * 1e-3
    B = r32["frame_bytes"]
    P = scene.width * scene.height
    line = {
        "metric": "Mrays/s + ms/frame at 1080p 16spp (FP32 vs FP16 G-buf); p50/p99 serve latency",
        "value": rays / frame_s / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {scene.width}x{scene.height}, "
                               f"{scene.params['spp']} spp, hierarchical-Z march (<= "
                               f"{scene.params['max_steps']} iterations, thickness 0.05), FP32 "
                               "G-buffer; plane + 40 spheres + 60 boxes; env 512x256 lognormal(0,2)",
                   "width": scene.width, "height": scene.height, "spp": scene.params["spp"],
                   "march": "hiz", "max_steps": scene.params["max_steps"]},
        # the frame's algorithmic bytes (every pixel and sample, which the
        # trace kernel processes) over the trace kernel's average duration
        "roofline": {"bound": "hbm", "achieved": B / trace_s / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": B / trace_s / 1e9 / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if args.config == "c2" else None,
                     "counters": measured_counters() if args.config == "c2" else None,
                     "kernel": "trace_hiz_kernel<f32>", "kernel_ms": r32["trace_ms"],
                     "algorithmic_bytes": B,
                     "bytes_model": "P (B_g + 12 + 16/3) + sum over samples (4 n_iter + B_r), "
                                    "B_g 48, B_r 12 (hit or env miss)",
                     "march_iterations": r32["iterations"], "rays": r32["rays"],
                     "mean_iterations_per_ray": r32["mean_iters"],
                     "frame": {"ms": r32["ms_per_step"], "gbs": B / frame_s / 1e9,
                               "frac": B / frame_s / 1e9 / HBM_PEAK_GBS},
                     "trace_share": {"bytes": r32["trace_bytes"],
                                     "gbs": r32["trace_bytes"] / trace_s / 1e9,
                                     "frac": r32["trace_bytes"] / trace_s / 1e9 / HBM_PEAK_GBS},
                     "alu": {"ops": r32["alu_ops"], "model": "200 per sample + 25 per iteration",
                             "tops": r32["alu_ops"] / trace_s / 1e12, "peak": VALU_PEAK_TOPS,
                             "frac": r32["alu_ops"] / trace_s / 1e12 / VALU_PEAK_TOPS},
                     "alu_impl_model": {"ops": r32["impl_ops_trace"],
                                        "tops": r32["impl_ops_trace"] / trace_s / 1e12,
                                        "frac": r32["impl_ops_trace"] / trace_s / 1e12 / VALU_PEAK_TOPS}},
        "resolve_ms": r32["resolve_ms"],
        "frame_ms_p50": r32["frame_ms_p50"], "frame_ms_p99": r32["frame_ms_p99"],
        "hiz_build_ms": r32["hiz_ms"],
        "hiz_build_gbs": P * 16 / 3 / (r32["hiz_ms"] * 1e-3) / 1e9,
    }
    if not args.no_variants:
        prec = time_precision({dt: res[dt]["step_fn"] for dt in res}, frames=max(100, args.steps))
        line["precision"] = prec
        for dt in ("f16", "bf16"):
            line[dt] = {"value": rays / (prec[dt]["frame_ms_p50"] * 1e-3) / 1e6,
                        "ms_per_step": res[dt]["ms_per_step"], **prec[dt],
                        "frame_bytes": res[dt]["frame_bytes"],
                        "hbm_frac_frame": res[dt]["frame_bytes"] / (prec[dt]["frame_ms_p50"] * 1e-3)
                        / 1e9 / HBM_PEAK_GBS}
        f32p, f16p = prec["f32"], prec["f16"]
        print(f"bench: frame p50 f32 {f32p['frame_ms_p50']:.4f} ms (p10-p90 "
              f"{f32p['frame_ms_p10']:.4f}-{f32p['frame_ms_p90']:.4f}), f16 "
              f"{f16p['frame_ms_p50']:.4f} ms ({f16p['frame_ms_p10']:.4f}-{f16p['frame_ms_p90']:.4f})",
              file=sys.stderr, flush=True)
    if sample is not None:
        line["error_vs_oracle"] = {
            dt: error_report(res[dt]["image"], res[dt]["codes"], sample, 1e-4 if dt == "f32" else 1e-3)
            for dt in res}
        line["error_vs_oracle"]["sample"] = ("the CPU baseline's rows; the oracle fed the FP32 "
                                             "G-buffer (for f16/bf16: the quantisation's own effect)")
    for r in res.values():
        for k in ("image", "codes", "step_fn"):
            r.pop(k, None)
    line["linear"] = time_linear(ctx, scene, dev, mips)
    print(f"bench: linear march {line['linear']['ms_per_step']:.3f} ms/frame", file=sys.stderr,
          flush=True)
    if not args.no_first_pass:
        line["first_pass"] = time_first_pass(ctx, scene, dev)
        fp = line["first_pass"]["first_pass_f32"]
        print(f"bench: first pass {fp['kernel_ms'] * 1e3:.1f} us ({fp['hbm_frac']:.2f} of HBM peak)",
              file=sys.stderr, flush=True)
    if not args.no_backward:
        line["backward"] = time_backward(ctx, dev)
        print(f"bench: backward {line['backward']['backward_ms']:.3f} ms at 800x800 8 spp",
              file=sys.stderr, flush=True)
    if serve_data is not None:
        ws = int(args.serve_workspace_gib * (1 << 30))
        line["serve"] = serve_run(serve_data, ws, dev)
        print(f"bench: serve p50 {line['serve']['latency_ms_p50']:.1f} ms p99 "
              f"{line['serve']['latency_ms_p99']:.1f} ms, {line['serve']['value']:.0f} Mrays/s",
              file=sys.stderr, flush=True)
        # capacity: the same requests all at once, graph replays and direct launches
        for key, graphs in (("serve_saturated", True), ("serve_saturated_direct", False)):
            line[key] = serve_run(serve_data, ws, dev, saturated=True, graphs=graphs)
            print(f"bench: {key} {line[key]['value']:.0f} Mrays/s delivered, p50 "
                  f"{line[key]['latency_ms_p50']:.1f} ms p99 {line[key]['latency_ms_p99']:.1f} ms",
                  file=sys.stderr, flush=True)
        line["serve_saturated"]["vs_fp32_single_frame"] = (
            line["serve_saturated"]["value"] / line["value"])
    if cpu is not None:
        line["cpu_baseline"] = cpu
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
