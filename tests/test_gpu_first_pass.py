"""The first shading pass on the GPU (depth normals, the split-sum table, the
radiance c1) against the FP64 oracle, through the C-ABI.

Bars: the table within one float32 ulp (both sides form float64 means and
round them); every depth normal within 64 float32 ulps times the pixel's
conditioning (one over the sine of the angle between its tangents) plus
1e-6, both signs allowed where the normal is perpendicular to the view ray
within that tolerance; every c1 channel within 1e-4 relative error plus the
oracle's first-order bound for a 1e-6 error in the stored normal, at least
99 % of pixels within 1e-4 outright; 16-bit outputs one ulp of their type
more.  The input normals of the 16-bit cases are the quantised values the
GPU reads.
"""

import numpy as np
import pytest
import torch

import scenes
from closed_form import floor_wall_scene
from gpu_util import DIR_EPS, compare, f32_camera, oracle_frame, rel_err
from oracle import camera as ocam
from oracle import first_pass as ofp
from scenes import quantise_gbuffer

pytestmark = pytest.mark.gpu

REL_TOL = 1e-4
F32_EPS = 2.0 ** -24
TDT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
ULP = {"f32": 0.0, "f16": 2.0 ** -10, "bf16": 2.0 ** -7}   # relative, one ulp at worst


@pytest.fixture(scope="module")
def ctx():
    from paper_2504_01358_amd import ssr
    c = ssr.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def lut128():
    # the table the context builds (128 x 128, 64 x 64 samples), from the oracle
    return ofp.brdf_lut(128, 64)


def _dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).to(torch.device("cuda", 0))


def _to_cam(cam, depth):
    """Unit vectors from each pixel's world point toward the camera."""
    c = ocam.unpack(cam)
    H, W = depth.shape
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    D = np.where(np.isfinite(depth), depth, 1.0).astype(np.float64)
    V = ocam.pixel_view_point(c, ii.astype(np.float64), jj.astype(np.float64), D)
    t = -ocam.view_to_world_dir(c, V.reshape(-1, 3)).reshape(H, W, 3)
    return t / np.linalg.norm(t, axis=-1, keepdims=True)


# ------------------------------------------------------------- the table --

@pytest.mark.parametrize("n", [2, 7, 32])
def test_brdf_table_matches_oracle(n):
    from paper_2504_01358_amd import ssr
    gpu = ssr.brdf_lut(n).cpu().numpy().astype(np.float64)
    ref = ofp.brdf_lut(n, 64)
    err = np.abs(gpu - ref)
    print(f"[lut n={n}] max rel {np.max(err / np.maximum(ref, 1e-30)):.3g}", flush=True)
    assert np.all(err <= 2.0 * F32_EPS * np.abs(ref) + 1e-30)


# --------------------------------------------------------- depth normals --

def _gpu_normals(cam, depth, dtype, fill=0.375):
    from paper_2504_01358_amd import ssr
    H, W = depth.shape
    nr = torch.full((H, W, 4), fill, dtype=TDT[dtype], device=torch.device("cuda", 0))
    ssr.depth_normals(cam, _dev(depth), nr)
    torch.cuda.synchronize()
    out = nr.float().cpu().numpy().astype(np.float64)
    assert np.all(out[..., 3] == fill), "channel 3 must be left as it is"
    return out[..., :3]


def _check_normals(gpu, cam, depth, dtype, label):
    ref = ofp.depth_normals(cam, depth)
    k = ofp.depth_normal_condition(cam, depth)
    fin = np.isfinite(depth)
    tol = 64.0 * F32_EPS * k + 1e-6 + ULP[dtype]
    err = np.abs(gpu - ref).max(-1)
    bad = fin & (err > tol)
    # perpendicular to the view ray: turning it toward the camera is a sign
    # decision within the rounding, both results are valid
    tc = _to_cam(cam, depth)
    flip_ok = (np.abs(gpu + ref).max(-1) <= tol) & (np.abs((ref * tc).sum(-1)) <= tol)
    bad &= ~flip_ok
    print(f"[{label}] pixels {int(fin.sum())} err max {err[fin].max() if fin.any() else 0:.3g} "
          f"p99 {np.quantile(err[fin], 0.99) if fin.any() else 0:.3g} sign-free {int((flip_ok & fin & (err > tol)).sum())} "
          f"bad {int(bad.sum())}", flush=True)
    assert not bad.any(), np.argwhere(bad)[:5]
    assert np.all(gpu[~fin] == 0.0)
    # every surface normal is unit length and faces the camera
    assert np.all(np.abs(np.linalg.norm(gpu[fin], axis=-1) - 1.0) <= 1e-6 + 2 * ULP[dtype])
    assert np.all((gpu * tc).sum(-1)[fin] >= -tol[fin])


@pytest.mark.parametrize("kind,w,h", [("c2", 203, 117), ("c1", 64, 48), ("c2", 96, 64)])
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_depth_normals_match_oracle(kind, w, h, dtype):
    sc = scenes.make_scene(kind, seed=5, width=w, height=h)
    cam = f32_camera(sc.camera)
    depth = np.asarray(sc.depth, np.float32)
    _check_normals(_gpu_normals(cam, depth, dtype), cam, depth, dtype, f"{kind} {w}x{h} {dtype}")


def test_depth_normals_of_planes_and_holes():
    cam, g, _ = floor_wall_scene(w=48, h=40)
    cam = f32_camera(cam)
    depth = np.asarray(g["depth"], np.float32).copy()
    depth[10:14, 20:23] = np.inf          # a hole: one-sided and fallback pixels around it
    depth[0, :] = np.inf                  # a background row along the top
    depth[25, 30] = np.inf                # an isolated background pixel
    _check_normals(_gpu_normals(cam, depth, "f32"), cam, depth, "f32", "planes+holes")


@pytest.mark.parametrize("w,h", [(1, 1), (2, 1), (1, 3), (4096, 1), (1, 2000), (0, 0)])
def test_depth_normals_degenerate_sizes(w, h):
    """No neighbour on an axis: the normal points at the camera."""
    sc = scenes.make_scene("c1", seed=9, width=max(w, 1), height=max(h, 1))
    cam = f32_camera(dict(sc.camera, width=w, height=h))
    depth = np.asarray(sc.depth, np.float32)[:h, :w]
    depth = np.where(np.isfinite(depth), depth, 3.0).astype(np.float32)
    if w * h == 0:
        from paper_2504_01358_amd import ssr
        ssr.depth_normals(cam, _dev(np.zeros((0, 0), np.float32)))
        return
    _check_normals(_gpu_normals(cam, depth, "f32"), cam, depth, "f32", f"{w}x{h}")


# -------------------------------------------------------------- first pass --

def _gpu_first_pass(ctx, sc, cam, dtype):
    """c1 from the GPU and the G-buffer values it read."""
    g = dict(depth=np.asarray(sc.depth, np.float32),
             normal_rough=np.asarray(sc.normal_rough, np.float32),
             albedo_metal=np.asarray(sc.albedo_metal, np.float32))
    if dtype == "f32":
        nr, am = _dev(g["normal_rough"]), _dev(g["albedo_metal"])
    else:
        bits, vals = quantise_gbuffer(sc, dtype)
        nr = _dev(bits["normal_rough"].view(np.int16), np.int16).view(TDT[dtype])
        am = _dev(bits["albedo_metal"].view(np.int16), np.int16).view(TDT[dtype])
        g["normal_rough"], g["albedo_metal"] = vals["normal_rough"], vals["albedo_metal"]
    out = ctx.first_pass(cam, _dev(g["depth"]), nr, am, _dev(sc.env))
    torch.cuda.synchronize()
    assert out.dtype == TDT[dtype]
    return out.float().cpu().numpy().astype(np.float64), g


def _check_c1(gpu, ref, bound, dtype, label, min_plain=0.999):
    """Every pixel within (1e-4 + one ulp of the storage type) relative plus
    the oracle's bound; the well-conditioned pixels (bound below that
    tolerance) within the plain tolerance on at least 99.9 %."""
    tol = REL_TOL + ULP[dtype]
    err = np.abs(gpu - ref)
    allowed = tol * np.abs(ref) + bound + 1e-30
    rel = rel_err(gpu[..., :3], ref[..., :3]).max(-1)
    brel = (bound[..., :3] / np.maximum(np.abs(ref[..., :3]), 1e-6)).max(-1)
    well = brel <= tol
    frac = float((rel <= tol).mean())
    frac_well = float((rel[well] <= tol).mean()) if well.any() else 1.0
    ex = float((err - allowed).max())
    print(f"[{label}] rel p50 {np.quantile(rel, 0.5):.3g} p99 {np.quantile(rel, 0.99):.3g} "
          f"max {rel.max():.3g} within {frac:.6f} (well-conditioned {frac_well:.6f} of "
          f"{int(well.sum())}) excess {ex:.3g}", flush=True)
    assert ex <= 0.0
    assert frac_well >= min_plain
    assert np.all(gpu[..., 3] == 0.0)


@pytest.mark.parametrize("dtype,w,h", [("f32", 203, 117), ("f16", 160, 90), ("bf16", 160, 90),
                                       ("f32", 64, 47)])
def test_first_pass_matches_oracle(ctx, lut128, dtype, w, h):
    sc = scenes.make_scene("c2", seed=13, width=w, height=h)
    cam = f32_camera(sc.camera)
    gpu, g = _gpu_first_pass(ctx, sc, cam, dtype)
    ref = ofp.first_pass(cam, g, sc.env, lut128)
    bound = ofp.first_pass_bound(cam, g, sc.env, lut128, eps=DIR_EPS)
    _check_c1(gpu, ref, bound, dtype, f"c1 {dtype} {w}x{h}")
    assert np.all(gpu[~np.isfinite(g["depth"])] == 0.0)


def test_first_pass_backfacing_and_unnormalised_normals(ctx, lut128):
    """Stored normals of any length; back-facing pixels get no specular term."""
    sc = scenes.make_scene("c2", seed=17, width=96, height=64)
    rng = np.random.default_rng(4)
    nr = sc.normal_rough.copy()
    nr[..., :3] *= rng.uniform(0.2, 3.0, nr.shape[:2])[..., None]
    flip = rng.random(nr.shape[:2]) < 0.2
    nr[flip, :3] *= -1.0
    sc.normal_rough = nr.astype(np.float32)
    cam = f32_camera(sc.camera)
    gpu, g = _gpu_first_pass(ctx, sc, cam, "f32")
    ref = ofp.first_pass(cam, g, sc.env, lut128)
    bound = ofp.first_pass_bound(cam, g, sc.env, lut128, eps=DIR_EPS)
    _check_c1(gpu, ref, bound, "f32", "c1 backfacing")


def test_first_pass_all_background_and_empty(ctx):
    from paper_2504_01358_amd import ssr
    sc = scenes.make_scene("c2", seed=3, width=40, height=30)
    sc.depth = np.full_like(sc.depth, np.inf)
    gpu, _ = _gpu_first_pass(ctx, sc, f32_camera(sc.camera), "f32")
    assert np.all(gpu == 0.0)
    cam = dict(f32_camera(sc.camera), width=0, height=0)
    z = _dev(np.zeros((0, 0), np.float32))
    e = _dev(np.zeros((0, 0, 4), np.float32))
    ctx.first_pass(cam, z, e, e, _dev(sc.env))
    with pytest.raises(ssr.SSRError):      # an env that is not 2:1 with a power-of-two height
        ctx.first_pass(f32_camera(sc.camera), _dev(sc.depth), _dev(sc.normal_rough),
                       _dev(sc.albedo_metal), _dev(sc.env[:, :-2]))


def test_first_pass_full_size_sampled(ctx, lut128):
    """1920 x 1080, the shading benchmark's frame: every pixel within 1e-4 for
    99 %, and 20000 sampled pixels against the per-pixel bound."""
    sc = scenes.make_scene("c2")
    cam = f32_camera(sc.camera)
    gpu, g = _gpu_first_pass(ctx, sc, cam, "f16")
    H, W = g["depth"].shape
    pix = np.random.default_rng(11).choice(W * H, 20000, replace=False)
    ref = ofp.first_pass(cam, g, sc.env, lut128, pix=pix)
    bound = ofp.first_pass_bound(cam, g, sc.env, lut128, eps=DIR_EPS, pix=pix)
    _check_c1(gpu.reshape(-1, 4)[pix], ref, bound, "f16", "c1 1080p sampled")
    full = ofp.first_pass(cam, g, sc.env, lut128)
    rel = rel_err(gpu[..., :3], full[..., :3]).max(-1)
    assert (rel <= REL_TOL + ULP["f16"]).mean() >= 0.99


def test_depth_normals_full_size():
    sc = scenes.make_scene("c2")
    cam = f32_camera(sc.camera)
    depth = np.asarray(sc.depth, np.float32)
    _check_normals(_gpu_normals(cam, depth, "f16"), cam, depth, "f16", "normals 1080p")


# ---------------------------------------------------------------- the chain --

def test_depth_to_image_chain(ctx, lut128):
    """depth -> depth normals -> first pass -> shading, each side computing its
    own intermediates: the GPU chain against the oracle chain.  The world is
    turned against the environment so that the floor's normal, which the
    finite differences give only to rounding, is not at the pole of the
    equirect map (where the lookup is discontinuous and the two precisions
    would pick different azimuths)."""
    from paper_2504_01358_amd import ssr
    sc = scenes.make_scene("c2", seed=23, width=160, height=90)
    a, b = np.radians(20.0), np.radians(15.0)
    rx = np.array([[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]])
    rz = np.array([[np.cos(b), -np.sin(b), 0], [np.sin(b), np.cos(b), 0], [0, 0, 1]])
    turn = rz @ rx
    cam = dict(sc.camera, rot=np.asarray(sc.camera["rot"], np.float64).reshape(3, 3) @ turn.T,
               pos=turn @ np.asarray(sc.camera["pos"], np.float64))
    cam = f32_camera(cam)
    depth = np.asarray(sc.depth, np.float32)
    params = dict(sc.params, spp=4, seed=77)
    # GPU
    dev = torch.device("cuda", 0)
    nr = _dev(sc.normal_rough)                  # channel 3: the roughness
    ssr.depth_normals(cam, _dev(depth), nr)
    am = _dev(sc.albedo_metal)
    env = _dev(sc.env)
    c1 = ctx.first_pass(cam, _dev(depth), nr, am, env)
    hits = torch.empty((90, 160, 4), dtype=torch.int32, device=dev)
    out = ctx.shade(cam, _dev(depth), nr, am, c1, env, params, hits=hits)
    torch.cuda.synchronize()
    # oracle
    n64 = ofp.depth_normals(cam, depth)
    g = dict(depth=depth, normal_rough=np.concatenate([n64, sc.normal_rough[..., 3:4]], -1),
             albedo_metal=np.asarray(sc.albedo_metal, np.float64))
    g["radiance"] = ofp.first_pass(cam, g, sc.env, lut128)
    ref = oracle_frame(cam, g, sc.env, params)
    gout = out.cpu().numpy().astype(np.float64)
    st = compare(gout, hits.cpu().numpy().astype(np.int64), ref["out"], ref["hits"], "chain")
    assert st["hit_agreement"] >= 0.999
    fg = np.isfinite(depth)
    l1 = np.abs(gout - ref["out"])[fg].sum() / np.abs(ref["out"])[fg].sum()
    print(f"[chain] relative L1 {l1:.3g}", flush=True)
    assert l1 <= 1e-4
    assert st["frac_within_1e4"] >= 0.99
