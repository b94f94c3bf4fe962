"""Analytic scenes ray-cast into G-buffers, plus lognormal HDR environment maps.

Conventions (the ones the shading library documents for its inputs):

* World space is right-handed with +y up.  The camera has position ``pos`` and
  three rows ``rot = (right, up, forward)``; a world point x has view
  coordinates X = (x-pos).right, Y = (x-pos).up, Z = (x-pos).forward, and Z is
  the linear depth stored in the depth buffer.
* Pixel (i, j) covers [i, i+1) x [j, j+1) in screen coordinates, row 0 on top.
  A view point projects to px = cx + fx*X/Z, py = cy - fy*Y/Z.
* Background pixels have depth +inf and all-zero G-buffer channels.
* The environment map is equirectangular, ``[He][We][3]`` with We = 2*He.

Everything is drawn from ``numpy.random.default_rng`` with a fixed seed per
configuration and computed in float64; the buffers handed to either side are
then rounded once to float32 (and, for the precision variants, to float16 or
bfloat16 with round-to-nearest-even).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

# Workload definitions.  Sizes, counts and distributions follow the synthetic
# configurations of the build's measurement plan: a 128x128 minimum slice,
# the 1080p/16 spp headline scene and its reduced-precision variants, the
# 800x800 differentiation scene, and the serving mix.
CONFIGS = {
    "c1": dict(
        width=128, height=128, cam_pos=(0.0, 1.5, 5.0), cam_target=(0.0, 0.0, 0.0),
        fov_y=60.0, z_near=0.01, n_spheres=4, sphere_r=(0.3, 1.0), n_boxes=0,
        box_size=(0.2, 1.5), region=2.0, env=(32, 64, 1.0), spp=1, march="linear",
        max_steps=32, step_len=0.125, max_dist=4.0, thickness=0.05, seed=1, frame=0),
    "c2": dict(
        width=1920, height=1080, cam_pos=(0.0, 1.5, 5.0), cam_target=(0.0, 0.0, 0.0),
        fov_y=60.0, z_near=0.01, n_spheres=40, sphere_r=(0.3, 1.0), n_boxes=60,
        box_size=(0.2, 1.5), region=2.0, env=(256, 512, 2.0), spp=16, march="hiz",
        max_steps=64, step_len=0.125, max_dist=100.0, thickness=0.05, seed=2, frame=0),
    "c4": dict(
        width=800, height=800, cam_pos=(0.0, 1.5, 5.0), cam_target=(0.0, 0.0, 0.0),
        fov_y=60.0, z_near=0.01, n_spheres=20, sphere_r=(0.3, 1.0), n_boxes=0,
        box_size=(0.2, 1.5), region=2.0, env=(128, 256, 2.0), spp=8, march="hiz",
        max_steps=64, step_len=0.125, max_dist=100.0, thickness=0.05, seed=4, frame=0),
}

MARCH_CODES = {"linear": 0, "hiz": 1}

# The serving mix: 8 resident scenes of 100-400 objects (spheres and boxes
# in equal expectation), each rasterised at four resolutions with the same
# objects and environment, FP16 G-buffers; 512 requests with exponential
# inter-arrival times at 200 requests/s, resolution, scene and spp uniform.
SERVE = dict(
    n_scenes=8, objects=(100, 400), seed=50,
    resolutions=((640, 360), (1280, 720), (1920, 1080), (3840, 2160)),
    spp=(4, 16, 64), n_requests=512, rate=200.0, dtype="f16")


def serving_scene(k, width, height) -> Scene:
    """Scene k of the serving mix at one resolution."""
    rng = np.random.default_rng([SERVE["seed"], k])
    n = int(rng.integers(SERVE["objects"][0], SERVE["objects"][1] + 1))
    n_spheres = int(rng.binomial(n, 0.5))
    cfg = dict(CONFIGS["c2"], width=width, height=height, n_spheres=n_spheres,
               n_boxes=n - n_spheres)
    return make_scene(cfg, seed=SERVE["seed"] * 1000 + k)


def serving_requests():
    """(arrival time s, scene index, resolution index, spp) of each request."""
    rng = np.random.default_rng([SERVE["seed"], 10 ** 6])
    n = SERVE["n_requests"]
    t = np.cumsum(rng.exponential(1.0 / SERVE["rate"], n))
    sc = rng.integers(0, SERVE["n_scenes"], n)
    res = rng.integers(0, len(SERVE["resolutions"]), n)
    spp = rng.choice(SERVE["spp"], n)
    return [(float(a), int(b), int(c), int(d)) for a, b, c, d in zip(t, sc, res, spp)]


@dataclasses.dataclass
class Scene:
    """One frame's inputs.  All arrays are C-contiguous float32."""

    camera: dict
    depth: np.ndarray         # [H][W] view-space linear depth, +inf = background
    normal_rough: np.ndarray  # [H][W][4] (n.x, n.y, n.z, roughness), world space
    albedo_metal: np.ndarray  # [H][W][4] (a.r, a.g, a.b, metallic)
    radiance: np.ndarray      # [H][W][4] (c1.r, c1.g, c1.b, 0): first-pass radiance
    env: np.ndarray           # [He][We][3] equirect HDR environment
    params: dict              # shading parameters (spp, march, ...)

    @property
    def width(self) -> int:
        return int(self.camera["width"])

    @property
    def height(self) -> int:
        return int(self.camera["height"])


def _normalize(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def look_at_camera(width, height, pos, target, fov_y_deg, z_near):
    """Pinhole camera looking from ``pos`` at ``target`` with +y up.

    Every value is rounded to float32 once, and the rasteriser below uses the
    rounded values, so the G-buffer agrees with the camera handed to the
    shader.
    """
    pos = np.asarray(pos, np.float64)
    f = _normalize(np.asarray(target, np.float64) - pos)
    r = _normalize(np.cross(f, np.array([0.0, 1.0, 0.0])))
    u = np.cross(r, f)
    fy = (height / 2.0) / math.tan(math.radians(fov_y_deg) / 2.0)
    f32 = np.float32
    return dict(
        width=int(width), height=int(height),
        pos=pos.astype(f32), rot=np.stack([r, u, f]).astype(f32),
        fx=f32(fy), fy=f32(fy), cx=f32(width / 2.0), cy=f32(height / 2.0),
        z_near=f32(z_near))


def make_env(height, width, sigma, rng):
    """Equirect HDR map with i.i.d. lognormal(0, sigma) texels per channel."""
    return np.exp(rng.normal(0.0, sigma, size=(height, width, 3))).astype(np.float32)


def _draw_material(rng):
    albedo = rng.uniform(0.0, 1.0, 3)
    rough = rng.uniform(0.05, 1.0)
    metal = float(rng.integers(0, 2))
    return albedo, rough, metal


def _draw_objects(cfg, rng):
    """Plane y=0 plus spheres and boxes resting on it, centres in U[-r,r]^2."""
    objs = [dict(kind="plane", mat=_draw_material(rng))]
    reg = cfg["region"]
    for _ in range(cfg["n_spheres"]):
        rad = rng.uniform(*cfg["sphere_r"])
        cx, cz = rng.uniform(-reg, reg, 2)
        objs.append(dict(kind="sphere", centre=np.array([cx, rad, cz]), radius=rad,
                         mat=_draw_material(rng)))
    for _ in range(cfg["n_boxes"]):
        size = rng.uniform(*cfg["box_size"], 3)
        cx, cz = rng.uniform(-reg, reg, 2)
        lo = np.array([cx - size[0] / 2, 0.0, cz - size[2] / 2])
        hi = np.array([cx + size[0] / 2, size[1], cz + size[2] / 2])
        objs.append(dict(kind="box", lo=lo, hi=hi, mat=_draw_material(rng)))
    return objs


def _intersect(obj, org, dirs):
    """Nearest positive ray parameter and the outward normal (inf where missed)."""
    n = dirs.shape[0]
    t = np.full(n, np.inf)
    nrm = np.zeros((n, 3))
    with np.errstate(divide="ignore", invalid="ignore"):
        if obj["kind"] == "plane":
            tt = -org[1] / dirs[:, 1]
            ok = (dirs[:, 1] < 0) & (tt > 0)
            t[ok] = tt[ok]
            nrm[ok] = (0.0, 1.0, 0.0)
        elif obj["kind"] == "sphere":
            oc = org - obj["centre"]
            a = np.einsum("ij,ij->i", dirs, dirs)
            b = dirs @ oc
            c = oc @ oc - obj["radius"] ** 2
            disc = b * b - a * c
            ok = disc >= 0
            tt = np.where(ok, (-b - np.sqrt(np.where(ok, disc, 0.0))) / a, np.inf)
            ok &= tt > 0
            t[ok] = tt[ok]
            nrm[ok] = (org + tt[ok, None] * dirs[ok] - obj["centre"]) / obj["radius"]
        else:
            t1 = (obj["lo"] - org) / dirs
            t2 = (obj["hi"] - org) / dirs
            tmin3 = np.minimum(t1, t2)
            tmax3 = np.maximum(t1, t2)
            tmin = tmin3.max(axis=1)
            tmax = tmax3.min(axis=1)
            ok = (tmax >= tmin) & (tmin > 0)
            t[ok] = tmin[ok]
            axis = tmin3.argmax(axis=1)
            rows = np.nonzero(ok)[0]
            nrm[rows, axis[rows]] = -np.sign(dirs[rows, axis[rows]])
    return t, nrm


def _env_nearest(env, d):
    """Input recipe for the first-pass radiance: the nearest env texel to d."""
    he, we, _ = env.shape
    u = 0.5 + np.arctan2(d[:, 0], -d[:, 2]) / (2.0 * math.pi)
    v = np.arccos(np.clip(d[:, 1], -1.0, 1.0)) / math.pi
    ix = np.floor(u * we).astype(np.int64) % we
    iy = np.clip(np.floor(v * he).astype(np.int64), 0, he - 1)
    return env[iy, ix].astype(np.float64)


def _screen_rect(obj, camera):
    """Flat indices of the pixels an object can cover (a conservative cull).

    The object's bounding sphere (centre C, radius R) spans view X in
    [X-R, X+R] and depth in [Z-R, Z+R]; X/Z over that box is extremal at its
    corners, which bounds the projected footprint.  The plane, and anything
    not wholly in front of the camera, keeps every pixel.
    """
    w, h = camera["width"], camera["height"]
    everything = np.arange(w * h)
    if obj["kind"] == "plane":
        return everything
    if obj["kind"] == "sphere":
        centre, rad = obj["centre"], obj["radius"]
    else:
        centre = 0.5 * (obj["lo"] + obj["hi"])
        rad = 0.5 * float(np.linalg.norm(obj["hi"] - obj["lo"]))
    rot = camera["rot"].astype(np.float64)
    v = rot @ (centre - camera["pos"].astype(np.float64))
    rad *= 1.0 + 1e-9
    if v[2] - rad <= 1e-6:
        return everything
    zs = (v[2] - rad, v[2] + rad)
    xs = [(v[0] + sx * rad) / z for sx in (-1, 1) for z in zs]
    ys = [(v[1] + sy * rad) / z for sy in (-1, 1) for z in zs]
    fx, fy = float(camera["fx"]), float(camera["fy"])
    cx, cy = float(camera["cx"]), float(camera["cy"])
    i0 = max(int(math.floor(cx + fx * min(xs))) - 1, 0)
    i1 = min(int(math.floor(cx + fx * max(xs))) + 2, w)
    j0 = max(int(math.floor(cy - fy * max(ys))) - 1, 0)
    j1 = min(int(math.floor(cy - fy * min(ys))) + 2, h)
    if i0 >= i1 or j0 >= j1:
        return np.zeros(0, np.int64)
    jj, ii = np.meshgrid(np.arange(j0, j1), np.arange(i0, i1), indexing="ij")
    return (jj * w + ii).reshape(-1)


def rasterize(camera, objs, env):
    """Ray-cast pixel centres against the objects into G-buffers (float64)."""
    w, h = camera["width"], camera["height"]
    pos = camera["pos"].astype(np.float64)
    rot = camera["rot"].astype(np.float64)
    fx, fy = float(camera["fx"]), float(camera["fy"])
    cx, cy = float(camera["cx"]), float(camera["cy"])
    jj, ii = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64),
                         indexing="ij")
    xs = ((ii + 0.5 - cx) / fx).reshape(-1)
    ys = (-(jj + 0.5 - cy) / fy).reshape(-1)
    dirs = xs[:, None] * rot[0] + ys[:, None] * rot[1] + rot[2]
    best_t = np.full(dirs.shape[0], np.inf)
    best_n = np.zeros((dirs.shape[0], 3))
    best_id = np.full(dirs.shape[0], -1)
    for k, obj in enumerate(objs):
        sel = _screen_rect(obj, camera)
        t, nrm = _intersect(obj, pos, dirs[sel])
        closer = t < best_t[sel]
        rows = sel[closer]
        best_t[rows] = t[closer]
        best_n[rows] = nrm[closer]
        best_id[rows] = k
    hit = best_id >= 0
    depth = np.full(dirs.shape[0], np.inf)
    depth[hit] = ((best_t[hit, None] * dirs[hit]) @ rot[2])
    # material of each pixel's object (row 0 of the tables: background, zeros)
    mat_a = np.zeros((len(objs) + 1, 3))
    mat_r = np.zeros(len(objs) + 1)
    mat_m = np.zeros(len(objs) + 1)
    for k, obj in enumerate(objs):
        mat_a[k + 1], mat_r[k + 1], mat_m[k + 1] = obj["mat"]
    albedo = mat_a[best_id + 1]
    rough = mat_r[best_id + 1]
    metal = mat_m[best_id + 1]
    nrm = np.zeros_like(best_n)
    nrm[hit] = _normalize(best_n[hit])
    rad = np.zeros((dirs.shape[0], 3))
    rad[hit] = albedo[hit] * _env_nearest(env, nrm[hit])
    f32 = np.float32
    z = np.zeros(dirs.shape[0])
    return (depth.reshape(h, w).astype(f32),
            np.stack([nrm[:, 0], nrm[:, 1], nrm[:, 2], rough], -1).reshape(h, w, 4).astype(f32),
            np.stack([albedo[:, 0], albedo[:, 1], albedo[:, 2], metal], -1).reshape(h, w, 4).astype(f32),
            np.stack([rad[:, 0], rad[:, 1], rad[:, 2], z], -1).reshape(h, w, 4).astype(f32))


def make_scene(cfg, seed=None, **overrides) -> Scene:
    """Build one frame's inputs from a configuration name or dict.

    ``overrides`` replace configuration entries (for instance a smaller
    ``width``/``height`` for a parity case that the oracle finishes quickly).
    """
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    cfg = dict(cfg)
    cfg.update(overrides)
    if seed is None:
        seed = cfg["seed"]
    rng = np.random.default_rng([seed, 0])
    env_rng = np.random.default_rng([seed, 1])
    he, we, sigma = cfg["env"]
    env = make_env(he, we, sigma, env_rng)
    camera = look_at_camera(cfg["width"], cfg["height"], cfg["cam_pos"], cfg["cam_target"],
                            cfg["fov_y"], cfg["z_near"])
    objs = _draw_objects(cfg, rng)
    depth, nr, am, rad = rasterize(camera, objs, env)
    params = dict(spp=int(cfg["spp"]), march=MARCH_CODES[cfg["march"]],
                  max_steps=int(cfg["max_steps"]), step_len=np.float32(cfg["step_len"]),
                  max_dist=np.float32(cfg["max_dist"]), thickness=np.float32(cfg["thickness"]),
                  seed=int(seed) & 0xFFFFFFFFFFFFFFFF, frame=int(cfg["frame"]), flags=0)
    return Scene(camera=camera, depth=depth, normal_rough=nr, albedo_metal=am, radiance=rad,
                 env=env, params=params)


def f16_round(x):
    """float32 -> IEEE binary16 bit patterns (round to nearest even)."""
    return np.ascontiguousarray(np.asarray(x, np.float32).astype(np.float16)).view(np.uint16)


def bf16_round(x):
    """float32 -> bfloat16 bit patterns (round to nearest even; inputs finite)."""
    b = np.ascontiguousarray(np.asarray(x, np.float32)).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return b.astype(np.uint16)


def _f16_to_f32(bits):
    return bits.view(np.float16).astype(np.float32)


def _bf16_to_f32(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32)


def quantise_gbuffer(scene: Scene, dtype: str):
    """Round the three packed G-buffers to ``dtype`` ('f16' or 'bf16').

    Returns ``(bits, values)``: ``bits`` maps buffer name to the uint16
    storage handed to the GPU, ``values`` to the same numbers widened back to
    float32 (the exact inputs the GPU reads), so the oracle can be fed the
    identical quantised G-buffer.  Depth stays float32.
    """
    enc, dec = {"f16": (f16_round, _f16_to_f32), "bf16": (bf16_round, _bf16_to_f32)}[dtype]
    bits, values = {}, {}
    for name in ("normal_rough", "albedo_metal", "radiance"):
        b = enc(getattr(scene, name))
        bits[name] = b
        values[name] = dec(b)
    return bits, values
