"""Pins of the FP64 oracle against things other than itself.

Each test ties one part of the oracle to a published value, a library
routine, a closed form, an invariant or brute force, chosen so that a
plausible slip (a dropped term, a wrong sign or index, a swapped operand)
fails at least one of them.  CPU only.
"""

import math
import os

import numpy as np
import pytest

from oracle import brdf, camera, env, march, philox, shade

from closed_form import floor_wall_scene, open_floor

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox ---

def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox4x32_known_answers():
    """Published Random123 known-answer vectors for Philox4x32-10."""
    for ctr, key, want in _kat():
        assert philox.philox([ctr], [key], bits=32).tolist() == [want]
        assert philox.philox4x32(np.array([ctr]), np.array(key)).tolist() == [want]


def test_philox_structure_matches_numpy_4x64():
    """The generic round/key schedule, instantiated at 64 bits, reproduces
    NumPy's independent Philox4x64-10 stream (counter incremented before use)."""
    ctr = np.array([11, 22, 33, 44], dtype=np.uint64)
    key = np.array([0x1234567890ABCDEF, 0xFEDCBA0987654321], dtype=np.uint64)
    g = np.random.Philox(counter=ctr, key=key)
    raw = g.random_raw(12).reshape(3, 4)
    mine = philox.philox([[12 + k, 22, 33, 44] for k in range(3)], [key.tolist()], bits=64)
    assert np.array_equal(raw, mine)


def test_philox_vectorised_equals_exact():
    rng = np.random.default_rng(5)
    c = rng.integers(0, 2 ** 32, (500, 4), dtype=np.uint64)
    k = rng.integers(0, 2 ** 32, (500, 2), dtype=np.uint64)
    assert np.array_equal(philox.philox(c, k), philox.philox4x32(c, k))


def test_uniforms_exact_grid_and_uniform():
    n = 200_000
    u1, u2 = philox.sample_uniforms(np.arange(n), 3, 0, 0x1234_5678_9ABC)
    for u in (u1, u2):
        assert u.min() >= 0.0 and u.max() < 1.0
        assert np.all(u * 2 ** 24 == np.floor(u * 2 ** 24))           # multiples of 2^-24
        assert np.all(u.astype(np.float32).astype(np.float64) == u)   # exact in f32
        counts = np.bincount((u * 64).astype(int), minlength=64)
        chi2 = ((counts - n / 64) ** 2 / (n / 64)).sum()
        assert chi2 < 120  # 63 dof: p ~ 1e-5
    assert abs(np.corrcoef(u1, u2)[0, 1]) < 0.01
    assert abs(np.corrcoef(u1[:-1], u1[1:])[0, 1]) < 0.01
    # a different sample index or frame gives a different stream
    v1, _ = philox.sample_uniforms(np.arange(1000), 4, 0, 0x1234_5678_9ABC)
    w1, _ = philox.sample_uniforms(np.arange(1000), 3, 1, 0x1234_5678_9ABC)
    assert not np.array_equal(u1[:1000], v1) and not np.array_equal(u1[:1000], w1)


# ------------------------------------------------------------ ONB / BRDF ---

def test_onb_orthonormal_right_handed():
    rng = np.random.default_rng(1)
    n = brdf.normalize(rng.normal(size=(2000, 3)))
    n = np.concatenate([n, [[0, 0, 1.0], [0, 0, -1.0], [1.0, 0, 0.0], [0.0, 1.0, 0.0],
                            [1.0, 0.0, -0.0], [0.6, 0.8, 0.0]]])
    t, b = brdf.onb(n)
    for u, v in ((t, b), (t, n), (b, n)):
        assert np.abs(brdf.dot(u, v)).max() < 1e-12
    for u in (t, b):
        assert np.abs(np.linalg.norm(u, axis=1) - 1).max() < 1e-12
    assert np.abs(np.cross(t, b) - n).max() < 1e-12
    # sign(+0) = +1 and sign(-0) = -1 both give a valid frame
    t0, b0 = brdf.onb(np.array([[0.6, 0.8, 0.0]]))
    assert np.allclose(t0, [[1 - 0.36, -0.48, -0.6]])


def _random_setup(rng, m, alpha=None):
    cos_no = rng.uniform(0.05, 1.0, m)
    wo = np.stack([np.sqrt(1 - cos_no ** 2), np.zeros(m), cos_no], axis=1)
    a = rng.uniform(0.05, 1.0, m) if alpha is None else np.full(m, alpha)
    return wo, a


def test_vndf_mirror_is_exact():
    """rho = 0: the visible-normal sample is the normal itself, for any u."""
    rng = np.random.default_rng(2)
    wo, _ = _random_setup(rng, 1000)
    h = brdf.sample_vndf(wo, np.zeros(1000), rng.uniform(0, 1, 1000), rng.uniform(0, 1 - 2 ** -24, 1000))
    assert np.array_equal(h, np.tile([0.0, 0.0, 1.0], (1000, 1)))


def test_weights_bounded_and_long_equals_short():
    rng = np.random.default_rng(3)
    m = 1_000_000
    wo, a = _random_setup(rng, m)
    u1, u2 = rng.uniform(0, 1, m), rng.uniform(0, 1, m)
    h = brdf.sample_vndf(wo, a, u1, u2)
    assert np.all(h[:, 2] > 0)
    cos_oh = brdf.dot(wo, h)
    assert np.all(cos_oh > 0)                      # visible normals only
    l = 2 * cos_oh[:, None] * h - wo
    cos_nl = l[:, 2]
    ok = cos_nl > 0
    f0 = rng.uniform(0, 1, (m, 3))
    ws = brdf.weight_short(f0[ok], cos_oh[ok], cos_nl[ok], a[ok])
    assert ws.max() <= 1.0 + 1e-15 and ws.min() >= 0.0
    sub = np.nonzero(ok)[0][:200_000]
    wl = brdf.weight_long(f0[sub], wo[sub, 2], cos_nl[sub], cos_oh[sub], h[sub, 2], a[sub])
    wsub = brdf.weight_short(f0[sub], cos_oh[sub], cos_nl[sub], a[sub])
    assert np.abs(wl - wsub).max() <= 1e-12


@pytest.mark.parametrize("alpha,cos_no", [(0.3, 0.9), (0.6, 0.5), (1.0, 0.2), (0.45, 0.15)])
@pytest.mark.parametrize("f0", [1.0, 0.0, 0.04])
def test_vndf_mean_weight_matches_quadrature(alpha, cos_no, f0):
    """E[w] under the sampler equals the integral of f_s cos over the
    hemisphere by quadrature, which uses only the closed-form D, F and G.
    F0 = 1 weighs by G1 alone, F0 = 0 by the Fresnel tail, so a wrong
    sampling density fails one of them."""
    rng = np.random.default_rng(int(alpha * 1000 + cos_no * 100 + f0 * 7))
    m = 400_000
    wo = np.tile([math.sqrt(1 - cos_no ** 2), 0.0, cos_no], (m, 1))
    h = brdf.sample_vndf(wo, np.full(m, alpha), rng.uniform(0, 1, m), rng.uniform(0, 1, m))
    cos_oh = brdf.dot(wo, h)
    l = 2 * cos_oh[:, None] * h - wo
    w = np.zeros(m)
    ok = l[:, 2] > 0
    w[ok] = brdf.weight_short(np.full((ok.sum(), 1), f0), cos_oh[ok], l[ok, 2], np.full(ok.sum(), alpha))[:, 0]
    mc, se = w.mean(), w.std() / math.sqrt(m)
    quad = brdf.specular_albedo_quadrature(np.array([f0]), cos_no, alpha, 1200, 600)[0]
    assert abs(mc - quad) < 4 * se + 2e-4 * max(quad, 1e-3), (mc, quad, se)


def test_vndf_below_surface_fraction_matches_pdf():
    """P(n.l > 0) from the sampler equals the integral of the closed-form
    reflected visible-normal density over the upper hemisphere."""
    alpha, cos_no = 0.8, 0.3
    rng = np.random.default_rng(11)
    m = 400_000
    wo = np.tile([math.sqrt(1 - cos_no ** 2), 0.0, cos_no], (m, 1))
    h = brdf.sample_vndf(wo, np.full(m, alpha), rng.uniform(0, 1, m), rng.uniform(0, 1, m))
    cos_oh = brdf.dot(wo, h)
    frac = ((2 * cos_oh[:, None] * h - wo)[:, 2] > 0).mean()
    nt, npd = 1200, 600
    mu = (np.arange(nt) + 0.5) / nt
    ph = (np.arange(npd) + 0.5) / npd * 2 * math.pi
    MU, PH = np.meshgrid(mu, ph, indexing="ij")
    s = np.sqrt(1 - MU ** 2)
    wi = np.stack([s * np.cos(PH), s * np.sin(PH), MU], -1)
    hh = brdf.normalize(wi + wo[0])
    pdf = brdf.vndf_pdf_l(cos_no, brdf.dot(hh, wo[0]), hh[..., 2], alpha)
    integral = pdf.sum() / nt * 2 * math.pi / npd
    assert abs(frac - integral) < 4 * math.sqrt(frac * (1 - frac) / m) + 1e-3


def test_microfacet_closed_forms():
    # D integrates to one over projected area: int D(h) (h.n) dh = 1
    for alpha in (0.2, 0.5, 1.0):
        mu = (np.arange(20000) + 0.5) / 20000
        assert abs((brdf.ndf(mu, alpha) * mu).sum() / 20000 * 2 * math.pi - 1) < 1e-3
    # alpha = 1: D = 1/pi, G1(z) = 2z / (1 + z); alpha = 0: G1 = 1
    assert np.allclose(brdf.ndf(np.linspace(0, 1, 9), 1.0), 1 / math.pi)
    z = np.linspace(0.01, 1, 9)
    assert np.allclose(brdf.smith_g1(z, 1.0), 2 * z / (1 + z))
    assert np.allclose(brdf.smith_g1(z, 0.0), 1.0)
    # Schlick: F(1) = F0, F(0) = 1, textbook (1 - c)^5 form
    f0 = np.array([[0.04, 0.5, 1.0]])
    assert np.allclose(brdf.schlick(f0, np.array([1.0])), f0)
    assert np.allclose(brdf.schlick(f0, np.array([0.0])), 1.0)
    assert np.allclose(brdf.schlick(np.array([[0.0]]), np.array([0.5])), 0.5 ** 5)


# ------------------------------------------------------------------- env ---

def test_env_uv_closed_forms():
    d = np.array([[0, 0, -1.0], [1.0, 0, 0], [0, 0, 1.0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0]])
    u, v = env.dir_to_uv(d)
    assert np.allclose(u[:4], [0.5, 0.75, 1.0, 0.25]) and np.allclose(v[:4], 0.5)
    assert v[4] == 0.0 and v[5] == 1.0


def test_env_bilinear_texel_centres_and_uniform():
    rng = np.random.default_rng(4)
    he, we = 8, 16
    img = rng.uniform(0.5, 2, (he, we, 3))
    for y in range(he):
        for x in range(we):
            u = (x + 0.5) / we
            v = (y + 0.5) / he
            phi = (u - 0.5) * 2 * math.pi
            th = v * math.pi
            d = np.array([[math.sin(th) * math.sin(phi), math.cos(th), -math.sin(th) * math.cos(phi)]])
            assert np.allclose(env.bilinear(img, d)[0], img[y, x], rtol=1e-12)
    # wrap: halfway between the last and first column
    th = 0.5 * math.pi * (2 * 3 + 1) / he * 2 / 2
    v = (3 + 0.5) / he
    th = v * math.pi
    d = np.array([[math.sin(th) * math.sin(-math.pi), math.cos(th), -math.sin(th) * math.cos(-math.pi)]])
    assert np.allclose(env.bilinear(img, d)[0], 0.5 * (img[3, 0] + img[3, we - 1]), rtol=1e-12)
    # constant map: every filter returns the constant
    const = np.full((he, we, 3), 3.25)
    mips = env.build_mips(const)
    dd = brdf.normalize(rng.normal(size=(1000, 3)))
    assert np.abs(env.bilinear(const, dd) - 3.25).max() < 1e-14
    assert np.abs(env.trilinear(mips, dd, rng.uniform(0, 3, 1000)) - 3.25).max() < 1e-14


def test_env_bilinear_equals_scipy_linear_interpolation():
    """Between texel centres: the lookup is linear interpolation at texel
    coordinates (u W - 1/2, v H - 1/2), wrapping in u and clamping in v,
    which SciPy's order-1 map_coordinates gives on the map padded by one
    wrapped column each side and one repeated row above and below.  Random
    directions, the poles' rows and the seam included."""
    from scipy import ndimage
    rng = np.random.default_rng(41)
    he, we = 16, 32
    img = np.exp(rng.normal(0, 1, (he, we, 3)))
    d = brdf.normalize(rng.normal(size=(4000, 3)))
    # directions near the poles and on both sides of the seam (u near 0 and 1)
    near_pole = brdf.normalize(np.stack([rng.normal(size=200) * 0.05, np.sign(rng.normal(size=200)),
                                         rng.normal(size=200) * 0.05], axis=1))
    seam = brdf.normalize(np.stack([rng.normal(size=200) * 1e-3, rng.normal(size=200),
                                    np.full(200, 1.0)], axis=1))
    d = np.concatenate([d, near_pole, seam])
    u, v = env.dir_to_uv(d)
    padded = np.pad(np.pad(img, ((0, 0), (1, 1), (0, 0)), mode="wrap"),
                    ((1, 1), (0, 0), (0, 0)), mode="edge")
    coords = [v * he - 0.5 + 1.0, u * we - 0.5 + 1.0]
    want = np.stack([ndimage.map_coordinates(padded[..., c], coords, order=1, mode="nearest")
                     for c in range(3)], axis=1)
    got = env.bilinear(img, d)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_env_mips_are_block_means():
    rng = np.random.default_rng(6)
    img = np.exp(rng.normal(0, 2, (32, 64, 3)))
    mips = env.build_mips(img)
    assert len(mips) == 6 and mips[-1].shape == (1, 2, 3)
    for k, m in enumerate(mips):
        b = 2 ** k
        direct = np.array([[img[y * b:(y + 1) * b, x * b:(x + 1) * b].reshape(-1, 3).mean(0)
                            for x in range(64 // b)] for y in range(32 // b)])
        assert np.allclose(m, direct, rtol=1e-13)
    assert env.roughness_level(mips, 1.0) == 5.0 and env.roughness_level(mips, 0.0) == 0.0


def _texel_centre_dir(x, y, we, he):
    """Unit direction to the centre of texel (x, y) of a we x he equirect
    level (u = (x + 1/2)/we, v = (y + 1/2)/he; u = 1/2 + atan2(d.x, -d.z)/(2 pi),
    v = theta/pi)."""
    phi = ((x + 0.5) / we - 0.5) * 2 * math.pi
    th = (y + 0.5) / he * math.pi
    return np.array([math.sin(th) * math.sin(phi), math.cos(th), -math.sin(th) * math.cos(phi)])


def test_roughness_level_interior_values():
    """lambda = log2(1 + rho) lambda_max (Sec. 3.2, SampleEnvMap) at interior
    roughness values whose logarithm is known by hand: rho = sqrt(2) - 1 gives
    lambda_max / 2, rho = 2^(1/4) - 1 a quarter, rho = 2^(3/4) - 1 three
    quarters.  A linear reading (rho lambda_max) gives 0.414, 0.189 and 0.682
    of lambda_max and fails."""
    mips = env.build_mips(np.ones((64, 128, 3)))       # lambda_max = 6
    assert env.lambda_max(mips) == 6
    for rho, frac in ((math.sqrt(2.0) - 1.0, 0.5), (2 ** 0.25 - 1.0, 0.25), (2 ** 0.75 - 1.0, 0.75)):
        assert abs(env.roughness_level(mips, rho) - 6 * frac) < 1e-12


def test_trilinear_blends_adjacent_levels_by_the_fraction():
    """A level-0 checkerboard of 1 and 3 (8 x 4) has the constant 2 on every
    level above it.  At a level-0 texel centre holding 1, E_lambda at
    lambda = 1/4 is (1 - 1/4) * 1 + 1/4 * 2 = 1.25 (a swapped blend gives
    1.75); at lambda = 1/2 it is 1.5 for a texel holding 1 and 2.5 for one
    holding 3; at lambda >= 1 it is 2."""
    he, we = 4, 8
    yy, xx = np.meshgrid(np.arange(he), np.arange(we), indexing="ij")
    img = np.where((xx + yy) % 2 == 0, 1.0, 3.0)[..., None] * np.ones(3)
    mips = env.build_mips(img)
    assert np.all(mips[1] == 2.0) and np.all(mips[2] == 2.0)
    d1 = _texel_centre_dir(2, 0, we, he)[None]            # (2 + 0) even: holds 1
    d3 = _texel_centre_dir(3, 2, we, he)[None]            # (3 + 2) odd: holds 3
    assert np.allclose(env.bilinear(img, d1), 1.0, rtol=0, atol=1e-12)
    assert np.allclose(env.trilinear(mips, d1, np.array([0.25])), 1.25, rtol=0, atol=1e-12)
    assert np.allclose(env.trilinear(mips, d1, np.array([0.5])), 1.5, rtol=0, atol=1e-12)
    assert np.allclose(env.trilinear(mips, d3, np.array([0.5])), 2.5, rtol=0, atol=1e-12)
    assert np.allclose(env.trilinear(mips, d3, np.array([1.7])), 2.0, rtol=0, atol=1e-12)


def test_direct_term_at_interior_roughness_closed_form():
    """The whole direct term c_d = (1 - m) a E_lambda(n) through the pixel
    estimator: normal aimed at a level-0 texel centre of the checkerboard
    above, rho = 2^(1/8) - 1 so lambda = 2 * 1/8 = 1/4, metallic 0.25,
    albedo (0.2, 0.4, 0.8), specular off: c_d = 0.75 a (0.75 * 1 + 0.25 * 2)."""
    he, we = 4, 8
    yy, xx = np.meshgrid(np.arange(he), np.arange(we), indexing="ij")
    img = np.where((xx + yy) % 2 == 0, 1.0, 3.0)[..., None] * np.ones(3)
    cam = dict(width=2, height=1, pos=np.zeros(3), rot=np.eye(3), fx=2.0, fy=2.0, cx=1.0,
               cy=0.5, z_near=0.01)
    n = _texel_centre_dir(2, 0, we, he)
    g = dict(depth=np.full((1, 2), 2.0),
             normal_rough=np.tile(np.r_[n, 2 ** 0.125 - 1.0], (1, 2, 1)),
             albedo_metal=np.tile(np.array([0.2, 0.4, 0.8, 0.25]), (1, 2, 1)),
             radiance=np.zeros((1, 2, 4)))
    p = dict(spp=1, march=1, max_steps=64, step_len=0.1, max_dist=10.0, thickness=0.05, seed=0,
             frame=0, flags=2)
    out = shade.shade_frame(cam, g, img, p)["out"]
    want = 0.75 * np.array([0.2, 0.4, 0.8]) * (0.75 * 1.0 + 0.25 * 2.0)
    assert np.allclose(out, want, rtol=0, atol=1e-12)


# --------------------------------------------------------------- pyramid ---

@pytest.mark.parametrize("h,w", [(1, 1), (1, 7), (5, 3), (9, 13), (16, 16), (33, 17)])
def test_hiz_pyramids_are_block_min_max(h, w):
    rng = np.random.default_rng(h * 100 + w)
    d = rng.uniform(1, 10, (h, w))
    d[rng.uniform(size=(h, w)) < 0.2] = np.inf
    lv = march.hiz_pyramid(d)
    lx = march.hiz_max_pyramid(d)
    assert lv[-1].shape == (1, 1) and len(lx) == len(lv)
    for L, (img, imx) in enumerate(zip(lv, lx)):
        b = 2 ** L
        assert img.shape == (-(-h // b), -(-w // b)) == imx.shape
        for y in range(img.shape[0]):
            for x in range(img.shape[1]):
                assert img[y, x] == d[y * b:(y + 1) * b, x * b:(x + 1) * b].min()
                assert imx[y, x] == d[y * b:(y + 1) * b, x * b:(x + 1) * b].max()


# ----------------------------------------------------------------- march ---

def _tiny_camera(w, h):
    return dict(width=w, height=h, pos=np.zeros(3), rot=np.eye(3), fx=w * 0.9, fy=w * 0.9,
                cx=w / 2, cy=h / 2, z_near=0.01)


def _random_rays(rng, cam, depth, m):
    c = camera.unpack(cam)
    h, w = depth.shape
    fin = np.argwhere(np.isfinite(depth))
    pick = fin[rng.integers(0, fin.shape[0], m)]
    org = np.stack([pick[:, 1], pick[:, 0]], 1)
    V0 = camera.pixel_view_point(c, org[:, 0].astype(float), org[:, 1].astype(float),
                                 depth[pick[:, 0], pick[:, 1]])
    Dv = brdf.normalize(rng.normal(size=(m, 3)))
    return org, V0, Dv


@pytest.mark.parametrize("h,w", [(4, 4), (9, 13), (16, 16), (21, 7), (32, 32)])
def test_hiz_march_equals_brute_force(h, w):
    """Cap lifted, the pyramid traversal finds exactly the first hit of the
    pixel-by-pixel scan; with the cap on, rays that need at most the cap
    agree too and the rest report -4."""
    rng = np.random.default_rng(h * 31 + w)
    cam = _tiny_camera(w, h)
    ok_rays = 0
    for trial in range(6):
        depth = rng.uniform(1.0, 3.0, (h, w))
        if trial % 2:
            depth[rng.uniform(size=(h, w)) < 0.3] = np.inf
        if trial == 4:  # a smooth slanted surface: exercises the in-front-first rule
            jj, ii = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
            depth = 1.5 + 0.08 * jj + 0.03 * ii
        org, V0, Dv = _random_rays(rng, cam, depth, 150)
        pyr = (march.hiz_pyramid(depth), march.hiz_max_pyramid(depth))
        for thick in (0.05, 0.5):
            want = march.brute_force_first_hit(cam, depth, org, V0, Dv, 6.0, thick)
            # the bounding-box restriction drops only pixels the segment cannot cross
            assert np.array_equal(
                march.brute_force_first_hit(cam, depth, org, V0, Dv, 6.0, thick, bbox=True), want)
            got, it = march.march_hiz(cam, pyr, org, V0, Dv, 10 ** 6, 6.0, thick)
            assert np.array_equal(got, want)
            capped, itc = march.march_hiz(cam, pyr, org, V0, Dv, 12, 6.0, thick)
            within = it <= 12
            assert np.array_equal(capped[within], want[within])
            assert np.all(capped[~within] == march.HIT_CAP)
            assert np.all(itc <= 12)
            ok_rays += within.sum()
    assert ok_rays > 0


def test_linear_march_wall_closed_form():
    """A ray from depth 2 toward a fronto-parallel wall at depth 5: it is in
    front at the first sample, then hits at sample k* = ceil(3/(step*dz))
    exactly when that sample lies inside the slab, in the pixel it projects to."""
    w = h = 64
    cam = _tiny_camera(w, h)
    c = camera.unpack(cam)
    depth = np.full((h, w), 5.0)
    rng = np.random.default_rng(8)
    n_checked = 0
    for _ in range(400):
        i, j = rng.integers(8, 56, 2)
        depth_o = 2.0
        V0 = camera.pixel_view_point(c, np.array([float(i)]), np.array([float(j)]), np.array([depth_o]))
        Dv = brdf.normalize(np.array([[rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), 1.0]]))
        step = 0.125
        thick = 0.05
        kstar = math.ceil(3.0 / (step * Dv[0, 2]))
        zk = depth_o + kstar * step * Dv[0, 2]
        p = V0[0] + kstar * step * Dv[0]
        px, py = c["cx"] + c["fx"] * p[0] / p[2], c["cy"] - c["fy"] * p[1] / p[2]
        if not (0 <= px < w and 0 <= py < h) or kstar > 32:
            continue
        # first sample must leave the origin pixel for the ray to be "in front"
        p1 = V0[0] + step * Dv[0]
        if (math.floor(c["cx"] + c["fx"] * p1[0] / p1[2]), math.floor(c["cy"] - c["fy"] * p1[1] / p1[2])) == (i, j):
            continue
        want = int(math.floor(py)) * w + int(math.floor(px)) if zk - 5.0 <= thick else march.HIT_CAP
        if want == march.HIT_CAP and kstar < 32:
            continue  # it would go on marching behind the wall until the cap; checked below
        got, it = march.march_linear(cam, depth, np.array([[i, j]]), V0, Dv, step, 32, 4.0, thick)
        assert got[0] == want and it[0] == kstar
        n_checked += 1
    assert n_checked > 50


# -------------------------------------------------- closed-form scenes ---

def test_mirror_floor_hits_wall_at_closed_form_pixel():
    cam, g, is_floor = floor_wall_scene()
    c = camera.unpack(cam)
    W, H = c["W"], c["H"]
    envmap = np.full((8, 16, 3), 0.25)
    params = dict(spp=1, march=1, max_steps=10 ** 6, step_len=0.125, max_dist=100.0,
                  thickness=0.05, seed=7, frame=0, flags=shade.NO_DIRECT)
    pix = np.nonzero(is_floor.reshape(-1))[0]
    r = shade.shade_pixels(cam, g, envmap, params, pix)
    checked = 0
    for k, q in enumerate(pix):
        i, j = q % W, q // W
        D = g["depth"][j, i]
        p = c["pos"] + camera.view_to_world_dir(c, camera.pixel_view_point(c, np.array(i, float), np.array(j, float), np.array(D)))
        wo = (c["pos"] - p) / np.linalg.norm(c["pos"] - p)
        l = np.array([-wo[0], wo[1], -wo[2]])          # mirror about +y
        t = (p[2] + 6.0) / (-l[2])
        x = p + t * l
        v = x - c["pos"]
        px = c["cx"] + c["fx"] * v[0] / (-v[2])
        py = c["cy"] - c["fy"] * v[1] / (-v[2])
        if not (0 <= px < W and 0 <= py < H):
            assert r["hits"][k, 0] == march.HIT_OFFSCREEN
            assert np.allclose(r["out"][k], 0.25)       # miss reads the env
            continue
        if min(px - math.floor(px), math.ceil(px) - px, py - math.floor(py), math.ceil(py) - py) < 1e-6:
            continue
        want = int(py) * W + int(px)
        assert r["hits"][k, 0] == want
        # F0 = 1 and G1 = 1 for a perfect mirror: the output is the hit's radiance
        assert np.allclose(r["out"][k], g["radiance"].reshape(-1, 4)[want, :3], rtol=1e-13)
        checked += 1
    assert checked > 300


def test_white_furnace():
    """Uniform environment L, specular off, dielectric: out = a * L exactly."""
    L = 1.75
    cam, g = open_floor(metal=0.0, rough=0.4)
    rng = np.random.default_rng(9)
    g["albedo_metal"][..., :3] = rng.uniform(0, 1, g["albedo_metal"][..., :3].shape)
    g["normal_rough"][..., 3] = rng.uniform(0, 1, g["normal_rough"][..., 3].shape)
    tilt = brdf.normalize(rng.normal(size=(32, 48, 3)) * 0.2 + [0, 1, 0])
    g["normal_rough"][..., :3] = tilt
    envmap = np.full((16, 32, 3), L)
    params = dict(spp=4, march=1, max_steps=64, step_len=0.125, max_dist=100.0,
                  thickness=0.05, seed=1, frame=0, flags=shade.NO_SPECULAR)
    r = shade.shade_frame(cam, g, envmap, params)
    assert np.abs(r["out"] - g["albedo_metal"][..., :3] * L).max() < 1e-14
    assert np.all(r["hits"] == shade.HIT_SKIPPED)


def test_mirror_furnace():
    """Perfect mirror (a = 1, m = 1, rho = 0) over an open floor under a
    uniform environment: every ray leaves the screen and out = L exactly."""
    L = 2.5
    cam, g = open_floor()
    envmap = np.full((16, 32, 3), L)
    params = dict(spp=2, march=1, max_steps=64, step_len=0.125, max_dist=100.0,
                  thickness=0.05, seed=3, frame=0, flags=0)
    r = shade.shade_frame(cam, g, envmap, params)
    assert np.all(r["hits"] == march.HIT_OFFSCREEN)
    assert np.abs(r["out"] - L).max() < 1e-14


def test_rough_furnace_equals_directional_albedo():
    """Rough metal under a uniform environment with nothing to hit: the
    pixel mean over many samples converges to L * int f_s cos (quadrature)."""
    L = 1.0
    alpha = 0.5
    cam, g = open_floor(w=8, h=8, rough=alpha, metal=1.0, albedo=0.8)
    envmap = np.full((16, 32, 3), L)
    params = dict(spp=4096, march=1, max_steps=64, step_len=0.125, max_dist=100.0,
                  thickness=0.05, seed=12, frame=0, flags=0)
    W = 8
    q = 3 * W + 5
    r = shade.shade_pixels(cam, g, envmap, params, np.array([q]))
    c = camera.unpack(cam)
    p = c["pos"] + camera.view_to_world_dir(c, camera.pixel_view_point(c, np.array(5.0), np.array(3.0), np.array(3.0)))
    cos_no = (c["pos"] - p)[1] / np.linalg.norm(c["pos"] - p)
    quad = brdf.specular_albedo_quadrature(np.array([0.8]), cos_no, alpha, 1200, 600)[0]
    assert np.all(r["hits"] < 0)
    assert abs(r["out"][0, 0] - quad) < 0.02 * quad


def test_background_reads_environment():
    cam, g = open_floor(w=8, h=8)
    g["depth"][:] = np.inf
    rng = np.random.default_rng(2)
    envmap = rng.uniform(1, 2, (8, 16, 3))
    params = dict(spp=1, march=0, max_steps=32, step_len=0.125, max_dist=4.0,
                  thickness=0.05, seed=0, frame=0, flags=0)
    r = shade.shade_frame(cam, g, envmap, params)
    c = camera.unpack(cam)
    jj, ii = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
    d = camera.view_ray_dir(c, ii.reshape(-1), jj.reshape(-1))
    assert np.allclose(r["out"].reshape(-1, 3), env.bilinear(envmap, d), rtol=1e-14)
    assert np.all(r["hits"] == shade.HIT_BACKGROUND)


# ------------------------------------------------- derivatives (fixed hits) --

def _small_scene(w=24, h=16, spp=4, seed=5):
    import scenes
    sc = scenes.make_scene("c2", seed=seed, width=w, height=h, spp=spp)
    g = dict(depth=sc.depth, normal_rough=sc.normal_rough, albedo_metal=sc.albedo_metal,
             radiance=sc.radiance)
    return sc, g


def test_replaying_hits_reproduces_the_forward():
    sc, g = _small_scene()
    pix = np.arange(sc.width * sc.height)
    a = shade.shade_pixels(sc.camera, g, sc.env, sc.params, pix)
    b = shade.shade_pixels(sc.camera, g, sc.env, sc.params, pix, replay_hits=a["hits"])
    assert np.array_equal(a["out"], b["out"]) and np.array_equal(a["hits"], b["hits"])


def test_pixel_gradients_closed_form_in_a_furnace():
    """Uniform environment (L per channel), specular off: out = (1 - m) a L,
    so d/da_c = (1 - m) L_c g_c, d/dm = -sum_c g_c a_c L_c and the normal and
    roughness derivatives vanish."""
    from oracle import grad
    Lc = np.array([1.5, 0.7, 2.2])
    cam, g = open_floor(w=12, h=8, metal=0.3, rough=0.4)
    rng = np.random.default_rng(4)
    g["albedo_metal"][..., :3] = rng.uniform(0, 1, g["albedo_metal"][..., :3].shape)
    g["albedo_metal"][..., 3] = rng.uniform(0.1, 0.9, g["albedo_metal"][..., 3].shape)
    g["normal_rough"][..., 3] = rng.uniform(0.1, 0.9, g["normal_rough"][..., 3].shape)
    envmap = np.broadcast_to(Lc, (8, 16, 3)).copy()
    params = dict(spp=2, march=1, max_steps=64, step_len=0.125, max_dist=100.0,
                  thickness=0.05, seed=1, frame=0, flags=shade.NO_SPECULAR)
    pix = np.arange(12 * 8)
    hits = np.full((pix.size, 2), shade.HIT_SKIPPED)
    g_out = rng.normal(size=(pix.size, 3))
    d = grad.pixel_grads(cam, g, envmap, params, pix, hits, g_out)
    am = g["albedo_metal"].reshape(-1, 4)
    assert np.allclose(d[:, 4:7], (1 - am[:, 3:4]) * Lc * g_out, atol=1e-8)
    assert np.allclose(d[:, 7], -(g_out * am[:, :3] * Lc).sum(1), atol=1e-8)
    assert np.abs(d[:, :4]).max() < 1e-8


def test_pixel_gradients_converge_with_the_step():
    """Central differences at eps and eps/4 agree: the fixed-hit estimator is
    smooth in every per-pixel input (up to the kinks of bilinear filtering at
    texel boundaries, kept small here by a smoothly varying map)."""
    from oracle import grad
    sc, g = _small_scene(w=12, h=8, spp=4)
    he, we = sc.env.shape[:2]
    yy, xx = np.meshgrid(np.arange(he), np.arange(we), indexing="ij")
    smooth = 1.0 + 0.5 * np.sin(2 * np.pi * xx / we)[..., None] * np.cos(np.pi * yy / he)[..., None] \
        * np.array([1.0, 0.5, -0.7])
    pix = np.arange(12 * 8)
    hits = shade.shade_pixels(sc.camera, g, smooth, sc.params, pix)["hits"]
    g_out = np.random.default_rng(1).normal(size=(pix.size, 3))
    a = grad.pixel_grads(sc.camera, g, smooth, sc.params, pix, hits, g_out, eps=1e-6)
    b = grad.pixel_grads(sc.camera, g, smooth, sc.params, pix, hits, g_out, eps=2.5e-7)
    scale = np.abs(b).max(axis=0) + 1e-12
    assert (np.abs(a - b) / scale).max() < 1e-6
    assert np.abs(b[:, :4]).max() > 0          # normal / roughness really matter here


def test_env_gradients_sum_to_the_diffuse_weight():
    """Specular off: the trilinear weights sum to one over the texels of every
    level and each mip texel is a block mean, so the derivative summed over
    all texels of channel c is sum_p g_pc (1 - m_p) a_pc over surface pixels
    plus sum_p g_pc over background pixels (which show the map itself)."""
    from oracle import grad
    sc, g = _small_scene(w=10, h=6, spp=1)
    envmap = np.random.default_rng(3).uniform(0.5, 2.0, (4, 8, 3))
    params = dict(sc.params, flags=shade.NO_SPECULAR)
    hits = np.full((6, 10, 1), shade.HIT_SKIPPED)
    g_out = np.random.default_rng(2).normal(size=(6, 10, 3))
    tex = [(y, x, c) for y in range(4) for x in range(8) for c in range(3)]
    d = grad.env_grads(sc.camera, g, envmap, params, hits, g_out, tex).reshape(4, 8, 3)
    am = np.asarray(g["albedo_metal"], np.float64)
    fg = np.isfinite(np.asarray(g["depth"]))
    want = (g_out * (1 - am[..., 3:4]) * am[..., :3])[fg].sum(0) + g_out[~fg].sum(0)
    assert (~fg).any() and fg.any()
    assert np.allclose(d.sum(axis=(0, 1)), want, rtol=1e-9, atol=1e-9)


def test_radiance_gradients_match_a_direct_difference():
    from oracle import grad
    sc, g = _small_scene(w=16, h=10, spp=4, seed=8)
    pix = np.arange(16 * 10)
    r = shade.shade_pixels(sc.camera, g, sc.env, sc.params, pix)
    hits = r["hits"].reshape(10, 16, 4)
    g_out = np.random.default_rng(6).normal(size=(10, 16, 3))
    d = grad.radiance_grads(sc.camera, g, sc.env, sc.params, hits, g_out)
    q = int(np.bincount(hits[hits >= 0]).argmax())          # the most-hit pixel
    for c in range(3):
        gg = {k: np.array(v, np.float64) for k, v in g.items()}
        vals = []
        for sgn in (1, -1):
            rad = gg["radiance"].copy().reshape(-1, 4)
            rad[q, c] += sgn * 1e-3
            o = shade.shade_pixels(sc.camera, dict(gg, radiance=rad.reshape(10, 16, 4)), sc.env,
                                   sc.params, pix, replay_hits=hits.reshape(-1, 4))["out"]
            vals.append((o * g_out.reshape(-1, 3)).sum())
        assert abs((vals[0] - vals[1]) / 2e-3 - d.reshape(-1, 3)[q, c]) < 1e-8
    assert np.abs(d).sum() > 0


# ------------------------------------------------ NDF sampling (Walter 2007) --

@pytest.mark.parametrize("alpha,cos_no,f0", [(0.3, 0.8, 0.04), (0.6, 0.5, 0.9), (0.9, 0.95, 0.5),
                                             (0.15, 0.3, 0.2)])
def test_ndf_mean_weight_matches_quadrature(alpha, cos_no, f0):
    """Unbiased like the visible-normal sampler: the mean NDF-sampled weight
    converges to the same integral of f_s cos (within 4 standard errors)."""
    rng = np.random.default_rng(int(alpha * 100 + cos_no * 10))
    n = 400_000
    u1, u2 = rng.uniform(size=n), rng.uniform(size=n)
    h = brdf.sample_ndf(np.full(n, alpha), u1, u2)
    wo = np.array([math.sqrt(1 - cos_no ** 2), 0.0, cos_no])
    cos_oh = h @ wo
    l = 2 * cos_oh[:, None] * h - wo
    ok = (l[:, 2] > 0) & (cos_oh > 0)
    w = np.zeros(n)
    w[ok] = brdf.weight_ndf_short(np.array([f0]), np.full(ok.sum(), cos_no), l[ok, 2], cos_oh[ok],
                                  h[ok, 2], np.full(ok.sum(), alpha))[:, 0]
    quad = brdf.specular_albedo_quadrature(np.array([f0]), cos_no, alpha, 800, 400)[0]
    assert abs(w.mean() - quad) < 4 * w.std() / math.sqrt(n) + 1e-4


def test_ndf_half_vectors_follow_d_cos():
    """The sampled cos(theta_h) has the distribution of D(h) (n.h): compare the
    empirical CDF with the closed-form CDF u2(cos^2) = (1 - c^2)/(1 + (a^2 - 1) c^2)."""
    alpha = 0.4
    rng = np.random.default_rng(1)
    u1, u2 = rng.uniform(size=200_000), rng.uniform(size=200_000)
    c = brdf.sample_ndf(np.full(u1.size, alpha), u1, u2)[:, 2]
    grid = np.linspace(0.2, 0.99, 9)
    a2 = alpha * alpha
    # P(cos theta_h <= c) = P(u2 >= u2(c)), u2(c) solving cos^2 = (1 - u2)/(1 + (a2 - 1) u2)
    u_c = (1 - grid ** 2) / (1 + (a2 - 1) * grid ** 2)
    emp = np.array([(c <= g).mean() for g in grid])
    assert np.abs(emp - (1 - u_c)).max() < 5e-3
    # and D(h) cos over the hemisphere integrates to one (the density is normalised)
    th = np.linspace(0, math.pi / 2, 20001)
    integral = np.trapezoid(brdf.ndf(np.cos(th), alpha) * np.cos(th) * np.sin(th) * 2 * math.pi, th)
    assert abs(integral - 1) < 1e-6


def test_ndf_and_vndf_frames_agree_in_the_mean():
    """Whole estimator: a rough pixel of an open floor under a uniform map
    gives the same mean under both samplers (many samples)."""
    cam, g = open_floor(w=4, h=4, rough=0.5, metal=1.0, albedo=0.8)
    envmap = np.full((8, 16, 3), 1.0)
    base = dict(spp=8192, march=1, max_steps=64, step_len=0.125, max_dist=100.0,
                thickness=0.05, seed=4, frame=0, flags=0)
    q = np.array([1 * 4 + 2])
    rv = shade.shade_pixels(cam, g, envmap, base, q)
    rn = shade.shade_pixels(cam, g, envmap, dict(base, flags=shade.SAMPLER_NDF), q)
    assert abs(rv["out"][0, 0] - rn["out"][0, 0]) < 0.02 * rv["out"][0, 0]


# ------------------------------------------------------ first pass (c1) --

def test_depth_normals_of_planes_are_exact():
    from oracle import first_pass
    cam, g, is_floor = floor_wall_scene(w=48, h=40)
    n = first_pass.depth_normals(cam, g["depth"])
    # pixels whose four neighbours lie on the same plane
    same = is_floor.copy()
    inner = np.zeros_like(same)
    inner[1:-1, 1:-1] = True
    flo = inner & is_floor & np.roll(is_floor, 1, 0) & np.roll(is_floor, -1, 0)
    wal = inner & ~is_floor & ~np.roll(is_floor, 1, 0) & ~np.roll(is_floor, -1, 0)
    assert flo.sum() > 100 and wal.sum() > 100
    assert np.abs(n[flo] - [0, 1, 0]).max() < 1e-12
    assert np.abs(n[wal] - [0, 0, 1]).max() < 1e-12       # faces the camera (+z)


def test_depth_normals_of_spheres_converge():
    """On the analytic spheres the finite-difference normal approaches the
    true one; pixels next to an edge of the object are left out."""
    import scenes
    from oracle import first_pass
    sc = scenes.make_scene("c1", width=256, height=256)
    n = first_pass.depth_normals(sc.camera, sc.depth)
    true = sc.normal_rough[..., :3].astype(np.float64)
    ok = np.isfinite(sc.depth)
    for ax in (0, 1):
        for sh in (1, -1):
            ok &= (np.roll(true, sh, ax) * true).sum(-1) > 0.995
            ok &= np.isfinite(np.roll(sc.depth, sh, ax))
    ok[0, :] = ok[-1, :] = ok[:, 0] = ok[:, -1] = False
    ang = np.arccos(np.clip((n[ok] * true[ok]).sum(-1), -1, 1))
    assert ok.sum() > 5000
    assert np.quantile(ang, 0.99) < 0.01


def test_brdf_table_sums_to_the_directional_albedo():
    """F0 A + B is the integral of f_s cos with Schlick's F (linear in F0):
    the stratified table entries agree with the quadrature of that integral,
    and A + B = 1 for a perfect mirror."""
    from oracle import first_pass
    lut = first_pass.brdf_lut(n=8, k=64)
    # (rho >= 0.15: the quadrature itself resolves the lobe there)
    for (j, i) in ((1, 2), (2, 0), (4, 6), (7, 1), (6, 7), (3, 3)):
        rho, mu = (j + 0.5) / 8, (i + 0.5) / 8
        for f0 in (0.04, 0.5, 1.0):
            q = brdf.specular_albedo_quadrature(np.array([f0]), mu, rho, 2400, 1200)[0]
            assert abs(f0 * lut[j, i, 0] + lut[j, i, 1] - q) < 2e-3, (j, i, f0)
    mirror = first_pass.brdf_lut(n=1, k=4)          # rho = 0.5: still a table
    assert mirror.shape == (1, 1, 2)
    h = brdf.sample_vndf(np.array([[0.6, 0.0, 0.8]]), np.array([0.0]), np.array([0.3]), np.array([0.7]))
    assert np.allclose(h, [[0, 0, 1]])              # rho = 0: h = n, G1 = 1 -> A + B = 1


def test_split_sum_is_exact_under_a_uniform_environment():
    """With a constant environment the split-sum product is exact: the first
    pass's specular term equals the mean of the Monte-Carlo estimator (many
    samples, nothing to hit) and its diffuse term is a (1 - m) L."""
    from oracle import first_pass
    L = 1.3
    cam, g = open_floor(w=6, h=6, rough=0.45, metal=0.5, albedo=0.7)
    envmap = np.full((8, 16, 3), L)
    lut = first_pass.brdf_lut(n=32, k=64)
    c1 = first_pass.first_pass(cam, g, envmap, lut)
    params = dict(spp=8192, march=1, max_steps=64, step_len=0.125, max_dist=100.0,
                  thickness=0.05, seed=5, frame=0, flags=shade.NO_DIRECT)
    q = np.array([2 * 6 + 3])
    mc = shade.shade_pixels(cam, g, envmap, params, q)["out"][0]
    cd = (1 - 0.5) * 0.7 * L
    assert abs((c1.reshape(-1, 4)[q[0], 0] - cd) - mc[0]) < 0.01 * mc[0]


def test_depth_normal_condition_and_pixel_subset():
    """A wall facing the camera has perpendicular tangents (condition 1); the
    first pass on a subset of pixels equals the full frame at those pixels."""
    from oracle import first_pass
    cam, g, is_floor = floor_wall_scene(w=48, h=40)
    k = first_pass.depth_normal_condition(cam, g["depth"])
    wall = ~is_floor
    wall[0, :] = wall[-1, :] = wall[:, 0] = wall[:, -1] = False
    wall &= ~np.roll(is_floor, 1, 0) & ~np.roll(is_floor, -1, 0)
    assert wall.sum() > 100 and np.abs(k[wall] - 1.0).max() < 1e-9
    assert np.all(k[is_floor] >= 1.0)
    lut = first_pass.brdf_lut(n=8, k=8)
    env_rgb = np.exp(np.random.default_rng(2).normal(0, 1, (16, 32, 3)))
    full = first_pass.first_pass(cam, g, env_rgb, lut)
    pix = np.array([0, 5, 100, 48 * 40 - 1, 777])
    sub = first_pass.first_pass(cam, g, env_rgb, lut, pix=pix)
    assert np.array_equal(sub, full.reshape(-1, 4)[pix])
