"""Microfacet terms, GGX visible-normal sampling and the Monte-Carlo weight.

Oracle code (test infrastructure only).

Closed forms from Appendix B with alpha = rho, as the paper writes them
(its D and G use rho^2 where the Disney convention would use rho^4):

  D(h)   = rho^2 / (pi ((h.n)^2 (rho^2 - 1) + 1)^2)          (Eq. ndf)
  F      = F0 + (1 - F0)(1 - wo.h)^5,  F0 = lerp(0.04, a, m)  (Eq. fresnel,
           read with the textbook parenthesisation; the printed form raises
           only wo.h to the fifth power)
  G1(z)  = 2 z / (z + sqrt(rho^2 + (1 - rho^2) z^2))           (Eq. geometry)
  G      = G1(n.wi) G1(n.wo)
  f_s    = D F G / (4 (n.wi)(n.wo))                            (Eq. brdf)

The specular estimator of Sec. 3.3 averages f_s c1 (wi.n) / p(wi).  Its
directions are drawn here from the distribution of visible normals (reading
taken in place of the paper's citation of plain NDF sampling, so that every
weight is bounded by one): the spherical-cap method of Dupuy and Benyoub
(2023).  For that density, p(wi) = G1(wo) max(0, wo.h) D(h) / (n.wo) / (4 wo.h),
and the weight f_s (n.wi) / p(wi) reduces to F(wo.h) G1(n.wi).  Both forms are
computed here; tests check that they agree.

The tangent frame around n is the branchless basis of Duff et al. (JCGT
2017), with sign(+0) = +1.
"""

import math

import numpy as np


def normalize(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def dot(a, b):
    return np.sum(a * b, axis=-1)


def onb(n):
    """Tangent t and bitangent b with (t, b, n) right-handed orthonormal."""
    sign = np.copysign(1.0, n[..., 2])
    a = -1.0 / (sign + n[..., 2])
    b = n[..., 0] * n[..., 1] * a
    t = np.stack([1.0 + sign * n[..., 0] ** 2 * a, sign * b, -sign * n[..., 0]], axis=-1)
    bt = np.stack([b, sign + n[..., 1] ** 2 * a, -n[..., 1]], axis=-1)
    return t, bt


def sample_vndf(wo_local, alpha, u1, u2):
    """Half vector (local frame, z = normal) from the visible-normal density.

    Dupuy & Benyoub 2023: stretch the view direction to the alpha = 1
    configuration, pick a point on the unit sphere's cap z > -wi_std.z
    uniformly (phi from u1, z from u2), add wi_std to get the normal of the
    hemisphere configuration, and un-stretch.
    """
    alpha = np.asarray(alpha, np.float64)
    wi_std = normalize(np.stack([alpha * wo_local[..., 0], alpha * wo_local[..., 1],
                                 wo_local[..., 2]], axis=-1))
    phi = 2.0 * math.pi * u1
    z = (1.0 - u2) * (1.0 + wi_std[..., 2]) - wi_std[..., 2]
    sin_t = np.sqrt(np.clip(1.0 - z * z, 0.0, 1.0))
    c = np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), z], axis=-1)
    h_std = c + wi_std
    return normalize(np.stack([alpha * h_std[..., 0], alpha * h_std[..., 1], h_std[..., 2]],
                              axis=-1))


def sample_ndf(alpha, u1, u2):
    """Half vector (local frame, z = normal) from the distribution of normals
    itself, density D(h) (n.h) (Walter et al. 2007, the GGX sampling the paper
    cites): azimuth 2 pi u1 and tan^2 theta_h = alpha^2 u2 / (1 - u2), i.e.
    cos^2 theta_h = (1 - u2) / (1 + (alpha^2 - 1) u2)."""
    alpha = np.asarray(alpha, np.float64)
    phi = 2.0 * math.pi * u1
    cos2 = (1.0 - u2) / (1.0 + (alpha * alpha - 1.0) * u2)
    cos_t = np.sqrt(cos2)
    sin_t = np.sqrt(np.clip(1.0 - cos2, 0.0, 1.0))
    return np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t], axis=-1)


def ndf_pdf_l(cos_oh, cos_h, alpha):
    """Density of wi = reflect(wo, h) when h follows D(h) (n.h)."""
    return ndf(cos_h, alpha) * cos_h / (4.0 * cos_oh)


def weight_ndf_short(f0, cos_no, cos_nl, cos_oh, cos_h, alpha):
    """f_s (n.wi) / p(wi) under NDF sampling, reduced:
    F(wo.h) G1(n.wo) G1(n.wi) (wo.h) / ((n.wo) (n.h)).  Unbounded above."""
    g = smith_g1(cos_no, alpha) * smith_g1(cos_nl, alpha) * cos_oh / (cos_no * cos_h)
    return schlick(f0, cos_oh) * g[..., None]


def weight_ndf_long(f0, cos_no, cos_nl, cos_oh, cos_h, alpha):
    """The same with every factor evaluated separately (alpha > 0)."""
    d = ndf(cos_h, alpha)
    g = smith_g1(cos_nl, alpha) * smith_g1(cos_no, alpha)
    f = schlick(f0, cos_oh)
    fs = d[..., None] * f * g[..., None] / (4.0 * cos_nl * cos_no)[..., None]
    return fs * (cos_nl / ndf_pdf_l(cos_oh, cos_h, alpha))[..., None]


def ndf(cos_h, alpha):
    a2 = alpha * alpha
    return a2 / (math.pi * (cos_h * cos_h * (a2 - 1.0) + 1.0) ** 2)


def smith_g1(z, alpha):
    a2 = alpha * alpha
    return 2.0 * z / (z + np.sqrt(a2 + (1.0 - a2) * z * z))


def schlick(f0, cos_oh):
    return f0 + (1.0 - f0) * ((1.0 - cos_oh) ** 5)[..., None]


def vndf_pdf_l(cos_no, cos_oh, cos_h, alpha):
    """Density of wi = reflect(wo, h) when h follows the visible-normal density."""
    p_h = smith_g1(cos_no, alpha) * np.maximum(cos_oh, 0.0) * ndf(cos_h, alpha) / cos_no
    return p_h / (4.0 * cos_oh)


def weight_short(f0, cos_oh, cos_nl, alpha):
    """F(wo.h) G1(n.wi): the estimator's weight under visible-normal sampling."""
    return schlick(f0, cos_oh) * smith_g1(cos_nl, alpha)[..., None]


def weight_long(f0, cos_no, cos_nl, cos_oh, cos_h, alpha):
    """f_s (n.wi) / p(wi) with every factor evaluated separately (alpha > 0)."""
    d = ndf(cos_h, alpha)
    g = smith_g1(cos_nl, alpha) * smith_g1(cos_no, alpha)
    f = schlick(f0, cos_oh)
    fs = d[..., None] * f * g[..., None] / (4.0 * cos_nl * cos_no)[..., None]
    return fs * (cos_nl / vndf_pdf_l(cos_no, cos_oh, cos_h, alpha))[..., None]


def specular_albedo_quadrature(f0, cos_no, alpha, n_theta=400, n_phi=400):
    """int f_s (n.wi) dwi over the hemisphere by midpoint quadrature (float64).

    Used only to pin the sampler: the mean weight of visible-normal samples
    must converge to this integral.
    """
    sin_o = math.sqrt(max(0.0, 1.0 - cos_no * cos_no))
    wo = np.array([sin_o, 0.0, cos_no])
    # integrate in (mu = cos theta_i, phi); dwi = dmu dphi
    mu = (np.arange(n_theta) + 0.5) / n_theta
    ph = (np.arange(n_phi) + 0.5) / n_phi * 2.0 * math.pi
    MU, PH = np.meshgrid(mu, ph, indexing="ij")
    s = np.sqrt(1.0 - MU * MU)
    wi = np.stack([s * np.cos(PH), s * np.sin(PH), MU], axis=-1)
    h = normalize(wi + wo)
    cos_h = h[..., 2]
    cos_oh = dot(h, wo)
    f = schlick(np.asarray(f0, np.float64), cos_oh)
    g = smith_g1(MU, alpha) * smith_g1(cos_no, alpha)
    fs = ndf(cos_h, alpha)[..., None] * f * g[..., None] / (4.0 * MU * cos_no)[..., None]
    integrand = fs * MU[..., None]
    return integrand.sum(axis=(0, 1)) * (1.0 / n_theta) * (2.0 * math.pi / n_phi)
