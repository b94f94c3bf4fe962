// Per-pixel and per-sample shading steps shared by the forward kernels
// (trace, resolve) and the adjoint: G-buffer loads, pixel set-up, the direct
// term, the sample direction and the weighted radiance of one sample.
#pragma once

#include <hip/hip_fp16.h>

#include "device_math.h"
#include "kernels.h"

namespace ssr {

// -------------------------------------------------------- G-buffer loads --

template <int DT>
struct Texel4;

template <>
struct Texel4<0> {  // float32
    __device__ static float4 load(const void* p, int64_t i) {
        return reinterpret_cast<const float4*>(p)[i];
    }
    // the first three channels only (a 12 B load: no register is written
    // that the caller does not read, so nothing waits on it before its use)
    __device__ static float3 load3(const void* p, int64_t i) {
        return *reinterpret_cast<const float3*>(reinterpret_cast<const float4*>(p) + i);
    }
};

template <>
struct Texel4<1> {  // float16
    __device__ static float4 load(const void* p, int64_t i) {
        const ushort4 b = reinterpret_cast<const ushort4*>(p)[i];
        return make_float4(__half2float(__ushort_as_half(b.x)), __half2float(__ushort_as_half(b.y)),
                           __half2float(__ushort_as_half(b.z)), __half2float(__ushort_as_half(b.w)));
    }
    __device__ static float3 load3(const void* p, int64_t i) {
        const float4 v = load(p, i);
        return make_float3(v.x, v.y, v.z);
    }
};

template <>
struct Texel4<2> {  // bfloat16: the high half of a float32
    __device__ static float4 load(const void* p, int64_t i) {
        const ushort4 b = reinterpret_cast<const ushort4*>(p)[i];
        return make_float4(__uint_as_float(static_cast<uint32_t>(b.x) << 16),
                           __uint_as_float(static_cast<uint32_t>(b.y) << 16),
                           __uint_as_float(static_cast<uint32_t>(b.z) << 16),
                           __uint_as_float(static_cast<uint32_t>(b.w) << 16));
    }
    __device__ static float3 load3(const void* p, int64_t i) {
        const float4 v = load(p, i);
        return make_float3(v.x, v.y, v.z);
    }
};

__device__ __forceinline__ EnvLevel env_level(const ShadeArgs& a, int k) {
    return EnvLevel{a.env + a.env_lay.offset[k], a.env_lay.w[k], a.env_lay.h[k]};
}

__device__ __forceinline__ V3 view_to_world(const ShadeArgs& a, float X, float Y, float Z) {
    return v3(X * a.right[0] + Y * a.up[0] + Z * a.fwd[0], X * a.right[1] + Y * a.up[1] + Z * a.fwd[1],
              X * a.right[2] + Y * a.up[2] + Z * a.fwd[2]);
}

__device__ __forceinline__ V3 world_to_view(const ShadeArgs& a, V3 l) {
    return v3(dot(l, v3(a.right[0], a.right[1], a.right[2])), dot(l, v3(a.up[0], a.up[1], a.up[2])),
              dot(l, v3(a.fwd[0], a.fwd[1], a.fwd[2])));
}


// ------------------------------------------------------------ per pixel --

struct Pixel {
    bool bg;              // background (depth not finite)
    float D, X0, Y0;      // view-space point of the pixel centre
    V3 wo, n;             // toward the camera; shading normal
    float rho, m;
    V3 alb, f0;
    float cos_no;
    bool trace;           // specular samples are drawn
    V3 t, b, ws;          // tangent frame; stretched view vector (visible normals)
};

template <int DT>
__device__ __forceinline__ Pixel setup_pixel(const ShadeArgs& a, int i, int j, int64_t q) {
    Pixel P;
    P.D = a.depth[q];
    P.bg = !(P.D < INFINITY);
    const float D = P.bg ? 1.0f : P.D;
    const float4 nr = Texel4<DT>::load(a.normal_rough, q);
    const float4 am = Texel4<DT>::load(a.albedo_metal, q);
    // (reciprocal focal lengths from the host: a multiply, not a division)
    P.X0 = (static_cast<float>(i) + 0.5f - a.cx) * D * a.inv_fx;
    P.Y0 = -(static_cast<float>(j) + 0.5f - a.cy) * D * a.inv_fy;
    P.wo = -1.0f * normalize(view_to_world(a, P.X0, P.Y0, D));
    P.n = normalize(v3(nr.x, nr.y, nr.z));
    P.rho = fminf(fmaxf(nr.w, 0.0f), 1.0f);
    P.m = fminf(fmaxf(am.w, 0.0f), 1.0f);
    P.alb = v3(am.x, am.y, am.z);
    P.f0 = v3(0.04f * (1.0f - P.m) + P.alb.x * P.m, 0.04f * (1.0f - P.m) + P.alb.y * P.m,
              0.04f * (1.0f - P.m) + P.alb.z * P.m);
    P.cos_no = dot(P.n, P.wo);
    P.trace = !P.bg && !(a.flags & SSR_NO_SPECULAR) && P.cos_no > 0.0f;
    onb(P.n, P.t, P.b);
    const V3 wl = v3(dot(P.wo, P.t), dot(P.wo, P.b), P.cos_no);
    // visible-normal sampling (Dupuy & Benyoub 2023): stretched view vector
    P.ws = normalize(v3(P.rho * wl.x, P.rho * wl.y, wl.z));
    return P;
}

// Mip level lambda = log2(1 + rho) * lambda_max of the roughness lookups
// (Sec. 3.2), via log1p (no rounding of 1 + rho), clamped to [0, top].
__device__ __forceinline__ float roughness_lod(const ShadeArgs& a, float rho) {
    const int top = a.env_lay.levels - 1;
    return fminf(fmaxf(log1pf(rho) * (static_cast<float>(top) * 1.44269504f), 0.0f),
                 static_cast<float>(top));
}

// E_lambda(d): the two mip levels around lambda, each read bilinearly, blended.
__device__ __forceinline__ float3 env_lod(const ShadeArgs& a, const EnvAngles& ang, float lam) {
    const int top = a.env_lay.levels - 1;
    const int k0 = static_cast<int>(floorf(lam));
    const int k1 = min(k0 + 1, top);
    const float t = lam - static_cast<float>(k0);
    const float3 e0 = env_bilinear(env_level(a, k0), ang);
    if (!(t > 0.0f)) return e0;
    const float3 e1 = env_bilinear(env_level(a, k1), ang);
    return make_float3((1.0f - t) * e0.x + t * e1.x, (1.0f - t) * e0.y + t * e1.y,
                       (1.0f - t) * e0.z + t * e1.z);
}

// Direct diffuse c_d = (1 - m) a E_lambda(n), or the environment seen directly
// for a background pixel.
__device__ __forceinline__ float3 direct_term(const ShadeArgs& a, const Pixel& P, int i, int j) {
    if (P.bg) {
        const V3 d = normalize(view_to_world(a, (static_cast<float>(i) + 0.5f - a.cx) / a.fx,
                                             -(static_cast<float>(j) + 0.5f - a.cy) / a.fy, 1.0f));
        return env_bilinear(env_level(a, 0), env_angles(d));
    }
    if (a.flags & SSR_NO_DIRECT) return make_float3(0.0f, 0.0f, 0.0f);
    const float3 e = env_lod(a, env_angles(P.n), roughness_lod(a, P.rho));
    const float k = 1.0f - P.m;
    return make_float3(k * P.alb.x * e.x, k * P.alb.y * e.y, k * P.alb.z * e.z);
}

// ----------------------------------------------------------- per sample --

struct SampleDir {
    V3 l;         // reflected ray direction (world)
    float cos_oh, cos_nl, cos_nh;
    bool valid;   // the sample reflects into the upper hemisphere
};

// Sample s of pixel q: Philox4x32-10 at counter (q, s, frame, 0) gives u1
// (azimuth) and u2 (cap height, or polar angle) of the half vector h; l
// reflects wo about h.
__device__ __forceinline__ SampleDir sample_dir(const ShadeArgs& a, const Pixel& P, int64_t q,
                                                int s) {
    const uint4 x = philox4x32_10(
        make_uint4(static_cast<uint32_t>(q), static_cast<uint32_t>(s), a.frame, 0u), a.key0, a.key1);
    const float u1 = unit24(x.x), u2 = unit24(x.y);
    float sphi, cphi;
    sincos_rev(u1, &sphi, &cphi);
    V3 hl;
    const bool ndf = a.flags & SSR_SAMPLER_NDF;
    if (ndf) {
        // distribution of normals: cos^2 theta = (1 - u2) / den and
        // sin^2 theta = rho^2 u2 / den, den = 1 + (rho^2 - 1) u2 (no cancellation)
        const float a2 = P.rho * P.rho;
        const float inv = __builtin_amdgcn_rcpf(1.0f + (a2 - 1.0f) * u2);
        const float ct = __builtin_amdgcn_sqrtf((1.0f - u2) * inv);
        const float st = P.rho * __builtin_amdgcn_sqrtf(u2 * inv);
        hl = v3(st * cphi, st * sphi, ct);
    } else {
        // visible normals: point on the spherical cap z > -ws.z, azimuth
        // 2 pi u1, height from u2.  h_std.z = z + ws.z = (1 - u2)(1 + ws.z)
        // and 1 - z^2 = (1 - z)(1 + z) with 1 - z = u2 (1 + ws.z),
        // 1 + z = (1 - u2)(1 + ws.z) + (1 - ws.z): no cancellation.
        const float one_m_u2 = 1.0f - u2;
        const float opz = 1.0f + P.ws.z;
        const float hz = one_m_u2 * opz;
        const float sin2 = (u2 * opz) * (hz + (1.0f - P.ws.z));
        const float st = __builtin_amdgcn_sqrtf(fmaxf(sin2, 0.0f));
        hl = normalize(v3(P.rho * (st * cphi + P.ws.x), P.rho * (st * sphi + P.ws.y), hz));
    }
    const V3 h = v3(hl.x * P.t.x + hl.y * P.b.x + hl.z * P.n.x,
                    hl.x * P.t.y + hl.y * P.b.y + hl.z * P.n.y,
                    hl.x * P.t.z + hl.y * P.b.z + hl.z * P.n.z);
    SampleDir d;
    d.cos_oh = dot(P.wo, h);
    d.l = (2.0f * d.cos_oh) * h - P.wo;
    d.cos_nl = dot(P.n, d.l);
    d.cos_nh = hl.z;
    // (a visible normal always faces wo; a half vector from D may not)
    d.valid = d.cos_nl > 0.0f && (!ndf || d.cos_oh > 0.0f);
    return d;
}

// Weight F(wo.h) G1(n.l) (visible normals; NDF sampling: the weight above)
// times the radiance Lr found along the sample (c1 at a hit pixel, the
// unfiltered environment otherwise), Kahan-accumulated per channel.
__device__ __forceinline__ void accumulate(const ShadeArgs& a, const Pixel& P, const SampleDir& d,
                                           float3 Lr, float* sum, float* cmp) {
    const float fc = 1.0f - d.cos_oh;
    const float fc2 = fc * fc;
    const float fr = fc2 * fc2 * fc;
    float g1 = smith_g1(fmaxf(d.cos_nl, 0.0f), P.rho * P.rho);
    if (a.flags & SSR_SAMPLER_NDF) {
        // F G1(n.wo) G1(n.l) (wo.h) / ((n.wo) (n.h)); nothing below the surface
        g1 = d.valid ? g1 * smith_g1(P.cos_no, P.rho * P.rho) * d.cos_oh / (P.cos_no * d.cos_nh)
                     : 0.0f;
    }
    kahan_add(sum[0], cmp[0], (P.f0.x + (1.0f - P.f0.x) * fr) * g1 * Lr.x);
    kahan_add(sum[1], cmp[1], (P.f0.y + (1.0f - P.f0.y) * fr) * g1 * Lr.y);
    kahan_add(sum[2], cmp[2], (P.f0.z + (1.0f - P.f0.z) * fr) * g1 * Lr.z);
}

__device__ __forceinline__ int fill_code(const ShadeArgs& a, const Pixel& P) {
    return P.bg ? SSR_HIT_BACKGROUND
                : ((a.flags & SSR_NO_SPECULAR) ? SSR_HIT_SKIPPED : SSR_HIT_INVALID);
}

// Index of sample k of pixel (i, j) in a per-sample buffer (hit codes,
// iteration counts): [H][W][S], or with SSR_CODES_TILED tile-major over 8 x 8
// pixel tiles, [ceil(H/8) ceil(W/8)][S][64] with the pixel at (j % 8) 8 +
// i % 8 of its tile (a tile's codes of one sample fill 256 contiguous bytes,
// so the rays a wave draws together write a few cache lines).
// The hot kernels take the layout as a template argument (TL: 1 tile-major,
// 0 public, -1 read from the flags at run time).
template <int TL = -1>
__device__ __forceinline__ int64_t code_index(const ShadeArgs& a, int i, int j, int k) {
    const bool tiled = TL < 0 ? (a.flags & SSR_CODES_TILED) != 0 : TL == 1;
    if (tiled) {
        const int t = (j >> 3) * ((a.W + 7) >> 3) + (i >> 3);
        return (static_cast<int64_t>(t) * a.spp + k) * 64 + ((j & 7) << 3) + (i & 7);
    }
    return (static_cast<int64_t>(j) * a.W + i) * a.spp + k;
}

__device__ __forceinline__ void write_out(const ShadeArgs& a, int64_t q, float3 cd, const float* sum) {
    const float invS = 1.0f / static_cast<float>(a.spp);
    // one 12-byte store per pixel: a row of lanes writes one contiguous run
    reinterpret_cast<float3*>(a.out)[q] =
        make_float3(cd.x + sum[0] * invS, cd.y + sum[1] * invS, cd.z + sum[2] * invS);
}


}  // namespace ssr
