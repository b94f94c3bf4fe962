// The adjoint of the shading estimator with the hit selection held fixed.
//
// For a loss whose gradient with respect to the output image is g, this
// computes, per pixel, d(g . out)/d of its normal (stored, before
// normalisation), roughness, albedo and metallic, and accumulates the
// derivatives with respect to the environment texels and to the first-pass
// radiance of the hit pixels.  The hit codes of the forward pass are replayed
// (the march selects pixels and has no useful derivative; the paper
// differentiates the shading with the tracing treated as a fixed selection).
//
// Per pixel, the roughness and the three normal components are propagated
// forward together as four-direction dual numbers through everything they
// touch: normalisation, the tangent frame, the visible-normal sample, the
// reflection, Fresnel (through wo.h), masking G1 (through n.l and alpha =
// rho), the roughness mip level and the environment lookups (through their
// angles and bilinear weights).  Albedo and metallic enter only through
// F0 = 0.04 (1 - m) + a m and the diffuse factor (1 - m) a, so their
// derivatives are written out directly.  The output is linear in the
// environment texels and in the radiance, whose derivatives are the lookup
// weights times the multiplying factor.
//
// Environment derivatives first go to a per-mip-level buffer (the direct
// term reads mip levels); the small, heavily shared top levels are summed
// per workgroup in LDS, and the texels of the lower levels a workgroup
// touches in an LDS hash table, before one atomic per texel.  A second
// kernel pushes each level down to the level-0 texels it is the box mean of.
#include "shading.h"

namespace ssr {

// --------------------------------------------------------- dual numbers --
//
// d[0]: stored roughness; d[1..3]: stored normal x, y, z.
constexpr int kDirs = 4;

struct Dual {
    float v;
    float d[kDirs];
};

__device__ __forceinline__ Dual dconst(float v) {
    Dual r;
    r.v = v;
#pragma unroll
    for (int k = 0; k < kDirs; ++k) r.d[k] = 0.0f;
    return r;
}
__device__ __forceinline__ Dual operator+(Dual a, Dual b) {
    Dual r;
    r.v = a.v + b.v;
#pragma unroll
    for (int k = 0; k < kDirs; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
__device__ __forceinline__ Dual operator-(Dual a, Dual b) {
    Dual r;
    r.v = a.v - b.v;
#pragma unroll
    for (int k = 0; k < kDirs; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
__device__ __forceinline__ Dual operator*(Dual a, Dual b) {
    Dual r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < kDirs; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
__device__ __forceinline__ Dual operator*(float s, Dual a) {
    Dual r;
    r.v = s * a.v;
#pragma unroll
    for (int k = 0; k < kDirs; ++k) r.d[k] = s * a.d[k];
    return r;
}
__device__ __forceinline__ Dual operator+(float s, Dual a) {
    a.v += s;
    return a;
}
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    Dual r;
    r.v = a.v / b.v;
    const float ib = 1.0f / b.v;
#pragma unroll
    for (int k = 0; k < kDirs; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
    return r;
}
__device__ __forceinline__ Dual dsqrt(Dual a) {
    Dual r;
    r.v = sqrtf(a.v);
    const float h = r.v > 0.0f ? 0.5f / r.v : 0.0f;
#pragma unroll
    for (int k = 0; k < kDirs; ++k) r.d[k] = a.d[k] * h;
    return r;
}
__device__ __forceinline__ Dual dmax0(Dual a) { return a.v > 0.0f ? a : dconst(0.0f); }

struct DV3 {
    Dual x, y, z;
};
__device__ __forceinline__ Dual ddot(const DV3& a, const DV3& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ Dual ddot(const DV3& a, V3 b) {
    return b.x * a.x + b.y * a.y + b.z * a.z;
}
__device__ __forceinline__ DV3 dnormalize(const DV3& a) {
    const Dual inv = dconst(1.0f) / dsqrt(ddot(a, a));
    return DV3{a.x * inv, a.y * inv, a.z * inv};
}
__device__ __forceinline__ V3 value(const DV3& a) { return v3(a.x.v, a.y.v, a.z.v); }

// --------------------------------------------- environment lookups (dual) --

// Bilinear lookup at direction d of one level: value, derivative of each
// channel along the four directions, and the four taps with their weights
// (for the environment derivatives).
struct EnvTaps {
    int idx[4];      // texel index within the level
    float w[4];
};

struct DualRGB {
    float v[3];
    float d[3][kDirs];
};

__device__ __forceinline__ DualRGB env_bilinear_dual(const EnvLevel& lv, const DV3& dir,
                                                     EnvTaps& taps) {
    const V3 d = value(dir);
    const EnvAngles a = env_angles(d);
    const float wf = static_cast<float>(lv.w), hf = static_cast<float>(lv.h);
    TexelCoord cx, cy;
    env_texel(lv, a, cx, cy);
    int x0, x1;
    env_columns(cx.i0, lv.w, x0, x1);
    const int y0 = min(max(cy.i0, 0), lv.h - 1);
    const int y1 = min(max(cy.i0 + 1, 0), lv.h - 1);
    const float4 t00 = lv.texels[y0 * lv.w + x0], t01 = lv.texels[y0 * lv.w + x1];
    const float4 t10 = lv.texels[y1 * lv.w + x0], t11 = lv.texels[y1 * lv.w + x1];
    const float fx = cx.f, fy = cy.f;
    taps.idx[0] = y0 * lv.w + x0;
    taps.idx[1] = y0 * lv.w + x1;
    taps.idx[2] = y1 * lv.w + x0;
    taps.idx[3] = y1 * lv.w + x1;
    taps.w[0] = (1.0f - fx) * (1.0f - fy);
    taps.w[1] = fx * (1.0f - fy);
    taps.w[2] = (1.0f - fx) * fy;
    taps.w[3] = fx * fy;
    // d phi = (x dz - z dx) / (x^2 + z^2); d theta = (y dr - r dy) / (r^2 + y^2)
    const float r2 = d.x * d.x + d.z * d.z;
    const float r = sqrtf(r2);
    const float ir2 = r2 > 0.0f ? 1.0f / r2 : 0.0f;
    const float ir = r > 0.0f ? 1.0f / r : 0.0f;
    const float iq = 1.0f / (r2 + d.y * d.y);
    float dfx[kDirs], dfy[kDirs];
#pragma unroll
    for (int k = 0; k < kDirs; ++k) {
        const float dphi = (d.x * dir.z.d[k] - d.z * dir.x.d[k]) * ir2;
        const float dr = (d.x * dir.x.d[k] + d.z * dir.z.d[k]) * ir;
        const float dth = (d.y * dr - r * dir.y.d[k]) * iq;
        dfx[k] = dphi * (wf * kInv2PiHi);
        dfy[k] = dth * (hf * kInvPiHi);
    }
    // the clamped rows of the poles do not move with the direction
    const bool ymove = cy.i0 >= 0 && cy.i0 + 1 <= lv.h - 1;
    const float c00[3] = {t00.x, t00.y, t00.z}, c01[3] = {t01.x, t01.y, t01.z};
    const float c10[3] = {t10.x, t10.y, t10.z}, c11[3] = {t11.x, t11.y, t11.z};
    DualRGB out;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        out.v[c] = taps.w[0] * c00[c] + taps.w[1] * c01[c] + taps.w[2] * c10[c] + taps.w[3] * c11[c];
        const float bx = (1.0f - fy) * (c01[c] - c00[c]) + fy * (c11[c] - c10[c]);
        const float by = ymove ? (1.0f - fx) * (c10[c] - c00[c]) + fx * (c11[c] - c01[c]) : 0.0f;
#pragma unroll
        for (int k = 0; k < kDirs; ++k) out.d[c][k] = bx * dfx[k] + by * dfy[k];
    }
    return out;
}

// ------------------------------------------------------------- the adjoint --

#ifndef SSR_BW_PRIV_TEXELS
#define SSR_BW_PRIV_TEXELS 4096
#endif
#ifndef SSR_BW_TABLE_BITS
#define SSR_BW_TABLE_BITS 11
#endif
#ifndef SSR_BW_PROBES
#define SSR_BW_PROBES 2
#endif
// top mip levels summed in LDS per workgroup (48 KB), and a table of
// 2^SSR_BW_TABLE_BITS slots (16 KB) that sums the other texels the
// workgroup touches before they go out as global atomics: 64 KB, two
// workgroups per CU, which the register use allows anyway
constexpr int kPrivTexels = SSR_BW_PRIV_TEXELS;
constexpr int kTableBits = SSR_BW_TABLE_BITS;
constexpr int kTableSlots = 1 << kTableBits;

struct BackArgs {
    const float* g_out;       // [H][W][3]
    const int32_t* hits;      // [H][W][spp]
    float* g_nr;              // [H][W][4] or null
    float* g_am;              // [H][W][4] or null
    float4* g_mips;           // this workgroup's copy: [env texels of all levels] (RGB)
    float* g_rad;             // [H][W][4] or null (channels 0..2 accumulated)
    int priv_first;           // first mip level summed in LDS
    int priv_offset;          // its texel offset in the level layout
    int priv_texels;          // texels of that level and all above
    int replicas;             // copies of the per-texel sums
    int64_t texels;           // texels of one copy
};

// The workgroup's sums of the top mip levels, and the table: slot k holds
// the texel lds_tag[k] (-1: free) and its RGB sum (file scope, so that the
// compiler sees LDS and issues LDS atomics).
__shared__ float lds_env[3 * kPrivTexels];
__shared__ int lds_tag[kTableSlots];
__shared__ float lds_tab[3 * kTableSlots];

// Add (r, g, bl) to texel `texel` of the lower levels: into the table slot
// the texel owns, or claims while it is free (two probes); else (both slots
// owned by other texels) straight to the global sums.  Device-scope float
// atomics are performed beyond the per-XCD L2 caches, so each one saved
// here is a round trip over the fabric.
__device__ __forceinline__ void add_lower(const BackArgs& b, int texel, float r, float g, float bl) {
    const unsigned h = (static_cast<unsigned>(texel) * 2654435761u) >> (32 - kTableBits);
#pragma unroll
    for (int p = 0; p < SSR_BW_PROBES; ++p) {
        const unsigned slot = (h + p) & (kTableSlots - 1);
        int cur = lds_tag[slot];
        if (cur == -1) {
            const int old = atomicCAS(&lds_tag[slot], -1, texel);
            cur = old == -1 ? texel : old;
        }
        if (cur == texel) {
            atomicAdd(&lds_tab[3 * slot + 0], r);
            atomicAdd(&lds_tab[3 * slot + 1], g);
            atomicAdd(&lds_tab[3 * slot + 2], bl);
            return;
        }
    }
    float* q = reinterpret_cast<float*>(b.g_mips + texel);
    atomicAdd(q + 0, r);
    atomicAdd(q + 1, g);
    atomicAdd(q + 2, bl);
}

__device__ __forceinline__ void add_env(const BackArgs& b, int level_offset, int level,
                                        const EnvTaps& t, const float coef[3]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float w = t.w[k];
        if (w == 0.0f) continue;
        const int texel = level_offset + t.idx[k];
        if (level >= b.priv_first) {
            const int at = 3 * (texel - b.priv_offset);
            atomicAdd(&lds_env[at + 0], w * coef[0]);
            atomicAdd(&lds_env[at + 1], w * coef[1]);
            atomicAdd(&lds_env[at + 2], w * coef[2]);
        } else {
            add_lower(b, texel, w * coef[0], w * coef[1], w * coef[2]);
        }
    }
}

template <int DT>
__global__ __launch_bounds__(256) void backward_kernel(const ShadeArgs a, const BackArgs b0) {
    for (int k = threadIdx.x; k < 3 * b0.priv_texels; k += blockDim.x) lds_env[k] = 0.0f;
    for (int k = threadIdx.x; k < kTableSlots; k += blockDim.x) {
        lds_tag[k] = -1;
        lds_tab[3 * k + 0] = 0.0f;
        lds_tab[3 * k + 1] = 0.0f;
        lds_tab[3 * k + 2] = 0.0f;
    }
    // workgroups spread their global atomics over `replicas` copies of the
    // per-texel sums, so that many pixels reading the same texels do not
    // all queue on one address
    BackArgs b = b0;
    b.g_mips = b0.g_mips + static_cast<int64_t>(blockIdx.x % b0.replicas) * b0.texels;
    __syncthreads();

    const int tiles_x = (a.W + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = (blockIdx.x % tiles_x) * 16 + (wave & 1) * 8 + (lane & 7);
    const int j = (blockIdx.x / tiles_x) * 16 + (wave >> 1) * 8 + (lane >> 3);
    if (i < a.W && j < a.H) {
        const int64_t q = static_cast<int64_t>(j) * a.W + i;
        const int S = a.spp;
        const float g[3] = {b.g_out[3 * q], b.g_out[3 * q + 1], b.g_out[3 * q + 2]};
        const Pixel P = setup_pixel<DT>(a, i, j, q);
        float G[kDirs] = {0.0f, 0.0f, 0.0f, 0.0f};   // d/d(rho, n.x, n.y, n.z)
        float ga[3] = {0.0f, 0.0f, 0.0f}, gm = 0.0f;
        if (P.bg) {
            // the background shows the map along the view ray
            const V3 d = normalize(view_to_world(a, (static_cast<float>(i) + 0.5f - a.cx) / a.fx,
                                                 -(static_cast<float>(j) + 0.5f - a.cy) / a.fy, 1.0f));
            EnvTaps t;
            const DV3 dd{dconst(d.x), dconst(d.y), dconst(d.z)};
            (void)env_bilinear_dual(env_level(a, 0), dd, t);
            add_env(b, 0, 0, t, g);
        } else {
            const float4 nr = Texel4<DT>::load(a.normal_rough, q);
            const float4 am = Texel4<DT>::load(a.albedo_metal, q);
            // dual inputs: roughness (clamped to [0, 1]) and the stored normal
            Dual rho = dconst(P.rho);
            rho.d[0] = (nr.w >= 0.0f && nr.w <= 1.0f) ? 1.0f : 0.0f;
            DV3 ns{dconst(nr.x), dconst(nr.y), dconst(nr.z)};
            ns.x.d[1] = 1.0f;
            ns.y.d[2] = 1.0f;
            ns.z.d[3] = 1.0f;
            const DV3 n = dnormalize(ns);
            const float dm = (am.w >= 0.0f && am.w <= 1.0f) ? 1.0f : 0.0f;
            const float m = P.m;
            const float alb[3] = {P.alb.x, P.alb.y, P.alb.z};
            const float f0[3] = {P.f0.x, P.f0.y, P.f0.z};

            if (!(a.flags & SSR_NO_DIRECT)) {
                const int top = a.env_lay.levels - 1;
                const float scale = static_cast<float>(top) * 1.44269504f;
                const float lam_raw = log1pf(P.rho) * scale;
                const bool lam_in = lam_raw > 0.0f && lam_raw < static_cast<float>(top);
                const float lam = fminf(fmaxf(lam_raw, 0.0f), static_cast<float>(top));
                const int k0 = static_cast<int>(floorf(lam));
                const int k1 = min(k0 + 1, top);
                Dual t = dconst(lam - static_cast<float>(k0));
                // d lambda / d rho = scale / (1 + rho)
                t.d[0] = lam_in ? rho.d[0] * scale / (1.0f + P.rho) : 0.0f;
                EnvTaps t0, t1;
                const DualRGB e0 = env_bilinear_dual(env_level(a, k0), n, t0);
                const bool two = t.v > 0.0f;
                DualRGB e1 = e0;
                if (two) e1 = env_bilinear_dual(env_level(a, k1), n, t1);
                float coef0[3], coef1[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    // E = (1 - t) E0 + t E1
                    const float Ev = (1.0f - t.v) * e0.v[c] + t.v * e1.v[c];
                    const float kf = (1.0f - m) * alb[c] * g[c];
#pragma unroll
                    for (int k = 0; k < kDirs; ++k) {
                        const float dE = (1.0f - t.v) * e0.d[c][k] + t.v * e1.d[c][k] +
                                         t.d[k] * (e1.v[c] - e0.v[c]);
                        G[k] += kf * dE;
                    }
                    ga[c] += g[c] * (1.0f - m) * Ev;
                    gm -= g[c] * alb[c] * Ev;
                    coef0[c] = kf * (1.0f - t.v);
                    coef1[c] = kf * t.v;
                }
                add_env(b, a.env_lay.offset[k0], k0, t0, coef0);
                if (two) add_env(b, a.env_lay.offset[k1], k1, t1, coef1);
            }

            if (P.trace) {
                const float invS = 1.0f / static_cast<float>(S);
                // tangent frame and stretched view vector as duals
                const float sign = copysignf(1.0f, n.z.v);
                const Dual ia = dconst(-1.0f) / (sign + n.z);
                const Dual bb = n.x * n.y * ia;
                const DV3 T{1.0f + sign * (n.x * n.x * ia), sign * bb, -sign * n.x};
                const DV3 B{bb, sign + n.y * n.y * ia, -1.0f * n.y};
                const Dual wlx = ddot(T, P.wo), wly = ddot(B, P.wo), cos_no = ddot(n, P.wo);
                const DV3 ws = dnormalize(DV3{rho * wlx, rho * wly, cos_no});
                const Dual a2 = rho * rho;
#pragma unroll 1
                for (int s = 0; s < S; ++s) {
                    int code = b.hits[code_index(a, i, j, s)];
                    if (code >= a.W * a.H || code < SSR_HIT_SKIPPED) code = SSR_HIT_INVALID;
                    if (!(code >= 0 || code == SSR_HIT_OFFSCREEN || code == SSR_HIT_CAP)) continue;
                    const uint4 x = philox4x32_10(
                        make_uint4(static_cast<uint32_t>(q), static_cast<uint32_t>(s), a.frame, 0u),
                        a.key0, a.key1);
                    const float u1 = unit24(x.x), u2 = unit24(x.y);
                    float sphi, cphi;
                    sincos_rev(u1, &sphi, &cphi);
                    // the visible-normal sample, as in the forward (sample_dir)
                    const Dual opz = 1.0f + ws.z;
                    const Dual hz = (1.0f - u2) * opz;
                    const Dual sin2 = (u2 * opz) * (hz + (1.0f + (-1.0f * ws.z)));
                    const Dual st = dsqrt(dmax0(sin2));
                    const DV3 hl = dnormalize(DV3{rho * (cphi * st + ws.x), rho * (sphi * st + ws.y), hz});
                    const DV3 h{hl.x * T.x + hl.y * B.x + hl.z * n.x, hl.x * T.y + hl.y * B.y + hl.z * n.y,
                                hl.x * T.z + hl.y * B.z + hl.z * n.z};
                    const Dual cos_oh = ddot(h, P.wo);
                    const Dual c2 = 2.0f * cos_oh;
                    const DV3 l{c2 * h.x + dconst(-P.wo.x), c2 * h.y + dconst(-P.wo.y),
                                c2 * h.z + dconst(-P.wo.z)};
                    const Dual cos_nl = ddot(n, l);
                    if (!(cos_nl.v > 0.0f)) continue;   // weight 0 (G1 of max(n.l, 0))
                    // Schlick term fr = (1 - wo.h)^5 and Smith G1 with alpha = rho
                    const Dual fc = 1.0f + (-1.0f * cos_oh);
                    const Dual fc2 = fc * fc;
                    const Dual fr = fc2 * fc2 * fc;
                    const Dual z = cos_nl;
                    const Dual g1 = (2.0f * z) / (z + dsqrt(a2 + (1.0f + (-1.0f * a2)) * (z * z)));
                    // radiance along the sample
                    DualRGB L;
                    EnvTaps te;
                    if (code >= 0) {
                        const float3 c1 = Texel4<DT>::load3(a.radiance, code);
                        const float cv[3] = {c1.x, c1.y, c1.z};
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            L.v[c] = cv[c];
#pragma unroll
                            for (int k = 0; k < kDirs; ++k) L.d[c][k] = 0.0f;
                        }
                    } else {
                        L = env_bilinear_dual(env_level(a, 0), l, te);
                    }
                    float coef[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        // contribution F_c G1 L_c with F_c = F0_c + (1 - F0_c) fr
                        const float Fv = f0[c] + (1.0f - f0[c]) * fr.v;
                        const float gs = g[c] * invS;
#pragma unroll
                        for (int k = 0; k < kDirs; ++k) {
                            const float dF = (1.0f - f0[c]) * fr.d[k];
                            G[k] += gs * (dF * g1.v * L.v[c] + Fv * g1.d[k] * L.v[c] + Fv * g1.v * L.d[c][k]);
                        }
                        const float dFdF0 = (1.0f - fr.v) * g1.v * L.v[c];
                        ga[c] += gs * m * dFdF0;
                        gm += gs * (alb[c] - 0.04f) * dFdF0;
                        coef[c] = gs * Fv * g1.v;
                    }
                    if (code >= 0) {
                        if (b.g_rad) {
                            atomicAdd(b.g_rad + 4 * static_cast<int64_t>(code) + 0, coef[0]);
                            atomicAdd(b.g_rad + 4 * static_cast<int64_t>(code) + 1, coef[1]);
                            atomicAdd(b.g_rad + 4 * static_cast<int64_t>(code) + 2, coef[2]);
                        }
                    } else {
                        add_env(b, 0, 0, te, coef);
                    }
                }
            }
            if (b.g_nr)
                reinterpret_cast<float4*>(b.g_nr)[q] = make_float4(G[1], G[2], G[3], G[0]);
            if (b.g_am)
                reinterpret_cast<float4*>(b.g_am)[q] = make_float4(ga[0], ga[1], ga[2], gm * dm);
        }
        if (P.bg) {
            if (b.g_nr) reinterpret_cast<float4*>(b.g_nr)[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (b.g_am) reinterpret_cast<float4*>(b.g_am)[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    }
    // this workgroup's sums of the top levels and of the table's texels, one
    // atomic per texel and channel
    __syncthreads();
    for (int k = threadIdx.x; k < b.priv_texels; k += blockDim.x) {
        const float* p = lds_env + 3 * k;
        if (p[0] != 0.0f || p[1] != 0.0f || p[2] != 0.0f) {
            float* dst = reinterpret_cast<float*>(b.g_mips + b.priv_offset + k);
            atomicAdd(dst + 0, p[0]);
            atomicAdd(dst + 1, p[1]);
            atomicAdd(dst + 2, p[2]);
        }
    }
    for (int k = threadIdx.x; k < kTableSlots; k += blockDim.x) {
        const int texel = lds_tag[k];
        if (texel < 0) continue;
        const float* p = lds_tab + 3 * k;
        float* dst = reinterpret_cast<float*>(b.g_mips + texel);
        atomicAdd(dst + 0, p[0]);
        atomicAdd(dst + 1, p[1]);
        atomicAdd(dst + 2, p[2]);
    }
}

__global__ void zero_kernel(float4* p, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Copy 0 += copies 1..R-1.
__global__ void sum_replicas_kernel(float4* g, int64_t texels, int replicas) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= texels) return;
    float4 acc = g[i];
    for (int r = 1; r < replicas; ++r) {
        const float4 v = g[r * texels + i];
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
    }
    g[i] = acc;
}

// g_env[y][x] += sum over levels k of g_level_k[y >> k][x >> k] / 4^k: level k
// texel is the mean of the 4^k level-0 texels it covers.
__global__ void env_pushdown_kernel(const float4* __restrict__ g_mips, EnvLayout lay,
                                    float* __restrict__ g_env) {
    const int w0 = lay.w[0];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= w0 * lay.h[0]) return;
    const int x = i % w0, y = i / w0;
    float r = 0.0f, g = 0.0f, bl = 0.0f;
    float scale = 1.0f;
    for (int k = 0; k < lay.levels; ++k) {
        const float4 v = g_mips[lay.offset[k] + (y >> k) * lay.w[k] + (x >> k)];
        r += scale * v.x;
        g += scale * v.y;
        bl += scale * v.z;
        scale *= 0.25f;
    }
    g_env[3 * i + 0] += r;
    g_env[3 * i + 1] += g;
    g_env[3 * i + 2] += bl;
}

hipError_t launch_backward(const ShadeArgs& args, const BackwardBuffers& bufs, int dtype,
                           hipStream_t stream) {
    const EnvLayout& el = args.env_lay;
    BackArgs b;
    b.g_out = bufs.grad_rgb;
    b.hits = bufs.hits;
    b.g_nr = bufs.g_normal_rough;
    b.g_am = bufs.g_albedo_metal;
    b.g_mips = bufs.g_mips;
    b.g_rad = bufs.g_radiance;
    // the levels summed in LDS: the smallest top part of the chain that fits
    int first = el.levels;
    int64_t tex = 0;
    while (first > 0) {
        const int64_t t = static_cast<int64_t>(el.w[first - 1]) * el.h[first - 1];
        if (tex + t > kPrivTexels) break;
        tex += t;
        --first;
    }
    b.priv_first = first;
    b.priv_offset = first < el.levels ? static_cast<int>(el.offset[first]) : 0;
    b.priv_texels = static_cast<int>(tex);
    b.replicas = bufs.replicas;
    b.texels = el.total;
    const int64_t all = el.total * bufs.replicas;
    hipLaunchKernelGGL(zero_kernel, dim3(static_cast<unsigned>((all + 255) / 256)), dim3(256), 0,
                       stream, bufs.g_mips, all);
    const dim3 grid(((args.W + 15) / 16) * ((args.H + 15) / 16));
    if (dtype == SSR_F32)
        hipLaunchKernelGGL((backward_kernel<0>), grid, dim3(256), 0, stream, args, b);
    else if (dtype == SSR_F16)
        hipLaunchKernelGGL((backward_kernel<1>), grid, dim3(256), 0, stream, args, b);
    else
        hipLaunchKernelGGL((backward_kernel<2>), grid, dim3(256), 0, stream, args, b);
    if (bufs.g_env) {
        if (bufs.replicas > 1)
            hipLaunchKernelGGL(sum_replicas_kernel, dim3(static_cast<unsigned>((el.total + 255) / 256)),
                               dim3(256), 0, stream, bufs.g_mips, el.total, bufs.replicas);
        const int n0 = el.w[0] * el.h[0];
        hipLaunchKernelGGL(env_pushdown_kernel, dim3((n0 + 255) / 256), dim3(256), 0, stream,
                           bufs.g_mips, el, bufs.g_env);
    }
    return hipGetLastError();
}

}  // namespace ssr
