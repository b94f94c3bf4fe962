// The shading kernel: one thread per pixel, all of that pixel's samples.
//
// Per pixel (Sec. 3.2 and Sec. 3.3):
//   load the G-buffer, un-project the pixel centre, wo = toward the camera;
//   c_d = (1 - m) a E_lambda(n), lambda = log2(1 + rho) lambda_max;
//   for each sample: Philox(q, s, frame, 0) -> (u1, u2); visible-normal GGX
//   half vector h; l = reflect(-wo, h); march l in screen space; radiance at
//   the hit pixel (c1) or, if the ray left the screen or ran out of
//   iterations, the environment at l; weight F(wo.h) G1(n.l);
//   Kahan-accumulate weight * radiance;
//   out = c_d + sum / S.
//
// The two marches implement the hit rule the library documents: a sample
// point (linear) or a pixel crossing (hierarchical) hits when the ray lies in
// the slab [D, D + thickness] behind the depth buffer after having been in
// front of it at some earlier point outside the origin pixel.
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
};

template <>
struct Texel4<1> {  // float16
    __device__ static float4 load(const void* p, int64_t i) {
        const ushort4 b = reinterpret_cast<const ushort4*>(p)[i];
        return make_float4(__half2float(__ushort_as_half(b.x)), __half2float(__ushort_as_half(b.y)),
                           __half2float(__ushort_as_half(b.z)), __half2float(__ushort_as_half(b.w)));
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
};

__device__ __forceinline__ EnvLevel env_level(const ShadeArgs& a, int k) {
    return EnvLevel{a.env + a.env_lay.offset[k], a.env_lay.w[k], a.env_lay.h[k]};
}

__device__ __forceinline__ V3 view_to_world(const ShadeArgs& a, float X, float Y, float Z) {
    return v3(X * a.right[0] + Y * a.up[0] + Z * a.fwd[0], X * a.right[1] + Y * a.up[1] + Z * a.fwd[1],
              X * a.right[2] + Y * a.up[2] + Z * a.fwd[2]);
}

// ------------------------------------------------------------- marches --

struct MarchResult {
    int code;
    int iters;
};

// Fixed world-space steps (Appendix D, Algorithm 1, with the documented hit
// rule).  V0 view-space origin, Dv view-space direction.
__device__ __forceinline__ MarchResult march_linear(const ShadeArgs& a, int i, int j, V3 V0, V3 Dv) {
    bool armed = false;
    for (int k = 1; k <= a.linear_samples; ++k) {
        const float t = static_cast<float>(k) * a.step_len;
        const float X = V0.x + t * Dv.x, Y = V0.y + t * Dv.y, Z = V0.z + t * Dv.z;
        if (!(Z > a.z_near)) return MarchResult{SSR_HIT_OFFSCREEN, k};
        const float px = a.cx + a.fx * X / Z;
        const float py = a.cy - a.fy * Y / Z;
        if (!(px >= 0.0f && px < static_cast<float>(a.W) && py >= 0.0f &&
              py < static_cast<float>(a.H)))
            return MarchResult{SSR_HIT_OFFSCREEN, k};
        const int ix = min(static_cast<int>(floorf(px)), a.W - 1);
        const int iy = min(static_cast<int>(floorf(py)), a.H - 1);
        if (ix == i && iy == j) continue;
        const float dz = Z - a.depth[static_cast<int64_t>(iy) * a.W + ix];
        if (armed && dz >= 0.0f && dz <= a.thickness) return MarchResult{iy * a.W + ix, k};
        if (dz < 0.0f) armed = true;
    }
    return MarchResult{SSR_HIT_CAP, a.linear_samples};
}

// Exact first hit on the depth heightfield, hierarchical over the min
// pyramid.  The ray is clipped at max_dist and the near plane and projected
// to the screen segment P0 + s dP; its depth 1/(iz0 + s (iz1 - iz0)) is
// monotone in s.  Each iteration skips the current level-L cell (ray in
// front of the cell's minimum depth) and goes up a level, or goes down a
// level, or tests one level-0 pixel.
__device__ __forceinline__ MarchResult march_hiz(const ShadeArgs& a, int i, int j, V3 V0, V3 Dv) {
    float t_end = a.max_dist;
    if (Dv.z < 0.0f) t_end = fminf(t_end, (a.z_near - V0.z) / Dv.z);
    if (!(t_end > 0.0f)) return MarchResult{SSR_HIT_OFFSCREEN, 0};
    const float EX = V0.x + t_end * Dv.x, EY = V0.y + t_end * Dv.y, EZ = V0.z + t_end * Dv.z;
    const float P0x = static_cast<float>(i) + 0.5f, P0y = static_cast<float>(j) + 0.5f;
    const float dPx = (a.cx + a.fx * EX / EZ) - P0x;
    const float dPy = (a.cy - a.fy * EY / EZ) - P0y;
    const float Wf = static_cast<float>(a.W), Hf = static_cast<float>(a.H);
    float s_max = 1.0f;
    if (dPx > 0.0f) s_max = fminf(s_max, (Wf - P0x) / dPx);
    if (dPx < 0.0f) s_max = fminf(s_max, (0.0f - P0x) / dPx);
    if (dPy > 0.0f) s_max = fminf(s_max, (Hf - P0y) / dPy);
    if (dPy < 0.0f) s_max = fminf(s_max, (0.0f - P0y) / dPy);
    const float iz0 = 1.0f / V0.z;
    const float diz = 1.0f / EZ - iz0;
    const int top = a.hiz_lay.levels - 1;

    float s = 0.0f, d_in = V0.z;
    int L = 0, ix = i, iy = j;
    bool armed = false;
    for (int it = 1; it <= a.max_steps; ++it) {
        const int cx0 = (ix >> L) << L, cy0 = (iy >> L) << L;
        const int cx1 = min(cx0 + (1 << L), a.W), cy1 = min(cy0 + (1 << L), a.H);
        float sx = INFINITY, sy = INFINITY;
        if (dPx > 0.0f) sx = (static_cast<float>(cx1) - P0x) / dPx;
        if (dPx < 0.0f) sx = (static_cast<float>(cx0) - P0x) / dPx;
        if (dPy > 0.0f) sy = (static_cast<float>(cy1) - P0y) / dPy;
        if (dPy < 0.0f) sy = (static_cast<float>(cy0) - P0y) / dPy;
        const float s_exit = fminf(fminf(sx, sy), s_max);
        const float d_out = 1.0f / (iz0 + s_exit * diz);
        const float hi = fmaxf(d_in, d_out), lo = fminf(d_in, d_out);
        const float zc = (L == 0)
                             ? a.depth[static_cast<int64_t>(iy) * a.W + ix]
                             : a.hiz[a.hiz_lay.offset[L] +
                                     static_cast<int64_t>(iy >> L) * a.hiz_lay.w[L] + (ix >> L)];
        bool advance;
        if (hi < zc) {
            if (s_exit > s) armed = true;
            advance = true;
        } else if (L > 0) {
            --L;
            advance = false;
        } else if (ix == i && iy == j) {
            advance = true;
        } else {
            if (lo <= zc + a.thickness && (armed || d_in < zc))
                return MarchResult{iy * a.W + ix, it};
            if (lo < zc) armed = true;
            advance = true;
        }
        if (advance) {
            if (s_exit >= s_max) return MarchResult{SSR_HIT_OFFSCREEN, it};
            int nx, ny;
            if (sx == s_exit) {
                nx = dPx > 0.0f ? cx1 : cx0 - 1;
            } else {
                const float px = P0x + s_exit * dPx;
                nx = min(max(static_cast<int>(floorf(px)), cx0), cx1 - 1);
            }
            if (sy == s_exit) {
                ny = dPy > 0.0f ? cy1 : cy0 - 1;
            } else {
                const float py = P0y + s_exit * dPy;
                ny = min(max(static_cast<int>(floorf(py)), cy0), cy1 - 1);
            }
            if (nx < 0 || nx >= a.W || ny < 0 || ny >= a.H) return MarchResult{SSR_HIT_OFFSCREEN, it};
            ix = nx;
            iy = ny;
            s = s_exit;
            d_in = d_out;
            L = min(L + 1, top);
        }
    }
    return MarchResult{SSR_HIT_CAP, a.max_steps};
}

// ------------------------------------------------------------- kernel --

// Workgroups of 256 threads shade 16 x 16 pixel tiles; each wave64 takes an
// 8 x 8 quadrant so that its rays start close together on the screen.
template <int DT, int MARCH>
__global__ __launch_bounds__(256) void shade_kernel(const ShadeArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
    const int j = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
    if (i >= a.W || j >= a.H) return;
    const int64_t q = static_cast<int64_t>(j) * a.W + i;
    const int S = a.spp;
    const float D = a.depth[q];

    if (!(D < INFINITY)) {
        // background: the environment seen directly
        const V3 d = normalize(view_to_world(a, (static_cast<float>(i) + 0.5f - a.cx) / a.fx,
                                             -(static_cast<float>(j) + 0.5f - a.cy) / a.fy, 1.0f));
        const float3 e = env_bilinear(env_level(a, 0), env_angles(d));
        a.out[3 * q + 0] = e.x;
        a.out[3 * q + 1] = e.y;
        a.out[3 * q + 2] = e.z;
        for (int s = 0; s < S; ++s) {
            if (a.hits) a.hits[q * S + s] = SSR_HIT_BACKGROUND;
            if (a.steps) a.steps[q * S + s] = 0;
        }
        return;
    }

    const float4 nr = Texel4<DT>::load(a.normal_rough, q);
    const float4 am = Texel4<DT>::load(a.albedo_metal, q);
    const float X0 = (static_cast<float>(i) + 0.5f - a.cx) * D / a.fx;
    const float Y0 = -(static_cast<float>(j) + 0.5f - a.cy) * D / a.fy;
    const V3 wo = -1.0f * normalize(view_to_world(a, X0, Y0, D));
    const V3 n = normalize(v3(nr.x, nr.y, nr.z));
    const float rho = fminf(fmaxf(nr.w, 0.0f), 1.0f);
    const float m = fminf(fmaxf(am.w, 0.0f), 1.0f);
    const V3 alb = v3(am.x, am.y, am.z);
    const V3 f0 = v3(0.04f * (1.0f - m) + alb.x * m, 0.04f * (1.0f - m) + alb.y * m,
                     0.04f * (1.0f - m) + alb.z * m);

    float3 cd = make_float3(0.0f, 0.0f, 0.0f);
    if (!(a.flags & SSR_NO_DIRECT)) {
        const int top = a.env_lay.levels - 1;
        const float lam = fminf(fmaxf(log2f(rho + 1.0f) * static_cast<float>(top), 0.0f),
                                static_cast<float>(top));
        const int k0 = static_cast<int>(floorf(lam));
        const int k1 = min(k0 + 1, top);
        const float t = lam - static_cast<float>(k0);
        const EnvAngles ang = env_angles(n);
        const float3 e0 = env_bilinear(env_level(a, k0), ang);
        float3 e = e0;
        if (t > 0.0f) {
            const float3 e1 = env_bilinear(env_level(a, k1), ang);
            e = make_float3((1.0f - t) * e0.x + t * e1.x, (1.0f - t) * e0.y + t * e1.y,
                            (1.0f - t) * e0.z + t * e1.z);
        }
        cd = make_float3((1.0f - m) * alb.x * e.x, (1.0f - m) * alb.y * e.y,
                         (1.0f - m) * alb.z * e.z);
    }

    float sum_r = 0.0f, sum_g = 0.0f, sum_b = 0.0f;
    float cmp_r = 0.0f, cmp_g = 0.0f, cmp_b = 0.0f;
    const float cos_no = dot(n, wo);
    const bool trace = !(a.flags & SSR_NO_SPECULAR) && cos_no > 0.0f;
    const int fill = (a.flags & SSR_NO_SPECULAR) ? SSR_HIT_SKIPPED : SSR_HIT_INVALID;
    if (trace) {
        V3 t, b;
        onb(n, t, b);
        const V3 wl = v3(dot(wo, t), dot(wo, b), cos_no);
        // visible-normal sampling (Dupuy & Benyoub 2023): stretched view vector
        const V3 ws = normalize(v3(rho * wl.x, rho * wl.y, wl.z));
        const float a2 = rho * rho;
        const V3 V0 = v3(X0, Y0, D);
        for (int s = 0; s < S; ++s) {
            const uint4 x = philox4x32_10(
                make_uint4(static_cast<uint32_t>(q), static_cast<uint32_t>(s), a.frame, 0u), a.key0,
                a.key1);
            const float u1 = unit24(x.x), u2 = unit24(x.y);
            // point on the spherical cap z > -ws.z: azimuth 2 pi u1, height from u2.
            // h_std.z = z + ws.z = (1 - u2)(1 + ws.z) and 1 - z^2 = (1 - z)(1 + z) with
            // 1 - z = u2 (1 + ws.z), 1 + z = (1 - u2)(1 + ws.z) + (1 - ws.z): no cancellation.
            float sphi, cphi;
            sincospif(2.0f * u1, &sphi, &cphi);
            const float one_m_u2 = 1.0f - u2;
            const float opz = 1.0f + ws.z;
            const float hz = one_m_u2 * opz;
            const float sin2 = (u2 * opz) * (hz + (1.0f - ws.z));
            const float st = sqrtf(fmaxf(sin2, 0.0f));
            const V3 hl = normalize(v3(rho * (st * cphi + ws.x), rho * (st * sphi + ws.y), hz));
            const V3 h = v3(hl.x * t.x + hl.y * b.x + hl.z * n.x, hl.x * t.y + hl.y * b.y + hl.z * n.y,
                            hl.x * t.z + hl.y * b.z + hl.z * n.z);
            const float cos_oh = dot(wo, h);
            const V3 l = (2.0f * cos_oh) * h - wo;
            const float cos_nl = dot(n, l);
            int code = SSR_HIT_INVALID, iters = 0;
            if (cos_nl > 0.0f) {
                const V3 Dv = v3(dot(l, v3(a.right[0], a.right[1], a.right[2])),
                                 dot(l, v3(a.up[0], a.up[1], a.up[2])),
                                 dot(l, v3(a.fwd[0], a.fwd[1], a.fwd[2])));
                const MarchResult r = MARCH == 0 ? march_linear(a, i, j, V0, Dv)
                                                 : march_hiz(a, i, j, V0, Dv);
                code = r.code;
                iters = r.iters;
                float3 Lr;
                if (code >= 0) {
                    const float4 c1 = Texel4<DT>::load(a.radiance, code);
                    Lr = make_float3(c1.x, c1.y, c1.z);
                } else {
                    Lr = env_bilinear(env_level(a, 0), env_angles(l));
                }
                const float fc = 1.0f - cos_oh;
                const float fc2 = fc * fc;
                const float fr = fc2 * fc2 * fc;
                const float g1 = smith_g1(cos_nl, a2);
                kahan_add(sum_r, cmp_r, (f0.x + (1.0f - f0.x) * fr) * g1 * Lr.x);
                kahan_add(sum_g, cmp_g, (f0.y + (1.0f - f0.y) * fr) * g1 * Lr.y);
                kahan_add(sum_b, cmp_b, (f0.z + (1.0f - f0.z) * fr) * g1 * Lr.z);
            }
            if (a.hits) a.hits[q * S + s] = code;
            if (a.steps) a.steps[q * S + s] = iters;
        }
    } else {
        for (int s = 0; s < S; ++s) {
            if (a.hits) a.hits[q * S + s] = fill;
            if (a.steps) a.steps[q * S + s] = 0;
        }
    }
    const float invS = 1.0f / static_cast<float>(S);
    a.out[3 * q + 0] = cd.x + sum_r * invS;
    a.out[3 * q + 1] = cd.y + sum_g * invS;
    a.out[3 * q + 2] = cd.z + sum_b * invS;
}

hipError_t launch_shade(const ShadeArgs& args, int dtype, int march, hipStream_t stream) {
    const dim3 grid((args.W + 15) / 16, (args.H + 15) / 16);
    const dim3 block(256);
#define SSR_LAUNCH(DT, MR) \
    hipLaunchKernelGGL((shade_kernel<DT, MR>), grid, block, 0, stream, args)
    if (march == 0) {
        if (dtype == 0) SSR_LAUNCH(0, 0);
        else if (dtype == 1) SSR_LAUNCH(1, 0);
        else SSR_LAUNCH(2, 0);
    } else {
        if (dtype == 0) SSR_LAUNCH(0, 1);
        else if (dtype == 1) SSR_LAUNCH(1, 1);
        else SSR_LAUNCH(2, 1);
    }
#undef SSR_LAUNCH
    return hipGetLastError();
}

}  // namespace ssr
