// Device helpers shared by the shading kernels: counter-based random numbers,
// equirect environment filtering and the GGX microfacet pieces.  Everything
// is float32 (the shading kernels use no float64); where a plain formula would lose
// accuracy that the environment map's contrast turns into visible error, the
// evaluation is rearranged (comments say how) so that it stays exact to a few
// float32 ulps of the sampled direction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssr {

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies whose high halves are mixed with the other counter words and the
// round key; the key advances by two Weyl constants between rounds.
// ----------------------------------------------------------------------------
struct Philox {
    static constexpr uint32_t kMul0 = 0xD2511F53u;
    static constexpr uint32_t kMul1 = 0xCD9E8D57u;
    static constexpr uint32_t kWeyl0 = 0x9E3779B9u;
    static constexpr uint32_t kWeyl1 = 0xBB67AE85u;
};

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += Philox::kWeyl0;
            k1 += Philox::kWeyl1;
        }
        // full 64-bit products: one v_mad_u64_u32 each instead of a
        // separate low and high multiply
        const uint64_t p0 = static_cast<uint64_t>(Philox::kMul0) * c.x;
        const uint64_t p1 = static_cast<uint64_t>(Philox::kMul1) * c.z;
        const uint32_t lo0 = static_cast<uint32_t>(p0), hi0 = static_cast<uint32_t>(p0 >> 32);
        const uint32_t lo1 = static_cast<uint32_t>(p1), hi1 = static_cast<uint32_t>(p1 >> 32);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// sin and cos of 2 pi u (u in revolutions) from the hardware sine and cosine
// units: absolute error at most 1.3e-7 over u = k 2^-24 in [0, 1) (measured
// against float64), a direction error far below the other float32 steps.
__device__ __forceinline__ void sincos_rev(float u, float* s, float* c) {
    *s = __builtin_amdgcn_sinf(u);
    *c = __builtin_amdgcn_cosf(u);
}

// 24 random bits -> [0, 1), a multiple of 2^-24 (exact in float32).
__device__ __forceinline__ float unit24(uint32_t x) {
    return static_cast<float>(x >> 8) * (1.0f / 16777216.0f);
}

// ----------------------------------------------------------------------------
// Small vector helpers.
// ----------------------------------------------------------------------------
struct V3 {
    float x, y, z;
};

__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 normalize(V3 a) {
    // hardware reciprocal square root (about 1 ulp): the scale of a direction,
    // whose error does not turn it
    const float inv = __builtin_amdgcn_rsqf(dot(a, a));
    return inv * a;
}

// ----------------------------------------------------------------------------
// Equirect lookup.  Direction d -> azimuth phi = atan2(d.x, -d.z) in (-pi, pi]
// and polar angle theta = atan2(|d.xz|, d.y) in [0, pi] (the atan2 form keeps
// full accuracy near the poles, where acos(d.y) does not).  Texel coordinate
// x = (W/2 - 1/2) + phi * W/(2 pi), y = theta * H/pi - 1/2.
//
// Near phi = +-pi (the seam, d.z > 0) and theta = pi (the lower pole) a
// float32 angle has an absolute error of an ulp of pi, far more than the
// direction's own.  There the angle is measured from the nearer reference
// instead: for d.z > 0, x = -1/2 - atan2(d.x, d.z) W/(2 pi) (the same
// position modulo W, as the map wraps), and for d.y < 0,
// y = (H - 1/2) - atan2(|d.xz|, -d.y) H/pi.  Both have the derivatives of
// phi and theta.
//
// The products are carried as float-float values: the scale constants come
// in (hi, lo) pairs, the product error is recovered with an FMA and the sum
// with the offset by an exact two-sum, so the fractional texel position is
// accurate to ~1e-7 of a texel instead of the ~1.5e-5 that rounding x itself
// to float32 at magnitude 256 would give.
// ----------------------------------------------------------------------------
struct EnvLevel {
    const float4* texels;  // [h][w] RGBA
    int w, h;
};

struct TexelCoord {
    int i0;     // integer part (outside [0, size) near the edges and, for the
                // other reference angle, the caller wraps or clamps it)
    float f;    // fractional part in [0, 1)
};

__device__ __forceinline__ TexelCoord texel_coord(float ang, float scale_hi, float scale_lo,
                                                  float offset) {
#pragma clang fp contract(off)
    const float t = ang * scale_hi;
    const float te = fmaf(ang, scale_hi, -t) + ang * scale_lo;
    const float x = offset + t;
    const float bp = x - offset;
    const float e = (offset - (x - bp)) + (t - bp);
    const float fl = floorf(x);
    const float fr = (x - fl) + (e + te);
    // the error terms are far below one, so fr lies in (-1, 2) and its floor
    // (-1, 0 or 1) moves the carry into the integer part
    const float c = floorf(fr);
    return TexelCoord{static_cast<int>(fl + c), fr - c};
}

struct EnvAngles {
    float phi, theta;  // measured from the references above
    bool front, low;   // d.z > 0 (from the seam), d.y < 0 (from the lower pole)
};

// atan2(a, b) for b >= 0 (including b = -0), without branches: with
// t = min(|a|, b) / max(|a|, b) in [0, 1], atan(t) = t q(t^2), q the
// degree-9 polynomial fitted (least squares on Chebyshev nodes) to atan(t)/t,
// max error 2e-9 (1e-7 once evaluated in float32); pi/2 - atan(t) when
// |a| > b; the signs of zero follow IEEE atan2 (atan2(+-0, -0) = +-pi).
__device__ __forceinline__ float atan2_right(float a, float b) {
    constexpr float kC[10] = {1.0f,           -0.33333284f,  0.19998230f,   -0.14261574f,
                              0.10940199f,    -0.083720639f, 0.057463557f,  -0.030717509f,
                              0.010680719f,   -0.0017437012f};
    const float aa = fabsf(a);
    const float mx = fmaxf(aa, b), mn = fminf(aa, b);
    const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    const float u = t * t;
    float q = kC[9];
#pragma unroll
    for (int k = 8; k >= 0; --k) q = fmaf(q, u, kC[k]);
    float p = t * q;
    p = aa > b ? 1.57079633f - p : p;
    p = (mx == 0.0f && signbit(b)) ? 3.14159265f : p;
    return copysignf(p, a);
}

__device__ __forceinline__ EnvAngles env_angles(V3 d) {
    const bool front = d.z > 0.0f, low = d.y < 0.0f;
    const float r = __builtin_amdgcn_sqrtf(d.x * d.x + d.z * d.z);
    // (the reference is chosen through the arguments, so that a wave whose
    // lanes look both ways evaluates each arctangent once)
    const float phi = atan2_right(d.x, front ? d.z : -d.z);
    const float theta = atan2_right(r, low ? -d.y : d.y);
    return EnvAngles{front ? -phi : phi, low ? -theta : theta, front, low};
}

// 1/(2 pi) and 1/pi as float-float pairs (hi + lo to ~1e-15).
constexpr float kInv2PiHi = 0x1.45f306p-3f;   // 0.15915494
constexpr float kInv2PiLo = 0x1.b93910p-28f;  // 6.4206382e-09
constexpr float kInvPiHi = 0x1.45f306p-2f;    // 0.31830987
constexpr float kInvPiLo = 0x1.b93910p-27f;   // 1.2841276e-08

// Texel coordinates of the angles in a w x h level.
__device__ __forceinline__ void env_texel(const EnvLevel& lv, const EnvAngles& a, TexelCoord& cx,
                                          TexelCoord& cy) {
    const float wf = static_cast<float>(lv.w);
    const float hf = static_cast<float>(lv.h);
    cx = texel_coord(a.phi, kInv2PiHi * wf, kInv2PiLo * wf, a.front ? -0.5f : 0.5f * wf - 0.5f);
    cy = texel_coord(a.theta, kInvPiHi * hf, kInvPiLo * hf, a.low ? hf - 0.5f : -0.5f);
}

// Columns of the two taps of a bilinear lookup whose integer part is i0 (any
// integer: the map wraps in azimuth) in a level of width w, a power of two,
// so that the masks are i0 mod w and i0 + 1 mod w.
__device__ __forceinline__ void env_columns(int i0, int w, int& x0, int& x1) {
    x0 = i0 & (w - 1);
    x1 = (x0 + 1) & (w - 1);
}

__device__ __forceinline__ float3 env_bilinear(const EnvLevel& lv, EnvAngles a) {
    TexelCoord cx, cy;
    env_texel(lv, a, cx, cy);
    int x0, x1;
    env_columns(cx.i0, lv.w, x0, x1);
    const int y0 = min(max(cy.i0, 0), lv.h - 1);
    const int y1 = min(max(cy.i0 + 1, 0), lv.h - 1);
    // RGB of the four taps (12 B loads from the 16 B texels), at 32-bit byte
    // offsets (a level holds at most 2^27 texels; rows and widths are below
    // 2^24, so the 24-bit multiply is exact)
    const char* base = reinterpret_cast<const char*>(lv.texels);
    const unsigned r0 = __umul24(static_cast<unsigned>(y0), static_cast<unsigned>(lv.w));
    const unsigned r1 = __umul24(static_cast<unsigned>(y1), static_cast<unsigned>(lv.w));
    const float3 t00 = *reinterpret_cast<const float3*>(base + ((r0 + x0) << 4));
    const float3 t01 = *reinterpret_cast<const float3*>(base + ((r0 + x1) << 4));
    const float3 t10 = *reinterpret_cast<const float3*>(base + ((r1 + x0) << 4));
    const float3 t11 = *reinterpret_cast<const float3*>(base + ((r1 + x1) << 4));
    const float fx = cx.f, fy = cy.f;
    const float w00 = (1.0f - fx) * (1.0f - fy), w01 = fx * (1.0f - fy);
    const float w10 = (1.0f - fx) * fy, w11 = fx * fy;
    return make_float3(w00 * t00.x + w01 * t01.x + w10 * t10.x + w11 * t11.x,
                       w00 * t00.y + w01 * t01.y + w10 * t10.y + w11 * t11.y,
                       w00 * t00.z + w01 * t01.z + w10 * t10.z + w11 * t11.z);
}

// Compensated (Kahan) accumulation of one channel: sum + comp carries the
// running total to about one float32 ulp regardless of the sample count.
__device__ __forceinline__ void kahan_add(float& sum, float& comp, float v) {
#pragma clang fp contract(off)
    const float y = v - comp;
    const float t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

// ----------------------------------------------------------------------------
// GGX with alpha = rho (Appendix B as written).
// ----------------------------------------------------------------------------
__device__ __forceinline__ float smith_g1(float z, float a2) {
    // (hardware square root and reciprocal, about 1 ulp each)
    return 2.0f * z * __builtin_amdgcn_rcpf(z + __builtin_amdgcn_sqrtf(a2 + (1.0f - a2) * z * z));
}

// Branchless tangent frame (Duff et al., JCGT 2017); sign(+0) = +1.
__device__ __forceinline__ void onb(V3 n, V3& t, V3& b) {
    const float sign = copysignf(1.0f, n.z);
    // (the hardware reciprocal, about 1 ulp: the frame stays orthonormal to
    // that accuracy; sign + n.z >= 1 in magnitude, so it is never near zero)
    const float a = -__builtin_amdgcn_rcpf(sign + n.z);
    const float bb = n.x * n.y * a;
    t = v3(1.0f + sign * n.x * n.x * a, sign * bb, -sign * n.x);
    b = v3(bb, sign + n.y * n.y * a, -n.y);
}

}  // namespace ssr
