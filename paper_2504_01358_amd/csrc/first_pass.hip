// The first shading pass (Sec. 3.2): depth normals by finite differences, the
// split-sum BRDF table (Appendix C) and the first-pass radiance
// c1 = c_d + c_s that the specular rays of the second pass read at their hits.
#include <hip/hip_fp16.h>

#include "kernels.h"
#include "shading.h"

namespace ssr {

namespace {

constexpr int kTileX = 64;  // one wave per 64 pixels of a row
constexpr int kTileY = 4;

// Store channels 0..2 (and 3 when `all4`) of a [H][W][4] texel in the
// storage type DT (round to nearest even for the 16-bit types).
template <int DT>
struct Store4;

template <>
struct Store4<0> {
    __device__ static void put(void* p, int64_t q, float4 v, bool all4) {
        float* t = reinterpret_cast<float*>(p) + 4 * q;
        if (all4) {
            *reinterpret_cast<float4*>(t) = v;
        } else {
            t[0] = v.x;
            t[1] = v.y;
            t[2] = v.z;
        }
    }
};

template <>
struct Store4<1> {
    __device__ static void put(void* p, int64_t q, float4 v, bool all4) {
        unsigned short* t = reinterpret_cast<unsigned short*>(p) + 4 * q;
        const ushort4 b = make_ushort4(__half_as_ushort(__float2half_rn(v.x)),
                                       __half_as_ushort(__float2half_rn(v.y)),
                                       __half_as_ushort(__float2half_rn(v.z)),
                                       __half_as_ushort(__float2half_rn(v.w)));
        if (all4) {
            *reinterpret_cast<ushort4*>(t) = b;
        } else {
            t[0] = b.x;
            t[1] = b.y;
            t[2] = b.z;
        }
    }
};

template <>
struct Store4<2> {
    // bfloat16 = the high half of a float32, rounded to nearest even (the
    // values here are finite)
    __device__ static unsigned short bf16(float f) {
        const uint32_t u = __float_as_uint(f);
        return static_cast<unsigned short>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
    }
    __device__ static void put(void* p, int64_t q, float4 v, bool all4) {
        unsigned short* t = reinterpret_cast<unsigned short*>(p) + 4 * q;
        const ushort4 b = make_ushort4(bf16(v.x), bf16(v.y), bf16(v.z), bf16(v.w));
        if (all4) {
            *reinterpret_cast<ushort4*>(t) = b;
        } else {
            t[0] = b.x;
            t[1] = b.y;
            t[2] = b.z;
        }
    }
};

// ------------------------------------------------------------ depth normals --

// View-space difference V(a) - V(b) of two pixel points on one row (along x)
// or one column (along y).  V(i, j) = (x_i D, y_j D, D) with
// x_i = (i + 1/2 - cx)/fx and y_j = -(j + 1/2 - cy)/fy; the x part of a row
// difference is written x_a (D_a - D_b) + (x_a - x_b) D_b, so that nothing
// cancels when the two depths are close (the usual case).
__device__ __forceinline__ V3 row_diff(const ShadeArgs& a, float xa, float yj, int da, float Da,
                                       float Db) {
    const float dD = Da - Db;
    return v3(xa * dD + (static_cast<float>(da) / a.fx) * Db, yj * dD, dD);
}

__device__ __forceinline__ V3 col_diff(const ShadeArgs& a, float xi, float ya, int da, float Da,
                                       float Db) {
    const float dD = Da - Db;
    return v3(xi * dD, ya * dD - (static_cast<float>(da) / a.fy) * Db, dD);
}

template <int DT>
__global__ __launch_bounds__(kTileX* kTileY) void depth_normals_kernel(ShadeArgs a, void* out) {
    const int i = blockIdx.x * kTileX + threadIdx.x;
    const int j = blockIdx.y * kTileY + threadIdx.y;
    if (i >= a.W || j >= a.H) return;
    const int64_t q = static_cast<int64_t>(j) * a.W + i;
    const float D = a.depth[q];
    if (!isfinite(D)) {
        Store4<DT>::put(out, q, make_float4(0.0f, 0.0f, 0.0f, 0.0f), false);
        return;
    }
    const float xi = (static_cast<float>(i) + 0.5f - a.cx) / a.fx;
    const float yj = -(static_cast<float>(j) + 0.5f - a.cy) / a.fy;
    // neighbours that are surface pixels inside the image
    const float Dl = i > 0 ? a.depth[q - 1] : INFINITY;
    const float Dr = i + 1 < a.W ? a.depth[q + 1] : INFINITY;
    const float Du = j > 0 ? a.depth[q - a.W] : INFINITY;
    const float Dd = j + 1 < a.H ? a.depth[q + a.W] : INFINITY;
    const bool hl = isfinite(Dl), hr = isfinite(Dr), hu = isfinite(Du), hd = isfinite(Dd);
    // tangents: central where both neighbours are there, else one-sided (the
    // scale of each does not matter, only its direction)
    V3 tx, ty;
    if (hl && hr) {
        tx = row_diff(a, (static_cast<float>(i) + 1.5f - a.cx) / a.fx, yj, 2, Dr, Dl);
    } else if (hr) {
        tx = row_diff(a, (static_cast<float>(i) + 1.5f - a.cx) / a.fx, yj, 1, Dr, D);
    } else {
        tx = row_diff(a, xi, yj, 1, D, Dl);
    }
    if (hu && hd) {
        ty = col_diff(a, xi, -(static_cast<float>(j) + 1.5f - a.cy) / a.fy, 2, Dd, Du);
    } else if (hd) {
        ty = col_diff(a, xi, -(static_cast<float>(j) + 1.5f - a.cy) / a.fy, 1, Dd, D);
    } else {
        ty = col_diff(a, xi, yj, 1, D, Du);
    }
    const V3 V = v3(xi * D, yj * D, D);
    V3 n = v3(tx.y * ty.z - tx.z * ty.y, tx.z * ty.x - tx.x * ty.z, tx.x * ty.y - tx.y * ty.x);
    const float len2 = dot(n, n);
    if (!((hl || hr) && (hu || hd) && len2 > 0.0f)) n = -1.0f * V;  // toward the camera
    if (dot(n, V) > 0.0f) n = -1.0f * n;                             // face the camera
    // (rows of the rotation are orthonormal: the cross product commutes with it)
    const V3 w = normalize(view_to_world(a, n.x, n.y, n.z));
    Store4<DT>::put(out, q, make_float4(w.x, w.y, w.z, 0.0f), false);
}

// --------------------------------------------------------- split-sum table --

// One workgroup per table entry; each lane takes 16 of the K x K stratified
// visible-normal samples.  The table is computed once per context, so it is
// evaluated in float64: its entries are the float32 roundings of the
// float64 means.
constexpr int kLutThreads = 256;

__global__ __launch_bounds__(kLutThreads) void brdf_lut_kernel(float2* lut, int n, int k) {
    const int e = blockIdx.x;
    const int ri = e / n, mi = e % n;
    const double rho = (ri + 0.5) / n;
    const double mu = (mi + 0.5) / n;
    const double wx = sqrt(1.0 - mu * mu), wz = mu;  // wo in the tangent frame (wo.y = 0)
    // stretched view vector of the visible-normal sampler (Dupuy & Benyoub 2023)
    const double sx = rho * wx, sz = wz;
    const double sl = sqrt(sx * sx + sz * sz);
    const double vx = sx / sl, vz = sz / sl;
    double sa = 0.0, sb = 0.0;
    for (int s = threadIdx.x; s < k * k; s += kLutThreads) {
        const double u1 = (s / k + 0.5) / k;
        const double u2 = (s % k + 0.5) / k;
        double sphi, cphi;
        sincospi(2.0 * u1, &sphi, &cphi);
        const double z = (1.0 - u2) * (1.0 + vz) - vz;
        const double st = sqrt(fmin(fmax(1.0 - z * z, 0.0), 1.0));
        const double hx0 = rho * (st * cphi + vx), hy0 = rho * (st * sphi), hz0 = z + vz;
        const double hl = sqrt(hx0 * hx0 + hy0 * hy0 + hz0 * hz0);
        const double hx = hx0 / hl, hz = hz0 / hl;
        const double coh = hx * wx + hz * wz;
        const double lz = 2.0 * coh * hz - wz;  // n.l
        if (lz > 0.0) {
            const double a2 = rho * rho;
            const double g1 = 2.0 * lz / (lz + sqrt(a2 + (1.0 - a2) * lz * lz));
            const double c = 1.0 - coh;
            const double fc = c * c * c * c * c;
            sa += (1.0 - fc) * g1;
            sb += fc * g1;
        }
    }
    // wave64 reduction, then across the four waves
    for (int off = 32; off > 0; off >>= 1) {
        sa += __shfl_xor(sa, off);
        sb += __shfl_xor(sb, off);
    }
    __shared__ double part[2][kLutThreads / 64];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        part[0][wave] = sa;
        part[1][wave] = sb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
        for (int w = 0; w < kLutThreads / 64; ++w) {
            ta += part[0][w];
            tb += part[1][w];
        }
        const double inv = 1.0 / (static_cast<double>(k) * k);
        lut[e] = make_float2(static_cast<float>(ta * inv), static_cast<float>(tb * inv));
    }
}

// ------------------------------------------------------------ first pass --

// Bilinear read of the table at (n.v, rho): texel centres at (i + 1/2)/n,
// clamped to the edges.
__device__ __forceinline__ float2 lut_read(const float2* lut, int n, float mu, float rho) {
    const float fn = static_cast<float>(n);
    const float x = fminf(fmaxf(mu * fn - 0.5f, 0.0f), fn - 1.0f);
    const float y = fminf(fmaxf(rho * fn - 0.5f, 0.0f), fn - 1.0f);
    const int x0 = min(static_cast<int>(floorf(x)), n - 2);
    const int y0 = min(static_cast<int>(floorf(y)), n - 2);
    const float fx = x - static_cast<float>(x0), fy = y - static_cast<float>(y0);
    const float2 t00 = lut[y0 * n + x0], t01 = lut[y0 * n + x0 + 1];
    const float2 t10 = lut[(y0 + 1) * n + x0], t11 = lut[(y0 + 1) * n + x0 + 1];
    const float w00 = (1.0f - fx) * (1.0f - fy), w01 = fx * (1.0f - fy);
    const float w10 = (1.0f - fx) * fy, w11 = fx * fy;
    return make_float2(w00 * t00.x + w01 * t01.x + w10 * t10.x + w11 * t11.x,
                       w00 * t00.y + w01 * t01.y + w10 * t10.y + w11 * t11.y);
}

template <int DT>
__global__ __launch_bounds__(kTileX* kTileY) void first_pass_kernel(ShadeArgs a, const float2* lut,
                                                                   int n, void* out) {
    const int i = blockIdx.x * kTileX + threadIdx.x;
    const int j = blockIdx.y * kTileY + threadIdx.y;
    if (i >= a.W || j >= a.H) return;
    const int64_t q = static_cast<int64_t>(j) * a.W + i;
    const Pixel P = setup_pixel<DT>(a, i, j, q);
    if (P.bg) {
        Store4<DT>::put(out, q, make_float4(0.0f, 0.0f, 0.0f, 0.0f), true);
        return;
    }
    const float lam = roughness_lod(a, P.rho);
    // c_d = (1 - m) a E_lambda(n)
    const float3 en = env_lod(a, env_angles(P.n), lam);
    const float kd = 1.0f - P.m;
    float3 c = make_float3(kd * P.alb.x * en.x, kd * P.alb.y * en.y, kd * P.alb.z * en.z);
    // c_s = E_lambda(r) (F0 A + B), r the mirror direction; nothing when n.v <= 0
    if (P.cos_no > 0.0f) {
        const V3 r = (2.0f * P.cos_no) * P.n - P.wo;
        const float3 er = env_lod(a, env_angles(r), lam);
        const float2 ab = lut_read(lut, n, fminf(P.cos_no, 1.0f), P.rho);
        c.x += er.x * (P.f0.x * ab.x + ab.y);
        c.y += er.y * (P.f0.y * ab.x + ab.y);
        c.z += er.z * (P.f0.z * ab.x + ab.y);
    }
    Store4<DT>::put(out, q, make_float4(c.x, c.y, c.z, 0.0f), true);
}

dim3 pixel_grid(int W, int H) {
    return dim3(static_cast<unsigned>((W + kTileX - 1) / kTileX),
                static_cast<unsigned>((H + kTileY - 1) / kTileY));
}

}  // namespace

#define SSR_DISPATCH(DTYPE, LAUNCH)         \
    do {                                    \
        if ((DTYPE) == SSR_F32) LAUNCH(0);  \
        else if ((DTYPE) == SSR_F16) LAUNCH(1); \
        else LAUNCH(2);                     \
    } while (0)

hipError_t launch_depth_normals(const ShadeArgs& a, int dtype, void* out, hipStream_t stream) {
#define SSR_LAUNCH(DT) \
    depth_normals_kernel<DT><<<pixel_grid(a.W, a.H), dim3(kTileX, kTileY), 0, stream>>>(a, out)
    SSR_DISPATCH(dtype, SSR_LAUNCH);
#undef SSR_LAUNCH
    return hipGetLastError();
}

hipError_t launch_brdf_lut(float2* lut, int n, int k, hipStream_t stream) {
    brdf_lut_kernel<<<n * n, kLutThreads, 0, stream>>>(lut, n, k);
    return hipGetLastError();
}

hipError_t launch_first_pass(const ShadeArgs& a, int dtype, const float2* lut, int n, void* out,
                             hipStream_t stream) {
#define SSR_LAUNCH(DT)                                                                \
    first_pass_kernel<DT><<<pixel_grid(a.W, a.H), dim3(kTileX, kTileY), 0, stream>>>( \
        a, lut, n, out)
    SSR_DISPATCH(dtype, SSR_LAUNCH);
#undef SSR_LAUNCH
    return hipGetLastError();
}

#undef SSR_DISPATCH

}  // namespace ssr
