// Builders for the two pyramids the shading kernel reads:
//  * the environment mip chain (Sec. 3.2, SampleEnvMap at level lambda):
//    level k is the 2x2 box mean of level k-1;
//  * the depth pyramid used by the hierarchical march, kept in inverse depth
//    over the hit slab [D, D + thickness] of each pixel: a level-0 texel is
//    (1/D, 1/(D + thickness)), the near and the far side of the slab, and a
//    level-L texel holds the maximum of the first and the minimum of the
//    second over its (up to four) level L-1 children (that is, one over the
//    minimum depth and one over the maximum depth plus thickness of the
//    pixels it covers), ceil-halving to 1 x 1.  A background pixel
//    (D = +inf) has inverse depth 0 on both sides.
#include "device_math.h"
#include "kernels.h"

namespace ssr {

bool make_env_layout(int w, int h, EnvLayout* out) {
    if (h < 1 || h > 8192 || (h & (h - 1)) != 0 || w != 2 * h) return false;
    int levels = 0;
    int64_t off = 0;
    for (int k = 0;; ++k) {
        out->w[k] = w >> k;
        out->h[k] = h >> k;
        out->offset[k] = off;
        off += static_cast<int64_t>(out->w[k]) * out->h[k];
        levels = k + 1;
        if (out->h[k] == 1) break;
    }
    out->levels = levels;
    out->total = off;
    return true;
}

bool make_hiz_layout(int w, int h, HizLayout* out) {
    if (w < 1 || h < 1 || w > 16384 || h > 16384) return false;
    int lw = w, lh = h, L = 0;
    int64_t off = 0;
    for (;;) {
        out->w[L] = lw;
        out->h[L] = lh;
        out->offset[L] = static_cast<int>(off);
        off += static_cast<int64_t>(lw) * ((lh + 1) & ~1);   // rows in pairs
        if (lw == 1 && lh == 1) break;
        lw = (lw + 1) / 2;
        lh = (lh + 1) / 2;
        ++L;
    }
    out->levels = L + 1;
    out->total = off;
    // the march addresses texels with 32-bit byte offsets
    return off * static_cast<int64_t>(sizeof(float4)) <= (int64_t(1) << 32) - 16;
}

// ---------------------------------------------------------------- env mips --

__global__ void env_level0_kernel(const float* __restrict__ rgb, float4* __restrict__ dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = make_float4(rgb[3 * i + 0], rgb[3 * i + 1], rgb[3 * i + 2], 0.0f);
}

__global__ void env_down_kernel(const float4* __restrict__ src, float4* __restrict__ dst, int sw,
                                int dw, int dh) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dw * dh) return;
    const int x = i % dw, y = i / dw;
    const float4 a = src[(2 * y) * sw + 2 * x], b = src[(2 * y) * sw + 2 * x + 1];
    const float4 c = src[(2 * y + 1) * sw + 2 * x], d = src[(2 * y + 1) * sw + 2 * x + 1];
    dst[i] = make_float4(((a.x + b.x) + (c.x + d.x)) * 0.25f, ((a.y + b.y) + (c.y + d.y)) * 0.25f,
                         ((a.z + b.z) + (c.z + d.z)) * 0.25f, 0.0f);
}

// Box mean of four texels: the two of row 2y (a, b) and the two of row
// 2y + 1 (c, d), summed in that order (the same arithmetic in every pass).
__device__ __forceinline__ float4 box4(float4 a, float4 b, float4 c, float4 d) {
    return make_float4(((a.x + b.x) + (c.x + d.x)) * 0.25f, ((a.y + b.y) + (c.y + d.y)) * 0.25f,
                       ((a.z + b.z) + (c.z + d.z)) * 0.25f, 0.0f);
}

// Levels 0..5 of a 32 x 32 texel tile of the map (the map is at least 64 x 32,
// a power of two in each direction, so tiles never cross its edge): each of
// the 256 threads converts a 2 x 2 block and writes its level-1 mean, and
// the 16 x 16 level-1 texels go through LDS for levels 2..5.  Every texel is
// the same box mean of the same four values as in the level-by-level pass.
constexpr int kEnvTile = 32;
__global__ __launch_bounds__(256) void env_tile_kernel(const float* __restrict__ rgb,
                                                       float4* __restrict__ mips, EnvLayout lay) {
    __shared__ float4 lds[2][16 * 16];
    const int W = lay.w[0];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int x0 = blockIdx.x * kEnvTile + 2 * tx, y0 = blockIdx.y * kEnvTile + 2 * ty;
    float4 t[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const float* row = rgb + 3 * (static_cast<int64_t>(y0 + r) * W + x0);
#pragma unroll
        for (int c = 0; c < 2; ++c) t[r][c] = make_float4(row[3 * c], row[3 * c + 1], row[3 * c + 2], 0.0f);
        float4* dst = mips + static_cast<int64_t>(y0 + r) * W + x0;
        dst[0] = t[r][0];
        dst[1] = t[r][1];
    }
    const float4 m1 = box4(t[0][0], t[0][1], t[1][0], t[1][1]);
    mips[lay.offset[1] + static_cast<int64_t>(y0 / 2) * lay.w[1] + x0 / 2] = m1;
    lds[0][ty * 16 + tx] = m1;
    int n = 16, cur = 0;
    for (int L = 2; L <= 5; ++L) {
        __syncthreads();
        const int m = n / 2;
        if (static_cast<int>(threadIdx.x) < m * m) {
            const int a = threadIdx.x % m, b = threadIdx.x / m;
            const float4* src = lds[cur];
            const float4 v = box4(src[(2 * b) * n + 2 * a], src[(2 * b) * n + 2 * a + 1],
                                  src[(2 * b + 1) * n + 2 * a], src[(2 * b + 1) * n + 2 * a + 1]);
            lds[cur ^ 1][b * m + a] = v;
            const int lx = blockIdx.x * (kEnvTile >> L) + a, ly = blockIdx.y * (kEnvTile >> L) + b;
            mips[lay.offset[L] + static_cast<int64_t>(ly) * lay.w[L] + lx] = v;
        }
        cur ^= 1;
        n = m;
    }
}

// The levels from `first` up, in one workgroup, through LDS (level first-1
// holds at most kEnvTopTexels texels).
constexpr int kEnvTopTexels = 2048;
__global__ __launch_bounds__(1024) void env_top_kernel(float4* __restrict__ mips, EnvLayout lay,
                                                       int first) {
    __shared__ float4 buf[kEnvTopTexels + kEnvTopTexels / 4];
    const int sw0 = lay.w[first - 1], sh0 = lay.h[first - 1];
    float4* a = buf;
    float4* b = buf + sw0 * sh0;
    for (int i = threadIdx.x; i < sw0 * sh0; i += blockDim.x) a[i] = mips[lay.offset[first - 1] + i];
    for (int L = first; L < lay.levels; ++L) {
        __syncthreads();
        const int sw = lay.w[L - 1], dw = lay.w[L], dh = lay.h[L];
        for (int i = threadIdx.x; i < dw * dh; i += blockDim.x) {
            const int x = i % dw, y = i / dw;
            const float4 v = box4(a[(2 * y) * sw + 2 * x], a[(2 * y) * sw + 2 * x + 1],
                                  a[(2 * y + 1) * sw + 2 * x], a[(2 * y + 1) * sw + 2 * x + 1]);
            b[i] = v;
            mips[lay.offset[L] + i] = v;
        }
        float4* tmp = a;
        a = b;
        b = tmp;
    }
}

hipError_t launch_env_mips(const float* rgb, const EnvLayout& lay, float4* mips,
                           hipStream_t stream) {
    int next = 1;   // the first level the passes below still have to build
    if (lay.h[0] >= kEnvTile) {
        // levels 0..5 by tiles, then the top in one workgroup when it is small
        hipLaunchKernelGGL(env_tile_kernel, dim3(lay.w[0] / kEnvTile, lay.h[0] / kEnvTile), dim3(256),
                           0, stream, rgb, mips, lay);
        next = 6;
        if (next < lay.levels && lay.w[next - 1] * lay.h[next - 1] <= kEnvTopTexels) {
            hipLaunchKernelGGL(env_top_kernel, dim3(1), dim3(1024), 0, stream, mips, lay, next);
            next = lay.levels;
        }
    } else {
        const int n0 = lay.w[0] * lay.h[0];
        hipLaunchKernelGGL(env_level0_kernel, dim3((n0 + 255) / 256), dim3(256), 0, stream, rgb,
                           mips, n0);
    }
    for (int k = next; k < lay.levels; ++k) {
        const int n = lay.w[k] * lay.h[k];
        hipLaunchKernelGGL(env_down_kernel, dim3((n + 255) / 256), dim3(256), 0, stream,
                           mips + lay.offset[k - 1], mips + lay.offset[k], lay.w[k - 1], lay.w[k],
                           lay.h[k]);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ Hi-Z pyramid --
//
// Pass 1: one 256-thread workgroup per 32 x 32 depth tile writes levels 0..5
// of that tile.  Each thread reduces a 2 x 2 pixel block to its
// (1/D, 1/(D + thickness)) level-0 pairs and one level-1 texel in
// registers; levels 2..4 are wave reductions across lanes, level 5 joins
// the four waves through LDS (see hiz_tile_kernel).
// (Small blocks give eight waves per SIMD at 1080p, enough to cover the
// latency of the depth loads; 4 x 4 blocks ran at two and took 25 % longer.)
// A texel at level L is the (max, min) of those pairs over the
// 2^L x 2^L pixel block it covers, clipped to the image (pixels outside
// count as -inf for the max and +inf for the min), which equals the
// ceil-halving recursion.  Texels that do not exist at their level
// (index >= W_L or H_L) are not written.  Both quotients are correctly
// rounded and rounding is monotone, so a texel equals the rounded inverse of
// the block's minimum depth and of its maximum (depth + thickness) exactly.
//
// Pass 2: the levels above 5.  When level 5 fits in LDS, one workgroup does
// them all there; otherwise one launch per level from global memory.
//
// Texels are stored as (own pair, parent's pair), see put_level.

constexpr int kTile = 32;
constexpr int kTileLevels = 5;

// (max inverse depth, min inverse depth) of two texels
__device__ __forceinline__ float2 mm(float2 a, float2 b) {
    return make_float2(fmaxf(a.x, b.x), fminf(a.y, b.y));
}

// A texel is stored as float4: its own pair, then its parent's pair (the top
// texel: its own again), so that the march reads a cell and its parent with
// one load.  Each pass writes the own pairs of the texels it computes and the
// parent pairs of their children; the pass that computes the top level also
// completes the top texel.
__device__ __forceinline__ void put(float4* __restrict__ pyr, int64_t i, float2 v) {
    *reinterpret_cast<float2*>(pyr + i) = v;
}
__device__ __forceinline__ void put_parent(float4* __restrict__ pyr, int64_t i, float2 v) {
    reinterpret_cast<float2*>(pyr + i)[1] = v;
}
__device__ __forceinline__ float2 own(const float4* __restrict__ p, int64_t i) {
    const float4 t = p[i];
    return make_float2(t.x, t.y);
}

// Texel (x, y) of level L >= 1 holds v: write it, hand v to its children as
// their parent, and complete it if it is the top texel.
__device__ __forceinline__ void put_level(float4* __restrict__ pyr, const HizLayout& lay, int L,
                                          int x, int y, float2 v) {
    const int64_t at = hiz_index(lay, L, x, y);
    put(pyr, at, v);
    if (L == lay.levels - 1) put_parent(pyr, at, v);
    const int cw = lay.w[L - 1], ch = lay.h[L - 1];
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx)
            if (2 * x + dx < cw && 2 * y + dy < ch)
                put_parent(pyr, hiz_index(lay, L - 1, 2 * x + dx, 2 * y + dy), v);
}

// The pair of the lane whose index differs from this lane's in bit M
// (M = 1, 2: a DPP quad permutation; 4, 8, 16: a swizzle within 32 lanes;
// 32: a permute across the halves of the wave).
template <int M>
__device__ __forceinline__ float lane_xor(float v) {
    const int x = __float_as_int(v);
    int y;
    if constexpr (M == 1) {
        y = __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    } else if constexpr (M == 2) {
        y = __builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    } else if constexpr (M < 32) {
        y = __builtin_amdgcn_ds_swizzle(x, 0x1F | (M << 10));           // and 0x1F, xor M
    } else {
        y = __builtin_amdgcn_ds_bpermute(static_cast<int>((__lane_id() ^ 32u) << 2), x);
    }
    return __int_as_float(y);
}

// (max, min) of the pairs of the lanes that differ from this one in bits
// M and 2M: the texel one level up of a 2 x 2 group of Morton-ordered lanes.
template <int M>
__device__ __forceinline__ float2 reduce_quad(float2 v) {
    v = mm(v, make_float2(lane_xor<M>(v.x), lane_xor<M>(v.y)));
    return mm(v, make_float2(lane_xor<2 * M>(v.x), lane_xor<2 * M>(v.y)));
}

// Levels 0..5 of a 32 x 32 pixel tile, one workgroup of four waves, each
// wave a 16 x 16 quadrant.  A lane holds the 2 x 2 pixels under one level-1
// texel; the lanes are in Morton order over the quadrant's 8 x 8 level-1
// texels (lane bits 0, 2, 4: x; 1, 3, 5: y), so that the texels of level
// L + 1 are reductions over lanes that differ in bits 2L - 2 and 2L - 1:
// levels 2, 3 and 4 come from cross-lane exchanges within the wave, level 5
// from the four waves' level-4 texels through LDS.  Every lane of a group
// ends with the group's pair, so each texel's parent pair is at hand where
// the texel is written.
__global__ __launch_bounds__(256) void hiz_tile_kernel(const float* __restrict__ depth,
                                                       float4* __restrict__ pyr, HizLayout lay,
                                                       float thickness, int tile_levels) {
    __shared__ float2 quad[4];
    const int W = lay.w[0], H = lay.h[0];
    const int top = lay.levels - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the lane's level-1 texel within the quadrant (Morton order)
    const int a = (lane & 1) | ((lane >> 1) & 2) | ((lane >> 2) & 4);
    const int b = ((lane >> 1) & 1) | ((lane >> 2) & 2) | ((lane >> 3) & 4);
    const int q1x = blockIdx.x * 16 + (wave & 1) * 8 + a;   // level-1 texel
    const int q1y = blockIdx.y * 16 + (wave >> 1) * 8 + b;
    const int x0 = 2 * q1x, y0 = 2 * q1y;
    float2 p[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int x = x0 + c, y = y0 + r;
            const bool in = x < W && y < H;
            const float D = in ? depth[static_cast<int64_t>(y) * W + x] : 1.0f;
            p[r][c] = in ? make_float2(1.0f / D, 1.0f / (D + thickness))
                         : make_float2(-INFINITY, INFINITY);
        }
    }
    // the pairs of this lane's texels at levels 1..4 (pixels outside the
    // image count as -inf for the max and +inf for the min)
    const float2 m1 = mm(mm(p[0][0], p[0][1]), mm(p[1][0], p[1][1]));
    const float2 m2 = reduce_quad<1>(m1);
    const float2 m3 = reduce_quad<4>(m2);
    const float2 m4 = reduce_quad<16>(m3);
    if (lane == 0) quad[wave] = m4;
    __syncthreads();
    const float2 m5 = mm(mm(quad[0], quad[1]), mm(quad[2], quad[3]));
    const float2 m[kTileLevels + 1] = {p[0][0], m1, m2, m3, m4, m5};   // m[L]: level L (L >= 1)
    // level 0: the lane's four pixels (rows y0, y0 + 1 of the row pair y0 / 2:
    // four consecutive texels), each with its parent m1 (or itself at the top)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int x = x0 + c, y = y0 + r;
            if (x < W && y < H) {
                const float2 par = top >= 1 ? m1 : p[r][c];
                pyr[hiz_index(lay, 0, x, y)] = make_float4(p[r][c].x, p[r][c].y, par.x, par.y);
            }
        }
    // levels 1..tile_levels: texel (q1x >> (L - 1), q1y >> (L - 1)), written
    // by the first lane of its group; its parent is the next level's pair,
    // or its own at the top; level 5's parent comes from the pass above
#pragma unroll
    for (int L = 1; L <= kTileLevels; ++L) {
        if (L > tile_levels) break;
        const int low = (1 << (2 * (L - 1))) - 1;   // the lane bits within the group
        const bool first = L < kTileLevels ? (lane & low) == 0 : threadIdx.x == 0;
        const int lx = q1x >> (L - 1), ly = q1y >> (L - 1);
        if (first && lx < lay.w[L] && ly < lay.h[L]) {
            const int64_t at = hiz_index(lay, L, lx, ly);
            if (L < top) {
                if (L < kTileLevels)
                    pyr[at] = make_float4(m[L].x, m[L].y, m[L + 1].x, m[L + 1].y);
                else
                    put(pyr, at, m[L]);
            } else {
                pyr[at] = make_float4(m[L].x, m[L].y, m[L].x, m[L].y);
            }
        }
    }
}

// (max, min) over the up-to-four children (2x + dx, 2y + dy) of texel (x, y)
// of the level above a sw x sh level, read through get(x, y).
template <typename Get>
__device__ __forceinline__ float2 children(Get get, int sw, int sh, int x, int y) {
    float2 v = get(2 * x, 2 * y);
    if (2 * x + 1 < sw) v = mm(v, get(2 * x + 1, 2 * y));
    if (2 * y + 1 < sh) {
        v = mm(v, get(2 * x, 2 * y + 1));
        if (2 * x + 1 < sw) v = mm(v, get(2 * x + 1, 2 * y + 1));
    }
    return v;
}

// One level L >= 1 from the level below it (global memory).
__global__ void hiz_level_kernel(float4* __restrict__ pyr, HizLayout lay, int L) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int dw = lay.w[L];
    if (i >= dw * lay.h[L]) return;
    const float2 v = children([&](int xx, int yy) { return own(pyr, hiz_index(lay, L - 1, xx, yy)); },
                              lay.w[L - 1], lay.h[L - 1], i % dw, i / dw);
    put_level(pyr, lay, L, i % dw, i / dw, v);
}

constexpr int kTopLdsTexels = 8192;  // 64 KB of LDS for the levels above the tile pass

// All levels from `first` up, in one workgroup, ping-ponging through LDS.
__global__ __launch_bounds__(1024) void hiz_top_kernel(float4* __restrict__ pyr, HizLayout lay,
                                                       int first) {
    extern __shared__ float2 lds2[];
    const int sw0 = lay.w[first - 1], sh0 = lay.h[first - 1];
    float2* a = lds2;
    float2* b = lds2 + sw0 * sh0;
    for (int i = threadIdx.x; i < sw0 * sh0; i += blockDim.x)
        a[i] = own(pyr, hiz_index(lay, first - 1, i % sw0, i / sw0));
    for (int L = first; L < lay.levels; ++L) {
        __syncthreads();
        const int sw = lay.w[L - 1], sh = lay.h[L - 1], dw = lay.w[L], dh = lay.h[L];
        for (int i = threadIdx.x; i < dw * dh; i += blockDim.x) {
            const float2 v = children([&](int xx, int yy) { return a[yy * sw + xx]; }, sw, sh, i % dw,
                                      i / dw);
            b[i] = v;
            put_level(pyr, lay, L, i % dw, i / dw, v);
        }
        float2* t = a;
        a = b;
        b = t;
    }
}

void plan_hiz(const float* depth, const HizLayout& lay, float thickness, float4* pyramid,
              Plan& plan) {
    const int top = lay.levels - 1;
    const int tile_levels = top < kTileLevels ? top : kTileLevels;
    const dim3 grid((lay.w[0] + kTile - 1) / kTile, (lay.h[0] + kTile - 1) / kTile);
    Launch& t = plan.add(reinterpret_cast<const void*>(&hiz_tile_kernel), grid, dim3(256));
    t.arg(depth);
    t.arg(pyramid);
    t.arg(lay);
    t.arg(thickness);
    t.arg(tile_levels);
    if (top > kTileLevels) {
        const int first = kTileLevels + 1;
        const int64_t need = static_cast<int64_t>(lay.w[first - 1]) * lay.h[first - 1] +
                             static_cast<int64_t>(lay.w[first]) * lay.h[first];
        if (need <= kTopLdsTexels) {
            Launch& u = plan.add(reinterpret_cast<const void*>(&hiz_top_kernel), dim3(1),
                                 dim3(1024), static_cast<unsigned>(need * sizeof(float2)));
            u.arg(pyramid);
            u.arg(lay);
            u.arg(first);
        } else {
            for (int L = first; L <= top; ++L) {
                const int n = lay.w[L] * lay.h[L];
                Launch& u = plan.add(reinterpret_cast<const void*>(&hiz_level_kernel),
                                     dim3((n + 255) / 256), dim3(256));
                u.arg(pyramid);
                u.arg(lay);
                u.arg(L);
            }
        }
    }
}

hipError_t launch_hiz(const float* depth, const HizLayout& lay, float thickness, float4* pyramid,
                      hipStream_t stream) {
    Plan plan;
    plan_hiz(depth, lay, thickness, pyramid, plan);
    return run_plan(plan, stream);
}

hipError_t run_plan(Plan& plan, hipStream_t stream) {
    for (int k = 0; k < plan.n; ++k) {
        Launch& x = plan.l[k];
        void* argv[kLaunchMaxArgs];
        x.argv(argv);
        const hipError_t e = hipLaunchKernel(x.func, x.grid, x.block, argv, x.shmem, stream);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ Philox --

__global__ void philox_kernel(const uint4* __restrict__ ctr, const uint2* __restrict__ key,
                              int64_t n, uint4* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint2 k = key[i];
    out[i] = philox4x32_10(ctr[i], k.x, k.y);
}

hipError_t launch_philox(const uint32_t* ctr, const uint32_t* key, int64_t n, uint32_t* out,
                         hipStream_t stream) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(philox_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       reinterpret_cast<const uint4*>(ctr), reinterpret_cast<const uint2*>(key), n,
                       reinterpret_cast<uint4*>(out));
    return hipGetLastError();
}

}  // namespace ssr
