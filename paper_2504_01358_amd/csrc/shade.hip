// The shading kernels.
//
// Per pixel (Sec. 3.2 and Sec. 3.3):
//   load the G-buffer, un-project the pixel centre, wo = toward the camera;
//   c_d = (1 - m) a E_lambda(n), lambda = log2(1 + rho) lambda_max;
//   for each sample: Philox(q, s, frame, 0) -> (u1, u2); visible-normal GGX
//   half vector h; l = reflect(-wo, h); march l in screen space; radiance at
//   the hit pixel (c1) or, if the ray left the screen or ran out of
//   iterations, the environment at l; weight F(wo.h) G1(n.l);
//   Kahan-accumulate weight * radiance in sample order;
//   out = c_d + sum / S.
//
// The two marches implement the hit rule the library documents: a sample
// point (linear) or a pixel crossing (hierarchical) hits when the ray lies in
// the slab [D, D + thickness] behind the depth buffer after having been in
// front of it at some earlier point outside the origin pixel.
#include <algorithm>

#include "shading.h"

namespace ssr {

// ---------------------------------------------------------- linear march --

struct MarchResult {
    int code;
    int iters;
};

// Fixed world-space steps (Appendix D, Algorithm 1, with the documented hit
// rule).  V0 view-space origin, Dv view-space direction.  The sample points
// are known in advance, so the depths of kLinearAhead of them are loaded
// together (at clamped, in-bounds pixels) and then tested in order: the
// march waits for one group of gathers instead of one gather per step.
#ifndef SSR_LINEAR_AHEAD
#define SSR_LINEAR_AHEAD 4
#endif
constexpr int kLinearAhead = SSR_LINEAR_AHEAD;

__device__ __forceinline__ MarchResult march_linear(const ShadeArgs& a, int i, int j, V3 V0, V3 Dv) {
    bool armed = false;
    const int K = a.linear_samples;
    for (int k0 = 1; k0 <= K; k0 += kLinearAhead) {
        float Z[kLinearAhead], D[kLinearAhead];
        int ix[kLinearAhead], iy[kLinearAhead];
        bool on[kLinearAhead];
#pragma unroll
        for (int u = 0; u < kLinearAhead; ++u) {
            const float t = static_cast<float>(k0 + u) * a.step_len;
            const float X = V0.x + t * Dv.x, Y = V0.y + t * Dv.y;
            Z[u] = V0.z + t * Dv.z;
            const float iz = 1.0f / Z[u];
            const float px = a.cx + a.fx * X * iz;
            const float py = a.cy - a.fy * Y * iz;
            on[u] = Z[u] > a.z_near && px >= 0.0f && px < static_cast<float>(a.W) && py >= 0.0f &&
                    py < static_cast<float>(a.H);
            // (off the screen the load reads pixel (0, 0) and is not used)
            ix[u] = min(static_cast<int>(floorf(on[u] ? px : 0.0f)), a.W - 1);
            iy[u] = min(static_cast<int>(floorf(on[u] ? py : 0.0f)), a.H - 1);
            D[u] = a.depth[static_cast<int64_t>(iy[u]) * a.W + ix[u]];
        }
#pragma unroll
        for (int u = 0; u < kLinearAhead; ++u) {
            const int k = k0 + u;
            if (k > K) break;
            if (!on[u]) return MarchResult{SSR_HIT_OFFSCREEN, k};
            if (ix[u] == i && iy[u] == j) continue;
            const float dz = Z[u] - D[u];
            if (armed && dz >= 0.0f && dz <= a.thickness) return MarchResult{iy[u] * a.W + ix[u], k};
            if (dz < 0.0f) armed = true;
        }
    }
    return MarchResult{SSR_HIT_CAP, K};
}

// ------------------------------------------------------ hierarchical march --
//
// Exact first hit on the depth heightfield, hierarchical over the depth
// pyramid.  The ray is clipped at max_dist and the near plane and projected
// to the screen segment P0 + s dP.  Its inverse depth iz(s) = iz0 + s diz is
// linear in s (perspective-correct interpolation), so the march runs in
// inverse depth and needs no division: the pyramid holds, per cell, one over
// the nearest depth and one over the farthest depth plus the thickness, the
// two sides of the union of the cell's hit slabs.  A cell can be skipped when
// the ray's part inside it lies wholly in front of that union (its smallest
// inverse depth exceeds the first) or wholly behind it (its largest inverse
// depth is below the second).  Each iteration looks at the level-L cell and
// its parent at once (one 16 B texel holds both pairs): skip the parent and
// go up a level, else skip the cell, else go down two levels, else (level 0)
// test the pixel and step to the next one.
//
// The march is resumable (one iteration per call) so that a wave can keep
// all its lanes busy with rays of different lengths.

// The part of a ray computed when it is drawn (and queued).
struct HizSegment {
    bool valid;             // false: clipped away before it started (code -1, 0 iterations)
    float dPx, dPy;         // P1 - P0 in pixels
    float iz0, diz;         // inverse depth at s = 0 and its change over the segment
};

__device__ __forceinline__ HizSegment hiz_segment(const ShadeArgs& a, int i, int j, V3 V0, V3 Dv) {
    HizSegment g;
    float t_end = a.max_dist;
    // (the near-plane crossing with the hardware reciprocal, about 1 ulp)
    if (Dv.z < 0.0f) t_end = fminf(t_end, (a.z_near - V0.z) * __builtin_amdgcn_rcpf(Dv.z));
    g.valid = t_end > 0.0f;
    const float EX = V0.x + t_end * Dv.x, EY = V0.y + t_end * Dv.y, EZ = V0.z + t_end * Dv.z;
    const float P0x = static_cast<float>(i) + 0.5f, P0y = static_cast<float>(j) + 0.5f;
    // (hardware reciprocals, about 1 ulp)
    const float iz1 = __builtin_amdgcn_rcpf(EZ);
    g.dPx = (a.cx + a.fx * EX * iz1) - P0x;
    g.dPy = (a.cy - a.fy * EY * iz1) - P0y;
    g.iz0 = __builtin_amdgcn_rcpf(V0.z);
    g.diz = iz1 - g.iz0;
    return g;
}

// A ray being marched.  A boundary x = b is crossed at s = b inv_dx + bx.  A
// zero component of dP counts as travelling in the positive direction with
// inv = +inf: its crossings are then NaN, which fminf ignores, and the far
// screen edge is never reached.
struct HizRay {
    float P0x, P0y;       // centre of the origin pixel
    float dPx, dPy;
    float inv_dx, inv_dy; // 1 / dP
    float bx, by;         // -P0 / dP
    int xp, yp;           // 1 when travelling toward +x (+y), else 0
    float s_max;          // where the segment leaves the screen (at most 1)
    float iz0, diz;
    float s;              // current point of the segment
    int L, ix, iy;        // level and the level-0 pixel containing the current point
    float armed;          // 1 once the ray has been in front of the depth buffer, else 0
                          // (a float: its tests compile to compares, not byte logic)
    int deadline;         // the wave's step count at which the ray reaches the
                          // iteration cap (its own count is kept by the wave)
    int2 lv;              // (offset, width) of level L, read ahead (see hiz_step)
};

// The next pixel after moving to segment parameter se across the boundary
// of a cell whose exits are ex, ey (crossing at sx, sy): on a crossed axis the
// first pixel past the boundary, on the other axis the pixel the point lies
// in, kept between the current pixel and the cell's last pixel in the
// direction of travel.  (Near a cell corner the rounded coordinate can fall
// on the far side of a boundary the ray has just crossed on that axis; two
// such steps back, one per axis, would repeat forever.  The point lies in
// the cell it leaves, and a ray's pixel index never goes back on either
// axis, so the clamp only removes rounding.)
// floor(x) as an int, one instruction (v_cvt_flr_i32_f32; x is a pixel
// coordinate, far inside the int range)
__device__ __forceinline__ int floor_to_int(float x) {
    int v;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(v) : "v"(x));
    return v;
}

// the median of three (one v_med3_i32)
__device__ __forceinline__ int med3i(int a, int b, int c) {
    return max(min(a, b), min(max(a, b), c));
}

__device__ __forceinline__ void next_pixel(const HizRay& r, float se, float sx, float sy, int ex,
                                           int ey, int& nx, int& ny) {
    const bool kx = sx == se, ky = sy == se;
    const int v = floor_to_int(fmaf(se, kx ? r.dPy : r.dPx, kx ? r.P0y : r.P0x));
    // (both candidates computed, then selected: no branch)
    const int cx = ex + r.xp - 1, cy = ey + r.yp - 1;
    const int vx = med3i(v, r.ix, ex - r.xp), vy = med3i(v, r.iy, ey - r.yp);
    nx = kx ? cx : vx;
    ny = ky ? cy : vy;
}

// The constants of a ray: origin pixel centre, screen delta, its
// reciprocals and the crossing offsets, the direction of travel, where the
// segment leaves the screen, and its inverse depths.  State at its start:
// level 0, not armed (its first iteration is taken when it is drawn, see
// hiz_first; the caller sets the iteration deadline and the level entry).
__device__ __forceinline__ void hiz_init(const ShadeArgs& a, HizRay& r, int i, int j, float dPx,
                                         float dPy, float iz0, float diz) {
    r.P0x = static_cast<float>(i) + 0.5f;
    r.P0y = static_cast<float>(j) + 0.5f;
    r.dPx = dPx;
    r.dPy = dPy;
    // (the hardware reciprocal: the crossings need not be correctly rounded)
    r.inv_dx = dPx != 0.0f ? __builtin_amdgcn_rcpf(dPx) : INFINITY;
    r.inv_dy = dPy != 0.0f ? __builtin_amdgcn_rcpf(dPy) : INFINITY;
    r.xp = dPx >= 0.0f ? 1 : 0;
    r.yp = dPy >= 0.0f ? 1 : 0;
    r.bx = -r.P0x * r.inv_dx;
    r.by = -r.P0y * r.inv_dy;
    r.s_max = fminf(fminf(fmaf(r.xp ? a.Wf : 0.0f, r.inv_dx, r.bx),
                          fmaf(r.yp ? a.Hf : 0.0f, r.inv_dy, r.by)),
                    1.0f);
    r.iz0 = iz0;
    r.diz = diz;
    r.L = 0;
    r.armed = 0.0f;
    r.ix = i;
    r.iy = j;
}

// The first iteration of a ray set up by hiz_init.  At s = 0 the ray lies
// in the slab of its own pixel and of every cell containing it (their
// nearest depth is at most the pixel's, their farthest depth plus thickness
// at least its own), so neither the pixel nor its parent can be skipped and
// the first iteration always crosses the origin pixel into the next one (no
// test, no load).  Moves r to that pixel and returns true when the move
// already ends the ray (it left the segment or the screen).
__device__ __forceinline__ bool hiz_first(const ShadeArgs& a, HizRay& r) {
    const int ex = r.ix + r.xp, ey = r.iy + r.yp;
    const float sx = fmaf(static_cast<float>(ex), r.inv_dx, r.bx);
    const float sy = fmaf(static_cast<float>(ey), r.inv_dy, r.by);
    const float se = fminf(fminf(sx, sy), r.s_max);
    int nx, ny;
    next_pixel(r, se, sx, sy, ex, ey, nx, ny);
    const bool leave = (se >= r.s_max) | (static_cast<unsigned>(nx) >= static_cast<unsigned>(a.W)) |
                       (static_cast<unsigned>(ny) >= static_cast<unsigned>(a.H));
    r.ix = nx;
    r.iy = ny;
    r.s = se;
    return leave;
}

// One iteration, branch-free.  `wit` counts the wave's steps, this one
// included.  Returns true when the ray is finished; then `hit` tells a hit at
// (ix, iy) from leaving the screen or the segment (or the iteration cap, when
// neither is set).  `lvl[L]` holds (offset, width) of level L; the entry of
// the next iteration's level is read as soon as that level is known, so that
// the next iteration does not start by waiting for it.  A texel holds the
// cell's pair and its parent's, so one 16 B load serves both; the top texel
// is its own parent, so the look-ahead needs no special case there (skipping
// it means leaving the screen, as skipping the top cell does).
__device__ __forceinline__ bool hiz_step(const ShadeArgs& a, const int2* lvl, HizRay& r, int wit,
                                         bool& hit, bool& leave) {
    const int L = r.L, Lp = L + 1;
    const int2 lv = r.lv;
    const int cx = r.ix >> L, cy = r.iy >> L, px = r.ix >> Lp, py = r.iy >> Lp;
    // 32-bit byte offsets from a base held in SGPRs (the pyramid is < 4 GiB;
    // row index and width are below 2^14, so the 24-bit multiply is exact);
    // texel (cx, cy) of the level at 2 (w (cy / 2) + cx) + cy % 2 (hiz_index;
    // cy / 2 is py)
    const char* base = reinterpret_cast<const char*>(a.hiz);
    const unsigned oc = ((lv.x + ((__umul24(py, lv.y) + cx) << 1)) + (cy & 1)) << 4;
    // (1/min D, 1/max(D + th)) of the cell, then of its parent
    const float4 z = *reinterpret_cast<const float4*>(base + oc);
    const float2 zc = make_float2(z.x, z.y), zp = make_float2(z.z, z.w);
    // the boundaries the segment leaves the cell and the parent through
    const int ecx = (cx + r.xp) << L, ecy = (cy + r.yp) << L;
    const int epx = (px + r.xp) << Lp, epy = (py + r.yp) << Lp;
    const float sxc = fmaf(static_cast<float>(ecx), r.inv_dx, r.bx);
    const float syc = fmaf(static_cast<float>(ecy), r.inv_dy, r.by);
    const float sxp = fmaf(static_cast<float>(epx), r.inv_dx, r.bx);
    const float syp = fmaf(static_cast<float>(epy), r.inv_dy, r.by);
    const float sec = fminf(fminf(sxc, syc), r.s_max), sep = fminf(fminf(sxp, syp), r.s_max);
    const float izc = fmaf(sec, r.diz, r.iz0), izp = fmaf(sep, r.diz, r.iz0);
    // far end (smaller inverse depth) and near end of the ray inside each cell
    // the ray's inverse depth at the current point (recomputed, not carried:
    // the same FMA that gave izc or izp when the point was reached)
    const float iz_in = fmaf(r.s, r.diz, r.iz0);
    const float fc = fminf(iz_in, izc), nc = fmaxf(iz_in, izc);
    const float fp = fminf(iz_in, izp), np = fmaxf(iz_in, izp);
    const bool front_c = fc > zc.x;
    const bool skip_c = front_c | (nc < zc.y);
    const bool front_p = fp > zp.x;
    const bool up = front_p | (np < zp.y);
    // outcomes: skip the parent / skip the cell / go down / level-0 pixel
    const bool stay = !up & !skip_c;
    const bool at0 = L == 0;
    // (every ray here has left its origin pixel: its first iteration is
    // taken when it starts)
    const bool test = stay & at0;
    const bool was_armed = r.armed > 0.0f;
    hit = test & (was_armed | (iz_in > zc.x));
    const bool move = !hit & (!stay | at0);
    // the cell the segment moves across
    const float se = up ? sep : sec;
    const float sx = up ? sxp : sxc, sy = up ? syp : syc;
    const int ex = up ? epx : ecx, ey = up ? epy : ecy;
    // (a skip is never a hit, so move & !stay is !stay; a skipped cell was
    // in front when its own test says so)
    // the next level (down two levels, not below 0: a saturating subtract;
    // at level 0 a stay is the pixel test, and L stays 0 either way; a ray
    // that leaves or hits no longer needs it)
    const int Ld = static_cast<int>(__builtin_elementwise_sub_sat(static_cast<unsigned>(L), 2u));
    const int nL = up ? Lp : (stay ? Ld : L);
    r.lv = lvl[nL];
    const bool arm = (((up & front_p) | (!up & front_c)) & (se > r.s)) | (test & (nc > zc.x));
    r.armed = arm ? 1.0f : r.armed;
    int nx, ny;
    next_pixel(r, se, sx, sy, ex, ey, nx, ny);
    leave = move & ((se >= r.s_max) | (static_cast<unsigned>(nx) >= static_cast<unsigned>(a.W)) |
                    (static_cast<unsigned>(ny) >= static_cast<unsigned>(a.H)));
    const bool step = move & !leave;
    r.ix = step ? nx : r.ix;
    r.iy = step ? ny : r.iy;
    r.s = step ? se : r.s;
    r.L = nL;
    return hit | leave | (wit >= r.deadline);
}


// ------------------------------------------------------ linear-march trace --
//
// Workgroups of 256 threads take 16 x 16 pixel tiles; each wave64 an 8 x 8
// quadrant; each thread marches its pixel's samples in order, in lockstep
// with the wave, and writes their hit codes.
template <int DT, int TL>
__global__ __launch_bounds__(256) void trace_linear_kernel(const ShadeArgs a) {
    const int tiles_x = (a.W + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = (blockIdx.x % tiles_x) * 16 + (wave & 1) * 8 + (lane & 7);
    const int j = (blockIdx.x / tiles_x) * 16 + (wave >> 1) * 8 + (lane >> 3);
    if (i >= a.W || j >= a.H) return;
    const int64_t q = static_cast<int64_t>(j) * a.W + i;
    const int S = a.spp;
    const Pixel P = setup_pixel<DT>(a, i, j, q);
    const int fill = fill_code(a, P);
    for (int s = 0; s < S; ++s) {
        int code = fill, iters = 0;
        if (P.trace) {
            const SampleDir d = sample_dir(a, P, q, s);
            if (d.valid) {
                const MarchResult r = march_linear(a, i, j, v3(P.X0, P.Y0, P.D), world_to_view(a, d.l));
                code = r.code;
                iters = r.iters;
            }
        }
        const int64_t c = code_index<TL>(a, i, j, s);
        a.codes[c] = code;
        if (a.steps) a.steps[c] = iters;
    }
}

// ---------------------------------------------------- hierarchical path --
//
// Two kernels.  The trace kernel marches every ray of the frame and writes
// each sample's hit code; the resolve kernel then shades each pixel from the
// codes of its samples.
//
// Trace: persistent wave64s take work units (an 8 x 8 pixel tile's samples,
// or a range of them near the end of the frame) from a global counter.  The
// rays flow through a per-wave pool instead of being marched in lockstep:
//   * generate: every lane draws its pixel's samples k of the current unit
//     (kGenBatch at a time); the rays that need marching go to an LDS ring
//     queue, compacted (ballot + popcount); the others get their hit code at
//     once.  When a unit's samples are all drawn the wave takes the next;
//   * march: lanes take rays from the queue, any lane any ray, and a lane
//     whose ray ends takes the next one.  Idle lanes are refilled together
//     once kRefillMin of them wait (or the queue is shorter); a refilled
//     lane first writes the code of the ray it marched before.
// New rays are drawn while older ones are still marching, across tile
// boundaries, so the lanes stay busy until the frame runs out of tiles.
//
// Resolve: one thread per pixel draws its samples again and accumulates
// weight x radiance in sample order (Kahan), reading each sample's hit code,
// so the result does not depend on which lane marched which ray.
#ifndef SSR_GEN_BATCH
#define SSR_GEN_BATCH 3
#endif
#ifndef SSR_QUEUE_LOW
#define SSR_QUEUE_LOW 32
#endif
#ifndef SSR_REFILL_MIN
#define SSR_REFILL_MIN 24
#endif
#ifndef SSR_STEP_UNROLL
#define SSR_STEP_UNROLL 5
#endif
#ifndef SSR_GUIDE_A
#define SSR_GUIDE_A 85
#endif
#ifndef SSR_GUIDE_B
#define SSR_GUIDE_B 95
#endif
#ifndef SSR_GUIDE_DIV
#define SSR_GUIDE_DIV 4
#endif
#ifndef SSR_WAVES_PER_EU
#define SSR_WAVES_PER_EU 5
#endif
constexpr int kGenBatch = SSR_GEN_BATCH;   // sample indices drawn at once
constexpr int kQueueLow = SSR_QUEUE_LOW;   // draw when fewer rays than this wait
constexpr int kRefillMin = SSR_REFILL_MIN;
constexpr int kTraceWavesPerEU = SSR_WAVES_PER_EU;
constexpr int kStepUnroll = SSR_STEP_UNROLL;   // march iterations between idle counts
constexpr int kGuideWhole = SSR_GUIDE_A;       // percent of tiles handed out whole,
constexpr int kGuideHalf = SSR_GUIDE_B;        //   up to this percent in halves,
constexpr int kGuideDiv = SSR_GUIDE_DIV;       //   the rest in this many parts
// the queue never holds more than kQueueLow - 1 + kGenBatch * 64 rays (28 B
// of LDS each: 6.3 KB per wave at the defaults, so that 20 waves fit a CU)
constexpr int kQueueCap = kQueueLow + kGenBatch * 64;
// (wrap_queue takes slots below 2 kQueueCap: a head or tail slot plus fewer
// than 64)
static_assert(kGenBatch >= 1 && kQueueLow >= 1 && kQueueCap >= 64, "ray queue settings");

// A queue slot in [0, 2 kQueueCap) wrapped into [0, kQueueCap) (the smaller
// of p and p - kQueueCap as unsigned numbers).
__device__ __forceinline__ int wrap_queue(int p) {
    return static_cast<int>(min(static_cast<unsigned>(p), static_cast<unsigned>(p - kQueueCap)));
}

// The counter starts past the units the waves take first (unit = wave index),
// so that the waves do not all queue on it at the start.
__global__ void reset_counter_kernel(int* counter, int first) { *counter = first; }

// A queued ray, 28 bytes of LDS: its segment (dPx, dPy, iz0, diz), the
// segment parameter after its first iteration, the origin pixel with the
// first step packed beside it (i in bits 0..13, dx + 1 in 14..15, j in
// 16..29, dy + 1 in 30..31) and where its code goes: the slot (tile S + k)
// of its 64 codes in the tile-major layout, or the sample index k in the
// public one.
__device__ __forceinline__ unsigned pack_origin(int i, int j, int nx, int ny) {
    return static_cast<unsigned>(i) | (static_cast<unsigned>(nx - i + 1) << 14) |
           (static_cast<unsigned>(j) << 16) | (static_cast<unsigned>(ny - j + 1) << 30);
}

// The number of lanes below this one whose bit is set in the wave mask m
// (v_mbcnt: no per-lane mask kept in registers).
__device__ __forceinline__ int lanes_below(unsigned long long m) {
    return static_cast<int>(__builtin_amdgcn_mbcnt_hi(static_cast<unsigned>(m >> 32),
                                                      __builtin_amdgcn_mbcnt_lo(static_cast<unsigned>(m), 0u)));
}

// Code index of a queued ray (see code_index).
template <int TL>
__device__ __forceinline__ int64_t queued_code_index(const ShadeArgs& a, int i, int j, unsigned slot) {
    if (TL == 1) return (static_cast<int64_t>(slot) << 6) | ((j & 7) << 3) | (i & 7);
    return code_index<TL>(a, i, j, static_cast<int>(slot));
}

// SPLIT: the frame has fewer tiles than resident waves, and every tile is
// handed out in `split` parts of its samples (then halves and quarters of
// those), so that all waves get work; otherwise whole tiles first (split is
// then unused).
template <int DT, int TL, bool SPLIT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(SSR_WAVES_PER_EU, 8)))
void trace_hiz_kernel(const ShadeArgs a, int split) {
    __shared__ int2 lvl[kMaxLevels];
    __shared__ float4 q_seg[kQueueCap];     // queued rays: (dPx, dPy, iz0, diz),
    __shared__ float q_s1[kQueueCap];       //   segment parameter after the first iteration,
    __shared__ uint2 q_ray[kQueueCap];      //   packed origin and first step, code slot
    // the code of a lane's ended ray, stored when the lane takes its next ray
    // (or when the wave ends): one store per refill instead of a store in
    // almost every march iteration
    __shared__ int pend[64];
    const int lane = threadIdx.x;
    {
        // levels past the top (never reached) alias the top texel
        const int top = a.hiz_lay.levels - 1;
        if (lane < kMaxLevels) {
            const int L = min(lane, top);
            lvl[lane] = make_int2(a.hiz_lay.offset[L], lane < top ? a.hiz_lay.w[L] : 0);
        }
    }
    const int tiles_x = (a.W + 7) / 8;
    const int n_tiles = tiles_x * ((a.H + 7) / 8);
    const int S = a.spp;
    // guided work units: whole tiles first, then the last tiles in chunks of
    // half and a quarter of their samples, so that the waves finish the
    // frame together (with whole tiles to the end, a wave that takes the
    // last tile marches ~0.3 ms after others ran dry) without many more
    // trips to the shared counter (units of one or two samples contend on it)
    // (SPLIT: units of c0 = S / split samples come first, k0 of them per tile)
    const int c0 = SPLIT ? max(1, S / split) : S;
    const int k0 = SPLIT ? (S + c0 - 1) / c0 : 1;
    const int c1 = max(1, c0 / 2), c2 = max(1, c0 / kGuideDiv);  // chunk sizes of the tail
    const int n1 = (n_tiles * kGuideWhole) / 100;              // tiles in units of c0
    const int n2 = (n_tiles * kGuideHalf) / 100;               // tiles in chunks of c1
    const int k1 = (S + c1 - 1) / c1, k2 = (S + c2 - 1) / c2;
    const int u1 = n1 * k0, u2 = u1 + (n2 - n1) * k1, n_units = u2 + (n_tiles - n2) * k2;
    auto next_unit = [&]() {
        int t = 0;
        if (lane == 0) t = atomicAdd(a.tile_counter, 1);
        // (wave-uniform: the unit arithmetic below stays in scalar registers)
        return __builtin_amdgcn_readlane(t, 0);
    };
    int tile = 0, kk = 0, kend = 0;
    auto set_unit = [&](int u) {
        if (u < u1) {
            if (SPLIT) {
                tile = u / k0; kk = (u % k0) * c0; kend = min(kk + c0, S);
            } else {
                tile = u; kk = 0; kend = S;
            }
        } else if (u < u2) {
            const int v = u - u1;
            tile = n1 + v / k1; kk = (v % k1) * c1; kend = min(kk + c1, S);
        } else {
            const int v = u - u2;
            tile = n2 + v / k2; kk = (v % k2) * c2; kend = min(kk + c2, S);
        }
    };
    __syncthreads();

    int unit = blockIdx.x;      // unit being drawn (n_units or more: none left)
    set_unit(unit);
    int qh = 0, qn = 0;         // queue head (a slot) and length
    int nidle = 64;             // lanes without a ray
    HizRay r;
    int32_t* dst = nullptr;     // where the marching ray's hit code goes
    bool active = false;
    // a lane's ray ended: keep its code (and write its iteration count)
    int wit = 0;                // the wave's march steps so far (see HizRay::deadline)
    auto finish = [&](bool hit, bool leave) {
        pend[lane] = hit ? r.iy * a.W + r.ix : (leave ? SSR_HIT_OFFSCREEN : SSR_HIT_CAP);
        if (a.steps) a.steps[dst - a.codes] = wit - r.deadline + a.max_steps;
        active = false;
    };
    for (;;) {
        // draw more rays while the queue runs low
        if (unit < n_units && qn < kQueueLow) {
            asm volatile("" ::: "memory");
            const int i = (tile % tiles_x) * 8 + (lane & 7), j = (tile / tiles_x) * 8 + (lane >> 3);
            const bool inb = i < a.W && j < a.H;
            const int64_t q = inb ? static_cast<int64_t>(j) * a.W + i : 0;
            const int g = min(kGenBatch, kend - kk);
            const Pixel P = setup_pixel<DT>(a, i, j, q);
            const bool trace = inb && P.trace;
            const int fill = fill_code(a, P);
#pragma unroll 1
            for (int k = kk; k < kk + g; ++k) {
                int code = fill, iters = 0;
                bool queue = false;
                HizRay f;
                if (trace) {
                    const SampleDir d = sample_dir(a, P, q, k);
                    if (d.valid) {
                        const HizSegment sg =
                            hiz_segment(a, i, j, v3(P.X0, P.Y0, P.D), world_to_view(a, d.l));
                        code = SSR_HIT_OFFSCREEN;
                        if (sg.valid) {
                            // the first iteration here, with every lane busy;
                            // a ray it already ends is not queued
                            hiz_init(a, f, i, j, sg.dPx, sg.dPy, sg.iz0, sg.diz);
                            const bool gone = hiz_first(a, f);
                            iters = 1;
                            queue = !gone & (a.max_steps > 1);
                            code = gone ? SSR_HIT_OFFSCREEN : SSR_HIT_CAP;
                        }
                    }
                }
                const unsigned long long m = __ballot(queue);
                if (queue) {
                    const int pos = wrap_queue(wrap_queue(qh + qn) + lanes_below(m));
                    q_seg[pos] = make_float4(f.dPx, f.dPy, f.iz0, f.diz);
                    q_s1[pos] = f.s;
                    q_ray[pos] = make_uint2(pack_origin(i, j, f.ix, f.iy),
                                            TL == 1 ? static_cast<unsigned>(tile * S + k)
                                                    : static_cast<unsigned>(k));
                } else if (inb) {
                    a.codes[code_index<TL>(a, i, j, k)] = code;
                    if (a.steps) a.steps[code_index<TL>(a, i, j, k)] = iters;
                }
                qn = __builtin_amdgcn_readfirstlane(qn + __popcll(m));
            }
            kk += g;
            if (kk == kend) {
                unit = next_unit();
                set_unit(unit);
            }
            __builtin_amdgcn_wave_barrier();
            continue;
        }
        // refill idle lanes together once enough of them wait (or the queue is shorter)
        const int rem = qn;
        if (rem > 0 && nidle >= min(kRefillMin, rem)) {
            const unsigned long long idle = __ballot(!active);
            const int rank = lanes_below(idle);
            if (!active && rank < rem) {
                if (dst) *dst = pend[lane];   // the code of the lane's previous ray
                const int pos = wrap_queue(qh + rank);
                const float4 gq = q_seg[pos];
                const float s1 = q_s1[pos];
                const uint2 ray = q_ray[pos];
                const int ri = ray.x & 0x3FFF, rj = (ray.x >> 16) & 0x3FFF;
                hiz_init(a, r, ri, rj, gq.x, gq.y, gq.z, gq.w);
                r.ix = ri + static_cast<int>((ray.x >> 14) & 3u) - 1;
                r.iy = rj + static_cast<int>(ray.x >> 30) - 1;
                r.s = s1;
                // (one iteration taken: the cap is reached max_steps - 1 steps on)
                r.deadline = wit + a.max_steps - 1;
                r.lv = lvl[0];
                dst = a.codes + queued_code_index<TL>(a, ri, rj, ray.y);
                active = true;
            }
            qh = __builtin_amdgcn_readfirstlane(wrap_queue(qh + min(nidle, rem)));
            qn = __builtin_amdgcn_readfirstlane(rem - min(nidle, rem));
            nidle = __builtin_amdgcn_readfirstlane(__popcll(__ballot(!active)));
        }
        if (nidle == 64) {
            if (unit >= n_units && qn == 0) {
                if (dst) *dst = pend[lane];
                break;
            }
            continue;
        }
        // march: one round when the queue wants more rays drawn, else until
        // enough lanes are idle to refill (all of them once nothing is queued)
        const bool gen = unit < n_units && qn < kQueueLow;
        const int want = qn > 0 ? min(kRefillMin, qn) : 64;
        // (kStepUnroll iterations between two counts of the idle lanes: the
        // count and the loop test cost as much as a fifth of an iteration)
        do {
#pragma unroll
            for (int u = 0; u < kStepUnroll; ++u) {
                ++wit;
                if (active) {
                    bool hit, leave;
                    if (hiz_step(a, lvl, r, wit, hit, leave)) finish(hit, leave);
                }
            }
            nidle = __builtin_amdgcn_readfirstlane(__popcll(__ballot(!active)));
        } while (!gen && nidle < want);
        __builtin_amdgcn_wave_barrier();
    }
}

// Workgroups of 256 threads shade 16 x 16 pixel tiles, one thread per pixel.
template <int DT, int TL>
__global__ __launch_bounds__(256) void resolve_kernel(const ShadeArgs a) {
    const int tiles_x = (a.W + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = (blockIdx.x % tiles_x) * 16 + (wave & 1) * 8 + (lane & 7);
    const int j = (blockIdx.x / tiles_x) * 16 + (wave >> 1) * 8 + (lane >> 3);
    if (i >= a.W || j >= a.H) return;
    const int64_t q = static_cast<int64_t>(j) * a.W + i;
    const int S = a.spp;
    const Pixel P = setup_pixel<DT>(a, i, j, q);
    float sum[3] = {0.0f, 0.0f, 0.0f}, cmp[3] = {0.0f, 0.0f, 0.0f};
    if (P.trace) {
        // the next sample's code is loaded one sample ahead, and a hit's
        // radiance before its direction is drawn again, so that both loads
        // overlap arithmetic
        int next = a.codes[code_index<TL>(a, i, j, 0)];
#pragma unroll 1
        for (int s = 0; s < S; ++s) {
            int code = next;
            if (s + 1 < S) next = a.codes[code_index<TL>(a, i, j, s + 1)];
            // (a code naming no pixel of this frame contributes nothing)
            if (code >= a.W * a.H || code < SSR_HIT_SKIPPED) code = SSR_HIT_INVALID;
            if (code >= 0 || code == SSR_HIT_OFFSCREEN || code == SSR_HIT_CAP) {
                const float3 c1 = code >= 0 ? Texel4<DT>::load3(a.radiance, code)
                                            : make_float3(0.0f, 0.0f, 0.0f);
                const SampleDir d = sample_dir(a, P, q, s);
                // a miss's environment lookup goes to registers of its own and
                // the choice comes after it, so the lookup does not wait for
                // the radiance loads of the wave's hit lanes
                float3 e = make_float3(0.0f, 0.0f, 0.0f);
                if (code < 0) e = env_bilinear(env_level(a, 0), env_angles(d.l));
                accumulate(a, P, d, code >= 0 ? c1 : e, sum, cmp);
            }
        }
    }
    write_out(a, q, direct_term(a, P, i, j), sum);
}

// The kernel of one storage type (DT) and per-sample layout (TL).
template <template <int, int> class K>
const void* pick(int dtype, bool tiled) {
    if (tiled) {
        if (dtype == SSR_F32) return K<0, 1>::fn();
        if (dtype == SSR_F16) return K<1, 1>::fn();
        return K<2, 1>::fn();
    }
    if (dtype == SSR_F32) return K<0, 0>::fn();
    if (dtype == SSR_F16) return K<1, 0>::fn();
    return K<2, 0>::fn();
}
template <int DT, int TL>
struct TraceLinearK {
    static const void* fn() { return reinterpret_cast<const void*>(&trace_linear_kernel<DT, TL>); }
};
template <int DT, int TL>
struct TraceHizK {
    static const void* fn() { return reinterpret_cast<const void*>(&trace_hiz_kernel<DT, TL, false>); }
};
template <int DT, int TL>
struct TraceHizSplitK {
    static const void* fn() { return reinterpret_cast<const void*>(&trace_hiz_kernel<DT, TL, true>); }
};
template <int DT, int TL>
struct ResolveK {
    static const void* fn() { return reinterpret_cast<const void*>(&resolve_kernel<DT, TL>); }
};

#ifndef SSR_SPLIT_UNITS
#define SSR_SPLIT_UNITS 4
#endif
// A frame with few tiles for the resident waves splits each tile's samples
// into `split` parts (a power of two) until there are about kSplitUnits
// units per resident wave: with fewer tiles than waves, keeping at least
// four samples in a part; with up to three tiles per wave, at least eight
// (units of one or two samples cost more in counter trips and pixel
// set-ups than they gain, and a draw of three samples then one wastes most
// of a round).  A frame that shares the device with others is split only in
// the first case: the other frames fill the waves its tail leaves idle.
// Returns 1 when the tiles are not split.
constexpr int kSplitUnits = SSR_SPLIT_UNITS;
int trace_split(int cu_count, int W, int H, int S, bool overlapped) {
    const int64_t n_tiles = static_cast<int64_t>((W + 7) / 8) * ((H + 7) / 8);
    const int64_t resident = static_cast<int64_t>(cu_count) * 4 * kTraceWavesPerEU;
    int f = 1;
    if (n_tiles >= (overlapped ? 1 : 3) * resident) return f;
    const int min_part = n_tiles < resident ? 4 : 8;
    while (S / (2 * f) >= min_part && n_tiles * f < kSplitUnits * resident) f *= 2;
    return f;
}

// One persistent wave per unit, up to the resident count (the unit count as
// the kernel computes it).
int trace_grid(int cu_count, int W, int H, int S, int split) {
    const int n_tiles = ((W + 7) / 8) * ((H + 7) / 8);
    int n_units = n_tiles;
    if (split > 1) {
        const int c0 = std::max(1, S / split), k0 = (S + c0 - 1) / c0;
        const int c1 = std::max(1, c0 / 2), c2 = std::max(1, c0 / kGuideDiv);
        const int n1 = (n_tiles * kGuideWhole) / 100, n2 = (n_tiles * kGuideHalf) / 100;
        const int k1 = (S + c1 - 1) / c1, k2 = (S + c2 - 1) / c2;
        n_units = n1 * k0 + (n2 - n1) * k1 + (n_tiles - n2) * k2;
    }
    const int resident = cu_count * 4 * kTraceWavesPerEU;
    return n_units < resident ? n_units : resident;
}

void plan_trace(const ShadeArgs& args, int dtype, int march, int cu_count, Plan& plan,
                bool overlapped) {
    const bool tiled = (args.flags & SSR_CODES_TILED) != 0;
    if (march == SSR_MARCH_LINEAR) {
        const dim3 grid(((args.W + 15) / 16) * ((args.H + 15) / 16));
        plan.add(pick<TraceLinearK>(dtype, tiled), grid, dim3(256)).arg(args);
        return;
    }
    const int split = trace_split(cu_count, args.W, args.H, args.spp, overlapped);
    const dim3 grid(trace_grid(cu_count, args.W, args.H, args.spp, split));
    Launch& r = plan.add(reinterpret_cast<const void*>(&reset_counter_kernel), dim3(1), dim3(1));
    r.arg(args.tile_counter);
    r.arg(static_cast<int>(grid.x));
    Launch& t = plan.add(split > 1 ? pick<TraceHizSplitK>(dtype, tiled) : pick<TraceHizK>(dtype, tiled),
                         grid, dim3(64));
    t.arg(args);
    t.arg(split);
}

void plan_resolve(const ShadeArgs& args, int dtype, Plan& plan) {
    const bool tiled = (args.flags & SSR_CODES_TILED) != 0;
    const dim3 grid(((args.W + 15) / 16) * ((args.H + 15) / 16));
    plan.add(pick<ResolveK>(dtype, tiled), grid, dim3(256)).arg(args);
}

hipError_t launch_trace(const ShadeArgs& args, int dtype, int march, int cu_count,
                        hipStream_t stream) {
    Plan plan;
    plan_trace(args, dtype, march, cu_count, plan);
    return run_plan(plan, stream);
}

hipError_t launch_resolve(const ShadeArgs& args, int dtype, hipStream_t stream) {
    Plan plan;
    plan_resolve(args, dtype, plan);
    return run_plan(plan, stream);
}

}  // namespace ssr
