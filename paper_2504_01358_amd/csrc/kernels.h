// Internal interface between the C-ABI layer and the HIP kernels: buffer
// layouts and launchers.  Not part of the public header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ssr.h"

namespace ssr {

constexpr int kMaxLevels = 16;

// Env mip chain: levels 0..top of a W x H equirect map (W = 2H, H a power of
// two), level k of size (W >> k) x (H >> k), stored as float4 RGBA texels,
// level after level.
struct EnvLayout {
    int levels;               // top + 1
    int w[kMaxLevels], h[kMaxLevels];
    int64_t offset[kMaxLevels];  // in float4 texels
    int64_t total;               // float4 texels
};

// Depth pyramid: levels 0..top, each texel a float4: its own pair
// (1/min D, 1/max(D + thickness)) over the pixels it covers, then its
// parent's pair (the top texel repeats its own), level after level.  Inside
// a level the rows go in pairs, each pair stored column by column (texel
// (x, y) at 2 (w (y / 2) + x) + y % 2; a level with an odd number of rows
// gets one row of padding), so that a 128 B line holds a 4 x 2 block of
// texels: rays marching near each other share lines in both directions.
struct HizLayout {
    int levels;               // top + 1
    int w[kMaxLevels], h[kMaxLevels];
    int offset[kMaxLevels];   // in texels
    int64_t total;            // texels, padding included
};

// Index of texel (x, y) of level L in the layout above.
__host__ __device__ inline int64_t hiz_index(const HizLayout& lay, int L, int x, int y) {
    return lay.offset[L] + ((static_cast<int64_t>(y >> 1) * lay.w[L] + x) << 1) + (y & 1);
}

bool make_env_layout(int w, int h, EnvLayout* out);
bool make_hiz_layout(int w, int h, HizLayout* out);

// Everything the shading kernel reads, by value.
struct ShadeArgs {
    int W, H;
    float Wf, Hf;             // W and H as floats (kernel arguments: scalar registers)
    float pos[3];
    float right[3], up[3], fwd[3];
    float fx, fy, cx, cy, z_near;
    float inv_fx, inv_fy;     // 1 / fx, 1 / fy (rounded once, on the host)
    const float* depth;
    const void* normal_rough;
    const void* albedo_metal;
    const void* radiance;
    const float4* env;        // mip chain (EnvLayout)
    EnvLayout env_lay;
    const float4* hiz;        // depth pyramid (HizLayout)
    HizLayout hiz_lay;
    int spp, max_steps, linear_samples;
    float step_len, max_dist, thickness;
    uint32_t key0, key1, frame, flags;
    float* out;
    int32_t* steps;
    int32_t* codes;           // per-sample hit codes [H][W][spp]
    int* tile_counter;        // hierarchical trace: next tile
};

// One kernel launch with its own copy of the arguments, so that a frame's
// launches can be run directly or become the kernel nodes of a HIP graph,
// whose parameters are later replaced launch by launch.
constexpr int kLaunchMaxArgs = 8;
constexpr int kLaunchArgBytes = 1024;
struct Launch {
    const void* func = nullptr;
    dim3 grid, block;
    unsigned shmem = 0;
    int nargs = 0;
    unsigned offset[kLaunchMaxArgs] = {};
    unsigned size = 0;
    alignas(16) unsigned char data[kLaunchArgBytes];
    template <class T>
    void arg(const T& v) {
        static_assert(alignof(T) <= 16, "argument alignment");
        size = (size + alignof(T) - 1) / alignof(T) * alignof(T);
        __builtin_memcpy(data + size, &v, sizeof(T));
        offset[nargs++] = size;
        size += sizeof(T);
    }
    // pointers to the argument copies (valid while this object lives)
    void argv(void** out) {
        for (int i = 0; i < nargs; ++i) out[i] = data + offset[i];
    }
};
static_assert(sizeof(ShadeArgs) + 64 <= kLaunchArgBytes, "launch argument space");

// The launches of a frame, in stream order.
struct Plan {
    static constexpr int kMax = 24;
    Launch l[kMax];
    int n = 0;
    Launch& add(const void* func, dim3 grid, dim3 block, unsigned shmem = 0) {
        Launch& x = l[n++];
        x.func = func;
        x.grid = grid;
        x.block = block;
        x.shmem = shmem;
        x.nargs = 0;
        x.size = 0;
        return x;
    }
};
hipError_t run_plan(Plan& plan, hipStream_t stream);

// The launches of the pyramid build, the trace (work counter reset, trace)
// and the resolve, appended to `plan` (the launchers below run exactly these).
// `overlapped`: the frame shares the device with other frames (a serving
// session), so the trace splits its tiles only when it has fewer of them
// than resident waves.
void plan_hiz(const float* depth, const HizLayout& lay, float thickness, float4* pyramid,
              Plan& plan);
void plan_trace(const ShadeArgs& args, int dtype, int march, int cu_count, Plan& plan,
                bool overlapped = false);
void plan_resolve(const ShadeArgs& args, int dtype, Plan& plan);

hipError_t launch_env_mips(const float* rgb, const EnvLayout& lay, float4* mips,
                           hipStream_t stream);
hipError_t launch_hiz(const float* depth, const HizLayout& lay, float thickness, float4* pyramid,
                      hipStream_t stream);
// Validate a camera, G-buffer, env (when need_env) and parameters and fill
// `a` with everything but the workspace and output pointers.  Returns SSR_OK,
// 1 for an empty image, or an error status.
int fill_args(const ssr_camera* cam, const ssr_gbuffer* g, const ssr_env* env, const ssr_params* p,
              bool need_env, ShadeArgs* a, EnvLayout* env_lay, HizLayout* hiz_lay);

// Per-sample hit codes into args.codes (and iteration counts into args.steps).
hipError_t launch_trace(const ShadeArgs& args, int dtype, int march, int cu_count,
                        hipStream_t stream);
// The image from the hit codes in args.codes.
hipError_t launch_resolve(const ShadeArgs& args, int dtype, hipStream_t stream);

// Buffers of the adjoint (see ssr_shade_backward).
struct BackwardBuffers {
    const int32_t* hits;
    const float* grad_rgb;
    float* g_normal_rough;
    float* g_albedo_metal;
    float* g_env;
    float* g_radiance;
    float4* g_mips;           // workspace: `replicas` copies of one texel per env mip texel
    int replicas;
};
hipError_t launch_backward(const ShadeArgs& args, const BackwardBuffers& bufs, int dtype,
                           hipStream_t stream);
// First pass: depth normals into channels 0..2 of `out` ([H][W][4] in the
// storage type `dtype`), the split-sum table ([n][n] (A, B) pairs from k x k
// samples each) and c1 into `out` ([H][W][4] in `dtype`).
hipError_t launch_depth_normals(const ShadeArgs& args, int dtype, void* out, hipStream_t stream);
hipError_t launch_brdf_lut(float2* lut, int n, int k, hipStream_t stream);
hipError_t launch_first_pass(const ShadeArgs& args, int dtype, const float2* lut, int n, void* out,
                             hipStream_t stream);
hipError_t launch_philox(const uint32_t* ctr, const uint32_t* key, int64_t n, uint32_t* out,
                         hipStream_t stream);

}  // namespace ssr
