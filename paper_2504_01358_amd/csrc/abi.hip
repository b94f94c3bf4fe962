// C-ABI entry points (declared in include/ssr.h): argument validation, the
// context's grow-only device workspace, and the launches.
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>

#include "kernels.h"
#include "ssr.h"

struct ssr_ctx {
    int device;
    int cu_count;
    // workspace: depth pyramid, env mip chain, per-sample hit codes of the
    // hierarchical path (when the caller asks for none) and its tile counter
    float4* hiz;
    int64_t hiz_cap;    // float4 texels
    float4* mips;
    int64_t mips_cap;   // float4 texels
    int32_t* codes;
    int64_t codes_cap;  // int32
    int* counter;
    float4* g_mips;     // adjoint: environment derivatives per mip texel
    int64_t g_mips_cap;
    float2* lut;        // first pass: split-sum table [kLutN][kLutN], built on first use
};

namespace {
constexpr int kLutN = 128;   // table entries per axis (n.v and roughness)
constexpr int kLutK = 64;    // stratified samples per axis of each entry
}  // namespace

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? SSR_OK : SSR_E_HIP; }

// Grow a workspace buffer.  The old buffer may still be read by work queued
// earlier, so the device is drained before it is freed (growth is rare: the
// buffers only ever get larger).
template <typename T>
int ensure(T** buf, int64_t* cap, int64_t need) {
    if (need <= *cap) return SSR_OK;
    if (*buf) {
        if (hipDeviceSynchronize() != hipSuccess) return SSR_E_HIP;
        if (hipFree(*buf) != hipSuccess) return SSR_E_HIP;
        *buf = nullptr;
        *cap = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, static_cast<size_t>(need) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return SSR_E_NOMEM;
    }
    *buf = static_cast<T*>(p);
    *cap = need;
    return SSR_OK;
}

bool finite_f(float v) { return isfinite(v) != 0; }

int check_camera(const ssr_camera* c) {
    if (!c) return SSR_E_ARG;
    if (c->width < 0 || c->height < 0 || c->width > 16384 || c->height > 16384) return SSR_E_ARG;
    for (int k = 0; k < 3; ++k)
        if (!finite_f(c->pos[k])) return SSR_E_ARG;
    for (int k = 0; k < 9; ++k)
        if (!finite_f(c->rot[k])) return SSR_E_ARG;
    if (!(c->fx > 0.0f) || !(c->fy > 0.0f) || !finite_f(c->fx) || !finite_f(c->fy) ||
        !finite_f(c->cx) || !finite_f(c->cy) || !(c->z_near > 0.0f) || !finite_f(c->z_near))
        return SSR_E_ARG;
    return SSR_OK;
}

int check_params(const ssr_params* p) {
    if (!p) return SSR_E_ARG;
    if (p->spp < 1 || p->spp > 4096) return SSR_E_ARG;
    if (p->march != SSR_MARCH_LINEAR && p->march != SSR_MARCH_HIZ) return SSR_E_ARG;
    if (p->max_steps < 1 || p->max_steps > (1 << 20)) return SSR_E_ARG;
    if (!(p->max_dist > 0.0f) || !finite_f(p->max_dist)) return SSR_E_ARG;
    if (!(p->thickness >= 0.0f) || !finite_f(p->thickness)) return SSR_E_ARG;
    if (p->march == SSR_MARCH_LINEAR && (!(p->step_len > 0.0f) || !finite_f(p->step_len)))
        return SSR_E_ARG;
    if (p->flags & ~static_cast<uint32_t>(SSR_NO_DIRECT | SSR_NO_SPECULAR | SSR_SAMPLER_NDF |
                                          SSR_CODES_TILED))
        return SSR_E_ARG;
    return SSR_OK;
}

// Zero `a` and fill its camera fields.
void camera_args(const ssr_camera* cam, ssr::ShadeArgs* a) {
    memset(a, 0, sizeof(*a));
    a->W = cam->width;
    a->H = cam->height;
    a->Wf = static_cast<float>(cam->width);
    a->Hf = static_cast<float>(cam->height);
    for (int k = 0; k < 3; ++k) {
        a->pos[k] = cam->pos[k];
        a->right[k] = cam->rot[k];
        a->up[k] = cam->rot[3 + k];
        a->fwd[k] = cam->rot[6 + k];
    }
    a->fx = cam->fx;
    a->fy = cam->fy;
    a->inv_fx = 1.0f / cam->fx;
    a->inv_fy = 1.0f / cam->fy;
    a->cx = cam->cx;
    a->cy = cam->cy;
    a->z_near = cam->z_near;
}

}  // namespace

// ------------------------------------------------ static scratch buffer --
//
// The workspace of ssr_shade_static: one array per device (each device that
// loads the library holds its own copy until the process ends).  Host code
// never uses the array's name as an address: its device address is looked up
// once per device with hipGetSymbolAddress and kept in `g_static`.
static __device__ __align__(256) char scratch[SSR_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

struct StaticDevice {
    char* ptr = nullptr;   // device address of `scratch` on this device
    int cu_count = 0;
    int status = 1;        // 1: not looked up yet; else SSR_OK or the error
};

std::mutex g_static_mu;
StaticDevice g_static[kMaxDevices];

// Look up the scratch array on `device` (made current by the caller) once,
// checking that the device is a gfx950.
int static_device(int device, StaticDevice* out) {
    if (device < 0 || device >= kMaxDevices) return SSR_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_static_mu);
    StaticDevice& d = g_static[device];
    if (d.status == 1) {
        hipDeviceProp_t prop;
        void* p = nullptr;
        if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
            (void)hipGetLastError();
            return SSR_E_HIP;   // not cached: a later call may succeed
        }
        if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            d.status = SSR_E_DEVICE;
        } else if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return SSR_E_HIP;
        } else {
            d.ptr = static_cast<char*>(p);
            d.cu_count = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
            d.status = SSR_OK;
        }
    }
    *out = d;
    return d.status;
}

}  // namespace

namespace ssr {

int fill_args(const ssr_camera* cam, const ssr_gbuffer* g, const ssr_env* env, const ssr_params* p,
              bool need_env, ShadeArgs* a, EnvLayout* env_lay, HizLayout* hiz_lay) {
    if (!g || (need_env && !env)) return SSR_E_ARG;
    int st = check_camera(cam);
    if (st != SSR_OK) return st;
    if (p) {
        st = check_params(p);
        if (st != SSR_OK) return st;
    }
    if (g->dtype != SSR_F32 && g->dtype != SSR_F16 && g->dtype != SSR_BF16) return SSR_E_DTYPE;
    if (need_env && (!env->rgb || !make_env_layout(env->width, env->height, env_lay)))
        return SSR_E_ARG;
    if (cam->width == 0 || cam->height == 0) return 1;
    if (!g->depth || !g->normal_rough || !g->albedo_metal || !g->radiance) return SSR_E_ARG;
    // (the hierarchical march needs the pyramid; the layout also bounds W H)
    if (!make_hiz_layout(cam->width, cam->height, hiz_lay)) return SSR_E_ARG;

    camera_args(cam, a);
    a->depth = g->depth;
    a->normal_rough = g->normal_rough;
    a->albedo_metal = g->albedo_metal;
    a->radiance = g->radiance;
    a->hiz_lay = *hiz_lay;
    if (need_env) a->env_lay = *env_lay;
    if (!p) return SSR_OK;
    // (the trace kernel addresses a (tile, sample) row of 64 codes with 32
    // bits: refuse frames past that, whose codes no device memory could hold)
    const int64_t tiles = static_cast<int64_t>((cam->width + 7) / 8) * ((cam->height + 7) / 8);
    if (tiles * p->spp >= (int64_t(1) << 32)) return SSR_E_ARG;
    a->spp = p->spp;
    a->max_steps = p->max_steps;
    // linear march: samples t_k = k * step_len for k = 1..K, K = min(max_steps,
    // floor(max_dist / step_len)), evaluated in double as the specification states
    if (p->march == SSR_MARCH_LINEAR) {
        const double k = floor(static_cast<double>(p->max_dist) / static_cast<double>(p->step_len));
        a->linear_samples = k < static_cast<double>(p->max_steps) ? static_cast<int>(k) : p->max_steps;
    }
    a->step_len = p->step_len;
    a->max_dist = p->max_dist;
    a->thickness = p->thickness;
    a->key0 = static_cast<uint32_t>(p->seed & 0xFFFFFFFFu);
    a->key1 = static_cast<uint32_t>(p->seed >> 32);
    a->frame = p->frame;
    a->flags = p->flags;
    return SSR_OK;
}

}  // namespace ssr

extern "C" {

const char* ssr_status_string(int status) {
    switch (status) {
        case SSR_OK: return "ok";
        case SSR_E_ARG: return "invalid argument";
        case SSR_E_DTYPE: return "unknown G-buffer storage type";
        case SSR_E_NOMEM: return "device workspace allocation failed";
        case SSR_E_HIP: return "HIP runtime error";
        case SSR_E_DEVICE: return "no such device or not a gfx950 device";
        case SSR_E_BUDGET: return "the session's device-memory budget cannot hold it";
        case SSR_E_BUSY: return "not allowed while the session is serving or stopping";
        case SSR_E_TICKET: return "no such request";
        case SSR_E_SCRATCH: return "the frame's workspace exceeds the static scratch buffer";
        case SSR_PENDING: return "pending";
        default: return "unknown status";
    }
}

int ssr_ctx_create(int device, ssr_ctx** out) {
    if (!out) return SSR_E_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return SSR_E_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return SSR_E_HIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SSR_E_DEVICE;
    ssr_ctx* c = new (std::nothrow) ssr_ctx;
    if (!c) return SSR_E_NOMEM;
    c->device = device;
    c->cu_count = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    c->hiz = nullptr;
    c->hiz_cap = 0;
    c->mips = nullptr;
    c->mips_cap = 0;
    c->codes = nullptr;
    c->codes_cap = 0;
    c->counter = nullptr;
    c->g_mips = nullptr;
    c->g_mips_cap = 0;
    c->lut = nullptr;
    if (hipSetDevice(device) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&c->counter), 256) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return SSR_E_NOMEM;
    }
    // (the static scratch buffer's address on this device, for
    // ssr_shade_static, looked up here so that it happens outside any graph
    // capture; a failure is not the context's: ssr_shade_static tries again
    // and reports it)
    StaticDevice sd;
    (void)static_device(device, &sd);
    *out = c;
    return SSR_OK;
}

void ssr_ctx_destroy(ssr_ctx* ctx) {
    if (!ctx) return;
    if (hipSetDevice(ctx->device) == hipSuccess) {
        (void)hipDeviceSynchronize();
        if (ctx->hiz) (void)hipFree(ctx->hiz);
        if (ctx->mips) (void)hipFree(ctx->mips);
        if (ctx->codes) (void)hipFree(ctx->codes);
        if (ctx->counter) (void)hipFree(ctx->counter);
        if (ctx->g_mips) (void)hipFree(ctx->g_mips);
        if (ctx->lut) (void)hipFree(ctx->lut);
    }
    delete ctx;
}

int64_t ssr_codes_count(int32_t width, int32_t height, int32_t spp, uint32_t flags) {
    if (width < 0 || height < 0 || spp < 0) return 0;
    if (flags & SSR_CODES_TILED)
        return static_cast<int64_t>((width + 7) / 8) * ((height + 7) / 8) * 64 * spp;
    return static_cast<int64_t>(width) * height * spp;
}

int64_t ssr_env_mips_floats(int32_t width, int32_t height) {
    ssr::EnvLayout lay;
    if (!ssr::make_env_layout(width, height, &lay)) return 0;
    return 4 * lay.total;
}

int ssr_env_build_mips(const float* rgb, int32_t width, int32_t height, float* mips,
                       void* stream) {
    ssr::EnvLayout lay;
    if (!rgb || !mips || !ssr::make_env_layout(width, height, &lay)) return SSR_E_ARG;
    return hip_status(ssr::launch_env_mips(rgb, lay, reinterpret_cast<float4*>(mips),
                                           static_cast<hipStream_t>(stream)));
}

int64_t ssr_hiz_floats(int32_t width, int32_t height) {
    ssr::HizLayout lay;
    if (!ssr::make_hiz_layout(width, height, &lay)) return 0;
    return 4 * lay.total;
}

int ssr_hiz_build(const float* depth, int32_t width, int32_t height, float thickness,
                  float* pyramid, void* stream) {
    ssr::HizLayout lay;
    if (!depth || !pyramid || !ssr::make_hiz_layout(width, height, &lay)) return SSR_E_ARG;
    if (!(thickness >= 0.0f) || !finite_f(thickness)) return SSR_E_ARG;
    return hip_status(ssr::launch_hiz(depth, lay, thickness, reinterpret_cast<float4*>(pyramid),
                                      static_cast<hipStream_t>(stream)));
}

int ssr_philox4x32_10(const uint32_t* ctr, const uint32_t* key, int64_t n, uint32_t* out,
                      void* stream) {
    if (n < 0 || n > (int64_t(1) << 31) * 255) return SSR_E_ARG;
    if (n == 0) return SSR_OK;
    if (!ctr || !key || !out) return SSR_E_ARG;
    return hip_status(ssr::launch_philox(ctr, key, n, out, static_cast<hipStream_t>(stream)));
}

}  // extern "C"

namespace {

// Validate the arguments common to the shading calls and fill `a` with
// everything but the output pointers.  Returns SSR_OK, or 1 for an empty
// image (nothing to do), or an error.
int prepare(ssr_ctx* ctx, const ssr_camera* cam, const ssr_gbuffer* g, const ssr_env* env,
            const ssr_params* p, bool need_env, ssr::ShadeArgs* a, ssr::EnvLayout* env_lay,
            ssr::HizLayout* hiz_lay) {
    if (!ctx) return SSR_E_ARG;
    const int st = ssr::fill_args(cam, g, need_env ? env : nullptr, p, need_env, a, env_lay, hiz_lay);
    if (st != SSR_OK) return st;
    if (hipSetDevice(ctx->device) != hipSuccess) return SSR_E_HIP;
    a->tile_counter = ctx->counter;
    return SSR_OK;
}

// The env mip chain: the caller's, or built in the workspace.
int env_mips(ssr_ctx* ctx, const ssr_env* env, const ssr::EnvLayout& lay, hipStream_t s,
             const float4** out) {
    *out = reinterpret_cast<const float4*>(env->mips);
    if (*out) return SSR_OK;
    int st = ensure(&ctx->mips, &ctx->mips_cap, lay.total);
    if (st != SSR_OK) return st;
    st = hip_status(ssr::launch_env_mips(env->rgb, lay, ctx->mips, s));
    *out = ctx->mips;
    return st;
}

// Trace into `codes`: the hierarchical march builds the pyramid first unless
// the caller supplies it.
int trace(ssr_ctx* ctx, const ssr_gbuffer* g, const ssr_params* p, ssr::ShadeArgs* a,
          const ssr::HizLayout& hiz_lay, int32_t* codes, int32_t* steps, hipStream_t s) {
    const float4* hiz = reinterpret_cast<const float4*>(g->hiz);
    if (p->march == SSR_MARCH_HIZ && !hiz) {
        int st = ensure(&ctx->hiz, &ctx->hiz_cap, hiz_lay.total);
        if (st != SSR_OK) return st;
        st = hip_status(ssr::launch_hiz(g->depth, hiz_lay, p->thickness, ctx->hiz, s));
        if (st != SSR_OK) return st;
        hiz = ctx->hiz;
    }
    a->hiz = hiz;
    a->codes = codes;
    a->steps = steps;
    return hip_status(ssr::launch_trace(*a, g->dtype, p->march, ctx->cu_count, s));
}

}  // namespace

extern "C" {

int ssr_trace(ssr_ctx* ctx, const ssr_camera* cam, const ssr_gbuffer* g, const ssr_params* p,
              int32_t* out_hits, int32_t* out_steps, void* stream) {
    ssr::ShadeArgs a;
    ssr::EnvLayout env_lay;
    ssr::HizLayout hiz_lay;
    int st = prepare(ctx, cam, g, nullptr, p, false, &a, &env_lay, &hiz_lay);
    if (st != SSR_OK) return st == 1 ? SSR_OK : st;
    if (!out_hits) return SSR_E_ARG;
    return trace(ctx, g, p, &a, hiz_lay, out_hits, out_steps, static_cast<hipStream_t>(stream));
}

int ssr_resolve(ssr_ctx* ctx, const ssr_camera* cam, const ssr_gbuffer* g, const ssr_env* env,
                const ssr_params* p, const int32_t* hits, float* out_rgb, void* stream) {
    ssr::ShadeArgs a;
    ssr::EnvLayout env_lay;
    ssr::HizLayout hiz_lay;
    int st = prepare(ctx, cam, g, env, p, true, &a, &env_lay, &hiz_lay);
    if (st != SSR_OK) return st == 1 ? SSR_OK : st;
    if (!hits || !out_rgb) return SSR_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = env_mips(ctx, env, env_lay, s, &a.env);
    if (st != SSR_OK) return st;
    a.codes = const_cast<int32_t*>(hits);  // read only by the resolve kernel
    a.out = out_rgb;
    return hip_status(ssr::launch_resolve(a, g->dtype, s));
}

int ssr_shade_backward(ssr_ctx* ctx, const ssr_camera* cam, const ssr_gbuffer* g,
                       const ssr_env* env, const ssr_params* p, const int32_t* hits,
                       const float* grad_rgb, float* g_normal_rough, float* g_albedo_metal,
                       float* g_env, float* g_radiance, void* stream) {
    ssr::ShadeArgs a;
    ssr::EnvLayout env_lay;
    ssr::HizLayout hiz_lay;
    int st = prepare(ctx, cam, g, env, p, true, &a, &env_lay, &hiz_lay);
    if (st != SSR_OK) return st == 1 ? SSR_OK : st;
    if (!hits || !grad_rgb || (p->flags & SSR_SAMPLER_NDF)) return SSR_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = env_mips(ctx, env, env_lay, s, &a.env);
    if (st != SSR_OK) return st;
    // copies of the environment sums that the workgroups' atomics spread
    // over: up to 32, within 256 MB
    const int64_t per = env_lay.total;
    int replicas = static_cast<int>((int64_t(256) << 20) / (per * 16));
    replicas = replicas < 1 ? 1 : (replicas > 32 ? 32 : replicas);
    st = ensure(&ctx->g_mips, &ctx->g_mips_cap, per * replicas);
    if (st != SSR_OK) return st;
    ssr::BackwardBuffers b{hits,      grad_rgb,   g_normal_rough, g_albedo_metal,
                           g_env,     g_radiance, ctx->g_mips,    replicas};
    return hip_status(ssr::launch_backward(a, b, g->dtype, s));
}

int ssr_shade(ssr_ctx* ctx, const ssr_camera* cam, const ssr_gbuffer* g, const ssr_env* env,
              const ssr_params* p, float* out_rgb, int32_t* out_hits, int32_t* out_steps,
              void* stream) {
    ssr::ShadeArgs a;
    ssr::EnvLayout env_lay;
    ssr::HizLayout hiz_lay;
    int st = prepare(ctx, cam, g, env, p, true, &a, &env_lay, &hiz_lay);
    if (st != SSR_OK) return st == 1 ? SSR_OK : st;
    if (!out_rgb) return SSR_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = env_mips(ctx, env, env_lay, s, &a.env);
    if (st != SSR_OK) return st;
    int32_t* codes = out_hits;
    if (!codes) {
        // the context's own codes go tile-major (unless the caller wants the
        // iteration counts, which share the codes' layout)
        if (!out_steps) a.flags |= SSR_CODES_TILED;
        const int64_t n = ssr_codes_count(cam->width, cam->height, p->spp, a.flags);
        st = ensure(&ctx->codes, &ctx->codes_cap, n);
        if (st != SSR_OK) return st;
        codes = ctx->codes;
    }
    st = trace(ctx, g, p, &a, hiz_lay, codes, out_steps, s);
    if (st != SSR_OK) return st;
    a.out = out_rgb;
    return hip_status(ssr::launch_resolve(a, g->dtype, s));
}

int ssr_shade_static(const ssr_camera* cam, const ssr_gbuffer* g, const ssr_env* env,
                     const ssr_params* p, float* out_rgb, int32_t* out_hits, int32_t* out_steps,
                     void* stream) {
    ssr::ShadeArgs a;
    ssr::EnvLayout env_lay;
    ssr::HizLayout hiz_lay;
    int st = ssr::fill_args(cam, g, env, p, true, &a, &env_lay, &hiz_lay);
    if (st != SSR_OK) return st == 1 ? SSR_OK : st;
    if (!out_rgb) return SSR_E_ARG;
    int device = -1;
    if (hipGetDevice(&device) != hipSuccess) {
        (void)hipGetLastError();
        return SSR_E_HIP;
    }
    StaticDevice sd;
    st = static_device(device, &sd);
    if (st != SSR_OK) return st;
    // the workspace: counter, then whatever the caller does not supply
    auto align = [](int64_t n) { return (n + 255) / 256 * 256; };
    int64_t off = 256;
    int64_t o_hiz = -1, o_codes = -1, o_mips = -1;
    if (p->march == SSR_MARCH_HIZ && !g->hiz) {
        o_hiz = off;
        off += align(hiz_lay.total * 16);
    }
    if (!out_hits) {
        if (!out_steps) a.flags |= SSR_CODES_TILED;
        o_codes = off;
        off += align(ssr_codes_count(cam->width, cam->height, p->spp, a.flags) * 4);
    }
    if (!env->mips) {
        o_mips = off;
        off += align(env_lay.total * 16);
    }
    if (off > SSR_STATIC_SCRATCH_BYTES) return SSR_E_SCRATCH;
    // (from here on the array is addressed through sd.ptr only)
    char* base = sd.ptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    a.tile_counter = reinterpret_cast<int*>(base);
    if (o_mips >= 0) {
        st = hip_status(ssr::launch_env_mips(env->rgb, env_lay, reinterpret_cast<float4*>(base + o_mips), s));
        if (st != SSR_OK) return st;
        a.env = reinterpret_cast<const float4*>(base + o_mips);
    } else {
        a.env = reinterpret_cast<const float4*>(env->mips);
    }
    a.hiz = reinterpret_cast<const float4*>(g->hiz);
    if (o_hiz >= 0) {
        float4* hiz = reinterpret_cast<float4*>(base + o_hiz);
        st = hip_status(ssr::launch_hiz(g->depth, hiz_lay, p->thickness, hiz, s));
        if (st != SSR_OK) return st;
        a.hiz = hiz;
    }
    a.codes = o_codes >= 0 ? reinterpret_cast<int32_t*>(base + o_codes) : out_hits;
    a.steps = out_steps;
    st = hip_status(ssr::launch_trace(a, g->dtype, p->march, sd.cu_count, s));
    if (st != SSR_OK) return st;
    a.out = out_rgb;
    return hip_status(ssr::launch_resolve(a, g->dtype, s));
}

int ssr_depth_normals(const ssr_camera* cam, const float* depth, int32_t dtype, void* normal_rough,
                      void* stream) {
    int st = check_camera(cam);
    if (st != SSR_OK) return st;
    if (dtype != SSR_F32 && dtype != SSR_F16 && dtype != SSR_BF16) return SSR_E_DTYPE;
    if (cam->width == 0 || cam->height == 0) return SSR_OK;
    if (!depth || !normal_rough) return SSR_E_ARG;
    ssr::ShadeArgs a;
    camera_args(cam, &a);
    a.depth = depth;
    return hip_status(ssr::launch_depth_normals(a, dtype, normal_rough,
                                                static_cast<hipStream_t>(stream)));
}

int ssr_brdf_lut(int32_t n, float* lut, void* stream) {
    if (n < 2 || n > 1024 || !lut) return SSR_E_ARG;
    return hip_status(ssr::launch_brdf_lut(reinterpret_cast<float2*>(lut), n, kLutK,
                                           static_cast<hipStream_t>(stream)));
}

int ssr_first_pass(ssr_ctx* ctx, const ssr_camera* cam, const ssr_gbuffer* g, const ssr_env* env,
                   void* out_radiance, void* stream) {
    if (!ctx || !g) return SSR_E_ARG;
    ssr_gbuffer gg = *g;
    gg.radiance = out_radiance;  // the output; the input radiance is not read
    ssr::ShadeArgs a;
    ssr::EnvLayout env_lay;
    ssr::HizLayout hiz_lay;
    int st = ssr::fill_args(cam, &gg, env, nullptr, true, &a, &env_lay, &hiz_lay);
    if (st != SSR_OK) return st == 1 ? SSR_OK : st;
    if (hipSetDevice(ctx->device) != hipSuccess) return SSR_E_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!ctx->lut) {
        // built once; the wait makes it visible to calls on any stream
        void* p = nullptr;
        if (hipMalloc(&p, sizeof(float2) * kLutN * kLutN) != hipSuccess) {
            (void)hipGetLastError();
            return SSR_E_NOMEM;
        }
        if (ssr::launch_brdf_lut(static_cast<float2*>(p), kLutN, kLutK, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            (void)hipFree(p);
            return SSR_E_HIP;
        }
        ctx->lut = static_cast<float2*>(p);
    }
    st = env_mips(ctx, env, env_lay, s, &a.env);
    if (st != SSR_OK) return st;
    return hip_status(ssr::launch_first_pass(a, g->dtype, ctx->lut, kLutN, out_radiance, s));
}

}  // extern "C"
