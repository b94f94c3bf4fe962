/*
 * ssr.h - screen-space GGX shading of a G-buffer on AMD Instinct MI355X (gfx950).
 *
 * The operation (3D Gaussian Inverse Rendering with Approximated Global
 * Illumination, Sec. 3.2 and Sec. 3.3): for every pixel of a deferred
 * G-buffer (Eq. g-buffer: depth, normal, albedo, roughness, metallic, plus the
 * first-pass radiance c1 of Sec. 3.2), output
 *
 *     c = c_d + c_s'
 *
 * where c_d = (1 - m) a E_lambda(n) is the direct diffuse light read from an
 * HDR environment map at the roughness mip level lambda = log2(1 + rho)
 * lambda_max (Sec. 3.2, "Shading"), and c_s' is the Monte-Carlo estimate of
 * the specular integral (Sec. 3.3, the estimator over N_s sampled rays): each
 * sample draws a GGX visible normal, reflects the view direction about it,
 * marches the ray in screen space against the depth buffer (Sec. 3.3 and
 * Appendix D, Algorithm 1, in fixed steps; or this library's own
 * hierarchical traversal of the same hit test over a min-max depth pyramid,
 * which the paper does not describe), and
 * weights the radiance found at the hit (c1 of the hit pixel; the environment
 * when the ray leaves the screen) by F(wo.h) G1(n.l) (Appendix B with
 * alpha = rho).
 *
 * Conventions.  World space is right-handed, +y up.  View coordinates of a
 * world point x: X = (x-pos).right, Y = (x-pos).up, Z = (x-pos).forward; Z is
 * the linear depth.  Pixel (i, j) covers [i, i+1) x [j, j+1), row 0 on top,
 * projects as px = cx + fx X/Z, py = cy - fy Y/Z and is un-projected at its
 * centre.  The environment is equirectangular: direction d maps to
 * u = 1/2 + atan2(d.x, -d.z)/(2 pi), v = acos(d.y)/pi.
 *
 * Memory.  Every buffer pointer below is a DEVICE pointer on the context's
 * device, owned by the caller; the library never frees caller memory.  Work
 * is enqueued on `stream` (a hipStream_t passed as void*; NULL = the null
 * stream) and returns before it finishes: the caller synchronises.
 *
 * Errors.  Every call returns an ssr_status.  Arguments are checked before
 * anything is enqueued; a rejected call enqueues nothing.  A failure reported
 * by the HIP runtime is returned as SSR_E_HIP (an earlier asynchronous fault
 * may surface there).  Nothing is thrown across this interface.
 *
 * Threads.  An ssr_ctx is used by one host thread at a time, and calls made
 * with the same context on different streams must be ordered by the caller
 * (they share the context's workspace).
 */
#ifndef SSR_H
#define SSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ssr_ctx ssr_ctx;

typedef enum {
    SSR_OK = 0,
    SSR_E_ARG = -1,    /* a pointer, size, mode or parameter is invalid          */
    SSR_E_DTYPE = -2,  /* unknown G-buffer storage type                          */
    SSR_E_NOMEM = -3,  /* the context's workspace could not be allocated         */
    SSR_E_HIP = -4,    /* the HIP runtime reported an error                      */
    SSR_E_DEVICE = -5, /* no such device, or it is not a gfx950 device          */
    SSR_E_BUDGET = -6, /* the session's device-memory budget cannot hold it     */
    SSR_E_BUSY = -7,   /* the session is serving (or stopping): not allowed now  */
    SSR_E_TICKET = -8, /* no such request (never submitted, or already retired) */
    SSR_E_SCRATCH = -9,/* the frame's workspace exceeds the static scratch buffer
                          of ssr_shade_static (SSR_STATIC_SCRATCH_BYTES)          */
    SSR_PENDING = 1    /* the request has not finished yet                       */
} ssr_status;

/* Storage type of the three packed G-buffers (depth is always float32). */
typedef enum { SSR_F32 = 0, SSR_F16 = 1, SSR_BF16 = 2 } ssr_dtype;

/* March modes.  LINEAR: fixed world-space steps (Appendix D, Algorithm 1).
 * HIZ: exact first hit on the depth heightfield under the same hit test,
 * traversed over a min-max depth pyramid with at most max_steps iterations
 * (skip a cell the ray passes wholly in front of or wholly behind, descend,
 * or test a pixel: one each).  The paper marches in fixed steps only (Sec. 3.3
 * cites a DDA tracer); the hierarchical traversal is this library's design,
 * and with the cap lifted it returns the first crossing a pixel-by-pixel scan
 * of the segment finds. */
enum { SSR_MARCH_LINEAR = 0, SSR_MARCH_HIZ = 1 };

/* Flags: drop the direct diffuse term, or the Monte-Carlo specular term;
 * SSR_SAMPLER_NDF draws half vectors from the distribution of normals,
 * density D(h) (n.h) (Walter et al. 2007, the GGX sampling Sec. 3.3 cites),
 * instead of the visible normals: the same expectation, weights
 * F G1(n.wo) G1(n.l) (wo.h) / ((n.wo) (n.h)), which are not bounded by one
 * (u1 picks the azimuth, u2 the polar angle, tan^2 theta_h =
 * rho^2 u2 / (1 - u2)). */
enum { SSR_NO_DIRECT = 1u, SSR_NO_SPECULAR = 2u, SSR_SAMPLER_NDF = 4u };

/* Layout flag of the per-sample buffers (hit codes and iteration counts) of
 * ssr_shade, ssr_trace, ssr_resolve and ssr_shade_backward.  Without it they
 * are [H][W][spp] int32.  With SSR_CODES_TILED they are tile-major over 8 x 8
 * pixel tiles: [ceil(H/8) ceil(W/8)][spp][64] int32 (ssr_codes_count
 * entries), tile (tx, ty) at ty ceil(W/8) + tx, pixel (i, j) at
 * (j % 8) 8 + i % 8 inside its tile; entries of pixels outside the image are
 * not written.  The hierarchical trace writes this layout with far less
 * memory traffic (the rays a wave draws together land in a few cache lines);
 * ssr_shade uses it for its own workspace when out_hits is NULL.  The codes'
 * values are the same in both layouts. */
enum { SSR_CODES_TILED = 8u };

/* Per-sample hit codes written to out_hits (>= 0: hit pixel index j*W + i). */
enum {
    SSR_HIT_OFFSCREEN = -1,  /* left the screen or the ray segment: env read    */
    SSR_HIT_INVALID = -2,    /* sampled direction below the surface, or the
                                pixel faces away from the camera: weight 0     */
    SSR_HIT_BACKGROUND = -3, /* background pixel (depth not finite)            */
    SSR_HIT_CAP = -4,        /* iteration cap reached: env read                */
    SSR_HIT_SKIPPED = -5     /* SSR_NO_SPECULAR set                            */
};

typedef struct {
    int32_t width, height; /* pixels; 0 <= width, height <= 16384              */
    float pos[3];          /* camera position (world)                           */
    float rot[9];          /* rows: right, up, forward (world, orthonormal)     */
    float fx, fy, cx, cy;  /* pinhole intrinsics in pixels                      */
    float z_near;          /* rays are clipped where view depth reaches z_near  */
} ssr_camera;

typedef struct {
    const float* depth;       /* [H][W] float32 view-space linear depth, > 0;
                                 +inf marks background; no NaN                   */
    const void* normal_rough; /* [H][W][4] (n.x, n.y, n.z, roughness), world n,
                                 need not be unit length but must be non-zero   */
    const void* albedo_metal; /* [H][W][4] (a.r, a.g, a.b, metallic)             */
    const void* radiance;     /* [H][W][4] (c1.r, c1.g, c1.b, unused): the
                                 first-pass radiance read at hit pixels         */
    int32_t dtype;            /* ssr_dtype of the three [H][W][4] buffers        */
    const float* hiz;         /* NULL, or the pyramid ssr_hiz_build wrote for this
                                 depth buffer with the thickness of the
                                 ssr_params it is shaded with (then ssr_shade
                                 does not build it)                              */
} ssr_gbuffer;

typedef struct {
    const float* rgb;  /* [He][We][3] float32 equirect map, texel (x, y) centred at
                          u = (x+1/2)/We, v = (y+1/2)/He                          */
    int32_t width;     /* We = 2 * He                                             */
    int32_t height;    /* He, a power of two, 1 <= He <= 8192                     */
    const float* mips; /* NULL, or the buffer ssr_env_build_mips filled from this
                          exact map (then no mip chain is built per call)        */
} ssr_env;

typedef struct {
    int32_t spp;       /* samples per pixel N_s, 1..4096 (Sec. 3.3 uses 8)        */
    int32_t march;     /* SSR_MARCH_LINEAR or SSR_MARCH_HIZ                       */
    int32_t max_steps; /* linear: samples; hiz: iterations; 1..2^20               */
    float step_len;    /* linear: world-space step (> 0); unused by hiz          */
    float max_dist;    /* world-space ray length (> 0)                            */
    float thickness;   /* depth slab behind a surface that counts as a hit (>= 0) */
    uint64_t seed;     /* Philox key: (seed mod 2^32, seed >> 32)                 */
    uint32_t frame;    /* third Philox counter word                               */
    uint32_t flags;    /* SSR_NO_DIRECT | SSR_NO_SPECULAR | SSR_SAMPLER_NDF |
                          SSR_CODES_TILED                                        */
} ssr_params;

/* Create a context on HIP device `device` (must be gfx950).  The context owns
 * a grow-only workspace (depth pyramid, env mip chain).  *out is set to
 * NULL on failure. */
int ssr_ctx_create(int device, ssr_ctx** out);

/* Free the context and its workspace after waiting for the device.  NULL is
 * accepted. */
void ssr_ctx_destroy(ssr_ctx* ctx);

/* Shade one frame (Sec. 3.2 diffuse + Sec. 3.3 Monte-Carlo specular):
 * ssr_trace followed by ssr_resolve on `stream`.
 *   out_rgb   [H][W][3] float32, written: linear HDR c_d + c_s' (no tone map).
 *   out_hits  NULL or [H][W][spp] int32 (tile-major with SSR_CODES_TILED):
 *             per-sample hit pixel or SSR_HIT_* code (NULL: the codes go to
 *             the context's workspace, tile-major).
 *   out_steps NULL or int32 in the layout of out_hits: march iterations each
 *             sample used.
 * Sample s of pixel q = j*W + i draws Philox4x32-10 with counter
 * (q, s, frame, 0): u1 = (x0 >> 8) 2^-24 picks the azimuth, u2 = (x1 >> 8) 2^-24
 * the cap height of the visible-normal sample.  width or height 0 is a no-op;
 * W H must leave the depth pyramid below 4 GiB (about 200 Mpixels), and
 * ceil(W/8) ceil(H/8) spp must stay below 2^32 (2^38 codes: more than any
 * device memory holds), else SSR_E_ARG.  In hiz mode the depth pyramid is built in the context's
 * workspace unless gbuf->hiz supplies it; the env mip chain likewise unless
 * env->mips does.  Both builds run on `stream` before the kernels. */
int ssr_shade(ssr_ctx* ctx, const ssr_camera* cam, const ssr_gbuffer* gbuf,
              const ssr_env* env, const ssr_params* params, float* out_rgb,
              int32_t* out_hits, int32_t* out_steps, void* stream);

/* Bytes of the static device scratch buffer that ssr_shade_static uses as
 * its workspace (192 MiB, on every device the library runs on, held until
 * the process ends). */
#define SSR_STATIC_SCRATCH_BYTES (192ll << 20)

/* ssr_shade for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same frame as ssr_shade (the same kernels; bit for bit the same outputs),
 * with no context and no allocation: nothing here calls hipMalloc, hipFree or
 * an allocating library routine.  Its workspace lives in a file-scope
 * static device array of SSR_STATIC_SCRATCH_BYTES per device: the trace
 * kernel's work counter (256 B), then, unless the caller supplies them, the
 * depth pyramid (gbuf->hiz NULL: ssr_hiz_floats(W, H) floats), the
 * per-sample hit codes (out_hits NULL: ssr_codes_count(W, H, spp,
 * SSR_CODES_TILED) int32, or the public layout when out_steps is given) and
 * the env mip chain (env->mips NULL: ssr_env_mips_floats floats), each
 * starting on a 256-byte boundary.  A frame whose workspace does not fit is
 * refused with SSR_E_SCRATCH before anything is enqueued (1920 x 1080 at
 * 16 spp fits with every part in scratch, about 180 MB; 3840 x 2160 at
 * 16 spp needs the caller's out_hits).
 * The device is the calling thread's current HIP device (hipSetDevice);
 * `stream` must belong to it.  The first call on a device looks up the
 * array's address there (hipGetSymbolAddress) and checks that it is a
 * gfx950 device (SSR_E_DEVICE otherwise); ssr_ctx_create does the same for
 * its device, so a caller can do it before any graph capture.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents; the counter is reset by a kernel at the start of each
 * frame and the other parts are written before they are read.  Calls whose
 * work overlaps on one device (different streams, or different host
 * threads, without ordering between them) race on the array: order them.
 * Other arguments, outputs and errors as ssr_shade. */
int ssr_shade_static(const ssr_camera* cam, const ssr_gbuffer* gbuf, const ssr_env* env,
                     const ssr_params* params, float* out_rgb, int32_t* out_hits,
                     int32_t* out_steps, void* stream);

/* The march half of ssr_shade (Sec. 3.3 sampling; the march of Appendix D,
 * Algorithm 1, or the library's hierarchical march, per params->march): write
 * every sample's hit code to out_hits ([H][W][spp] int32, or tile-major with
 * SSR_CODES_TILED; required) and,
 * unless NULL, its iteration count to out_steps.  Reads depth and the
 * normal/roughness buffer (and gbuf->hiz); the other buffers and the
 * environment are not used.  Same validation as ssr_shade. */
int ssr_trace(ssr_ctx* ctx, const ssr_camera* cam, const ssr_gbuffer* gbuf,
              const ssr_params* params, int32_t* out_hits, int32_t* out_steps, void* stream);

/* The shading half of ssr_shade (Sec. 3.2, Sec. 3.3 estimator): out_rgb from
 * per-sample hit codes `hits` ([H][W][spp] int32, or tile-major with
 * SSR_CODES_TILED; as ssr_trace writes them, or
 * any codes to replay).  The sample directions are drawn again from the same
 * Philox counters; a code >= 0 reads the first-pass radiance of that pixel,
 * SSR_HIT_OFFSCREEN and SSR_HIT_CAP the environment along the sample; a code
 * outside [SSR_HIT_SKIPPED, W H) counts as SSR_HIT_INVALID (weight 0). */
int ssr_resolve(ssr_ctx* ctx, const ssr_camera* cam, const ssr_gbuffer* gbuf,
                const ssr_env* env, const ssr_params* params, const int32_t* hits,
                float* out_rgb, void* stream);

/* The adjoint of ssr_resolve (the shading with the hit selection held fixed;
 * the paper differentiates its shading with the screen-space tracing treated
 * as a fixed selection): given the hit codes `hits` of a frame ([H][W][spp],
 * or tile-major with SSR_CODES_TILED) and
 * the gradient of a loss with respect to its image, grad_rgb [H][W][3], write
 * or accumulate the gradient with respect to the inputs:
 *   g_normal_rough [H][W][4]: written, d/d(n.x, n.y, n.z, rho) of the stored
 *                  values (n before normalisation; rho 0 outside [0, 1]);
 *   g_albedo_metal [H][W][4]: written, d/d(a.r, a.g, a.b, m) (m 0 outside
 *                  [0, 1]); zero for background pixels;
 *   g_env          [He][We][3]: ADDED to, d/d of every level-0 texel of the
 *                  map (through the mip chain of the direct term, the
 *                  environment read by rays that miss, and the background);
 *   g_radiance     [H][W][4]: channels 0..2 ADDED to, d/d first-pass
 *                  radiance of each hit pixel; channel 3 untouched.
 * Each output may be NULL.  Derivatives flow through the sampled directions
 * (visible-normal sample, reflection), Fresnel, masking, the roughness mip
 * level and the bilinear weights of every environment lookup; a bilinear
 * lookup is differentiated inside its texel cell, so the derivative is
 * discontinuous across texel boundaries, as the function's is.  Codes
 * outside [SSR_HIT_SKIPPED, W H) count as SSR_HIT_INVALID.  The adjoint
 * covers the visible-normal sampler (SSR_SAMPLER_NDF: SSR_E_ARG).  Other
 * arguments and errors as ssr_shade. */
int ssr_shade_backward(ssr_ctx* ctx, const ssr_camera* cam, const ssr_gbuffer* gbuf,
                       const ssr_env* env, const ssr_params* params, const int32_t* hits,
                       const float* grad_rgb, float* g_normal_rough, float* g_albedo_metal,
                       float* g_env, float* g_radiance, void* stream);

/* Entries of a per-sample buffer (hit codes, iteration counts) of a
 * width x height frame with spp samples in the layout `flags` selects
 * (SSR_CODES_TILED or not); 0 for negative sizes. */
int64_t ssr_codes_count(int32_t width, int32_t height, int32_t spp, uint32_t flags);

/* Number of floats of the env mip-chain buffer for a We x He map (0 if the
 * dimensions are invalid). */
int64_t ssr_env_mips_floats(int32_t width, int32_t height);

/* Fill `mips` (ssr_env_mips_floats floats) with levels 0..log2(He) of the map:
 * level k is the 2x2 box mean of level k-1 (Sec. 3.2, SampleEnvMap mip levels),
 * stored as RGBA float32 texels, level after level.  The layout is private to
 * the library; pass the buffer back through ssr_env.mips. */
int ssr_env_build_mips(const float* rgb, int32_t width, int32_t height, float* mips,
                       void* stream);

/* Number of floats of the depth pyramid of a W x H depth buffer (0 for an
 * empty image, or one whose pyramid would exceed 4 GiB: about 200 Mpixels,
 * beyond which the hierarchical march is unavailable and ssr_shade returns
 * SSR_E_ARG for it). */
int64_t ssr_hiz_floats(int32_t width, int32_t height);

/* Fill `pyramid` (ssr_hiz_floats floats) with levels 0..top of the depth
 * pyramid the hierarchical march traverses (the library's own acceleration
 * structure for the hit test of Sec. 3.3; the paper uses none), in inverse
 * depth over each pixel's hit slab [D, D + thickness]:
 * level 0 is W x H, level L has ceil(W_{L-1}/2) x ceil(H_{L-1}/2) texels and
 * the last level is 1 x 1.  The pair of a level-0 texel is
 * (1/D, 1/(D + thickness)), both correctly rounded float32 quotients (with
 * D + thickness rounded first); the pair of a texel above holds the maximum
 * of the first and the minimum of the second over its children, i.e. one
 * over the smallest depth and one over the largest depth plus thickness of
 * the pixels it covers.  Background (D = +inf) gives (0, 0).  Each texel is
 * stored as four floats, its own pair and then the pair of its parent (the
 * texel (x/2, y/2) one level up; the top texel repeats its own), level after
 * level.  A level of w x h texels takes w * 2 ceil(h/2) slots: its rows go in
 * pairs, each pair column by column, texel (x, y) in slot
 * 2 (w floor(y/2) + x) + (y mod 2), so that one 128-byte line holds a 4 x 2
 * block; the padding slots of a level with odd h are left unwritten.  Depths
 * must be positive, thickness finite and >= 0 (else SSR_E_ARG).  Pass the
 * buffer to ssr_shade through ssr_gbuffer.hiz to reuse it with the same
 * thickness. */
int ssr_hiz_build(const float* depth, int32_t width, int32_t height, float thickness,
                  float* pyramid, void* stream);

/* ------------------------------------------------------------------------
 * First shading pass (Sec. 3.2, "Shading"): the producer of the radiance c1
 * that ssr_shade reads at hit pixels.
 * ------------------------------------------------------------------------ */

/* Depth normals (Sec. 3.2, the G-buffer: the shading normal taken from the depth buffer by
 * finite differences).  Each surface pixel's world point is the camera ray
 * through its centre at its depth; the tangents along x and y are the central
 * differences of the points of its two neighbours on that axis where both are
 * surface pixels inside the image, the one-sided difference where only one is;
 * the normal is their cross product, normalised and turned to face the camera
 * (n . (camera - point) > 0).  A pixel with no neighbour on an axis, or a zero
 * cross product, gets the unit vector toward the camera.  Background pixels
 * (depth +inf) get (0, 0, 0).
 * depth: [H][W] float32 device buffer (as ssr_gbuffer.depth); normal_rough:
 * [H][W][4] device buffer in storage type `dtype` (ssr_dtype): channels 0..2
 * are written (rounded to nearest even for the 16-bit types), channel 3 (the
 * roughness) is left as it is, so the G-buffer's own buffer can be passed.
 * The camera's rotation rows must be orthonormal.  SSR_E_DTYPE for an unknown
 * dtype; SSR_E_ARG for a bad camera or a NULL buffer of a non-empty image. */
int ssr_depth_normals(const ssr_camera* cam, const float* depth, int32_t dtype, void* normal_rough,
                      void* stream);

/* The BRDF table of the split sum (Sec. 3.2, Eq. split-sum, and Appendix C):
 * with Schlick's Fresnel F = F0 + (1 - F0) Fc, Fc = (1 - wo.h)^5, the BRDF
 * integral over the hemisphere is F0 A + B with A the integral of
 * f/F (1 - Fc) cos and B that of f/F Fc cos.  lut: [n][n][2] float32 device
 * buffer, row r for roughness (r + 1/2)/n, column c for n.v = (c + 1/2)/n,
 * entries (A, B).  Each entry is the mean of G1(n.l) (1 - Fc) and G1(n.l) Fc
 * (zero where n.l <= 0) over the 64 x 64 visible-normal samples
 * (Dupuy & Benyoub 2023) at the stratified cell centres
 * u = ((a + 1/2)/64, (b + 1/2)/64) (a fixed rule: the table is deterministic),
 * computed in float64 and rounded to float32.  2 <= n <= 1024 (else
 * SSR_E_ARG). */
int ssr_brdf_lut(int32_t n, float* lut, void* stream);

/* First-pass radiance (Sec. 3.2): per surface pixel, c1 = c_d + c_s with
 * c_d = (1 - m) a E_lambda(n) (as the direct term of ssr_shade) and
 * c_s = E_lambda(r) (F0 A + B), r = 2 (v.n) n - v the mirror direction,
 * F0 = lerp(0.04, a, m), and (A, B) read bilinearly (texel centres at
 * (i + 1/2)/128, clamped) from the 128 x 128 table ssr_brdf_lut builds, at
 * (n.v, roughness); c_s = 0 where n.v <= 0.  E_lambda is the environment
 * mip chain read at lambda = log2(1 + roughness) lambda_max.  Background
 * pixels get 0.  Reads gbuf depth, normal_rough and albedo_metal (gbuf
 * radiance and hiz are not read); writes out_radiance, a [H][W][4] device
 * buffer in gbuf->dtype: (c1.r, c1.g, c1.b, 0), rounded to nearest even for
 * the 16-bit types, the layout ssr_gbuffer.radiance takes.  out_radiance must
 * not overlap the buffers read.  The context builds the table on its first
 * call (and waits for it there).  Errors as ssr_shade. */
int ssr_first_pass(ssr_ctx* ctx, const ssr_camera* cam, const ssr_gbuffer* gbuf,
                   const ssr_env* env, void* out_radiance, void* stream);

/* Philox4x32-10 (Salmon et al., SC'11) of n counters: ctr [n][4], key [n][2],
 * out [n][4], all uint32 device buffers.  The same generator ssr_shade draws
 * its samples from. */
int ssr_philox4x32_10(const uint32_t* ctr, const uint32_t* key, int64_t n, uint32_t* out,
                      void* stream);

/* Static description of a status code. */
const char* ssr_status_string(int status);

/* ------------------------------------------------------------------------
 * Serving session.  Scenes (camera, G-buffer, environment) are copied once
 * into device memory the session owns; render requests then name a scene and
 * the per-frame parameters.  A request waits until a slot is free and the
 * session's device-memory budget holds its workspace (depth pyramid and
 * per-sample hit codes: ssr_session_request_bytes); admitted requests run
 * concurrently, each on its own stream, and new requests are admitted as
 * earlier ones finish (continuous batching).  A frame is a fixed chain of
 * kernels (depth pyramid, work-counter reset, trace, resolve) whose shape
 * depends only on the image size, march mode and storage type: each slot
 * keeps one instantiated HIP graph per such shape class, built on the class's
 * first request, and replays it for later requests of the class with the
 * kernel nodes' parameters (buffers, samples, seed, frame, flags) replaced.  Waiting requests are admitted
 * oldest first; one that does not fit may be overtaken by later ones that do,
 * at most max_bypass times.  Each result is the frame ssr_shade renders for
 * the same scene and parameters, bit for bit, whatever else runs beside it.
 *
 * For callers that serve many frames from resident scenes (the persistent
 * request loop of the method's serving use): submit and poll are
 * thread-safe; add_scene is allowed only before the first submit.
 * ------------------------------------------------------------------------ */
typedef struct ssr_session ssr_session;

/* Session flag: launch each frame's kernels directly instead of replaying a
 * captured HIP graph (for comparison; the frames are the same). */
enum { SSR_SESSION_DIRECT = 1u };

typedef struct {
    int64_t hbm_budget_bytes; /* device memory for scenes and request workspaces  */
    int32_t max_slots;        /* requests on the device at once, 1..64            */
    int32_t max_bypass;       /* times the oldest waiting request may be overtaken */
    uint32_t flags;           /* 0 or SSR_SESSION_DIRECT                           */
} ssr_session_cfg;

typedef struct {
    int32_t scene_id;   /* from ssr_session_add_scene                             */
    ssr_params params;  /* as for ssr_shade                                       */
    float* out_rgb;     /* [H][W][3] float32 device buffer of the scene's size,
                           caller-owned; written when the request finishes and
                           must stay valid until poll / wait reports it        */
} ssr_request;

typedef struct {
    int32_t status;          /* SSR_OK, or the error the request's work hit     */
    double t_submit;         /* seconds since the session was created, host    */
    double t_admit;          /*   monotonic clock: submitted, launched, seen    */
    double t_done;           /*   finished by the session                       */
    int64_t workspace_bytes; /* device memory the request held                  */
} ssr_result;

typedef struct {
    int64_t scene_bytes;     /* device memory held by the resident scenes         */
    int64_t arena_bytes;     /* workspace arena (0 before the first submit)        */
    int64_t arena_used;      /* workspace held by running requests now             */
    int32_t running;         /* requests on the device now                         */
    int32_t waiting;         /* requests queued for admission                      */
    int64_t completed;       /* requests finished so far                           */
} ssr_session_stats;

/* Create a session on gfx950 device `device`.  Nothing is allocated until
 * scenes are added; the first submit reserves the rest of the budget as the
 * workspace arena and starts the session's worker thread. */
int ssr_session_create(int device, const ssr_session_cfg* cfg, ssr_session** out);

/* Copy a scene (all device buffers, as for ssr_shade; gbuf->hiz and env->mips
 * are ignored) into session memory and build its env mip chain, on `stream`,
 * then wait for the copy.  The copy counts against the budget
 * (SSR_E_BUDGET).  Only before the first submit (else SSR_E_BUSY). */
int ssr_session_add_scene(ssr_session* s, const ssr_camera* cam, const ssr_gbuffer* gbuf,
                          const ssr_env* env, int32_t* scene_id, void* stream);

/* Device-memory workspace a request needs, in bytes (-1 if invalid). */
int64_t ssr_session_request_bytes(ssr_session* s, const ssr_request* req);

/* Queue a request; *ticket names it.  SSR_E_BUDGET if its workspace can never
 * fit the budget left after the scenes. */
int ssr_session_submit(ssr_session* s, const ssr_request* req, uint64_t* ticket);

/* SSR_OK and *result once the request has finished (the ticket is then
 * retired), SSR_PENDING before, SSR_E_TICKET for an unknown ticket. */
int ssr_session_poll(ssr_session* s, uint64_t ticket, ssr_result* result);

/* As poll, but blocks until the request has finished. */
int ssr_session_wait(ssr_session* s, uint64_t ticket, ssr_result* result);

/* A snapshot of the session's occupancy. */
int ssr_session_get_stats(ssr_session* s, ssr_session_stats* out);

/* Stop the session: waiting requests are dropped, running ones finish, all
 * session memory is freed.  No other call on `s` may be in progress or
 * follow.  NULL is accepted. */
void ssr_session_destroy(ssr_session* s);

#ifdef __cplusplus
}
#endif

#endif /* SSR_H */
